"""The pins are strong enough: each plausible mistake planted in a copy of the
oracle source (CPU only) is caught by at least one pin.

Each mutation is a textual edit of ``oracle/eg_oracle.c`` that must match the
source exactly once, so the list stays in step with the oracle.
"""
import os

import numpy as np
import pytest

import pins
from oracle import oracle

MUTANTS = {
    # the codomain cap at "strictly above the bound" becomes "at or above"
    "cap_ge": ("if (a != ORC_TOP && a > bound) return ORC_TOP;",
               "if (a != ORC_TOP && a >= bound) return ORC_TOP;"),
    # the (-) operator loses its floor at 0
    "no_floor": ("return d > 0 ? d : 0;", "return d;"),
    # the (-) operator adds the weight instead of subtracting it
    "sign": ("int64_t d = a - b;", "int64_t d = a + b;"),
    # TOP is not absorbing under (-)
    "top_not_absorbing": ("if (a == ORC_TOP) return ORC_TOP;\n  int64_t d", "int64_t d"),
    # min and max swapped between the players
    "players_swapped": ("} else if (owner[v] == 0) {", "} else if (owner[v] != 0) {"),
    # player 1 takes min as well
    "both_min": ("      if (t > acc) acc = t; /* player 1: max */",
                 "      if (t < acc) acc = t; /* player 1: max */"),
    # the lift reads the source instead of the target of each edge
    "reads_source": ("int64_t t = clamp_to_codomain(ominus(f[tgt[e]], (int64_t)w[e]), bound);",
                     "int64_t t = clamp_to_codomain(ominus(f[v], (int64_t)w[e]), bound);"),
    # successors enqueued instead of predecessors
    "pushes_self": ("      psrc[slot] = v;", "      psrc[slot] = u;"),
    # initial list conditions of the two players exchanged
    "init_swapped": ("return owner[v] == 0 ? all_neg : some_neg;",
                     "return owner[v] == 0 ? some_neg : all_neg;"),
    # bound one vertex short
    "bound_short": ("return (int64_t)(n - 1) * (int64_t)W;", "return (int64_t)(n - 2) * (int64_t)W;"),
    # the first edge of each row is skipped
    "skip_first_edge": ("for (int64_t e = off[v]; e < off[v + 1]; e++) {\n    int64_t t",
                        "for (int64_t e = off[v] + 1; e < off[v + 1]; e++) {\n    int64_t t"),
    # the last edge of each row is skipped
    "skip_last_edge": ("for (int64_t e = off[v]; e < off[v + 1]; e++) {\n    int64_t t",
                       "for (int64_t e = off[v]; e + 1 < off[v + 1]; e++) {\n    int64_t t"),
}


def _battery(solve):
    """Run the pins; return the name of the first one that fails, or None."""
    checks = [("brute", lambda: pins.pin_brute(solve, count=400, seed0=70_000))]
    checks += [(p.__name__, (lambda p=p: p(solve))) for p in pins.CLOSED_FORMS]
    for g in pins.medium_games()[:2]:
        checks.append(("fixpoint", lambda g=g: pins.pin_fixpoint(g, solve(g), (g.n - 1) * g.W)))
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            return name
    return None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(oracle.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation {name} no longer matches the oracle source"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = oracle.build(force=True, src=str(msrc), out=str(tmp_path / f"lib_{name}.so"))
    solve = lambda g, **kw: oracle.solve(g, lib_path=lib, max_lifts=2_000_000, **kw).f
    caught = _battery(solve)
    assert caught is not None, f"no pin detects mutant {name}"


# mistakes in the strategy read off the measure (Lemma 1)
STRATEGY_MUTANTS = {
    # the last edge that achieves f(v) instead of the first
    "strategy_last": ("        choice[v] = (int32_t)(e - off[v]);\n        break;",
                      "        choice[v] = (int32_t)(e - off[v]);"),
    # only edges strictly below f(v) count
    "strategy_strict": ("if (term != ORC_TOP && term <= f[v]) {", "if (term != ORC_TOP && term < f[v]) {"),
    # the global edge index instead of the index within the row
    "strategy_global": ("choice[v] = (int32_t)(e - off[v]);", "choice[v] = (int32_t)e;"),
    # player-1 vertices get a choice too
    "strategy_p1": ("if (owner[v] != 0 || f[v] == ORC_TOP) continue;", "if (f[v] == ORC_TOP) continue;"),
    # the weight is added instead of subtracted
    "strategy_sign": ("int64_t term = clamp_to_codomain(ominus(f[tgt[e]], (int64_t)w[e]), bound);",
                      "int64_t term = clamp_to_codomain(ominus(f[tgt[e]], -(int64_t)w[e]), bound);"),
}


def _strategy_battery(strategy):
    for name, fn in [("cases", lambda: pins.pin_strategy_cases(strategy)),
                     ("brute", lambda: pins.pin_strategy_brute(strategy, count=300))]:
        try:
            fn()
        except AssertionError:
            return name
    return None


@pytest.mark.parametrize("name", sorted(STRATEGY_MUTANTS))
def test_strategy_mutant_is_caught(name, tmp_path):
    src = open(oracle.SRC).read()
    old, new = STRATEGY_MUTANTS[name]
    assert src.count(old) == 1, f"mutation {name} no longer matches the oracle source"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = oracle.build(force=True, src=str(msrc), out=str(tmp_path / f"lib_{name}.so"))
    caught = _strategy_battery(lambda g, f: oracle.strategy(g, f, lib_path=lib)[0])
    assert caught is not None, f"no pin detects mutant {name}"


def test_unmutated_strategy_passes_battery():
    assert _strategy_battery(lambda g, f: oracle.strategy(g, f)[0]) is None


def test_unmutated_passes_battery():
    assert _battery(lambda g, **kw: oracle.solve(g, **kw).f) is None
