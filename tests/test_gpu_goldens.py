"""Device credits against stored oracle results of larger instances
(tests/golden/credit_goldens.json, written by tests/golden/make_credit_goldens.py
from the CPU oracle alone): R-MAT 2^18 (and 2^20 when stored), the uniform game
at 2^16, tori of 128^2 and 256^2 and the first 32 serving-stream games, at
sizes where running the oracle inside a test would take minutes.

Each game is regenerated and checked against the stored instance hash, solved
through the C-ABI in the launch shape bench.py uses for its class (tuned shape,
renumbering and cut tiles automatic), plain and with TOP seeding, and its
credits are compared element by element through their SHA-256 (on a mismatch
the stored samples name differing vertices)."""
import hashlib
import json
import os

import numpy as np
import pytest

from golden.make_credit_goldens import instances
from paper_1710_03647_amd import eg, tune

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "credit_goldens.json")))
GiB = 1 << 30


def make(name):
    """Regenerate an instance with the golden script's own generator call."""
    call, gen = instances()[name]
    entry = GOLD[name]
    assert call == entry["generator"]
    game = gen()
    assert game.sha256() == entry["instance_sha256"], f"{call}: instance differs from the stored one"
    return game


def check(name, f):
    entry = GOLD[name]
    got = hashlib.sha256(np.ascontiguousarray(f, dtype="<i8").tobytes()).hexdigest()
    if got != entry["credits_sha256"]:
        bad = [(i, int(f[i]), v) for i, v in entry["samples"] if int(f[i]) != v]
        top = int(np.sum(f == eg.EG_TOP))
        raise AssertionError(f"{name}: credits differ from the oracle's (TOP {top} vs {entry['top']}; "
                             f"sampled vertices differing: {bad[:8]})")


LARGE = [k for k in ("rmat18", "rmat20", "uniform16", "torus128", "torus256") if k in GOLD]
STREAM = sorted((k for k in GOLD if k.startswith("stream")), key=lambda k: int(k[6:]))


@pytest.mark.parametrize("seeded", [0, 1], ids=["plain", "seeded"])
@pytest.mark.parametrize("name", LARGE)
def test_large_instance(name, seeded):
    if name == "torus256" and not seeded:
        pytest.skip("the 256^2 torus needs millions of rounds either way: one solve (the seeded one) is checked")
    game = make(name)
    shape = tune.config_for(game)
    with eg.Context(0, top_seeding=seeded, **shape) as ctx:
        with ctx.create(game) as g:
            f, st, rc = g.solve()
    print(f"{name} seeded={seeded}: rounds {st['rounds']}, t_solve {st['t_solve']:.2f} s", flush=True)
    check(name, f)


@pytest.mark.parametrize("seeded", [0, 1], ids=["plain", "seeded"])
def test_stream_games_one_at_a_time(seeded):
    with eg.Context(0, top_seeding=seeded) as ctx:
        for name in STREAM:
            game = make(name)
            with ctx.create(game) as g:
                f, st, rc = g.solve()
            check(name, f)


@pytest.mark.parametrize("seeded", [0, 1], ids=["plain", "seeded"])
def test_stream_games_served_together(seeded):
    """The 32 stream games submitted at once to a server with 8 slots: each
    game's credits in the mix are the oracle's."""
    games = {name: make(name) for name in STREAM}
    with eg.Context(0, hbm_budget_bytes=2 * GiB, max_slots=8, top_seeding=seeded) as ctx:
        tickets = {name: ctx.submit(g) for name, g in games.items()}
        for name, t in tickets.items():
            rc, f, st = ctx.wait(t, games[name].n)
            check(name, f)
