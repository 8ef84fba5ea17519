"""The benchmarked configurations at their full sizes, in the launch shapes
bench.py times.  The oracle cannot finish these, so they are checked through
properties that hold at any size: the result is a fixpoint of Def. 6 with
finite values in [0, B] (I1, I2); seeded and plain solves agree bit for bit;
full-frontier rounds from the result change nothing in every round
representation; and a budgeted solve stops at a post-fixpoint (f <= lift(f))."""
import numpy as np
import pytest

import pins
from paper_1710_03647_amd import eg, synth, tune

pytestmark = pytest.mark.gpu
TOP = pins.TOP


def solve(game, **cfg):
    with eg.Context(0, **cfg) as c:
        with c.create(game) as g:
            f, st, rc = g.solve(allow_timeout=True)
    return f, st, rc


def bound_of(game):
    return (game.n - 1) * game.W


def test_uniform_full_seeded_equals_plain():
    game = synth.gen_uniform_full()
    shape = tune.config_for(game)
    fs, sts, _ = solve(game, top_seeding=1, **shape)
    pins.pin_fixpoint(game, fs, bound_of(game), "uniform 2^20 seeded")
    fp, stp, _ = solve(game, **shape)
    pins.expect_equal(fp, fs, "uniform 2^20 plain against seeded")
    assert sts["seeded"] > 0 and stp["rounds"] > 1000 * sts["rounds"]


@pytest.mark.parametrize("label,over", [("unsliced", {}), ("uncut", {"seg_edges": -1}), ("sliced", {"partition": 2}),
                                        ("slice-major", {"partition": 3})])
def test_rmat_full_fixpoint_is_stable(label, over):
    game = synth.gen_rmat_full()
    shape = dict(tune.config_for(game), **over)
    f, st, _ = solve(game, top_seeding=1, **shape)
    pins.pin_fixpoint(game, f, bound_of(game), "R-MAT 2^22")
    with eg.Context(0, **shape) as c:
        with c.create(game) as g:
            g.set_measure(f)
            f1, st1, rc = g.solve(max_rounds=1, resume=True, allow_timeout=True)
    assert st1["lifts"] == game.n and st1["changes"] == 0
    pins.expect_equal(f1, f, f"R-MAT 2^22 one full round from the fixpoint ({label})")


def test_torus_full_budget_is_a_post_fixpoint():
    game = synth.gen_torus_full()
    with eg.Context(0, max_rounds=20000) as c:
        with c.create(game) as g:
            f, st, rc = g.solve(allow_timeout=True)
    assert rc == eg.EG_ETIMEDOUT
    lifted = pins.lift_all_numpy(game, f, bound_of(game))
    assert np.all(f <= lifted), "a stop point of the iteration from 0 is below its own lift"
    fin = f[f != TOP]
    assert fin.min() >= 0 and fin.max() <= bound_of(game)


@pytest.mark.parametrize("which", ["uniform", "rmat"])
def test_full_strategy_properties(which):
    """Player 0's strategy at full size, in the benchmarked launch shape: -1 exactly
    on player-1 and TOP vertices, else the first edge that witnesses Def. 5."""
    game = synth.gen_uniform_full() if which == "uniform" else synth.gen_rmat_full()
    with eg.Context(0, top_seeding=1, **tune.config_for(game)) as c:
        with c.create(game) as g:
            f, st, rc = g.solve()
            choice, t = g.strategy()
    pins.pin_fixpoint(game, f, bound_of(game), f"{which} seeded")
    pins.pin_strategy_properties(game, f, bound_of(game), choice, f"{which} strategy")
    assert t > 0
