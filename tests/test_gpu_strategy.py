"""Player 0's positional strategy on the device (eg_strategy) against the CPU
oracle's, index for index (Def. 5, Lemma 1).

Both sides read the strategy off their own least fixpoint, so the comparison
also repeats the credit parity.  Long rows (a wave per row) are exercised with
hand-built hubs whose witness sits at each boundary of the lane and wave
scans; renumbered and cut-tile launch shapes must give the same indices."""
import numpy as np
import pytest

import pins
from paper_1710_03647_amd import eg, synth

pytestmark = pytest.mark.gpu
TOP = pins.TOP


@pytest.fixture(scope="module")
def ctx():
    c = eg.Context(0)
    yield c
    c.close()


def gpu_strategy(ctx, game):
    with ctx.create(game) as g:
        f, st, rc = g.solve()
        choice, t = g.strategy()
    return f, choice, t


def check(ctx, oracle_mod, game, what):
    f, choice, _ = gpu_strategy(ctx, game)
    want_f = oracle_mod.solve(game).f
    pins.expect_equal(f, want_f, f"{what} credits")
    want, missing = oracle_mod.strategy(game, want_f)
    assert missing == 0
    pins.expect_equal(choice, want, f"{what} strategy")


GAMES = [
    ("plain", lambda: synth.gen_plain()),
    ("uniform-ragged", lambda: synth.gen_uniform(12345, 5, 300, 21)),
    ("uniform-16k", lambda: synth.gen_uniform(1 << 14, 16, 1000, 2)),
    ("rmat-12", lambda: synth.gen_rmat(12, 16, seed=3)),
    ("rmat-14", lambda: synth.gen_rmat(14, 16, seed=3)),
    ("torus-32", lambda: synth.gen_torus(32, seed=4)),
    ("rmat-16-int64", lambda: synth.gen_rmat(16, 16, wlim=40000, seed=5)),
    ("stream-3", lambda: synth.gen_stream_game(3, scale_n=0.05)),
]


@pytest.mark.parametrize("name,make", GAMES, ids=[g[0] for g in GAMES])
def test_strategy_matches_oracle(ctx, oracle_mod, name, make):
    check(ctx, oracle_mod, make(), name)


def test_strategy_tiny_brute_force(ctx):
    """On tiny games the device strategy passes the brute-force pins directly."""
    def strat(game, f):
        fg, choice, _ = gpu_strategy(ctx, game)
        pins.expect_equal(fg, f, "tiny credits")
        return choice
    pins.pin_strategy_brute(strat, count=150, seed0=91_000)


def test_strategy_cases(ctx):
    def strat(game, f):
        fg, choice, _ = gpu_strategy(ctx, game)
        pins.expect_equal(fg, f, "case credits")
        return choice
    pins.pin_strategy_cases(strat)


def hub_rows_game(specs):
    """Vertex 0: a -1 self-loop trap (TOP); vertex 1: a 0-sink.  Then one
    player-0 vertex per (deg, k): deg edges into the trap, except edge k into
    the sink with weight 0, so its credit is 0 and its choice is k."""
    edges = [(0, 0, -1), (1, 1, 0)]
    for i, (deg, k) in enumerate(specs):
        v = 2 + i
        edges += [(v, 1 if j == k else 0, 0 if j == k else 3) for j in range(deg)]
    n = 2 + len(specs)
    return synth.make_game(n, edges, [1, 0] + [0] * len(specs), W=1), [k for _, k in specs]


def test_long_rows_first_witness(ctx, oracle_mod):
    specs = []
    for deg in (1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 129, 300, 5000):
        for k in sorted({0, 1, deg // 2, 31, 32, 33, 63, 64, 65, deg - 1}):
            if k < deg:
                specs.append((deg, k))
    game, want_k = hub_rows_game(specs * 3)  # several long rows share a wave
    f, choice, _ = gpu_strategy(ctx, game)
    pins.expect_equal(f, [TOP, 0] + [0] * len(want_k), "hub credits")
    assert choice[:2].tolist() == [-1, 0]
    assert choice[2:].tolist() == want_k
    check(ctx, oracle_mod, game, "hub rows")


def test_strategy_is_invisible_to_launch_shape(oracle_mod):
    game = synth.gen_rmat(13, 16, seed=7)
    want_f = oracle_mod.solve(game).f
    want, _ = oracle_mod.strategy(game, want_f)
    for shape in (dict(), dict(relabel=1), dict(relabel=2, seg_edges=512), dict(partition=2),
                  dict(seg_edges=-1, relabel=1)):
        with eg.Context(0, **shape) as c:
            f, choice, _ = gpu_strategy(c, game)
        pins.expect_equal(f, want_f, f"credits {shape}")
        pins.expect_equal(choice, want, f"strategy {shape}")


def test_strategy_needs_a_fixpoint(ctx):
    game = pins.cf8_game(40)
    with ctx.create(game) as g:
        with pytest.raises(eg.EgError) as e:
            g.strategy()
        assert e.value.code == eg.EG_EINVAL
        f, st, rc = g.solve(max_rounds=3, allow_timeout=True)
        assert rc == eg.EG_ETIMEDOUT
        with pytest.raises(eg.EgError) as e:
            g.strategy()
        assert e.value.code == eg.EG_EINVAL
        f, st, rc = g.solve(resume=True)
        assert rc == eg.EG_OK
        choice, _ = g.strategy()
        assert choice.tolist() == [-1] + [0] * 40
        g.set_measure(f)
        with pytest.raises(eg.EgError):
            g.strategy()


def test_all_player1_and_all_top(ctx):
    g1 = synth.gen_uniform(3000, 4, 10, 5)
    g1.owner[:] = 1
    _, choice, _ = gpu_strategy(ctx, g1)
    assert np.all(choice == -1)
    gn = synth.gen_uniform(3000, 4, 10, 6)
    gn = synth.Game(gn.n, gn.off, gn.tgt, (-np.abs(gn.w) - 1).astype(np.int32), gn.owner, W=11)
    f, choice, _ = gpu_strategy(ctx, gn)
    assert np.all(f == TOP) and np.all(choice == -1)
