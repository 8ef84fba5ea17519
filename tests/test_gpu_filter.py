"""The player-1 frontier filter (p1_filter: a player-1 predecessor joins the
next active set only if f(p) < f(v) (-) w(p, v), Alg. 1's test) changes the
work, never the credits: every game below is checked against the oracle in
every representation of the active set (list rounds, flag rounds, all-vertex
rounds, the single-block small mode, target-sliced rounds, cut tiles), with
seeding, resumed, batched and served, and across launch shapes."""
import numpy as np
import pytest

import pins
from paper_1710_03647_amd import eg, synth

pytestmark = pytest.mark.gpu
GiB = 1 << 30


def solve(game, **cfg):
    with eg.Context(0, p1_filter=1, **cfg) as ctx:
        with ctx.create(game) as g:
            f, st, rc = g.solve()
    return f, st


def test_filter_brute_force():
    pins.pin_brute(lambda g: solve(g)[0], count=300, seed0=82_000)


@pytest.mark.parametrize("pin", pins.CLOSED_FORMS, ids=lambda p: p.__name__)
def test_filter_closed_forms(pin):
    pin(lambda g: solve(g)[0])


GAMES = [
    ("plain", synth.gen_plain),
    ("uniform-4k", lambda: synth.gen_uniform(1 << 12, 16, 1000, 2)),
    ("uniform-16k", lambda: synth.gen_uniform(1 << 14, 16, 1000, 2)),
    ("uniform-ragged", lambda: synth.gen_uniform(12345, 5, 300, 21)),
    ("rmat-12", lambda: synth.gen_rmat(12, 16, seed=3)),
    ("rmat-14", lambda: synth.gen_rmat(14, 16, seed=3)),
    ("torus-32", lambda: synth.gen_torus(32, seed=4)),
    ("rmat-16-int64", lambda: synth.gen_rmat(16, 16, wlim=40000, seed=5)),
]

# launch shapes that force each representation of the active set
SHAPES = [
    ("default", {}),
    ("flags", {"dense_div": 1 << 20, "small_limit": 1}),      # flag sweeps (or all-vertex rounds) throughout
    ("lists", {"dense_div": 1, "small_limit": 1}),            # list rounds almost throughout
    ("small", {"small_limit": 65536}),                        # the single-block mode takes most rounds
    ("uncut", {"seg_edges": -1, "relabel": 1, "blocks_per_cu": 2}),
    ("cut-256", {"seg_edges": 256}),                          # many cut tiles
    ("sliced", {"partition": 2}),
    ("slice-major", {"partition": 3}),
    ("seeded", {"top_seeding": 1}),
]


@pytest.mark.parametrize("shape", [s[1] for s in SHAPES], ids=[s[0] for s in SHAPES])
@pytest.mark.parametrize("name,make", GAMES, ids=[g[0] for g in GAMES])
def test_filter_matches_oracle(oracle_mod, name, make, shape):
    game = make()
    f, st = solve(game, **shape)
    pins.expect_equal(f, oracle_mod.solve(game).f, f"{name} {shape}")


def test_filter_cuts_lifts_and_keeps_credits(oracle_mod):
    """Same credits with and without the filter; the filter leaves predecessors
    out and so lifts fewer vertices.  List rounds throughout (all-vertex
    rounds scan no predecessors, so the default shape may leave nothing to
    filter)."""
    game = synth.gen_uniform(1 << 14, 16, 1000, 2)
    want = oracle_mod.solve(game).f
    lists = {"dense_div": 1, "small_limit": 1}
    with eg.Context(0, **lists) as ctx:
        with ctx.create(game) as g:
            f0, st0, _ = g.solve()
    f1, st1 = solve(game, **lists)
    pins.expect_equal(f0, want, "unfiltered")
    pins.expect_equal(f1, want, "filtered")
    assert st1["filtered_preds"] > 0
    assert st0["filtered_preds"] == 0
    print(f"lifts {st0['lifts']} -> {st1['lifts']}, rounds {st0['rounds']} -> {st1['rounds']}, "
          f"filtered {st1['filtered_preds']}")


def test_filter_resume_from_below(oracle_mod):
    game = synth.gen_torus(32, seed=4)
    want = oracle_mod.solve(game).f
    noise = synth.to_int(synth.draws(6, 2, 0, game.n), 0, 60)
    with eg.Context(0, p1_filter=1) as ctx:
        with ctx.create(game) as g:
            g.set_measure(np.minimum(want, noise))
            f, _, _ = g.solve(resume=True)
    pins.expect_equal(f, want, "resumed with the filter")


def test_filter_in_batch_and_serving(oracle_mod):
    games = [synth.gen_stream_game(i, scale_n=0.05) for i in range(8)]
    games += [synth.gen_random_small(950 + i, n_max=7) for i in range(6)]
    games += [pins.cf8_game(200), synth.gen_rmat(11, 16, seed=3)]
    with eg.Context(0, hbm_budget_bytes=GiB, p1_filter=1) as ctx:
        res = ctx.solve_batch(games)
    for g, (f, st) in zip(games, res):
        pins.expect_equal(f, oracle_mod.solve(g).f, f"{g.name}: batched with the filter")
    with eg.Context(0, hbm_budget_bytes=GiB, max_slots=4, p1_filter=1, top_seeding=1) as ctx:
        tickets = [ctx.submit(g) for g in games]
        for g, t in zip(games, tickets):
            rc, f, st = ctx.wait(t, g.n)
            pins.expect_equal(f, oracle_mod.solve(g).f, f"{g.name}: served with the filter and seeding")


def test_filter_stress_launch_shapes(oracle_mod):
    """Many random mid-size games, each under a different launch shape: the
    in-place races between lifts and filter tests differ from run to run and
    from shape to shape; the credits never do."""
    shapes = [s[1] for s in SHAPES]
    for i in range(24):
        game = synth.gen_uniform(500 + 97 * i, 2 + i % 7, 5 + 11 * i, 300 + i)
        want = oracle_mod.solve(game).f
        f, _ = solve(game, **shapes[i % len(shapes)])
        pins.expect_equal(f, want, f"{game.name} shape {i % len(shapes)}")
