"""Device solver (through the C-ABI) against the CPU oracle: bit-exact credits.

Sizes span several tiles of the launch grid and ragged tails; the closed forms
and tiny brute-force games cover the degenerate cases (single vertices,
self-loops, duplicates, TOP everywhere, credits exactly at the bound)."""
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


def gpu_solve(ctx, game, **kw):
    g = ctx.create(game)
    try:
        f, st, rc = g.solve(**kw)
    finally:
        g.destroy()
    return f, st


def test_plain_config(ctx, oracle_mod):
    game = synth.gen_plain()
    f, st = gpu_solve(ctx, game)
    want = oracle_mod.solve(game).f
    pins.expect_equal(f, want, "plain")
    assert st["rounds"] > 0 and st["lifts"] >= st["changes"] > 0
    assert st["relaxed_edges"] >= 4 * st["lifts"] - 1


def test_tiny_brute_force(ctx):
    pins.pin_brute(lambda g: gpu_solve(ctx, g)[0], count=300, seed0=80_000)


@pytest.mark.parametrize("pin", pins.CLOSED_FORMS, ids=lambda p: p.__name__)
def test_closed_forms(ctx, pin):
    pin(lambda g: gpu_solve(ctx, g)[0])


def test_cf8_lift_count(ctx):
    for k in (1, 7, 100):
        f, st = gpu_solve(ctx, pins.cf8_game(k))
        pins.expect_equal(f, [TOP] + [0] * k, "CF8")
        assert st["changes"] == k + 1 and st["lifts"] == k + 2


SCALED = [
    ("uniform-1k", lambda: synth.gen_uniform(1 << 10, 16, 1000, 2)),
    ("uniform-4k", lambda: synth.gen_uniform(1 << 12, 16, 1000, 2)),
    ("uniform-16k", lambda: synth.gen_uniform(1 << 14, 16, 1000, 2)),
    ("uniform-ragged", lambda: synth.gen_uniform(12345, 5, 300, 21)),
    ("rmat-10", lambda: synth.gen_rmat(10, 16, seed=3)),
    ("rmat-12", lambda: synth.gen_rmat(12, 16, seed=3)),
    ("rmat-14", lambda: synth.gen_rmat(14, 16, seed=3)),
    ("torus-32", lambda: synth.gen_torus(32, seed=4)),
    ("torus-48", lambda: synth.gen_torus(48, seed=4)),
    ("rmat-16-int64", lambda: synth.gen_rmat(16, 16, wlim=40000, seed=5)),
]


@pytest.mark.parametrize("name,make", SCALED, ids=[s[0] for s in SCALED])
def test_scaled_configs(ctx, oracle_mod, name, make):
    game = make()
    f, st = gpu_solve(ctx, game)
    want = oracle_mod.solve(game).f
    pins.expect_equal(f, want, name)


def test_stream_games(ctx, oracle_mod):
    for i in range(12):
        game = synth.gen_stream_game(i, scale_n=0.1)
        f, _ = gpu_solve(ctx, game)
        pins.expect_equal(f, oracle_mod.solve(game).f, game.name)


def test_device_pointer_input(ctx, oracle_mod):
    import torch

    game = synth.gen_uniform(3000, 6, 40, 17)
    dev = torch.device("cuda", 0)
    off = torch.from_numpy(game.off).to(dev)
    tgt = torch.from_numpy(game.tgt).to(dev)
    w = torch.from_numpy(game.w).to(dev)
    bits = torch.from_numpy(game.owner_bits()).to(dev)
    torch.cuda.synchronize()
    g = ctx.create(n=game.n, offsets=off, targets=tgt, weights=w, owner_bits=bits, W=game.W, device=True)
    try:
        f, st, rc = g.solve()
    finally:
        g.destroy()
    pins.expect_equal(f, oracle_mod.solve(game).f, "device pointers")


def test_torch_stream(oracle_mod):
    import torch

    s = torch.cuda.Stream()
    game = synth.gen_uniform(2000, 4, 20, 5)
    with eg.Context(0, stream=s) as c:
        f, _ = gpu_solve(c, game)
    pins.expect_equal(f, oracle_mod.solve(game).f, "torch stream")


def test_bound_mg(oracle_mod):
    game = synth.gen_uniform(3000, 3, 20, 11)
    with eg.Context(0, bound_mode=eg.EG_BOUND_MG) as c:
        f, _ = gpu_solve(c, game)
    pins.expect_equal(f, oracle_mod.solve(game, bound_mode=1).f, "M_G bound")
    pins.expect_equal(f, oracle_mod.solve(game).f, "M_G bound = (n-1)W result")


def test_budget_gives_lower_bound_and_resume(ctx, oracle_mod):
    game = synth.gen_torus(32, seed=4)
    want = oracle_mod.solve(game).f
    g = ctx.create(game)
    try:
        f, st, rc = g.solve(max_rounds=50, allow_timeout=True)
        assert rc == eg.EG_ETIMEDOUT and st["rounds"] == 50
        assert np.all(f <= want)  # a lower bound; TOP only where proven
        g.set_measure(f)
        f2, st2, rc2 = g.solve(resume=True)
        assert rc2 == eg.EG_OK
        pins.expect_equal(f2, want, "resume")
    finally:
        g.destroy()


def test_resume_from_below(ctx, oracle_mod):
    game = synth.gen_uniform(4000, 4, 30, 9)
    want = oracle_mod.solve(game).f
    noise = synth.to_int(synth.draws(3, 2, 0, game.n), 0, 50)
    g = ctx.create(game)
    try:
        g.set_measure(np.minimum(want, noise))
        f, _, _ = g.solve(resume=True)
        pins.expect_equal(f, want, "resume from below")
        f, _, _ = g.solve()  # a fresh solve after a resumed one
        pins.expect_equal(f, want, "fresh after resume")
    finally:
        g.destroy()


def test_repeated_solves_identical(ctx, oracle_mod):
    game = synth.gen_rmat(13, 16, seed=7)
    want = oracle_mod.solve(game).f
    g = ctx.create(game)
    try:
        for _ in range(5):
            f, _, _ = g.solve()
            pins.expect_equal(f, want, "repeat")
    finally:
        g.destroy()


def test_set_measure_rejects_out_of_range(ctx):
    game = synth.gen_plain()
    g = ctx.create(game)
    try:
        bad = np.zeros(game.n, dtype=np.int64)
        bad[3] = 10 ** 9
        with pytest.raises(eg.EgError) as ei:
            g.set_measure(bad)
        assert ei.value.code == eg.EG_EINVAL
    finally:
        g.destroy()


PARTITIONED = [
    ("uniform-20k", lambda: synth.gen_uniform(20000, 16, 1000, 2)),
    ("uniform-ragged-int32", lambda: synth.gen_uniform(12345, 7, 300, 21)),
    ("rmat-13-int64", lambda: synth.gen_rmat(13, 16, wlim=400000, seed=5)),
    ("rmat-14", lambda: synth.gen_rmat(14, 16, seed=3)),
    ("torus-40", lambda: synth.gen_torus(40, seed=4)),
]


@pytest.mark.parametrize("mode", [2, 3], ids=["per-xcd", "slice-major"])
@pytest.mark.parametrize("name,make", PARTITIONED, ids=[s[0] for s in PARTITIONED])
def test_partitioned_dense_rounds(oracle_mod, name, make, mode):
    """Dense rounds over the target-sliced edge copy (forced on small games):
    per-XCD slices with partial keys, and slice-major sweeps with keys in LDS."""
    game = make()
    with eg.Context(0, partition=mode) as c:
        f, st = gpu_solve(c, game)
    assert st["dense_rounds"] > 0
    pins.expect_equal(f, oracle_mod.solve(game).f, name)


@pytest.mark.parametrize("mode", [2, 3], ids=["per-xcd", "slice-major"])
@pytest.mark.parametrize("name,make", PARTITIONED[:4], ids=[s[0] for s in PARTITIONED[:4]])
def test_partitioned_round_is_one_jacobi_step(oracle_mod, name, make, mode):
    """A partitioned dense round reads only the values of the previous round:
    from any measure below the fixpoint, one resumed round with every vertex
    active is exactly one application of the lifting operator everywhere,
    kept only where it raises the value (writes never lower a value)."""
    game = make()
    want = oracle_mod.solve(game)
    noise = synth.to_int(synth.draws(11, 2, 0, game.n), 0, 4 * game.W)
    f0 = np.minimum(want.f, noise)
    with eg.Context(0, partition=mode) as c:
        g = c.create(game)
        try:
            g.set_measure(f0)
            f1, st, rc = g.solve(max_rounds=1, resume=True, allow_timeout=True)
        finally:
            g.destroy()
    assert st["dense_rounds"] == 1
    pins.expect_equal(f1, np.maximum(f0, pins.lift_all_numpy(game, f0, want.bound)), name)


SYNCHRONOUS = [
    ("rmat-11", lambda: synth.gen_rmat(11, 16, seed=3)),
    ("rmat-11-int64", lambda: synth.gen_rmat(11, 16, wlim=2_000_000, seed=3)),
    ("uniform-3000", lambda: synth.gen_uniform(3000, 4, 30, 9)),
]


@pytest.mark.parametrize("name,make", SYNCHRONOUS, ids=[s[0] for s in SYNCHRONOUS])
def test_partitioned_rounds_are_synchronous(oracle_mod, name, make):
    """With every round a target-sliced dense round, the solve is Alg. 3 with
    synchronous rounds: the same lifts, changes and relaxed edges as the numpy
    iteration, round for round.  A slice key that missed an edge (an LDS update
    not yet visible to the wave that stores the key) changes these counts."""
    game = make()
    want = oracle_mod.solve(game)
    f_np, rounds, lifts, changes, edges = pins.synchronous_rounds_numpy(game, want.bound)
    with eg.Context(0, partition=2, dense_div=1 << 20, small_limit=1) as c:
        f, st = gpu_solve(c, game)
    pins.expect_equal(f, want.f, name)
    assert st["dense_rounds"] >= st["rounds"] >= rounds
    assert (st["lifts"], st["changes"], st["relaxed_edges"]) == (lifts, changes, edges)


def hub_game(seed=31):
    """Uniform game plus a few hub vertices with tens of thousands of
    out-edges, two of them in one tile: dense rounds cut those tiles into
    segments taken by different blocks."""
    base = synth.gen_uniform(6000, 4, 50, seed)
    src = [np.repeat(np.arange(base.n), 4)]
    dst, w = [base.tgt.astype(np.int64)], [base.w.astype(np.int64)]
    for hub, k, s in ((7, 30000, 1), (200, 20000, 2), (4100, 9000, 3)):
        x = synth.draws(seed, 40 + s, 0, 2 * k)
        src.append(np.full(k, hub))
        dst.append(synth.to_int(x[:k], 0, base.n - 1))
        w.append(synth.to_int(x[k:], -50, 50))
    return synth.from_edges(base.n, np.concatenate(src), np.concatenate(dst), np.concatenate(w), base.owner,
                            W=50, name="uniform-with-hubs")


def test_hub_tiles_are_cut(ctx, oracle_mod):
    game = hub_game()
    want = oracle_mod.solve(game).f
    for _ in range(2):
        f, st = gpu_solve(ctx, game)
        pins.expect_equal(f, want, game.name)
    with eg.Context(0, top_seeding=1) as c:
        f, st = gpu_solve(c, game)
    pins.expect_equal(f, want, game.name + " seeded")


@pytest.mark.parametrize("relabel", [1, 2])
def test_renumbering_is_invisible(oracle_mod, relabel):
    """Credits come back in the caller's numbering whether or not the game is
    renumbered internally, also through set_measure and resumed solves."""
    for game in (synth.gen_rmat(12, 16, seed=3), synth.gen_uniform(5000, 6, 40, 3)):
        want = oracle_mod.solve(game).f
        noise = synth.to_int(synth.draws(17, 2, 0, game.n), 0, 3 * game.W)
        with eg.Context(0, relabel=relabel) as c:
            with c.create(game) as g:
                f, st, rc = g.solve()
                pins.expect_equal(f, want, f"{game.name} relabel={relabel}")
                g.set_measure(np.minimum(want, noise))
                f, st, rc = g.solve(resume=True)
                pins.expect_equal(f, want, f"{game.name} resumed, relabel={relabel}")


SHAPES = [dict(), dict(blocks_per_cu=4), dict(blocks_per_cu=16, dense_div=4), dict(small_limit=64),
          dict(small_limit=8192, dense_div=256), dict(seg_edges=256), dict(seg_edges=-1, relabel=1),
          dict(partition=2), dict(partition=3), dict(relabel=2, seg_edges=512),
          dict(relabel=2, seg_edges=512, hub_cache=1), dict(relabel=2, hub_cache=-1), dict(relabel=2, hub_cache=40)]


def test_launch_shapes_give_identical_credits(oracle_mod):
    """The credits do not depend on the launch shape: occupancy, representation
    thresholds, tile cutting, renumbering, slicing and the LDS copy of the most
    gathered values (bit-identical results)."""
    for game in (synth.gen_rmat(13, 16, seed=7), synth.gen_uniform(9999, 7, 80, 29)):
        want = oracle_mod.solve(game).f
        for shape in SHAPES:
            with eg.Context(0, **shape) as c:
                f, st = gpu_solve(c, game)
            pins.expect_equal(f, want, f"{game.name} {shape}")
