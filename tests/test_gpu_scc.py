"""The component schedule (scc_schedule: strongly connected components solved
level by level from the sink components up, the refinement the paper proposes
after its results, Sec. 6).

The device's components (eg_components) are compared with scipy's strong
components (a library routine, used here as the reference partition) and its
levels with the longest-path levels of the condensation computed in numpy from
scipy's labels.  The schedule changes the work, never the credits: every game
is checked against the oracle, plain, seeded, with the player-1 filter and in
several launch shapes."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as cg

import pins
from paper_1710_03647_amd import eg, synth

pytestmark = pytest.mark.gpu


def reference_components(game):
    """scipy's strong components and the condensation levels (0 for sink
    components, else 1 + the largest level of a component reached by an edge)."""
    src = np.repeat(np.arange(game.n), np.diff(game.off))
    a = sp.csr_matrix((np.ones(game.m, dtype=np.int8), (src, game.tgt)), shape=(game.n, game.n))
    nc, lab = cg.connected_components(a, directed=True, connection="strong")
    cs, ct = lab[src], lab[game.tgt]
    cross = cs != ct
    es, et = cs[cross], ct[cross]
    lev = np.zeros(nc, dtype=np.int64)
    while True:
        nxt = lev.copy()
        np.maximum.at(nxt, es, lev[et] + 1)
        if np.array_equal(nxt, lev):
            break
        lev = nxt
    return nc, lab, lev[lab]


def same_partition(a, b):
    pairs = np.unique(np.stack([a.astype(np.int64), b.astype(np.int64)], 1), axis=0)
    return len(pairs) == len(np.unique(a)) == len(np.unique(b))


def chain_of_cycles(k, size, seed):
    """k cycles of `size` vertices, cycle i with an edge into cycle i+1, the last
    cycle a sink component; ids decrease along the chain (the colouring then
    assigns one component per phase) and owners and weights are random."""
    rng = np.random.default_rng(seed)
    n = k * size
    rows = [[] for _ in range(n)]
    for c in range(k):
        base = (k - 1 - c) * size  # cycle c occupies ids [base, base + size)
        for j in range(size):
            v = base + j
            rows[v].append((base + (j + 1) % size, int(rng.integers(-3, 4))))
        if c + 1 < k:
            nb = (k - 2 - c) * size
            rows[base].append((nb + int(rng.integers(0, size)), int(rng.integers(-3, 4))))
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    tgt = np.array([t for r in rows for t, _ in r], dtype=np.int32)
    w = np.array([x for r in rows for _, x in r], dtype=np.int32)
    owner = rng.integers(0, 2, n).astype(np.uint8)
    return synth.Game(n=n, off=off, tgt=tgt, w=w, owner=owner, W=3, name=f"chain-{k}x{size}")


def dag_with_sinks(n, seed):
    """Edges only to smaller ids (every vertex its own component), vertex 0 a
    sink with a self-loop: n levels."""
    rng = np.random.default_rng(seed)
    rows = [[(0, 0)]] + [[(int(rng.integers(0, v)), int(rng.integers(-5, 6))) for _ in range(1 + v % 3)]
                         for v in range(1, n)]
    rows[1:] = [r if any(t == v - 1 for t, _ in r) else r + [(v - 1, 1)] for v, r in enumerate(rows[1:], 1)]
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    tgt = np.array([t for r in rows for t, _ in r], dtype=np.int32)
    w = np.array([x for r in rows for _, x in r], dtype=np.int32)
    owner = rng.integers(0, 2, n).astype(np.uint8)
    return synth.Game(n=n, off=off, tgt=tgt, w=w, owner=owner, W=5, name=f"dag-{n}")


GAMES = [
    ("plain", synth.gen_plain),
    ("uniform-ragged", lambda: synth.gen_uniform(12345, 2, 300, 21)),
    ("uniform-16k", lambda: synth.gen_uniform(1 << 14, 16, 1000, 2)),
    ("rmat-12", lambda: synth.gen_rmat(12, 16, seed=3)),
    ("rmat-16", lambda: synth.gen_rmat(16, 16, seed=3)),
    ("rmat-16-int64", lambda: synth.gen_rmat(16, 16, wlim=40000, seed=5)),
    ("torus-32", lambda: synth.gen_torus(32, seed=4)),
    ("stream-3", lambda: synth.gen_stream_game(3)),
    ("chain-40x5", lambda: chain_of_cycles(40, 5, 1)),
    ("chain-300x1", lambda: chain_of_cycles(300, 1, 2)),
    ("dag-700", lambda: dag_with_sinks(700, 3)),
]


@pytest.mark.parametrize("name,make", GAMES, ids=[g[0] for g in GAMES])
def test_components_and_levels_match_reference(name, make):
    game = make()
    nc, lab, lev = reference_components(game)
    with eg.Context(0) as ctx:
        with ctx.create(game) as g:
            comp, level, ncomp, nlev = g.components()
    assert ncomp == nc, f"{name}: {ncomp} components, scipy finds {nc}"
    assert same_partition(comp, lab), f"{name}: the partition differs from scipy's"
    assert nlev == int(lev.max()) + 1
    bad = np.nonzero(level != lev)[0]
    assert len(bad) == 0, f"{name}: levels differ at {bad[:8]} ({level[bad[:8]]} vs {lev[bad[:8]]})"


SHAPES = [
    ("default", {}),
    ("seeded", {"top_seeding": 1}),
    ("filter", {"p1_filter": 1}),
    ("flags", {"dense_div": 1 << 20, "small_limit": 1}),  # flag sweeps (dense_at = 1)
    ("lists", {"dense_div": 1, "small_limit": 1}),  # list rounds (dense_at = n)
    ("small", {"small_limit": 65536}),
]


_WANT = {}  # oracle credits per game name (the same game under every shape)


# the schedule against the oracle: the same classes, R-MAT at scale 14 (scale 16
# plain solves take tens of seconds per shape; the components test keeps 16)
SCHEDULE_GAMES = [g for g in GAMES if not g[0].startswith("rmat-16")] + [
    ("rmat-14", lambda: synth.gen_rmat(14, 16, seed=3)),
    ("rmat-14-int64", lambda: synth.gen_rmat(14, 16, wlim=200000, seed=5)),
]


@pytest.mark.parametrize("shape", [s[1] for s in SHAPES], ids=[s[0] for s in SHAPES])
@pytest.mark.parametrize("name,make", SCHEDULE_GAMES, ids=[g[0] for g in SCHEDULE_GAMES])
def test_schedule_matches_oracle(oracle_mod, name, make, shape):
    game = make()
    if name not in _WANT:
        _WANT[name] = oracle_mod.solve(game).f
    want = _WANT[name]
    with eg.Context(0, scc_schedule=1, **shape) as ctx:
        with ctx.create(game) as g:
            f, st, rc = g.solve()
            f2, st2, _ = g.solve()  # the components are kept: the second solve reuses them
    pins.expect_equal(f, want, f"{name} {shape}")
    pins.expect_equal(f2, want, f"{name} {shape} (second solve)")
    assert st["scc_components"] >= 1 and st["scc_levels"] >= 1


def test_schedule_brute_force():
    def solve(game):
        with eg.Context(0, scc_schedule=1) as ctx:
            with ctx.create(game) as g:
                return g.solve()[0]

    pins.pin_brute(solve, count=300, seed0=71_000)


def climb_chain(k, seed):
    """Vertex 0 is a player-1 sink with a self-loop of weight -1: its value
    climbs by one per lift up to the bound and then becomes TOP (W = 1, so B + 2
    lifts).  Vertices 1..k each have one edge, of weight 0, to the vertex
    before: every rise of vertex 0 travels up the chain.  Each vertex is a
    component of its own, on level = its id."""
    rng = np.random.default_rng(seed)
    n = k + 1
    off = np.arange(n + 1, dtype=np.int64)
    tgt = np.concatenate([[0], np.arange(k)]).astype(np.int32)
    w = np.concatenate([[-1], np.zeros(k)]).astype(np.int32)
    owner = rng.integers(0, 2, n).astype(np.uint8)
    owner[0] = 1
    return synth.Game(n=n, off=off, tgt=tgt, w=w, owner=owner, W=1, name=f"climb-{k}")


def test_schedule_lifts_each_level_once_its_successors_are_final(oracle_mod):
    """Plain iteration re-lifts the chain every time the sink's value rises
    (about (B + 2) * k lifts); the schedule lifts the sink to TOP alone and then
    each chain vertex once per level (about B + 2 + 2k lifts).  Same credits."""
    game = climb_chain(50, 7)
    want = oracle_mod.solve(game).f
    assert np.all(want == eg.EG_TOP)
    with eg.Context(0) as ctx:
        with ctx.create(game) as g:
            f0, st0, _ = g.solve()
    with eg.Context(0, scc_schedule=1) as ctx:
        with ctx.create(game) as g:
            f1, st1, _ = g.solve()
    pins.expect_equal(f0, want, "plain")
    pins.expect_equal(f1, want, "component schedule")
    assert st1["scc_levels"] == 51 and st1["scc_components"] == 51
    print(f"lifts {st0['lifts']} -> {st1['lifts']}, rounds {st0['rounds']} -> {st1['rounds']}")
    assert 4 * st1["lifts"] < st0["lifts"]


def test_rmat_full_components_and_schedule():
    """R-MAT scale 22 in the benchmarked launch shape: components and levels
    against scipy's, and the seeded schedule's credits equal the seeded plain
    solve's."""
    from paper_1710_03647_amd import tune

    game = synth.gen_rmat_full()
    nc, lab, lev = reference_components(game)
    shape = tune.config_for(game)
    with eg.Context(0, top_seeding=1, **shape) as ctx:
        with ctx.create(game) as g:
            want, _, _ = g.solve()
    with eg.Context(0, top_seeding=1, scc_schedule=1, **shape) as ctx:
        with ctx.create(game) as g:
            f, st, _ = g.solve()
            comp, level, ncomp, nlev = g.components()
    assert ncomp == nc and same_partition(comp, lab)
    assert np.array_equal(level, lev)
    pins.expect_equal(f, want, "R-MAT 2^22 schedule vs plain (seeded)")
    print(f"components {ncomp}, levels {nlev}, t_scc {st['t_scc'] * 1e3:.1f} ms, rounds {st['rounds']}")
