"""Pins for the CPU oracle: checks against things other than the oracle itself.

Every pin takes ``solve(game, **kw) -> int64[n]`` (TOP = INT64_MAX) so that the
same battery runs on the oracle and on deliberately broken copies of it.  The
sources of truth are:

* brute force over positional strategies (Lemma 1, Eq. (1)/Def. 3, memoryless
  determinacy), two independent implementations in ``oracle.brute``;
* closed forms for chains, cycles, choices and one-player arenas;
* the fixpoint condition of the lifting operator (Def. 6), evaluated here with
  numpy, and order/bound/relabel/monotonicity/resume invariants.
"""
from __future__ import annotations

import numpy as np

from oracle import brute
from paper_1710_03647_amd import synth

TOP = np.iinfo(np.int64).max


def fmt(f):
    return ["T" if x == TOP else int(x) for x in f]


def expect_equal(got, want, what=""):
    got = np.asarray(got, dtype=np.int64)
    want = np.asarray(want, dtype=np.int64)
    if got.shape != want.shape or not np.array_equal(got, want):
        raise AssertionError(f"{what}: got {fmt(got)[:40]} want {fmt(want)[:40]}")


# --------------------------------------------------------------------------- brute force
def pin_brute(solve, count=2000, n_max=7, deg_max=3, wlim=4, seed0=10_000, owner_mode="mixed",
              checker="fw"):
    check = brute.credits_fw if checker == "fw" else brute.credits_dfs
    for s in range(count):
        g = synth.gen_random_small(seed0 + s, n_max=n_max, deg_max=deg_max, wlim=wlim,
                                   owner_mode=owner_mode)
        expect_equal(solve(g), check(g), f"brute[{checker}] seed={seed0 + s} n={g.n}")


# --------------------------------------------------------------------------- closed forms
def pin_cf1_self_loop(solve):
    """One vertex with a self-loop of weight w: credit 0 if w >= 0, TOP otherwise."""
    for owner in (0, 1):
        for w in (-7, -1, 0, 1, 9):
            g = synth.make_game(1, [(0, 0, w)], [owner], W=max(0, -w))
            expect_equal(solve(g), [0 if w >= 0 else TOP], f"CF1 owner={owner} w={w}")


def _chain_game(ws, owners):
    k = len(ws)  # chain vertices 0..k-1, sink k
    edges = [(i, i + 1, int(ws[i])) for i in range(k)] + [(k, k, 0)]
    return synth.make_game(k + 1, edges, list(owners) + [0], W=max(0, -min(list(ws) + [0])))


def _chain_credit(ws, i):
    best, acc = 0, 0
    for j in range(i, len(ws)):
        acc += ws[j]
        best = max(best, -acc)
    return best


def pin_cf2_chain(solve, trials=200, seed=7):
    """Chain v0 -> ... -> v_{k-1} -> sink (0 self-loop): c(v_i) is the worst
    suffix-prefix deficit max(0, max_{j>=i} -(w_i + ... + w_j)), whatever the owners."""
    x = synth.draws(seed, 1, 0, trials * 40)
    pos = 0
    for t in range(trials):
        k = int(x[pos] % np.uint64(12)) + 1
        pos += 1
        ws = [int(v) for v in synth.to_int(x[pos:pos + k], -9, 6)]
        pos += k
        owners = [int(v) for v in synth.to_bit(x[pos:pos + k])]
        pos += k
        g = _chain_game(ws, owners)
        want = [_chain_credit(ws, i) for i in range(k)] + [0]
        expect_equal(solve(g), want, f"CF2 ws={ws}")


def pin_cf3_tight_chain(solve):
    """n-1 edges of weight -W into a 0-sink: c(v0) = (n-1)W, exactly the bound,
    which must stay finite (values strictly above the bound become TOP)."""
    for n in (2, 3, 5, 9):
        for W in (1, 3, 10):
            edges = [(i, i + 1, -W) for i in range(n - 1)] + [(n - 1, n - 1, 0)]
            for owners in ([0] * n, [1] * n):
                g = synth.make_game(n, edges, owners, W=W)
                want = [(n - 1 - i) * W for i in range(n)]
                expect_equal(solve(g), want, f"CF3 n={n} W={W}")


def pin_cf4_cycle(solve, trials=200, seed=8):
    """Cycle of length L with sum S: all TOP if S < 0, otherwise
    c(v_i) = max(0, max_{k=1..L-1} -(w_i + ... + w_{i+k-1}))."""
    x = synth.draws(seed, 1, 0, trials * 40)
    pos = 0
    for t in range(trials):
        L = int(x[pos] % np.uint64(9)) + 1
        pos += 1
        ws = [int(v) for v in synth.to_int(x[pos:pos + L], -6, 6)]
        pos += L
        owners = [int(v) for v in synth.to_bit(x[pos:pos + L])]
        pos += L
        edges = [(i, (i + 1) % L, ws[i]) for i in range(L)]
        g = synth.make_game(L, edges, owners, W=max(0, -min(ws)))
        S = sum(ws)
        if S < 0:
            want = [TOP] * L
        else:
            want = []
            for i in range(L):
                best, acc = 0, 0
                for k in range(1, L):
                    acc += ws[(i + k - 1) % L]
                    best = max(best, -acc)
                want.append(best)
        expect_equal(solve(g), want, f"CF4 ws={ws}")


def pin_cf5_choice(solve):
    """A vertex with edges of weights a, b into two 0-sinks: player 0 pays
    max(0, -max(a, b)), player 1 makes it pay max(0, -min(a, b))."""
    for a in (-5, -2, 0, 3):
        for b in (-4, -1, 0, 2):
            for owner in (0, 1):
                g = synth.make_game(3, [(0, 1, a), (0, 2, b), (1, 1, 0), (2, 2, 0)],
                                    [owner, 0, 1], W=5)
                want0 = max(0, -max(a, b)) if owner == 0 else max(0, -min(a, b))
                expect_equal(solve(g), [want0, 0, 0], f"CF5 a={a} b={b} owner={owner}")


def pin_cf6_top_propagation(solve):
    """TOP successors: a player-1 vertex with one TOP successor is TOP; a player-0
    vertex is TOP only when every successor term is TOP."""
    for a in (-3, 0, 4):
        # vertex 1 is a -1 self-loop trap (TOP); vertex 2 is a 0-sink
        g = synth.make_game(3, [(0, 1, 5), (0, 2, a), (1, 1, -1), (2, 2, 0)], [1, 0, 0], W=3)
        expect_equal(solve(g), [TOP, TOP, 0], f"CF6 p1 a={a}")
        g = synth.make_game(3, [(0, 1, 5), (0, 2, a), (1, 1, -1), (2, 2, 0)], [0, 0, 0], W=3)
        expect_equal(solve(g), [max(0, -a), TOP, 0], f"CF6 p0 a={a}")
    g = synth.make_game(3, [(0, 1, 5), (0, 2, 7), (1, 1, -1), (2, 2, -2)], [0, 1, 0], W=2)
    expect_equal(solve(g), [TOP, TOP, TOP], "CF6 p0 all top")


def pin_cf6b_positive_weight_into_top(solve):
    """Positive weights above W (W only bounds the negative ones) into a TOP
    successor still give TOP: TOP (-) b = TOP for every b."""
    for big in (2, 7, 1000, 2 ** 31 - 1):
        # 1 is a -1 self-loop trap; 0 can only move to 1, with weight +big
        g = synth.make_game(3, [(0, 1, big), (1, 1, -1), (2, 0, big), (2, 2, -1)], [0, 1, 1], W=1)
        expect_equal(solve(g), [TOP, TOP, TOP], f"CF6b big={big}")
        g = synth.make_game(3, [(0, 1, big), (0, 2, big), (1, 1, -1), (2, 2, 0)], [0, 0, 0], W=1)
        expect_equal(solve(g), [0, TOP, 0], f"CF6b choice big={big}")


def pin_cf7_sign(solve):
    """All weights >= 0: every credit 0.  All weights < 0: every vertex TOP."""
    for seed in (1, 2, 3):
        g = synth.gen_uniform(300, 3, 20, seed)
        gp = synth.Game(g.n, g.off, g.tgt, np.abs(g.w).astype(np.int32), g.owner, W=0)
        expect_equal(solve(gp), np.zeros(g.n, dtype=np.int64), f"CF7 nonneg seed={seed}")
        gn = synth.Game(g.n, g.off, g.tgt, (-np.abs(g.w) - 1).astype(np.int32), g.owner, W=21)
        expect_equal(solve(gn), np.full(g.n, TOP, dtype=np.int64), f"CF7 neg seed={seed}")


def cf8_game(k):
    """Vertex 0 has a -1 self-loop; vertices 1..k have 0 self-loops; W = 1, so
    the bound (n-1)W is k and f(0) climbs 0, 1, ..., k and then becomes TOP."""
    edges = [(0, 0, -1)] + [(i, i, 0) for i in range(1, k + 1)]
    return synth.make_game(k + 1, edges, [1] + [0] * k, W=1)


def pin_cf8_climb(solve):
    for k in (1, 5, 40):
        expect_equal(solve(cf8_game(k)), [TOP] + [0] * k, f"CF8 k={k}")


def pin_cf9_one_player(solve, trials=60, seed=9):
    """Arenas owned by player 1 only: TOP iff a negative cycle is reachable,
    else max(0, -min over reachable u of d(v, u)) with Floyd-Warshall distances."""
    for t in range(trials):
        n = 5 + (t % 25)
        g = synth.gen_uniform(n, 1 + t % 3, 6, seed * 1000 + t)
        g.owner[:] = 1
        expect_equal(solve(g), brute.credits_one_player_max(g), f"CF9 t={t} n={n}")


CLOSED_FORMS = [pin_cf1_self_loop, pin_cf2_chain, pin_cf3_tight_chain, pin_cf4_cycle, pin_cf5_choice,
                pin_cf6_top_propagation, pin_cf6b_positive_weight_into_top, pin_cf7_sign, pin_cf8_climb, pin_cf9_one_player]


# --------------------------------------------------------------------------- fixpoint (numpy)
def lift_all_numpy(game, f, bound):
    """delta(f, v)(v) for every v (Def. 6), evaluated with numpy."""
    f = np.asarray(f, dtype=np.int64)
    ft = f[game.tgt.astype(np.int64)]
    is_top = ft == TOP
    d = np.where(is_top, 0, ft) - game.w.astype(np.int64)
    t = np.where(is_top, TOP, np.maximum(d, 0))
    t = np.where((t != TOP) & (t > bound), TOP, t)
    starts = game.off[:-1].astype(np.int64)
    mn = np.minimum.reduceat(t, starts)
    mx = np.maximum.reduceat(t, starts)
    return np.where(game.owner == 0, mn, mx)



def initially_active_numpy(game):
    """L_1 of Alg. 3: player-0 vertices whose out-edges are all negative,
    player-1 vertices with some negative out-edge."""
    src = np.repeat(np.arange(game.n), np.diff(game.off))
    neg = np.bincount(src, weights=(game.w < 0), minlength=game.n)
    deg = np.diff(game.off)
    return np.where(game.owner == 0, neg == deg, neg > 0)


def synchronous_rounds_numpy(game, bound):
    """Alg. 3 with synchronous rounds: round r lifts every vertex of L_r from the
    values left by round r-1, and L_{r+1} holds the predecessors of the vertices
    whose value changed.  Returns (f, rounds, lifts, changes, relaxed edges)."""
    src = np.repeat(np.arange(game.n), np.diff(game.off))
    deg = np.diff(game.off).astype(np.int64)
    f = np.zeros(game.n, dtype=np.int64)
    act = initially_active_numpy(game)
    rounds = lifts = changes = edges = 0
    while act.any():
        new = lift_all_numpy(game, f, bound)
        changed = act & (new != f)
        f = np.where(act, new, f)
        rounds += 1
        lifts += int(act.sum())
        changes += int(changed.sum())
        edges += int(deg[act].sum())
        act = np.zeros(game.n, dtype=bool)
        act[src[changed[game.tgt]]] = True
    return f, rounds, lifts, changes, edges


def pin_fixpoint(game, f, bound, what=""):
    """I1 and I2: f is a fixpoint, finite values lie in [0, bound]."""
    f = np.asarray(f, dtype=np.int64)
    g = lift_all_numpy(game, f, bound)
    bad = np.nonzero(g != f)[0]
    if len(bad):
        raise AssertionError(f"{what}: not a fixpoint at {len(bad)} vertices, e.g. {bad[:5]}")
    fin = f[f != TOP]
    if len(fin) and (fin.min() < 0 or fin.max() > bound):
        raise AssertionError(f"{what}: finite value outside [0, {bound}]")


def medium_games():
    return [
        synth.gen_uniform(1500, 3, 20, 11),
        synth.gen_uniform(1000, 4, 10, 1),
        synth.gen_torus(24, seed=4),
        synth.gen_rmat(9, 8, wlim=50, seed=3),
        synth.gen_uniform(700, 3, 5, 13),
    ]


# --------------------------------------------------------------------------- strategy (Lemma 1)
def _sigma_dict(game, choice):
    """Full positional strategy {v: edge index}: the given choice, else v's first edge."""
    return {v: int(game.off[v]) + max(0, int(choice[v])) for v in range(game.n) if game.owner[v] == 0}


def _credit_under(game, sigma, v):
    """Credit player 0 needs at v when playing sigma: None if a negative cycle is
    reachable from v in G(sigma) (Lemma 1), else the worst deficit over the
    simple paths from v."""
    adj = brute._induced_edges(game, sigma)
    reach = brute._reachable(adj, v)
    if any(brute._has_negative_cycle_through(adj, u, set(range(game.n))) for u in reach):
        return None
    return brute._worst_deficit(adj, v)


def pin_strategy_brute(strategy, count=600, n_max=6, deg_max=3, wlim=4, seed0=90_000):
    """``strategy(game, f) -> choice`` on tiny games, against brute force over G(sigma0):
    * choice is -1 exactly on player-1 vertices and on TOP vertices;
    * from every v in W0 the chosen strategy wins (no negative cycle reachable,
      Lemma 1) with credit exactly f(v) (Def. 4: f(v) is the least credit);
    * at every player-0 v in W0, each earlier out-edge, played instead, needs more
      than f(v) or loses (the choice is the first edge that achieves f(v))."""
    for s in range(count):
        g = synth.gen_random_small(seed0 + s, n_max=n_max, deg_max=deg_max, wlim=wlim)
        f = brute.credits_fw(g)
        choice = np.asarray(strategy(g, f))
        what = f"strategy seed={seed0 + s} n={g.n}"
        want_neg = (g.owner == 1) | (f == TOP)
        if not np.array_equal(choice < 0, want_neg):
            raise AssertionError(f"{what}: choice {choice.tolist()} f {fmt(f)} owner {g.owner.tolist()}")
        if np.any(choice >= np.diff(g.off)):
            raise AssertionError(f"{what}: choice past the row end {choice.tolist()}")
        sigma = _sigma_dict(g, choice)
        for v in range(g.n):
            if f[v] == TOP:
                continue
            c = _credit_under(g, sigma, v)
            if c is None or c != f[v]:
                raise AssertionError(f"{what}: v={v} needs {c} under the strategy, f={f[v]}")
            if g.owner[v] == 0:
                for k in range(int(choice[v])):
                    alt = dict(sigma)
                    alt[v] = int(g.off[v]) + k
                    ca = _credit_under(g, alt, v)
                    if ca is not None and ca <= f[v]:
                        raise AssertionError(f"{what}: v={v} edge {k} < choice {choice[v]} also needs only {ca}")


def pin_strategy_cases(strategy):
    """Hand cases: two edges into 0-sinks with weights (a, b); a trap; a player-1 vertex."""
    for a, b, want in [(-3, -1, 1), (-1, -1, 0), (-1, -3, 0), (2, 5, 0), (-4, 0, 1)]:
        g = synth.make_game(3, [(0, 1, a), (0, 2, b), (1, 1, 0), (2, 2, 0)], [0, 0, 0], W=4)
        f = np.array([max(0, -max(a, b)), 0, 0], dtype=np.int64)
        got = np.asarray(strategy(g, f))
        if got.tolist() != [want, 0, 0]:
            raise AssertionError(f"strategy a={a} b={b}: got {got.tolist()} want {[want, 0, 0]}")
    # 1 is a -1 self-loop trap (TOP); 0 must avoid it through its second edge
    g = synth.make_game(3, [(0, 1, 5), (0, 2, -2), (1, 1, -1), (2, 2, 0)], [0, 0, 1], W=2)
    got = np.asarray(strategy(g, np.array([2, TOP, 0], dtype=np.int64)))
    if got.tolist() != [1, -1, -1]:
        raise AssertionError(f"strategy trap: got {got.tolist()} want [1, -1, -1]")


def pin_strategy_properties(game, f, bound, choice, what=""):
    """Properties of player 0's strategy that hold at any size (numpy, no oracle):
    -1 exactly on player-1 and TOP vertices; otherwise the chosen edge satisfies
    the first condition of Def. 5, f(v) >= f(u) (-) w, and no earlier edge does."""
    f = np.asarray(f, dtype=np.int64)
    choice = np.asarray(choice, dtype=np.int64)
    deg = np.diff(game.off).astype(np.int64)
    want_neg = (game.owner == 1) | (f == TOP)
    bad = np.nonzero((choice < 0) != want_neg)[0]
    if len(bad):
        raise AssertionError(f"{what}: -1 misplaced at {len(bad)} vertices, e.g. {bad[:5]}")
    if np.any(choice >= deg):
        raise AssertionError(f"{what}: choice past the end of its row")
    ft = f[game.tgt.astype(np.int64)]
    is_top = ft == TOP
    t = np.where(is_top, TOP, np.maximum(np.where(is_top, 0, ft) - game.w.astype(np.int64), 0))
    t = np.where((t != TOP) & (t > bound), TOP, t)
    src = np.repeat(np.arange(game.n), deg)
    ok = (t != TOP) & (t <= f[src])
    local = np.arange(len(game.tgt), dtype=np.int64) - game.off[:-1].astype(np.int64)[src]
    first = np.minimum.reduceat(np.where(ok, local, np.iinfo(np.int64).max), game.off[:-1].astype(np.int64))
    sel = ~want_neg
    diff = np.nonzero(first[sel] != choice[sel])[0]
    if len(diff):
        v = np.nonzero(sel)[0][diff[:5]]
        raise AssertionError(f"{what}: choice is not the first witnessing edge at {len(diff)} vertices, e.g. {v}")
