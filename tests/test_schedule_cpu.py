"""The round schedule around all-vertex rounds, pinned on the CPU (no device
code) against brute force over positional strategies.

The device starts a solve with all-vertex rounds when the initially active
vertices' predecessors would cover V, runs them in place (a lift may read
values written earlier in the same round, in any order), flags the vertices
each one raises, and on leaving them takes as the next active set the
predecessors of the vertices raised in the last all-vertex round only.  The
claim: every vertex that the last round left unstable has a successor raised
in that round, so the frontier rounds that follow (Alg. 3, also in place)
still end at the least fixpoint.  This file runs that schedule in Python in
random lift orders and compares the result with brute force; a planted
mistake (the raises of the round before the last) must fail."""
import numpy as np

from oracle import brute
from paper_1710_03647_amd import synth

import pins

TOP = pins.TOP


def lift(game, f, v, bound):
    """Def. 6 for one vertex: min (player 0) or max (player 1) over its edges
    of max(0, f(u) - w), TOP above the bound."""
    a, b = int(game.off[v]), int(game.off[v + 1])
    terms = []
    for e in range(a, b):
        u, w = int(game.tgt[e]), int(game.w[e])
        t = TOP if f[u] == TOP else max(0, f[u] - w)
        terms.append(TOP if t != TOP and t > bound else t)
    return min(terms) if game.owner[v] == 0 else max(terms)


def preds_of(game):
    p = [[] for _ in range(game.n)]
    for v in range(game.n):
        for e in range(int(game.off[v]), int(game.off[v + 1])):
            p[int(game.tgt[e])].append(v)
    return p


def schedule(game, rng, all_rounds, planted=False):
    bound = (game.n - 1) * game.W
    f = [0] * game.n
    pr = preds_of(game)
    raised_last, raised_before = set(), set()
    for _ in range(all_rounds):
        raised = set()
        for v in rng.permutation(game.n):
            nv = max(f[v], lift(game, f, int(v), bound))  # writes never lower a value
            if nv != f[v]:
                f[v] = nv
                raised.add(int(v))
        raised_before, raised_last = raised_last, raised
    src = raised_before if planted else raised_last
    act = {p for v in src for p in pr[v]}
    while act:
        raised = set()
        for v in rng.permutation(sorted(act)):
            nv = max(f[v], lift(game, f, int(v), bound))
            if nv != f[v]:
                f[v] = nv
                raised.add(int(v))
        act = {p for v in raised for p in pr[v]}
    return f


def test_frontier_after_all_vertex_rounds_reaches_the_least_fixpoint():
    rng = np.random.default_rng(11)
    for s in range(1200):
        g = synth.gen_random_small(80_000 + s, n_max=7, deg_max=3, wlim=4)
        want = brute.credits_fw(g)
        f = schedule(g, rng, all_rounds=1 + s % 3)
        pins.expect_equal(f, want, f"seed {80_000 + s}")


def test_frontier_from_an_earlier_all_vertex_round_is_caught():
    rng = np.random.default_rng(12)
    wrong = 0
    for s in range(1200):
        g = synth.gen_random_small(80_000 + s, n_max=7, deg_max=3, wlim=4)
        want = brute.credits_fw(g)
        f = schedule(g, rng, all_rounds=2 + s % 2, planted=True)
        wrong += not np.array_equal(np.asarray(f, dtype=np.int64), want)
    assert wrong > 0
