"""The mathematics behind TOP seeding, pinned on the CPU (no device code).

The device's seeding passes rest on two facts, checked here against brute
force over positional strategies (a source other than the oracle) on
thousands of tiny games:

* Lemma 1 applied to the forced subgraph (player-1 vertices and player-0
  vertices of out-degree 1): a cycle of chosen edges, one per forced vertex,
  whose weights sum below zero can be forced by player 1 forever, so every
  vertex on it has credit TOP, whichever edge each player-1 vertex chose.
* The Bellman-Ford passes: the lifting operator restricted to that subgraph
  (player 1 maximises over forced successors only, player 0 has no choice,
  every other vertex keeps its value), iterated in any order from a measure
  below the least fixpoint, stays below it; so a value above B proves TOP.

The passes here are written out in Python from those definitions, with the
update the device makes (the term of one chosen edge per vertex, not the
maximum), in random orders to stand for the device's in-place updates."""
import numpy as np

from oracle import brute
from paper_1710_03647_amd import synth

TOP = np.iinfo(np.int64).max


def forced_mask(game):
    deg = np.diff(game.off)
    return (game.owner == 1) | (deg == 1)


def choose(game, vals, forced, v, rng):
    """One candidate edge of v under vals: for player 1 a forced successor with
    a negative self-loop first, then the largest term max(0, vals[u] - w),
    ties broken at random (any choice must be sound); for player 0 of
    out-degree 1 its edge.  Returns (target, weight) or None."""
    a, b = int(game.off[v]), int(game.off[v + 1])
    if game.owner[v] == 0:
        return (int(game.tgt[a]), int(game.w[a])) if b - a == 1 else None
    best, keys = None, []
    for e in range(a, b):
        u, w = int(game.tgt[e]), int(game.w[e])
        if not forced[u]:
            continue
        keys.append(((u == v and w < 0), max(0, vals[u] - w), rng.random(), u, w))
    if keys:
        best = max(keys)
        return best[3], best[4]
    return None


def test_negative_cycles_of_any_choice_are_top():
    rng = np.random.default_rng(5)
    found = 0
    for s in range(1500):
        g = synth.gen_random_small(60_000 + s, n_max=7, deg_max=3, wlim=4)
        want = brute.credits_fw(g)
        forced = forced_mask(g)
        vals = [0] * g.n
        succ = [choose(g, vals, forced, v, rng) for v in range(g.n)]
        # every cycle of the chosen edges, by walking from each vertex
        for v0 in range(g.n):
            seen, x = [], v0
            while x is not None and x not in seen:
                seen.append(x)
                c = succ[x]
                x = c[0] if c is not None else None
            if x is None:
                continue
            cyc = seen[seen.index(x):]
            if sum(succ[y][1] for y in cyc) < 0:
                found += 1
                assert all(want[y] == TOP for y in cyc), (s, cyc, want)
    assert found > 100


def test_bellman_ford_values_stay_below_the_least_fixpoint():
    rng = np.random.default_rng(6)
    proved = 0
    for s in range(1500):
        g = synth.gen_random_small(70_000 + s, n_max=7, deg_max=3, wlim=4)
        want = brute.credits_fw(g)
        bound = (g.n - 1) * g.W
        forced = forced_mask(g)
        # start from 0, or from a random measure below the least fixpoint
        if s % 2:
            vals = [0] * g.n
        else:
            vals = [int(rng.integers(0, bound + 2)) if want[v] == TOP else int(rng.integers(0, want[v] + 1))
                    for v in range(g.n)]
            vals = [min(x, bound + 1) for x in vals]
        for _ in range(12):
            for v in rng.permutation(g.n):
                c = choose(g, vals, forced, int(v), rng)
                if c is None:
                    continue
                tm = min(bound + 1, max(0, vals[c[0]] - c[1]))
                vals[v] = max(vals[v], tm)
        for v in range(g.n):
            if want[v] == TOP:
                proved += vals[v] > bound
            else:
                assert vals[v] <= want[v], (s, v, vals, want)
    assert proved > 50
