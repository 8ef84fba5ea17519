"""Exhaustive checker for tiny energy games (test infrastructure only).

It computes the minimum initial credit straight from the game-theoretic
definitions, without the lifting operator:

* Eq. (1) and Def. 3: player 0 wins a play with credit c if c plus every
  finite prefix sum of the play's weights stays >= 0.
* Memoryless determinacy (Sec. 3): positional player-0 strategies suffice, so
  it enumerates every positional strategy sigma0 (one out-edge per player-0
  vertex; edges are a multiset, so a strategy picks an edge index).
* Lemma 1: sigma0 wins from v iff every cycle reachable from v in the graph
  G(sigma0) (player-0 vertices keep only their chosen edge) is non-negative.
* Then the credit sigma0 needs at v is the worst deficit over the finite paths
  from v in G(sigma0), max(0, max over paths p of -w(p)); removing a
  non-negative cycle from a path never lowers that deficit, so simple paths
  suffice.  The minimum initial credit is the least of these over the winning
  sigma0, and TOP when none wins (Def. 4).

Two independent evaluations are provided: ``credits_dfs`` enumerates simple
cycles and simple paths explicitly; ``credits_fw`` uses Floyd-Warshall shortest
paths (a textbook routine) batched over all strategies.
"""
from __future__ import annotations

import itertools

import numpy as np

TOP = np.iinfo(np.int64).max


def _strategies(game):
    """All positional player-0 strategies as {v: chosen edge index}."""
    p0 = [v for v in range(game.n) if game.owner[v] == 0]
    choices = [range(int(game.off[v]), int(game.off[v + 1])) for v in p0]
    for pick in itertools.product(*choices):
        yield dict(zip(p0, pick))


def _induced_edges(game, sigma):
    """Out-edge lists (target, weight) of G(sigma0)."""
    adj = []
    for v in range(game.n):
        if game.owner[v] == 0:
            es = [sigma[v]]
        else:
            es = range(int(game.off[v]), int(game.off[v + 1]))
        adj.append([(int(game.tgt[e]), int(game.w[e])) for e in es])
    return adj


def _reachable(adj, v):
    seen = {v}
    stack = [v]
    while stack:
        x = stack.pop()
        for y, _ in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return seen


def _has_negative_cycle_through(adj, s, allowed):
    """Is there a simple cycle through s, inside ``allowed``, with negative sum?"""
    # depth-first enumeration of simple paths starting at s
    stack = [(s, 0, frozenset([s]))]
    while stack:
        x, acc, used = stack.pop()
        for y, wt in adj[x]:
            if y not in allowed:
                continue
            if y == s:
                if acc + wt < 0:
                    return True
            elif y not in used:
                stack.append((y, acc + wt, used | {y}))
    return False


def _worst_deficit(adj, v):
    """max(0, max over simple paths p from v of -w(p))."""
    worst = 0
    stack = [(v, 0, frozenset([v]))]
    while stack:
        x, acc, used = stack.pop()
        worst = max(worst, -acc)
        for y, wt in adj[x]:
            if y not in used:
                stack.append((y, acc + wt, used | {y}))
    return worst


def credits_dfs(game) -> np.ndarray:
    """Minimum initial credits by explicit enumeration (TOP = INT64_MAX)."""
    n = game.n
    best = [None] * n
    for sigma in _strategies(game):
        adj = _induced_edges(game, sigma)
        neg = [_has_negative_cycle_through(adj, s, set(range(n))) for s in range(n)]
        for v in range(n):
            reach = _reachable(adj, v)
            if any(neg[u] for u in reach):
                continue  # Lemma 1: sigma0 loses from v
            c = _worst_deficit(adj, v)
            if best[v] is None or c < best[v]:
                best[v] = c
    return np.array([TOP if b is None else b for b in best], dtype=np.int64)


def credits_fw(game) -> np.ndarray:
    """Minimum initial credits with Floyd-Warshall over G(sigma0), vectorised over
    all positional strategies (TOP = INT64_MAX)."""
    n = game.n
    sigmas = list(_strategies(game))
    S = len(sigmas)
    INF = np.inf
    d = np.full((S, n, n), INF)
    for s, sigma in enumerate(sigmas):
        for v in range(n):
            if game.owner[v] == 0:
                es = [sigma[v]]
            else:
                es = range(int(game.off[v]), int(game.off[v + 1]))
            for e in es:
                u = int(game.tgt[e])
                d[s, v, u] = min(d[s, v, u], float(game.w[e]))
    # the empty path has weight 0; a negative self-loop stays below it
    idx = np.arange(n)
    d[:, idx, idx] = np.minimum(d[:, idx, idx], 0.0)
    for k in range(n):
        d = np.minimum(d, d[:, :, k:k + 1] + d[:, k:k + 1, :])
    neg_cycle = d[:, idx, idx] < 0  # (S, n): vertex lies on a negative cycle
    reach = d < INF  # (S, n, n)
    loses = (reach & neg_cycle[:, None, :]).any(axis=2)  # (S, n)
    deficit = np.maximum(0.0, -np.where(reach, d, INF).min(axis=2))
    cred = np.where(loses, INF, deficit)
    best = cred.min(axis=0)
    return np.array([TOP if not np.isfinite(b) else int(b) for b in best], dtype=np.int64)


def credits_one_player_max(game) -> np.ndarray:
    """Closed form for arenas owned entirely by player 1 (Lemma 1 with V0 empty):
    v is TOP iff a negative cycle is reachable from v, otherwise its credit is
    max(0, -min over reachable u of d(v, u)) with d the Floyd-Warshall distance."""
    assert all(int(o) == 1 for o in game.owner)
    return credits_fw(game)
