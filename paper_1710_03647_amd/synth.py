"""Seeded synthetic energy games.

This module only draws inputs: arenas (CSR out-edges, integer weights, owner
partition) of the shapes used to exercise the solver.  It contains none of the
solver's arithmetic, and both the device path and the CPU oracle take their
inputs from here.

Arena model (paper Sec. 2, "Weighted graphs" and "Graph games"): a total
directed graph with integer edge weights and a partition of the vertices into
player 0 (owner 0, takes the min in the lifting operator) and player 1 (owner 1,
takes the max).  Edges form a multiset: duplicates and self-loops are kept.

Randomness: one counter-based generator, SplitMix64 (S. Vigna, public domain).
Value i of stream s under seed k is ``mix(key(k, s) + (i + 1) * GAMMA)`` where
``mix`` is the SplitMix64 output finaliser.  An integer in [lo, hi] is
``lo + x mod (hi - lo + 1)`` (bias below 2**-50 for the ranges used here); a
real in [0, 1) is ``(x >> 11) * 2**-53``; a fair bit is ``x >> 63``.
"""
from __future__ import annotations

import hashlib
import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream ids (fixed so that instances are reproducible)
S_TARGET, S_WEIGHT, S_OWNER, S_RMAT, S_PERM, S_PARAM, S_ARRIVAL = 1, 2, 3, 4, 5, 6, 7


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _mix_scalar(z: int) -> int:
    return int(_mix(np.array([z & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0])


def stream_key(seed: int, stream: int) -> int:
    """Key of stream ``stream`` under ``seed``."""
    k = _mix_scalar((seed + int(GAMMA)) & 0xFFFFFFFFFFFFFFFF)
    return _mix_scalar((k + stream) & 0xFFFFFFFFFFFFFFFF)


def draws(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """uint64 values ``start .. start+count-1`` of the given stream."""
    key = np.uint64(stream_key(seed, stream))
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + idx * GAMMA)


def draws_at(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """uint64 values at arbitrary counters ``idx`` of the given stream."""
    key = np.uint64(stream_key(seed, stream))
    with np.errstate(over="ignore"):
        return _mix(key + (idx.astype(np.uint64) + np.uint64(1)) * GAMMA)


def to_int(x: np.ndarray, lo: int, hi: int) -> np.ndarray:
    span = np.uint64(hi - lo + 1)
    return (x % span).astype(np.int64) + lo


def to_unit(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def to_bit(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(63)).astype(np.uint8)


@dataclass
class Game:
    """A total weighted arena in CSR form.

    off[v]..off[v+1] index the out-edges of v in ``tgt``/``w``;
    ``owner[v]`` is 0 (player 0, min) or 1 (player 1, max);
    ``W`` is the weight magnitude passed to the solver (W >= max(0, max -w)).
    """

    n: int
    off: np.ndarray  # int64[n+1]
    tgt: np.ndarray  # int32[m]
    w: np.ndarray  # int32[m]
    owner: np.ndarray  # uint8[n], 0/1
    W: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.off[-1])

    def owner_bits(self) -> np.ndarray:
        """Owner partition packed LSB-first, bit = 1 for player 1."""
        return np.packbits(self.owner.astype(np.uint8), bitorder="little")

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (np.array([self.n, self.W], dtype=np.int64), self.off.astype(np.int64),
                  self.tgt.astype(np.int32), self.w.astype(np.int32), self.owner.astype(np.uint8)):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def outdeg(self) -> np.ndarray:
        return np.diff(self.off)


def _stable_argsort(keys: np.ndarray) -> np.ndarray:
    """The stable sort order of ``keys`` (unique, so any stable sort gives it);
    torch's multithreaded CPU sort when torch is present, numpy's otherwise."""
    if len(keys) >= 1 << 22:
        try:
            import torch

            return torch.sort(torch.from_numpy(np.ascontiguousarray(keys)), stable=True)[1].numpy()
        except ImportError:
            pass
    return np.argsort(keys, kind="stable")


def from_edges(n: int, src: np.ndarray, dst: np.ndarray, w: np.ndarray, owner: np.ndarray,
               W: int | None = None, name: str = "", sink_loops: bool = False) -> Game:
    """CSR by a stable counting sort on the source (row order = input order).

    With ``sink_loops`` every vertex without an out-edge gets one self-loop of
    weight 0 so that the arena is total.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    if sink_loops:
        deg = np.bincount(src, minlength=n)
        sinks = np.nonzero(deg == 0)[0]
        src = np.concatenate([src, sinks])
        dst = np.concatenate([dst, sinks])
        w = np.concatenate([w, np.zeros(len(sinks), dtype=np.int64)])
    order = _stable_argsort(src)
    deg = np.bincount(src, minlength=n)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    if W is None:
        W = int(max(0, -int(w.min()))) if len(w) else 0
    return Game(n=n, off=off, tgt=dst[order].astype(np.int32), w=w[order].astype(np.int32),
                owner=np.asarray(owner, dtype=np.uint8).copy(), W=int(W), name=name)


def gen_uniform(n: int, deg: int, wlim: int, seed: int, name: str | None = None) -> Game:
    """Every vertex gets exactly ``deg`` targets uniform on [0, n) (self-loops and
    duplicates allowed), weights uniform in [-wlim, wlim], owners Bernoulli(0.5).

    Edge i = v*deg + j is the j-th out-edge of v; its target and weight are value
    i of the target and weight streams.
    """
    m = n * deg
    tgt = to_int(draws(seed, S_TARGET, 0, m), 0, n - 1).astype(np.int32)
    w = to_int(draws(seed, S_WEIGHT, 0, m), -wlim, wlim).astype(np.int32)
    owner = to_bit(draws(seed, S_OWNER, 0, n))
    off = np.arange(n + 1, dtype=np.int64) * deg
    return Game(n=n, off=off, tgt=tgt, w=w, owner=owner, W=wlim,
                name=name or f"uniform-n{n}-d{deg}-W{wlim}-s{seed}",
                meta=dict(kind="uniform", n=n, deg=deg, wlim=wlim, seed=seed))


def gen_plain(seed: int = 1) -> Game:
    """Plain single game: n=1000, out-degree 4, weights in [-10, 10]."""
    return gen_uniform(1000, 4, 10, seed, name="plain-n1000-d4-W10")


def gen_uniform_full(seed: int = 2) -> Game:
    """Uniform random game: n=2**20, out-degree 16, weights in [-1000, 1000]."""
    return gen_uniform(1 << 20, 16, 1000, seed, name="uniform-n1048576-d16-W1000")


def gen_rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
             wlim: int = 10000, seed: int = 3, name: str | None = None) -> Game:
    """R-MAT graph (Graph500 style): ``edge_factor * 2**scale`` edges, each placed
    by ``scale`` recursive quadrant draws with probabilities (a, b, c, 1-a-b-c)
    and no parameter noise, then a seeded random relabelling of the vertices.
    Duplicates and self-loops are kept; every sink gets one 0-weight self-loop.
    Weights uniform in [-wlim, wlim] (drawn in generation order); owners
    Bernoulli(0.5) on the relabelled ids.
    """
    n = 1 << scale
    m0 = edge_factor * n
    src = np.zeros(m0, dtype=np.int64)
    dst = np.zeros(m0, dtype=np.int64)
    ab, abc = a + b, a + b + c

    def place(lo: int, hi: int) -> None:
        # edges [lo, hi): the same draws whatever the chunking
        eidx = np.arange(lo, hi, dtype=np.uint64)
        s_, d_ = src[lo:hi], dst[lo:hi]
        for lvl in range(scale):
            u = to_unit(draws_at(seed, S_RMAT, eidx * np.uint64(scale) + np.uint64(lvl)))
            s_ <<= 1
            s_ |= u >= ab  # quadrants c, d: source bit 1
            d_ <<= 1
            d_ |= ((u >= a) & (u < ab)) | (u >= abc)  # quadrants b, d

    chunk = 1 << 20
    spans = [(lo, min(m0, lo + chunk)) for lo in range(0, m0, chunk)]
    if len(spans) > 1:
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(lambda sp: place(*sp), spans))
    else:
        place(0, m0)
    perm = np.argsort(draws(seed, S_PERM, 0, n), kind="stable")  # vertex v -> perm[v]
    src = perm[src]
    dst = perm[dst]
    w = to_int(draws(seed, S_WEIGHT, 0, m0), -wlim, wlim)
    owner = to_bit(draws(seed, S_OWNER, 0, n))
    g = from_edges(n, src, dst, w, owner, W=wlim, sink_loops=True,
                   name=name or f"rmat-s{scale}-ef{edge_factor}-W{wlim}-s{seed}")
    g.meta = dict(kind="rmat", scale=scale, edge_factor=edge_factor, wlim=wlim, seed=seed)
    return g


def gen_rmat_full(seed: int = 3) -> Game:
    return gen_rmat(22, 16, seed=seed, name="rmat-s22-ef16-W10000")


def gen_torus(side: int, wlo: int = -100, whi: int = 100, bias: int = 2, seed: int = 4,
              name: str | None = None) -> Game:
    """side x side directed torus; vertex id r*side + c has out-edges to its N, S,
    W and E neighbours (in that order, with wraparound).  Weights uniform in
    [wlo, whi] plus ``bias``; owners Bernoulli(0.5)."""
    n = side * side
    v = np.arange(n, dtype=np.int64)
    r, c = v // side, v % side
    nbr = np.stack([((r - 1) % side) * side + c, ((r + 1) % side) * side + c,
                    r * side + (c - 1) % side, r * side + (c + 1) % side], axis=1).reshape(-1)
    m = 4 * n
    w = to_int(draws(seed, S_WEIGHT, 0, m), wlo, whi) + bias
    owner = to_bit(draws(seed, S_OWNER, 0, n))
    W = max(0, -(wlo + bias), whi + bias)
    return Game(n=n, off=np.arange(n + 1, dtype=np.int64) * 4, tgt=nbr.astype(np.int32),
                w=w.astype(np.int32), owner=owner, W=W,
                name=name or f"torus-{side}x{side}-s{seed}",
                meta=dict(kind="torus", side=side, seed=seed))


def gen_torus_full(seed: int = 4) -> Game:
    return gen_torus(2048, seed=seed, name="torus-2048x2048")


def stream_game_params(g: int, seed: int = 5) -> dict:
    """Parameters of game ``g`` of the serving stream: n log-uniform in [1e3, 1e5],
    out-degree uniform in {2..16}, W log-uniform in [10, 1000]."""
    x = draws(seed, S_PARAM, 4 * g, 4)
    n = int(math.floor(10.0 ** (3.0 + 2.0 * float(to_unit(x[0:1])[0]))))
    deg = int(to_int(x[1:2], 2, 16)[0])
    W = int(round(10.0 ** (1.0 + 2.0 * float(to_unit(x[2:3])[0]))))
    gseed = int(x[3] & np.uint64(0x7FFFFFFFFFFFFFFF))
    return dict(n=n, deg=deg, W=W, seed=gseed)


def gen_stream_game(g: int, seed: int = 5, scale_n: float = 1.0) -> Game:
    """Game ``g`` of the serving stream (uniform targets, weights in [-W, W])."""
    p = stream_game_params(g, seed)
    n = max(1, int(p["n"] * scale_n))
    game = gen_uniform(n, p["deg"], p["W"], p["seed"], name=f"stream{seed}-g{g}")
    game.meta.update(dict(kind="stream", index=g))
    return game


def poisson_arrivals(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    u = to_unit(draws(seed, S_ARRIVAL, 0, count))
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)


def gen_random_small(rng_seed: int, n_max: int = 7, deg_max: int = 3, wlim: int = 4,
                     owner_mode: str = "mixed") -> Game:
    """Tiny arena for exhaustive checks: n in [1, n_max], out-degree in
    [1, deg_max] per vertex, weights in [-wlim, wlim]; duplicates and self-loops
    allowed.  ``owner_mode`` is 'mixed', 'p0' (all player 0) or 'p1'."""
    x = draws(rng_seed, S_PARAM, 0, 2)
    n = int(to_int(x[0:1], 1, n_max)[0])
    degs = to_int(draws(rng_seed, S_PARAM, 2, n), 1, deg_max)
    m = int(degs.sum())
    tgt = to_int(draws(rng_seed, S_TARGET, 0, m), 0, n - 1)
    w = to_int(draws(rng_seed, S_WEIGHT, 0, m), -wlim, wlim)
    if owner_mode == "mixed":
        owner = to_bit(draws(rng_seed, S_OWNER, 0, n))
    else:
        owner = np.full(n, 0 if owner_mode == "p0" else 1, dtype=np.uint8)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(degs, out=off[1:])
    return Game(n=n, off=off, tgt=tgt.astype(np.int32), w=w.astype(np.int32), owner=owner,
                W=wlim, name=f"small-{rng_seed}")


def make_game(n: int, edges, owner, W: int | None = None, name: str = "") -> Game:
    """Arena from an explicit edge list [(src, dst, weight), ...] (row order kept)."""
    edges = list(edges)
    src = np.array([e[0] for e in edges], dtype=np.int64)
    dst = np.array([e[1] for e in edges], dtype=np.int64)
    w = np.array([e[2] for e in edges], dtype=np.int64)
    return from_edges(n, src, dst, w, np.asarray(owner, dtype=np.uint8), W=W, name=name)


CONFIGS = {
    "plain": gen_plain,
    "uniform": gen_uniform_full,
    "rmat": gen_rmat_full,
    "torus": gen_torus_full,
}
