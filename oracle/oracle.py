"""Python front end of the CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use this module.  It compiles ``eg_oracle.c`` with the host C compiler into
``liboracle.so`` next to it and calls it through ctypes.  Nothing here is shared
with, or imported by, the device solver.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

TOP = np.iinfo(np.int64).max  # the oracle's (and the API's) marker for TOP

FIFO, LIFO, RANDOM, JACOBI, ROUNDS, ALG1 = 0, 1, 2, 3, 4, 5
ORDERS = {"fifo": FIFO, "lifo": LIFO, "random": RANDOM, "jacobi": JACOBI, "rounds": ROUNDS,
          "alg1": ALG1}
BOUND_NW, BOUND_MG, BOUND_EXPLICIT = 0, 1, 2


class _Stats(ctypes.Structure):
    _fields_ = [("lifts", ctypes.c_uint64), ("relaxed_edges", ctypes.c_uint64),
                ("pushes", ctypes.c_uint64), ("changes", ctypes.c_uint64),
                ("rounds", ctypes.c_uint64), ("bound", ctypes.c_int64)]


@dataclass
class OracleResult:
    f: np.ndarray  # int64[n], TOP = INT64_MAX
    status: int  # 0 fixpoint, 1 stopped by the lift budget
    lifts: int
    relaxed_edges: int
    pushes: int
    changes: int
    rounds: int
    bound: int


def build(force: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle (gcc -O2, no shared code with the device solver)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, out)
    return out


_libs: dict = {}


def _load(path: str | None = None):
    key = path or LIB
    lib = _libs.get(key)
    if lib is None:
        if path is None:
            build()
        lib = ctypes.CDLL(key)
        p = ctypes.POINTER
        lib.orc_solve.argtypes = [ctypes.c_int32, p(ctypes.c_int64), p(ctypes.c_int32),
                                  p(ctypes.c_int32), p(ctypes.c_uint8), ctypes.c_int32, ctypes.c_int,
                                  ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, p(ctypes.c_int64),
                                  ctypes.c_uint64, p(ctypes.c_int64), p(_Stats)]
        lib.orc_solve.restype = ctypes.c_int
        lib.orc_bound.argtypes = [ctypes.c_int32, p(ctypes.c_int64), p(ctypes.c_int32),
                                  ctypes.c_int32, ctypes.c_int, ctypes.c_int64]
        lib.orc_bound.restype = ctypes.c_int64
        lib.orc_count_unstable.argtypes = [ctypes.c_int32, p(ctypes.c_int64), p(ctypes.c_int32),
                                           p(ctypes.c_int32), p(ctypes.c_uint8), ctypes.c_int64,
                                           p(ctypes.c_int64)]
        lib.orc_count_unstable.restype = ctypes.c_int64
        lib.orc_strategy.argtypes = [ctypes.c_int32, p(ctypes.c_int64), p(ctypes.c_int32),
                                     p(ctypes.c_int32), p(ctypes.c_uint8), ctypes.c_int64,
                                     p(ctypes.c_int64), p(ctypes.c_int32)]
        lib.orc_strategy.restype = ctypes.c_int64
        _libs[key] = lib
    return lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _arrays(game):
    off = np.ascontiguousarray(game.off, dtype=np.int64)
    tgt = np.ascontiguousarray(game.tgt, dtype=np.int32)
    w = np.ascontiguousarray(game.w, dtype=np.int32)
    owner = np.ascontiguousarray(game.owner, dtype=np.uint8)
    if len(tgt) == 0:  # keep valid pointers for empty edge arrays
        tgt = np.zeros(1, dtype=np.int32)
        w = np.zeros(1, dtype=np.int32)
    return off, tgt, w, owner


def solve(game, order: str | int = "fifo", bound_mode: int = BOUND_NW, bound: int = 0,
          f_init: np.ndarray | None = None, max_lifts: int = 0, seed: int = 1,
          lib_path: str | None = None) -> OracleResult:
    """Least energy progress measure of ``game`` (TOP = INT64_MAX)."""
    lib = _load(lib_path)
    off, tgt, w, owner = _arrays(game)
    n = int(game.n)
    f = np.empty(max(n, 1), dtype=np.int64)
    st = _Stats()
    fi = None
    if f_init is not None:
        fi = np.ascontiguousarray(f_init, dtype=np.int64)
    order_id = ORDERS[order] if isinstance(order, str) else int(order)
    rc = lib.orc_solve(n, _ptr(off, ctypes.c_int64), _ptr(tgt, ctypes.c_int32),
                       _ptr(w, ctypes.c_int32), _ptr(owner, ctypes.c_uint8), int(game.W),
                       int(bound_mode), int(bound), order_id, int(seed),
                       _ptr(fi, ctypes.c_int64) if fi is not None else None, int(max_lifts),
                       _ptr(f, ctypes.c_int64), ctypes.byref(st))
    if rc < 0:
        raise MemoryError("oracle allocation failed")
    return OracleResult(f=f[:n], status=rc, lifts=st.lifts, relaxed_edges=st.relaxed_edges,
                        pushes=st.pushes, changes=st.changes, rounds=st.rounds, bound=st.bound)


def bound_of(game, bound_mode: int = BOUND_NW, bound: int = 0, lib_path: str | None = None) -> int:
    lib = _load(lib_path)
    off, tgt, w, owner = _arrays(game)
    return int(lib.orc_bound(int(game.n), _ptr(off, ctypes.c_int64), _ptr(w, ctypes.c_int32),
                             int(game.W), int(bound_mode), int(bound)))


def count_unstable(game, f: np.ndarray, bound: int, lib_path: str | None = None) -> int:
    """Number of vertices where ``f`` is not a fixpoint of the lifting operator."""
    lib = _load(lib_path)
    off, tgt, w, owner = _arrays(game)
    fa = np.ascontiguousarray(f, dtype=np.int64)
    return int(lib.orc_count_unstable(int(game.n), _ptr(off, ctypes.c_int64),
                                      _ptr(tgt, ctypes.c_int32), _ptr(w, ctypes.c_int32),
                                      _ptr(owner, ctypes.c_uint8), int(bound),
                                      _ptr(fa, ctypes.c_int64)))


def strategy(game, f: np.ndarray, bound: int | None = None, lib_path: str | None = None):
    """Player 0's positional strategy from the progress measure ``f`` (Def. 5, Lemma 1).

    Returns (choice, missing): choice[v] is the index, within v's out-edges, of
    the first edge e with f(v) >= f(target) (-) w(e), for player-0 vertices with
    finite f(v), else -1; missing counts player-0 vertices with finite f(v) and
    no such edge (0 when f is a progress measure).  ``bound`` defaults to (n-1)W.
    """
    lib = _load(lib_path)
    off, tgt, w, owner = _arrays(game)
    n = int(game.n)
    if bound is None:
        bound = bound_of(game, lib_path=lib_path)
    fa = np.ascontiguousarray(f, dtype=np.int64)
    choice = np.empty(max(n, 1), dtype=np.int32)
    missing = lib.orc_strategy(n, _ptr(off, ctypes.c_int64), _ptr(tgt, ctypes.c_int32),
                               _ptr(w, ctypes.c_int32), _ptr(owner, ctypes.c_uint8), int(bound),
                               _ptr(fa, ctypes.c_int64), _ptr(choice, ctypes.c_int32))
    return choice[:n], int(missing)
