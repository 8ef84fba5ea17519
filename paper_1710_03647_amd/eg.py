"""Python binding of libeg (ctypes).  Argument marshalling only: every step of
the solve runs in the library's HIP kernels.  Torch is used, when given, only
for device buffers (``data_ptr``) and stream handles.

Raises ``RuntimeError`` if ``libeg.so`` has not been built: there is no other
implementation behind these calls.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libeg.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "eg.h")

EG_TOP = np.iinfo(np.int64).max
EG_OK, EG_PENDING = 0, 1
EG_EINVAL, EG_ENOMEM, EG_EDEVICE, EG_ETIMEDOUT, EG_EBUSY, EG_ENOTFOUND, EG_ECANCELED = -1, -2, -3, -4, -5, -6, -7
EG_BOUND_NW, EG_BOUND_MG = 0, 1
EG_MEM_HOST, EG_MEM_DEVICE = 0, 1
ERROR_NAMES = {EG_EINVAL: "EG_EINVAL", EG_ENOMEM: "EG_ENOMEM", EG_EDEVICE: "EG_EDEVICE",
               EG_ETIMEDOUT: "EG_ETIMEDOUT", EG_EBUSY: "EG_EBUSY", EG_ENOTFOUND: "EG_ENOTFOUND",
               EG_ECANCELED: "EG_ECANCELED", EG_PENDING: "EG_PENDING"}

EXPORTS = ["eg_ctx_create", "eg_ctx_destroy", "eg_check", "eg_create", "eg_destroy", "eg_solve",
           "eg_solve_ex", "eg_solve_seeded_noalloc", "eg_set_measure", "eg_strategy", "eg_components", "eg_submit", "eg_poll", "eg_cancel", "eg_wait", "eg_solve_batch",
           "eg_last_error"]


class EgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class eg_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hip_stream", ctypes.c_void_p),
                ("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int),
                ("bound_mode", ctypes.c_int), ("max_rounds", ctypes.c_uint64),
                ("time_budget_s", ctypes.c_double), ("max_pending", ctypes.c_int),
                ("partition", ctypes.c_int), ("blocks_per_cu", ctypes.c_int), ("dense_div", ctypes.c_int),
                ("small_limit", ctypes.c_int), ("top_seeding", ctypes.c_int), ("seg_edges", ctypes.c_int),
                ("relabel", ctypes.c_int), ("p1_filter", ctypes.c_int), ("scc_schedule", ctypes.c_int),
                ("hub_cache", ctypes.c_int)]


class eg_game_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("targets", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("owner_bits", ctypes.c_void_p), ("W", ctypes.c_int32), ("mem", ctypes.c_int)]


class eg_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("lifts", ctypes.c_uint64),
                ("relaxed_edges", ctypes.c_uint64), ("pushes", ctypes.c_uint64),
                ("changes", ctypes.c_uint64), ("scanned_preds", ctypes.c_uint64),
                ("t_upload", ctypes.c_double),
                ("t_rcsr", ctypes.c_double), ("t_solve", ctypes.c_double), ("t_d2h", ctypes.c_double),
                ("model_bytes", ctypes.c_double), ("achieved_gbps", ctypes.c_double),
                ("t_round_kernels", ctypes.c_double), ("t_queue", ctypes.c_double),
                ("t_latency", ctypes.c_double), ("launched_rounds", ctypes.c_uint64),
                ("dense_rounds", ctypes.c_uint64), ("seeded", ctypes.c_uint64), ("seed_passes", ctypes.c_uint64),
                ("all_rounds", ctypes.c_uint64), ("t_seed", ctypes.c_double),
                ("filtered_preds", ctypes.c_uint64), ("scc_components", ctypes.c_uint64),
                ("scc_levels", ctypes.c_uint64), ("t_scc", ctypes.c_double), ("t_slices", ctypes.c_double)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class eg_game_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("bound", ctypes.c_int64),
                ("value_bits", ctypes.c_int), ("device_bytes", ctypes.c_uint64),
                ("max_outdeg", ctypes.c_int32), ("max_indeg", ctypes.c_int32)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class eg_solve_opts(ctypes.Structure):
    _fields_ = [("max_rounds", ctypes.c_uint64), ("time_budget_s", ctypes.c_double),
                ("resume", ctypes.c_int), ("driver", ctypes.c_int)]


_lib = None


def lib():
    """The loaded libeg (RuntimeError if it was not built)."""
    global _lib
    if _lib is None:
        try:
            # One HIP runtime per process: when torch is installed its runtime is
            # loaded first and libeg binds to it, so torch streams and device
            # pointers can be handed to libeg.
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.eg_ctx_create.argtypes = [P(eg_config), P(vp)]
        L.eg_ctx_destroy.argtypes = [vp]
        L.eg_check.argtypes = [P(eg_game_desc), ctypes.c_int, P(eg_game_info), ctypes.c_char_p, ctypes.c_size_t]
        L.eg_create.argtypes = [vp, P(eg_game_desc), P(vp), P(eg_stats)]
        L.eg_destroy.argtypes = [vp]
        L.eg_solve.argtypes = [vp, vp, P(eg_stats)]
        L.eg_solve_ex.argtypes = [vp, P(eg_solve_opts), vp, P(eg_stats)]
        L.eg_solve_seeded_noalloc.argtypes = [vp, P(eg_solve_opts), vp, P(eg_stats)]
        L.eg_set_measure.argtypes = [vp, vp]
        L.eg_strategy.argtypes = [vp, vp, P(ctypes.c_double)]
        L.eg_components.argtypes = [vp, vp, vp, P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.eg_submit.argtypes = [vp, P(eg_game_desc), P(ctypes.c_uint64)]
        L.eg_poll.argtypes = [vp, ctypes.c_uint64, vp, P(eg_stats)]
        L.eg_cancel.argtypes = [vp, ctypes.c_uint64]
        L.eg_wait.argtypes = [vp, ctypes.c_uint64, vp, P(eg_stats), ctypes.c_double]
        L.eg_solve_batch.argtypes = [vp, P(eg_game_desc), ctypes.c_int, P(ctypes.c_void_p), P(eg_stats)]
        L.eg_last_error.argtypes = [vp]
        L.eg_last_error.restype = ctypes.c_char_p
        for name in EXPORTS[:-1]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _err(code: int, ctx=None) -> EgError:
    msg = lib().eg_last_error(ctx)
    return EgError(code, msg.decode() if msg else "")


def _ptr(a) -> int:
    if a is None:
        return 0
    if hasattr(a, "data_ptr"):
        return int(a.data_ptr())
    return int(a.ctypes.data)


@dataclass
class _HostGame:
    """Host arrays of a game kept alive for the duration of a call."""
    n: int
    off: np.ndarray
    tgt: np.ndarray
    w: np.ndarray
    bits: np.ndarray
    W: int


def _host_arrays(game) -> _HostGame:
    off = np.ascontiguousarray(game.off, dtype=np.int64)
    tgt = np.ascontiguousarray(game.tgt, dtype=np.int32)
    w = np.ascontiguousarray(game.w, dtype=np.int32)
    bits = np.ascontiguousarray(game.owner_bits(), dtype=np.uint8)
    return _HostGame(int(game.n), off, tgt, w, bits, int(game.W))


def make_desc(game=None, *, n=None, offsets=None, targets=None, weights=None, owner_bits=None, W=None,
              device=False):
    """Descriptor of a game.  Either a ``synth.Game`` (host arrays) or explicit
    arrays (numpy for host, torch device tensors with ``device=True``).
    Returns (desc, keepalive)."""
    if game is not None:
        h = _host_arrays(game)
        d = eg_game_desc(h.n, int(h.off[-1]), _ptr(h.off), _ptr(h.tgt), _ptr(h.w), _ptr(h.bits), h.W,
                         EG_MEM_HOST)
        return d, h
    m = int(targets.numel() if hasattr(targets, "numel") else len(targets))
    d = eg_game_desc(int(n), m, _ptr(offsets), _ptr(targets), _ptr(weights), _ptr(owner_bits), int(W),
                     EG_MEM_DEVICE if device else EG_MEM_HOST)
    return d, (offsets, targets, weights, owner_bits)


def check(game=None, bound_mode: int = EG_BOUND_NW, **arrays) -> dict:
    """Host-only validation (eg_check).  Raises EgError(EG_EINVAL) on a bad game."""
    desc, keep = make_desc(game, **arrays)
    info = eg_game_info()
    msg = ctypes.create_string_buffer(512)
    rc = lib().eg_check(ctypes.byref(desc), bound_mode, ctypes.byref(info), msg, 512)
    if rc != EG_OK:
        raise EgError(rc, msg.value.decode())
    return info.to_dict()


class Context:
    """An eg_ctx on one device.  ``stream`` may be a torch.cuda.Stream or a raw handle."""

    def __init__(self, device: int = 0, stream=None, hbm_budget_bytes: int = 0, max_slots: int = 0,
                 bound_mode: int = EG_BOUND_NW, max_rounds: int = 0, time_budget_s: float = 0.0,
                 max_pending: int = 0, partition: int = 0, blocks_per_cu: int = 0, dense_div: int = 0,
                 small_limit: int = 0, top_seeding: int = 0, seg_edges: int = 0, relabel: int = 0,
                 p1_filter: int = 0, scc_schedule: int = 0, hub_cache: int = 0):
        handle = getattr(stream, "cuda_stream", stream) or 0
        cfg = eg_config(device, handle, hbm_budget_bytes, max_slots, bound_mode, max_rounds, time_budget_s,
                        max_pending, partition, blocks_per_cu, dense_div, small_limit, int(top_seeding),
                        seg_edges, relabel, int(p1_filter), int(scc_schedule), int(hub_cache))
        p = ctypes.c_void_p()
        rc = lib().eg_ctx_create(ctypes.byref(cfg), ctypes.byref(p))
        if rc != EG_OK:
            raise _err(rc)
        self.handle = p
        self.device = device
        self._games = weakref.WeakSet()

    def close(self):
        """eg_ctx_destroy: cancels unfinished tickets and frees the context's
        games (their Game objects are marked destroyed)."""
        if self.handle:
            for g in list(self._games):
                g.handle = None
            lib().eg_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def create(self, game=None, **arrays) -> "Game":
        desc, keep = make_desc(game, **arrays)
        p = ctypes.c_void_p()
        st = eg_stats()
        rc = lib().eg_create(self.handle, ctypes.byref(desc), ctypes.byref(p), ctypes.byref(st))
        if rc != EG_OK:
            raise _err(rc, self.handle)
        g = Game(self, p, desc.n, st.to_dict())
        self._games.add(g)
        return g

    # serving
    def submit(self, game=None, **arrays) -> int:
        desc, keep = make_desc(game, **arrays)
        t = ctypes.c_uint64()
        rc = lib().eg_submit(self.handle, ctypes.byref(desc), ctypes.byref(t))
        if rc != EG_OK:
            raise _err(rc, self.handle)
        return int(t.value)

    def poll(self, ticket: int, n: int):
        """(status, credits or None, stats dict)."""
        out = np.empty(n, dtype=np.int64)
        st = eg_stats()
        rc = lib().eg_poll(self.handle, ticket, _ptr(out), ctypes.byref(st))
        if rc == EG_OK:
            return rc, out, st.to_dict()
        if rc == EG_PENDING:
            return rc, None, None
        raise _err(rc, self.handle)

    def cancel(self, ticket: int) -> int:
        return lib().eg_cancel(self.handle, ticket)

    def wait(self, ticket: int, n: int, timeout_s: float = 0.0):
        """Block until the ticket is done: (status, credits or None, stats dict or None)."""
        out = np.empty(n, dtype=np.int64)
        st = eg_stats()
        rc = lib().eg_wait(self.handle, ticket, _ptr(out), ctypes.byref(st), timeout_s)
        if rc == EG_OK:
            return rc, out, st.to_dict()
        if rc == EG_PENDING:
            return rc, None, None
        raise _err(rc, self.handle)

    def solve_batch(self, games):
        """Solve many games in the batched iteration: list of (credits, stats)."""
        keep = [make_desc(g) for g in games]
        descs = (eg_game_desc * len(games))(*[d for d, _ in keep])
        outs = [np.empty(g.n, dtype=np.int64) for g in games]
        ptrs = (ctypes.c_void_p * len(games))(*[o.ctypes.data for o in outs])
        stats = (eg_stats * len(games))()
        rc = lib().eg_solve_batch(self.handle, descs, len(games), ptrs, stats)
        if rc != EG_OK:
            raise _err(rc, self.handle)
        return [(outs[i], stats[i].to_dict()) for i in range(len(games))]


class Game:
    """A device-resident game (eg_game)."""

    def __init__(self, ctx: Context, handle, n: int, create_stats: dict):
        self.ctx = ctx
        self.handle = handle
        self.n = n
        self.create_stats = create_stats

    def solve(self, out=None, max_rounds: int = 0, time_budget_s: float = 0.0, resume: bool = False,
              allow_timeout: bool = False):
        """Solve to the least fixpoint.  Returns (credits int64[n], stats dict, status)."""
        if out is None:
            out = np.empty(self.n, dtype=np.int64)
        st = eg_stats()
        opts = eg_solve_opts(max_rounds, time_budget_s, 1 if resume else 0, 0)
        rc = lib().eg_solve_ex(self.handle, ctypes.byref(opts), _ptr(out), ctypes.byref(st))
        if rc != EG_OK and not (allow_timeout and rc == EG_ETIMEDOUT):
            raise _err(rc, self.ctx.handle)
        return out, st.to_dict(), rc

    def solve_noalloc(self, out=None, max_rounds: int = 0, time_budget_s: float = 0.0, resume: bool = False):
        """eg_solve_seeded_noalloc: a seeded solve that allocates nothing (its
        seeding scratch is the library's static per-device array).  Returns
        (credits int64[n], stats dict, status)."""
        if out is None:
            out = np.empty(self.n, dtype=np.int64)
        st = eg_stats()
        opts = eg_solve_opts(max_rounds, time_budget_s, 1 if resume else 0, 0)
        rc = lib().eg_solve_seeded_noalloc(self.handle, ctypes.byref(opts), _ptr(out), ctypes.byref(st))
        if rc != EG_OK:
            raise _err(rc, self.ctx.handle)
        return out, st.to_dict(), rc

    def set_measure(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.int64)
        rc = lib().eg_set_measure(self.handle, _ptr(f))
        if rc != EG_OK:
            raise _err(rc, self.ctx.handle)

    def strategy(self, out=None):
        """Player 0's positional strategy from the least fixpoint reached by the
        last solve (eg_strategy).  Returns (choice int32[n], kernel seconds):
        choice[v] indexes v's out-edges, -1 for player-1 and TOP vertices."""
        if out is None:
            out = np.empty(self.n, dtype=np.int32)
        t = ctypes.c_double(0.0)
        rc = lib().eg_strategy(self.handle, _ptr(out), ctypes.byref(t))
        if rc != EG_OK:
            raise _err(rc, self.ctx.handle)
        return out, t.value

    def components(self):
        """Strongly connected components and condensation levels (eg_components).
        Returns (comp int32[n], level int32[n], number of components, number of levels)."""
        comp = np.empty(self.n, dtype=np.int32)
        level = np.empty(self.n, dtype=np.int32)
        nc, nl = ctypes.c_uint32(0), ctypes.c_uint32(0)
        rc = lib().eg_components(self.handle, _ptr(comp), _ptr(level), ctypes.byref(nc), ctypes.byref(nl))
        if rc != EG_OK:
            raise _err(rc, self.ctx.handle)
        return comp, level, nc.value, nl.value

    def destroy(self):
        if self.handle:
            lib().eg_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()


def solve(game, device: int = 0, **kw):
    """One-shot helper: create a context and a game, solve, clean up."""
    with Context(device) as ctx:
        g = ctx.create(game)
        try:
            return g.solve(**kw)
        finally:
            g.destroy()
