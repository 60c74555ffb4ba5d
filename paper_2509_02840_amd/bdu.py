"""Python binding of the C ABI in include/bdu.h (argument marshalling only).

Every step of an update runs in the gfx950 kernels of libbdu.so; this module
only passes pointers and sizes.  Arrays may be numpy arrays (host memory) or
torch tensors on the GPU (device memory); both must be float64 and
column-major (Fortran order) for matrices.  The library copies its inputs.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbdu.so")

BDU_OK = 0
BDU_EINVAL = -1
BDU_ENOMEM = -2
BDU_EDEVICE = -3
BDU_ENONFINITE = -4
BDU_EBUSY = -5
BDU_ESPAN = -6
BDU_ESCRATCH = -7


class BduError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_strerror(status)} ({status})")
        self.status = status


_lib = None


def lib():
    """Load libbdu.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.bdu_create.argtypes = [i64, i64, vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.bdu_update.argtypes = [vp, vp, vp, i32]
        L.bdu_update_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(i32), i32]
        L.bdu_update_projected.argtypes = [vp, vp, vp]
        L.bdu_update_noalloc.argtypes = [vp, vp, vp, i32]
        L.bdu_update_noalloc.restype = i32
        L.bdu_noalloc_capacity.argtypes = []
        L.bdu_noalloc_capacity.restype = i64
        L.bdu_project.argtypes = [vp, vp, vp, vp, vp]
        L.bdu_read.argtypes = [vp, vp, vp, vp, vp]
        L.bdu_last_rotations.argtypes = [vp, vp, vp, vp, vp, i64]
        L.bdu_last_rotations.restype = i64
        L.bdu_set_stream.argtypes = [vp, vp]
        L.bdu_sync.argtypes = [vp]
        L.bdu_destroy.argtypes = [vp]
        L.bdu_strerror.argtypes = [i32]
        L.bdu_strerror.restype = ctypes.c_char_p
        L.bdu_footprint_bytes.argtypes = [i64, i64]
        L.bdu_footprint_bytes.restype = i64
        L.bdu_set_tiling.argtypes = [i32, i32, i32]
        L.bdu_get_tiling.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.bdu_plan_stats.argtypes = [i64, i64, ctypes.POINTER(i64)]
        L.bdu_givens_device.argtypes = [vp, vp, i32, vp, vp, vp, i64]
        L.bdu_timing_enable.argtypes = [i32]
        L.bdu_timing_read.argtypes = [vp, vp]
        L.bdu_plan_rotations.argtypes = [i64, i64, vp, vp, vp, vp, i64]
        L.bdu_plan_rotations.restype = i64
        L.bdu_autotune.argtypes = [i64, i64, i32, ctypes.POINTER(i64)]
        L.bdu_set_generation_in_lds.argtypes = [i32]
        L.bdu_set_finite_check.argtypes = [i32]
        L.bdu_set_split_pass.argtypes = [i32]
        L.bdu_plan_segments.argtypes = [i64, i64, vp, vp, vp, i64]
        L.bdu_plan_blocks.argtypes = [i64, i64, ctypes.c_int, vp, i64]
        L.bdu_update_householder.argtypes = [vp, vp, vp]
        L.bdu_orth_error.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.bdu_reorthogonalize.argtypes = [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]
        L.bdu_truncated_bd.argtypes = [vp, i64, vp, ctypes.POINTER(ctypes.c_double), vp, vp]
        L.bdu_track_create.argtypes = [i64, i64, i64, vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.bdu_track_update.argtypes = [vp, vp, vp]
        L.bdu_track_sync.argtypes = [vp]
        L.bdu_track_read.argtypes = [vp, vp, vp, vp, vp]
        L.bdu_track_last.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(i64)]
        L.bdu_track_last_projection.argtypes = [vp, vp, vp, vp, vp]
        dbl = ctypes.POINTER(ctypes.c_double)
        L.bdu_track_orth_error.argtypes = [vp, dbl, dbl]
        L.bdu_track_reorthogonalize.argtypes = [vp, ctypes.c_double, dbl, dbl]
        L.bdu_track_set_drift_check.argtypes = [vp, i64, ctypes.c_double]
        L.bdu_track_drift_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), dbl, dbl]
        L.bdu_track_destroy.argtypes = [vp]
        L.bdu_tune_save.argtypes = [ctypes.c_char_p]
        L.bdu_tune_load.argtypes = [ctypes.c_char_p]
        L.bdu_handle_tiling.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.bdu_server_create.argtypes = [i64, i32, i32, ctypes.POINTER(vp)]
        L.bdu_server_create_classes.argtypes = [i64, i32, i32, ctypes.POINTER(i64), i32, ctypes.POINTER(vp)]
        L.bdu_server_class_of.argtypes = [vp, i64]
        L.bdu_server_reset_stats.argtypes = [vp]
        L.bdu_server_open.argtypes = [vp, i64, i64, vp, vp, vp, vp, ctypes.POINTER(i32)]
        L.bdu_server_submit.argtypes = [vp, i32, vp, vp, i32, ctypes.POINTER(i64)]
        L.bdu_server_wait.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
        L.bdu_server_poll.argtypes = [vp, i64]
        L.bdu_server_drain.argtypes = [vp]
        L.bdu_server_pause.argtypes = [vp, i32]
        L.bdu_server_read.argtypes = [vp, i32, vp, vp, vp, vp]
        L.bdu_server_close.argtypes = [vp, i32]
        L.bdu_server_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
        L.bdu_server_destroy.argtypes = [vp]
        L.bdu_batch_create.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp)]
        L.bdu_batch_create_flags.argtypes = [ctypes.POINTER(vp), i32, i32, i32, ctypes.POINTER(vp)]
        L.bdu_batch_update.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32)]
        L.bdu_batch_sync.argtypes = [vp]
        L.bdu_batch_info.argtypes = [vp, ctypes.POINTER(i64)]
        L.bdu_batch_destroy.argtypes = [vp]
        for f in ("bdu_create", "bdu_update", "bdu_update_batched", "bdu_update_projected", "bdu_project",
                  "bdu_read", "bdu_set_stream", "bdu_sync", "bdu_destroy", "bdu_set_tiling",
                  "bdu_get_tiling", "bdu_plan_stats", "bdu_givens_device", "bdu_timing_enable",
                  "bdu_timing_read", "bdu_batch_create", "bdu_batch_update", "bdu_batch_sync",
                  "bdu_batch_info", "bdu_batch_destroy", "bdu_autotune", "bdu_tune_save", "bdu_tune_load",
                  "bdu_handle_tiling", "bdu_set_generation_in_lds", "bdu_set_finite_check", "bdu_set_split_pass", "bdu_plan_segments", "bdu_plan_blocks", "bdu_update_householder", "bdu_server_create", "bdu_server_open", "bdu_server_submit",
                  "bdu_server_wait", "bdu_server_poll", "bdu_server_drain", "bdu_server_pause",
                  "bdu_server_read", "bdu_server_close", "bdu_server_stats", "bdu_server_destroy"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _strerror(status: int) -> str:
    try:
        return lib().bdu_strerror(status).decode()
    except Exception:
        return "unknown"


def _check(status: int, what: str) -> int:
    if status < 0:
        raise BduError(status, what)
    return status


def _ptr(a, matrix: bool = False):
    """Data pointer of a float64 numpy array or CUDA tensor (kept alive by the caller)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64:
            raise TypeError("float64 required")
        if matrix and a.ndim == 2 and not a.flags["F_CONTIGUOUS"]:
            raise ValueError("matrices must be column-major (Fortran order)")
        if not (a.flags["F_CONTIGUOUS"] or a.flags["C_CONTIGUOUS"]):
            raise ValueError("array must be contiguous")
        return a.ctypes.data
    # torch tensor
    import torch
    if a.dtype != torch.float64:
        raise TypeError("float64 required")
    if matrix and a.dim() == 2 and a.stride(0) != 1:
        raise ValueError("matrices must be column-major (stride(0) == 1)")
    return a.data_ptr()


def _shape(a):
    return tuple(int(x) for x in a.shape)


def _packed(a) -> bool:
    """Column-major with leading dimension = rows (matrices), unit stride (vectors)."""
    if isinstance(a, np.ndarray):
        return a.flags["F_CONTIGUOUS"]
    st = a.stride()
    if a.dim() == 1:
        return a.shape[0] <= 1 or st[0] == 1
    return (a.shape[0] <= 1 or st[0] == 1) and (a.shape[1] <= 1 or st[1] == a.shape[0])


def _arg(a, shape, name: str):
    """Pointer of a float64 array or CUDA tensor of exactly this shape, packed
    column-major; None passes through.  The C side reads prod(shape) doubles
    from the pointer, so every shape and stride is checked here."""
    if a is None:
        return None
    if _shape(a) != tuple(shape):
        raise ValueError(f"{name}: shape {_shape(a)}, expected {tuple(shape)}")
    if not _packed(a):
        raise ValueError(f"{name}: must be packed column-major (leading dimension = rows)")
    return _ptr(a, len(shape) == 2)


def _cols(a, rows: int, name: str):
    """(pointer, r) of an update block: a vector of length rows (r = 1) or a
    rows x r matrix."""
    if a.ndim == 1:
        return _arg(a, (rows,), name), 1
    return _arg(a, (rows, int(a.shape[1])), name), int(a.shape[1])


def _pair(B, C, m: int, n: int):
    pb, rb = _cols(B, m, "B")
    pc, rc = _cols(C, n, "C")
    if rb != rc:
        raise ValueError(f"B has {rb} columns and C has {rc}")
    return pb, pc, rb


def set_tiling(k0: int, nw: int, rpl: int = 1) -> None:
    _check(lib().bdu_set_tiling(k0, nw, rpl), "bdu_set_tiling")


def set_finite_check(on: bool) -> None:
    _check(lib().bdu_set_finite_check(1 if on else 0), "bdu_set_finite_check")


def set_generation_in_lds(allow: bool) -> None:
    _check(lib().bdu_set_generation_in_lds(1 if allow else 0), "bdu_set_generation_in_lds")


def set_split_pass(mode) -> None:
    """0 / False: off; 1: phase 1 applied while phase 2 is generated; 2 / True
    (the default): also phase 2 in segments (handles created afterwards)."""
    _check(lib().bdu_set_split_pass(2 if mode is True else int(mode)), "bdu_set_split_pass")


def plan_segments(m: int, n: int):
    """(tcut, bcut, block) of the phase-2 segments; block in plan_rotations order."""
    L = lib()
    cnt = _check(L.bdu_plan_rotations(m, n, None, None, None, None, 0), "bdu_plan_rotations")
    tc = np.zeros(8, np.int32)
    bc = np.zeros(8, np.int32)
    blk = np.empty(cnt, np.int32)
    ns = _check(L.bdu_plan_segments(m, n, tc.ctypes.data, bc.ctypes.data, blk.ctypes.data, cnt), "bdu_plan_segments")
    return tc[:ns], bc[:ns], blk


def plan_blocks(m: int, n: int, side: int) -> np.ndarray:
    """Applier blocks of one side (0: Q, 1: P) under the current tiling: rows
    (base, lmax, nfront, phase, start, off)."""
    L = lib()
    nb = _check(L.bdu_plan_blocks(m, n, side, None, 0), "bdu_plan_blocks")
    out = np.zeros((max(nb, 1), 6), np.int64)
    _check(L.bdu_plan_blocks(m, n, side, out.ctypes.data, nb), "bdu_plan_blocks")
    return out[:nb]


def set_tiling_auto() -> None:
    """Handles created afterwards take the tiling recorded for their shape by autotune / tune_load."""
    _check(lib().bdu_set_tiling(0, 0, 0), "bdu_set_tiling")


def autotune(m: int, n: int, streams: int) -> dict:
    out = (ctypes.c_int64 * 4)()
    _check(lib().bdu_autotune(m, n, streams, out), "bdu_autotune")
    return {"k0": out[0], "nw": out[1], "rpl": out[2], "us_per_step": out[3]}


def tune_save(path: str) -> None:
    _check(lib().bdu_tune_save(path.encode()), "bdu_tune_save")


def tune_load(path: str) -> int:
    return _check(lib().bdu_tune_load(path.encode()), "bdu_tune_load")


def get_tiling():
    k0, nw, rpl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib().bdu_get_tiling(ctypes.byref(k0), ctypes.byref(nw), ctypes.byref(rpl))
    return k0.value, nw.value, rpl.value


def footprint_bytes(m: int, n: int) -> int:
    return _check(lib().bdu_footprint_bytes(m, n), "bdu_footprint_bytes")


def givens_device(a: np.ndarray, b: np.ndarray, mode: int):
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    c, s, r = np.empty_like(a), np.empty_like(a), np.empty_like(a)
    _check(lib().bdu_givens_device(a.ctypes.data, b.ctypes.data, mode, c.ctypes.data, s.ctypes.data,
                                   r.ctypes.data, len(a)), "bdu_givens_device")
    return c, s, r


STAGES = ("project", "spike", "generate", "apply")


def timing_enable(on: bool = True) -> None:
    _check(lib().bdu_timing_enable(1 if on else 0), "bdu_timing_enable")


def timing_read() -> dict:
    """{stage: (milliseconds summed over launches, launches)} since timing_enable(True)."""
    ms = np.zeros(4)
    cnt = np.zeros(4, np.int64)
    _check(lib().bdu_timing_read(ms.ctypes.data, cnt.ctypes.data), "bdu_timing_read")
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(STAGES)}


def plan_stats(m: int, n: int) -> dict:
    out = (ctypes.c_int64 * 9)()
    _check(lib().bdu_plan_stats(m, n, out), "bdu_plan_stats")
    keys = ["left", "right", "spike", "chains", "ticks", "left_slots", "right_slots", "gen_threads", "split"]
    return dict(zip(keys, list(out)))


def plan_rotations(m: int, n: int):
    L = lib()
    cnt = _check(L.bdu_plan_rotations(m, n, None, None, None, None, 0), "bdu_plan_rotations")
    side = np.empty(cnt, np.int32)
    idx = np.empty(cnt, np.int64)
    ph = np.empty(cnt, np.int32)
    tick = np.empty(cnt, np.int64)
    L.bdu_plan_rotations(m, n, side.ctypes.data, idx.ctypes.data, ph.ctypes.data, tick.ctypes.data, cnt)
    return side, idx, ph, tick


class Handle:
    """One factorization A = Q Bd P^T resident on the GPU."""

    def __init__(self, Q, d, e, P):
        m, n = int(Q.shape[0]), int(P.shape[0])
        h = ctypes.c_void_p()
        _check(lib().bdu_create(m, n, _arg(Q, (m, m), "Q"), _arg(d, (n,), "d"), _arg(e, (n - 1,), "e"),
                                _arg(P, (n, n), "P"), ctypes.byref(h)), "bdu_create")
        self._h = h
        self.m, self.n = m, n

    @property
    def ptr(self):
        return self._h

    def update(self, B, C) -> None:
        pb, pc, r = _pair(B, C, self.m, self.n)
        _check(lib().bdu_update(self._h, pb, pc, r), "bdu_update")

    def update_noalloc(self, B, C) -> None:
        """bdu_update_noalloc: the same update, staged in the library's fixed
        device scratch (no allocation)."""
        pb, pc, r = _pair(B, C, self.m, self.n)
        _check(lib().bdu_update_noalloc(self._h, pb, pc, r), "bdu_update_noalloc")

    def update_projected(self, u, v) -> None:
        _check(lib().bdu_update_projected(self._h, _arg(u, (self.m,), "u"), _arg(v, (self.n,), "v")),
               "bdu_update_projected")

    def update_householder(self, b, c) -> None:
        """A <- A + b c^T by the Householder bidiagonal update (Algorithm 1)."""
        _check(lib().bdu_update_householder(self._h, _arg(b, (self.m,), "b"), _arg(c, (self.n,), "c")),
               "bdu_update_householder")

    def project(self, b, c):
        u = np.empty(self.m)
        v = np.empty(self.n)
        _check(lib().bdu_project(self._h, _arg(b, (self.m,), "b"), _arg(c, (self.n,), "c"), u.ctypes.data,
                                 v.ctypes.data), "bdu_project")
        return u, v

    def read(self):
        Q = np.empty((self.m, self.m), order="F")
        P = np.empty((self.n, self.n), order="F")
        d = np.empty(self.n)
        e = np.empty(max(self.n - 1, 1))
        _check(lib().bdu_read(self._h, Q.ctypes.data, d.ctypes.data, e.ctypes.data, P.ctypes.data), "bdu_read")
        return Q, d, e[: self.n - 1], P

    def read_into(self, Q=None, d=None, e=None, P=None) -> None:
        m, n = self.m, self.n
        _check(lib().bdu_read(self._h, _arg(Q, (m, m), "Q"), _arg(d, (n,), "d"), _arg(e, (n - 1,), "e"),
                              _arg(P, (n, n), "P")), "bdu_read")

    def last_rotations(self):
        L = lib()
        cnt = _check(L.bdu_last_rotations(self._h, None, None, None, None, 0), "bdu_last_rotations")
        side = np.empty(cnt, np.int32)
        idx = np.empty(cnt, np.int64)
        c = np.empty(cnt)
        s = np.empty(cnt)
        L.bdu_last_rotations(self._h, side.ctypes.data, idx.ctypes.data, c.ctypes.data, s.ctypes.data, cnt)
        return side, idx, c, s

    def set_stream(self, stream) -> None:
        """stream: a torch.cuda.Stream, a raw hipStream_t (int) or None."""
        raw = getattr(stream, "cuda_stream", stream)
        _check(lib().bdu_set_stream(self._h, ctypes.c_void_p(raw) if raw else None), "bdu_set_stream")

    def sync(self) -> None:
        _check(lib().bdu_sync(self._h), "bdu_sync")

    def truncated_bd(self, r: int):
        """Best rank-r truncated bidiagonal approximation: (idx, err2, Qr, Pr)
        with A_r = Qr Pr^T (eqs. (trBD), (errtrBD))."""
        idx = np.empty(r, np.int64)
        Qr = np.empty((self.m, r), order="F")
        Pr = np.empty((self.n, r), order="F")
        err2 = ctypes.c_double()
        _check(lib().bdu_truncated_bd(self._h, r, idx.ctypes.data, ctypes.byref(err2), Qr.ctypes.data, Pr.ctypes.data),
               "bdu_truncated_bd")
        return idx, err2.value, Qr, Pr

    def orth_error(self):
        """(||Q^T Q - I||_F, ||P^T P - I||_F) measured on the device."""
        eq, ep = ctypes.c_double(), ctypes.c_double()
        _check(lib().bdu_orth_error(self._h, ctypes.byref(eq), ctypes.byref(ep)), "bdu_orth_error")
        return eq.value, ep.value

    def reorthogonalize(self, tol: float = 0.0):
        """One Newton-Schulz step on each factor whose drift exceeds tol
        (every factor if tol <= 0); returns the drifts measured before."""
        eq, ep = ctypes.c_double(), ctypes.c_double()
        _check(lib().bdu_reorthogonalize(self._h, tol, ctypes.byref(eq), ctypes.byref(ep)), "bdu_reorthogonalize")
        return eq.value, ep.value

    def tiling(self):
        k0, nw, rpl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().bdu_handle_tiling(self._h, ctypes.byref(k0), ctypes.byref(nw), ctypes.byref(rpl)),
               "bdu_handle_tiling")
        return k0.value, nw.value, rpl.value

    def close(self) -> None:
        if self._h:
            lib().bdu_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def update_batched(handles, Bs, Cs) -> None:
    """bdu_update_batched over distinct handles; Bs[i] is m_i x r_i, Cs[i] n_i x r_i."""
    n = len(handles)
    if len(Bs) != n or len(Cs) != n:
        raise ValueError("one B and one C per handle")
    args = [_pair(B, C, h.m, h.n) for h, B, C in zip(handles, Bs, Cs)]
    hp = (ctypes.c_void_p * n)(*[h.ptr.value for h in handles])
    bp = (ctypes.c_void_p * n)(*[a[0] for a in args])
    cp = (ctypes.c_void_p * n)(*[a[1] for a in args])
    rs = (ctypes.c_int * n)(*[a[2] for a in args])
    _check(lib().bdu_update_batched(hp, bp, cp, rs, n), "bdu_update_batched")


class Batch:
    """bdu_batch: a fixed set of distinct handles updated together, step after step."""

    def __init__(self, handles, max_rank: int = 1, eager: bool = False):
        """eager: launch every step eagerly on the first handle's stream (no
        graph capture; BDU_BATCH_EAGER)."""
        n = len(handles)
        self.handles = list(handles)  # the batch keeps them alive
        hp = (ctypes.c_void_p * n)(*[h.ptr.value for h in handles])
        b = ctypes.c_void_p()
        _check(lib().bdu_batch_create_flags(hp, n, max_rank, 1 if eager else 0, ctypes.byref(b)),
               "bdu_batch_create_flags")
        self._b = b

    def update(self, Bs, Cs, ranks=None) -> None:
        """Bs[i] is m_i x r_i (or a vector for r_i = 1), None for no update of handle i."""
        n = len(self.handles)
        if len(Bs) != n or len(Cs) != n:
            raise ValueError("one B and one C (or None) per handle")
        args = []
        for i, (h, B, C) in enumerate(zip(self.handles, Bs, Cs)):
            if (B is None) != (C is None):
                raise ValueError(f"handle {i}: B and C must both be given or both be None")
            args.append((None, None, 0) if B is None else _pair(B, C, h.m, h.n))
        rs = list(ranks) if ranks is not None else [a[2] for a in args]
        for i, (rk, a) in enumerate(zip(rs, args)):
            if rk > a[2]:
                raise ValueError(f"handle {i}: rank {rk} exceeds the {a[2]} columns given")
        bp = (ctypes.c_void_p * n)(*[a[0] for a in args])
        cp = (ctypes.c_void_p * n)(*[a[1] for a in args])
        ra = (ctypes.c_int * n)(*rs)
        _check(lib().bdu_batch_update(self._b, bp, cp, ra), "bdu_batch_update")

    def sync(self) -> None:
        _check(lib().bdu_batch_sync(self._b), "bdu_batch_sync")

    def info(self) -> dict:
        out = (ctypes.c_int64 * 5)()
        _check(lib().bdu_batch_info(self._b, out), "bdu_batch_info")
        return dict(zip(["handles", "max_rank", "groups", "graph", "steps"], list(out)))

    def close(self) -> None:
        if self._b:
            lib().bdu_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """bdu_server: resident streams, budget admission, bounded queues, continuous batching."""

    STAT_KEYS = ["completed", "rejected_busy", "rejected_memory", "rounds", "batched_passes",
                 "streams", "bytes_in_use", "pending", "failed"]

    def __init__(self, budget_bytes: int, queue_cap: int = 8, max_batch: int = 256, classes=None):
        """classes: ascending upper bounds of n of the size classes (None: the
        library's default 1024, 2048, 4096; [] for a single class)."""
        s = ctypes.c_void_p()
        if classes is None:
            _check(lib().bdu_server_create(budget_bytes, queue_cap, max_batch, ctypes.byref(s)), "bdu_server_create")
        else:
            b = (ctypes.c_int64 * max(len(classes), 1))(*classes)
            _check(lib().bdu_server_create_classes(budget_bytes, queue_cap, max_batch, b, len(classes),
                                                   ctypes.byref(s)), "bdu_server_create_classes")
        self._s = s
        self.shapes = {}

    def open(self, Q, d, e, P) -> int:
        """Stream id; raises BduError (status BDU_ENOMEM) when over the budget."""
        m, n = int(Q.shape[0]), int(P.shape[0])
        sid = ctypes.c_int()
        _check(lib().bdu_server_open(self._s, m, n, _arg(Q, (m, m), "Q"), _arg(d, (n,), "d"),
                                     _arg(e, (n - 1,), "e"), _arg(P, (n, n), "P"), ctypes.byref(sid)),
               "bdu_server_open")
        self.shapes[sid.value] = (m, n)
        return sid.value

    def submit(self, sid: int, B, C, detach: bool = False):
        """Ticket (None if detached); raises BduError (status BDU_EBUSY) when the stream's queue is full."""
        if sid not in self.shapes:
            raise ValueError(f"unknown stream {sid}")
        m, n = self.shapes[sid]
        pb, pc, r = _pair(B, C, m, n)
        t = ctypes.c_int64()
        _check(lib().bdu_server_submit(self._s, sid, pb, pc, r, None if detach else ctypes.byref(t)),
               "bdu_server_submit")
        return None if detach else t.value

    def wait(self, ticket: int) -> float:
        ms = ctypes.c_double()
        _check(lib().bdu_server_wait(self._s, ticket, ctypes.byref(ms)), "bdu_server_wait")
        return ms.value

    def poll(self, ticket: int) -> bool:
        return bool(_check(lib().bdu_server_poll(self._s, ticket), "bdu_server_poll"))

    def drain(self) -> None:
        _check(lib().bdu_server_drain(self._s), "bdu_server_drain")

    def pause(self, paused: bool = True) -> None:
        _check(lib().bdu_server_pause(self._s, 1 if paused else 0), "bdu_server_pause")

    def read(self, sid: int):
        m, n = self.shapes[sid]
        Q = np.empty((m, m), order="F")
        P = np.empty((n, n), order="F")
        d = np.empty(n)
        e = np.empty(max(n - 1, 1))
        _check(lib().bdu_server_read(self._s, sid, Q.ctypes.data, d.ctypes.data, e.ctypes.data, P.ctypes.data),
               "bdu_server_read")
        return Q, d, e[: n - 1], P

    def reset_stats(self) -> None:
        _check(lib().bdu_server_reset_stats(self._s), "bdu_server_reset_stats")

    def class_of(self, n: int) -> int:
        return _check(lib().bdu_server_class_of(self._s, n), "bdu_server_class_of")

    def close_stream(self, sid: int) -> None:
        _check(lib().bdu_server_close(self._s, sid), "bdu_server_close")
        self.shapes.pop(sid, None)

    def stats(self) -> dict:
        c = (ctypes.c_int64 * 9)()
        lat = (ctypes.c_double * 4)()
        _check(lib().bdu_server_stats(self._s, c, lat), "bdu_server_stats")
        out = dict(zip(self.STAT_KEYS, list(c)))
        out.update(p50_ms=lat[0], p99_ms=lat[1], mean_ms=lat[2], max_ms=lat[3])
        return out

    def close(self) -> None:
        if self._s:
            lib().bdu_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tracker:
    """Subspace tracking (Section 4): a thin rank-r factorization
    A = U B V^T on the GPU, updated with rank-1 b c^T and truncated back to
    rank r (bdu_track_*)."""

    def __init__(self, U, d, e, V):
        self.m, self.r = int(U.shape[0]), int(U.shape[1])
        self.n = int(V.shape[0])
        m, n, r = self.m, self.n, self.r
        h = ctypes.c_void_p()
        _check(lib().bdu_track_create(m, n, r, _arg(U, (m, r), "U"), _arg(d, (r,), "d"),
                                      _arg(e, (r - 1,), "e") if r > 1 else None, _arg(V, (n, r), "V"),
                                      ctypes.byref(h)), "bdu_track_create")
        self._h = h

    def update(self, b, c) -> None:
        _check(lib().bdu_track_update(self._h, _arg(b, (self.m,), "b"), _arg(c, (self.n,), "c")),
               "bdu_track_update")

    def last_projection(self):
        """(b_hat, c_hat, b_perp/delta, c_perp/gamma) of the last update."""
        bh, ch = np.empty(self.r), np.empty(self.r)
        qb, qc = np.empty(self.m), np.empty(self.n)
        _check(lib().bdu_track_last_projection(self._h, bh.ctypes.data, ch.ctypes.data, qb.ctypes.data,
                                               qc.ctypes.data), "bdu_track_last_projection")
        return bh, ch, qb, qc

    def sync(self) -> None:
        _check(lib().bdu_track_sync(self._h), "bdu_track_sync")

    def read(self):
        U = np.empty((self.m, self.r), order="F")
        V = np.empty((self.n, self.r), order="F")
        d = np.empty(self.r)
        e = np.empty(max(self.r - 1, 1))
        _check(lib().bdu_track_read(self._h, U.ctypes.data, d.ctypes.data, e.ctypes.data, V.ctypes.data),
               "bdu_track_read")
        return U, d, e[: self.r - 1], V

    def orth_error(self):
        """(||U^T U - I||_F, ||V^T V - I||_F)."""
        eu, ev = ctypes.c_double(), ctypes.c_double()
        _check(lib().bdu_track_orth_error(self._h, ctypes.byref(eu), ctypes.byref(ev)), "bdu_track_orth_error")
        return eu.value, ev.value

    def reorthogonalize(self, tol: float = 0.0):
        """One Newton-Schulz step on each side whose drift exceeds tol; the drift before it."""
        eu, ev = ctypes.c_double(), ctypes.c_double()
        _check(lib().bdu_track_reorthogonalize(self._h, tol, ctypes.byref(eu), ctypes.byref(ev)),
               "bdu_track_reorthogonalize")
        return eu.value, ev.value

    def set_drift_check(self, period: int, tol: float) -> None:
        _check(lib().bdu_track_set_drift_check(self._h, period, tol), "bdu_track_set_drift_check")

    def drift_stats(self) -> dict:
        c, k = ctypes.c_int64(), ctypes.c_int64()
        eu, ev = ctypes.c_double(), ctypes.c_double()
        _check(lib().bdu_track_drift_stats(self._h, ctypes.byref(c), ctypes.byref(k), ctypes.byref(eu),
                                           ctypes.byref(ev)), "bdu_track_drift_stats")
        return {"checks": c.value, "corrections": k.value, "eu": eu.value, "ev": ev.value}

    def last(self):
        """(delta, gamma, removed index) of the last update."""
        dl, gm, k = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().bdu_track_last(self._h, ctypes.byref(dl), ctypes.byref(gm), ctypes.byref(k)),
               "bdu_track_last")
        return dl.value, gm.value, k.value

    def close(self) -> None:
        if self._h:
            lib().bdu_track_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
