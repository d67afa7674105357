"""Python binding of libhschur (MI355X symmetric near-field Schur-complement
preconditioner for complex-symmetric H-matrix solves).

Argument marshalling only: every step of the method runs in the library's
host C++ and gfx950 HIP kernels. PyTorch supplies device memory (through the
context's allocator callback, i.e. torch's caching allocator) and streams.
The names follow the C-ABI in include/hschur.h.

Raises ``HschurError`` on every non-zero status except HS_NOT_CONVERGED,
which is reported through the returned statistics. Importing never loads a
fallback: without the built library ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhschur.so")

HS_OK, HS_NOT_CONVERGED = 0, 1
HS_EINVAL, HS_ENOMEM, HS_ENODEVICE, HS_EHIP, HS_ESINGULAR, HS_ENUMERIC, HS_ETIMEOUT = -1, -2, -3, -4, -5, -6, -7
ORDER = {"natural": 0, "rcm": 1, "cm": 2, "sloan": 3, "king": 4}
X_CODES = {"perm": 1, "leaf_off": 2, "boxes": 3, "near": 4, "far": 5, "order": 6, "rowptr": 7, "cols": 8, "orig": 9}
H_CODES = {"near_off": 101, "near_data": 102, "far_rank": 103, "far_off": 104, "far_uv": 105, "far_piv": 106}
P_CODES = {"d": 201, "alpha_kind": 202, "alpha_off": 203, "alpha": 204, "alpha_left": 205}


class HschurError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"hschur status {status}: {message}")
        self.status = status


class BuildOpts(ctypes.Structure):
    _fields_ = [("leaf_max", ctypes.c_int32), ("aca_tol", ctypes.c_double), ("rank_cap", ctypes.c_int32),
                ("store_c64", ctypes.c_int32)]


class PrecondOpts(ctypes.Structure):
    _fields_ = [("ordering", ctypes.c_int32), ("fill_tol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("sweep_chunk", ctypes.c_int32), ("sweep_fold_cols", ctypes.c_int32), ("kind", ctypes.c_int32)]


PC_KIND = {"schur": 0, "block_jacobi": 1, "schur_nonsym": 2, "schur_lowrank": 3}


class SolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("restart", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("fixed_iters", ctypes.c_int32), ("inner_steps", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("use_x0", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("relres", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("n", "nb", "nbox", "n_near", "n_far", "n_pattern", "n_fill", "n_lowrank", "max_dk", "max_rank",
                 "bytes_near", "bytes_far", "bytes_alpha", "bytes_d", "bytes_device")] + \
               [("flops_setup", ctypes.c_double), ("flops_fill", ctypes.c_double), ("bytes_estimate", ctypes.c_int64)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class RequestStats(ctypes.Structure):
    _fields_ = [("geometry", ctypes.c_int32), ("ncols", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("relres", ctypes.c_double), ("t_arrival", ctypes.c_double),
                ("t_done", ctypes.c_double), ("done", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_start", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_ if f[0] != "pad"}


class SolveItem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_void_p), ("P", ctypes.c_void_p), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("nrhs", ctypes.c_int64)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 7), ("total_ms", ctypes.c_double * 7),
                ("all_launches", ctypes.c_int64 * 7)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load(path: str = LIB_PATH):
    """Load libhschur.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HschurError(HS_ENODEVICE, f"{path} is not built; run paper_2111_13483_amd/build.py")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pvp = ctypes.POINTER(vp)
    sig = {
        "hs_context_create": (i32, [pvp, i32, vp, ALLOC_FN, FREE_FN, vp]),
        "hs_context_set_stream": (i32, [vp, vp]),
        "hs_context_set_wait_limit": (i32, [vp, dbl]),
        "hs_context_destroy": (None, [vp]),
        "hs_plan_create": (i32, [vp, i64, i32, i32, pvp]),
        "hs_plan_query": (i32, [vp, ctypes.POINTER(Info)]),
        "hs_plan_destroy": (None, [vp]),
        "hs_plan_export": (i32, [vp, i32, vp, i64, ctypes.POINTER(i64)]),
        "hs_h_build": (i32, [vp, vp, i64, dbl, dbl, ctypes.POINTER(BuildOpts), pvp]),
        "hs_query_hmatrix": (i32, [vp, ctypes.POINTER(Info)]),
        "hs_hmatrix_destroy": (None, [vp]),
        "hs_precond_setup": (i32, [vp, vp, ctypes.POINTER(PrecondOpts), pvp]),
        "hs_precond_setup_many": (i32, [vp, i64, pvp, ctypes.POINTER(PrecondOpts), pvp]),
        "hs_query_precond": (i32, [vp, ctypes.POINTER(Info)]),
        "hs_precond_tune": (i32, [vp, vp, ctypes.POINTER(PrecondOpts), i32, i32, ctypes.POINTER(PrecondOpts),
                                  ctypes.POINTER(dbl), ctypes.POINTER(i32)]),
        "hs_precond_destroy": (None, [vp]),
        "hs_solve": (i32, [vp, vp, vp, vp, vp, i64, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)]),
        "hs_matvec": (i32, [vp, vp, vp, vp, i64]),
        "hs_matvec_noalloc": (i32, [vp, vp, vp, vp, i64, ctypes.POINTER(i64)]),
        "hs_precond_apply": (i32, [vp, vp, vp, vp, i64]),
        "hs_hmatrix_export": (i32, [vp, i32, vp, i64, ctypes.POINTER(i64)]),
        "hs_precond_export": (i32, [vp, i32, vp, i64, ctypes.POINTER(i64)]),
        "hs_server_clock": (dbl, []),
        "hs_server_create": (i32, [vp, i64, i32, ctypes.POINTER(SolveOpts), pvp]),
        "hs_server_admit": (i32, [vp, vp, vp, ctypes.POINTER(i32)]),
        "hs_server_add_geometry": (i32, [vp, vp, i64, dbl, dbl, ctypes.POINTER(BuildOpts),
                                         ctypes.POINTER(PrecondOpts), ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "hs_server_geometry": (i32, [vp, i32, pvp, pvp, ctypes.POINTER(i64)]),
        "hs_solve_many": (i32, [vp, i64, ctypes.POINTER(SolveItem), ctypes.POINTER(SolveOpts),
                                ctypes.POINTER(SolveStats)]),
        "hs_server_submit": (i32, [vp, i32, vp, vp, i32, dbl, ctypes.POINTER(i64)]),
        "hs_server_step": (i32, [vp, ctypes.POINTER(i32)]),
        "hs_server_pending": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "hs_server_request": (i32, [vp, i64, ctypes.POINTER(RequestStats)]),
        "hs_server_destroy": (None, [vp]),
        "hs_timing_begin": (i32, [vp]),
        "hs_timing_begin_every": (i32, [vp, i32]),
        "hs_timing_end": (i32, [vp, ctypes.POINTER(KernelTimes)]),
        "hs_status_string": (ctypes.c_char_p, [i32]),
        "hs_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = (
    "hs_context_create", "hs_context_set_stream", "hs_context_set_wait_limit", "hs_context_destroy", "hs_plan_create", "hs_plan_query",
    "hs_plan_destroy", "hs_plan_export", "hs_h_build", "hs_query_hmatrix", "hs_hmatrix_destroy", "hs_precond_setup",
    "hs_precond_setup_many", "hs_precond_tune", "hs_query_precond", "hs_precond_destroy", "hs_solve", "hs_matvec", "hs_matvec_noalloc", "hs_precond_apply", "hs_hmatrix_export",
    "hs_precond_export", "hs_timing_begin", "hs_timing_begin_every", "hs_timing_end", "hs_server_clock",
    "hs_server_create",
    "hs_server_admit", "hs_server_add_geometry", "hs_server_geometry", "hs_solve_many", "hs_server_submit", "hs_server_step", "hs_server_pending", "hs_server_request",
    "hs_server_destroy", "hs_status_string", "hs_last_error",
)

KT_NAMES = ("sweep_fwd", "sweep_bwd", "near_mv", "far_mv", "factor", "schur", "elimination")


def _check(status: int, allow_not_converged: bool = False) -> int:
    if status == HS_OK or (allow_not_converged and status == HS_NOT_CONVERGED):
        return status
    msg = _lib.hs_last_error().decode(errors="replace")
    raise HschurError(status, msg)


def _export(fn, handle, code: int, dtype):
    needed = ctypes.c_int64(0)
    _check(fn(handle, code, None, 0, ctypes.byref(needed)))
    out = np.empty(needed.value // np.dtype(dtype).itemsize, dtype=dtype)
    _check(fn(handle, code, out.ctypes.data_as(ctypes.c_void_p), needed.value, ctypes.byref(needed)))
    return out


# ---------------------------------------------------------------- plan (host only)

class Plan:
    """Integer phases on the host: octree, partition, ordering, symbolic fill."""

    def __init__(self, points: np.ndarray, leaf_max: int, ordering: str = "rcm"):
        L = load()
        pts = np.ascontiguousarray(points, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(L.hs_plan_create(pts.ctypes.data_as(ctypes.c_void_p), pts.shape[0], leaf_max, ORDER[ordering],
                                ctypes.byref(h)))
        self._h = h

    def export(self, what: str) -> np.ndarray:
        return _export(_lib.hs_plan_export, self._h, X_CODES[what], np.int64)

    def info(self) -> dict:
        inf = Info()
        _check(_lib.hs_plan_query(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hs_plan_destroy(self._h)
            self._h = None


# ---------------------------------------------------------------- device handles

def _torch():
    import torch
    return torch


class Context:
    """A device + stream; device memory comes from torch's caching allocator."""

    def __init__(self, device: int = 0, stream=None, use_torch_allocator: bool = True):
        torch = _torch()
        L = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self._keep = []
        if use_torch_allocator:
            dev = device

            def _alloc(nbytes, user):
                try:
                    with torch.cuda.device(dev):
                        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.stream)
                except Exception:   # out of memory -> NULL -> HS_ENOMEM
                    return None

            def _free(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            a, f = ALLOC_FN(_alloc), FREE_FN(_free)
            self._keep = [a, f]
        else:
            a, f = ALLOC_FN(), FREE_FN()
        h = ctypes.c_void_p()
        _check(L.hs_context_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream), a, f, None))
        self._h = h

    def timing_begin(self, every: int = 1):
        """Start bracketing the sweep and matvec launches with HIP events
        (every `every`-th launch of each kernel)."""
        _check(_lib.hs_timing_begin_every(self._h, int(every)))

    def timing_end(self) -> dict:
        """Stop timing; {kernel: (timed launches, their total ms, all launches)}."""
        kt = KernelTimes()
        _check(_lib.hs_timing_end(self._h, ctypes.byref(kt)))
        return {name: (int(kt.launches[i]), float(kt.total_ms[i]), int(kt.all_launches[i]))
                for i, name in enumerate(KT_NAMES)}

    def set_wait_limit(self, seconds: float):
        """Bound on each device-side wait of the preconditioner sweeps."""
        _check(_lib.hs_context_set_wait_limit(self._h, float(seconds)))

    def set_stream(self, stream):
        _check(_lib.hs_context_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hs_context_destroy(self._h)
            self._h = None


def _dev_c128(t, n: int):
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.complex128):
        raise HschurError(HS_EINVAL, "expected a cuda complex128 tensor")
    if t.dim() == 1:
        t = t.reshape(n, 1)
    # column-major N x nrhs: store the transpose contiguously
    return t.t().contiguous(), t.shape[1]


class HMatrix:
    def __init__(self, ctx: Context, points, k: float, self_h: float, leaf_max: int, aca_tol: float = 1e-4,
                 rank_cap: int = 0, store_c64: bool = False):
        torch = _torch()
        pts = points if torch.is_tensor(points) else torch.as_tensor(np.ascontiguousarray(points, dtype=np.float64))
        pts = pts.to(device=f"cuda:{ctx.device}", dtype=torch.float64).contiguous()
        self.ctx = ctx
        self.n = int(pts.shape[0])
        opts = BuildOpts(leaf_max, aca_tol, rank_cap, int(bool(store_c64)))
        h = ctypes.c_void_p()
        _check(_lib.hs_h_build(ctx._h, ctypes.c_void_p(pts.data_ptr()), self.n, float(k), float(self_h),
                               ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    def info(self) -> dict:
        inf = Info()
        _check(_lib.hs_query_hmatrix(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def export(self, what: str) -> np.ndarray:
        if what in X_CODES:
            return _export(_lib.hs_hmatrix_export, self._h, X_CODES[what], np.int64)
        dt = np.complex128 if what in ("near_data", "far_uv") else np.int64
        return _export(_lib.hs_hmatrix_export, self._h, H_CODES[what], dt)

    def matvec(self, x):
        """y = Z_H x for a cuda complex128 tensor of shape (N,) or (N, nrhs)."""
        torch = _torch()
        xc, s = _dev_c128(x, self.n)
        y = torch.empty_like(xc)
        _check(_lib.hs_matvec(self.ctx._h, self._h, ctypes.c_void_p(xc.data_ptr()), ctypes.c_void_p(y.data_ptr()), s))
        y = y.t()
        return y.reshape(-1) if x.dim() == 1 else y

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hs_hmatrix_destroy(self._h)
            self._h = None


class Precond:
    def __init__(self, ctx: Context, H: HMatrix, ordering: str = "rcm", fill_tol: float = 1e-2, sweep_chunk: int = 0,
                 sweep_fold_cols: int = 0, mixed: bool = False, kind: str = "schur"):
        """kind="block_jacobi" sets up the comparator blockdiag(Z_kk)^-1 instead;
        kind="schur_nonsym" runs the non-symmetric elimination (left
        coefficients formed separately, export("alpha_left")); kind=
        "schur_lowrank" carries the fill-in blocks compressed through the
        elimination."""
        self.ctx, self.H = ctx, H
        opts = PrecondOpts(ORDER[ordering], float(fill_tol), 1 if mixed else 0, int(sweep_chunk), int(sweep_fold_cols),
                           PC_KIND[kind])
        h = ctypes.c_void_p()
        _check(_lib.hs_precond_setup(ctx._h, H._h, ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    @classmethod
    def many(cls, ctx: Context, Hs, ordering: str = "rcm", fill_tol: float = 1e-2, sweep_chunk: int = 0,
             sweep_fold_cols: int = 0, mixed: bool = False):
        """Batched setup (hs_precond_setup_many): one preconditioner per H-matrix,
        the elimination steps of all of them sharing launches."""
        opts = PrecondOpts(ORDER[ordering], float(fill_tol), 1 if mixed else 0, int(sweep_chunk), int(sweep_fold_cols))
        hs_arr = (ctypes.c_void_p * len(Hs))(*[H._h.value for H in Hs])
        outs = (ctypes.c_void_p * len(Hs))()
        _check(_lib.hs_precond_setup_many(ctx._h, len(Hs), hs_arr, ctypes.byref(opts), outs))
        res = []
        for H, h in zip(Hs, outs):
            P = cls.__new__(cls)
            P.ctx, P.H = ctx, H
            P._h = ctypes.c_void_p(h)
            res.append(P)
        return res

    @staticmethod
    def tune(ctx: Context, H: HMatrix, ordering: str = "rcm", fill_tol: float = 1e-2, nrhs: int = 1, reps: int = 10):
        """hs_precond_tune: the fastest apply layout; returns
        ((sweep_chunk, sweep_fold_cols), [average apply ms per layout])."""
        opts = PrecondOpts(ORDER[ordering], float(fill_tol), 0, 0, 0, 0)
        best = PrecondOpts()
        times = (ctypes.c_double * 9)()
        k = ctypes.c_int32()
        _check(_lib.hs_precond_tune(ctx._h, H._h, ctypes.byref(opts), int(nrhs), int(reps), ctypes.byref(best), times,
                                    ctypes.byref(k)))
        return (best.sweep_chunk, best.sweep_fold_cols), [times[i] for i in range(k.value)]

    def info(self) -> dict:
        inf = Info()
        _check(_lib.hs_query_precond(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def export(self, what: str) -> np.ndarray:
        if what in X_CODES:
            return _export(_lib.hs_precond_export, self._h, X_CODES[what], np.int64)
        dt = np.complex128 if what in ("d", "alpha", "alpha_left") else np.int64
        return _export(_lib.hs_precond_export, self._h, P_CODES[what], dt)

    def apply(self, v):
        """z = P^-1 v = alpha D^-1 alpha^T v."""
        torch = _torch()
        vc, s = _dev_c128(v, self.H.n)
        z = torch.empty_like(vc)
        _check(_lib.hs_precond_apply(self.ctx._h, self._h, ctypes.c_void_p(vc.data_ptr()),
                                     ctypes.c_void_p(z.data_ptr()), s))
        z = z.t()
        return z.reshape(-1) if v.dim() == 1 else z

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hs_precond_destroy(self._h)
            self._h = None


@dataclass
class Stats:
    iters: int
    converged: bool
    relres: float


def solve(ctx: Context, H: HMatrix, P: Precond | None, b, restart: int = 30, tol: float = 1e-6,
          max_iters: int = 0, fixed_iters: int = 0, mixed: bool = False, inner_steps: int = 0, inner_tol: float = 0.0,
          x0=None, transformed: bool = False, block: bool = False):
    """Solve Z x = b: right-preconditioned GMRES, or with mixed=True FP64
    flexible GMRES whose preconditioning steps are inner GMRES solves on the
    complex64 copies, or with mixed="refined" GMRES whose Arnoldi steps use
    the complex64 copies and whose restarts recompute the FP64 residual; x0 (GMRES only) is the initial guess; transformed=True
    solves the paper's transformed system (Eq. 25-28) instead, its stats
    holding the true residual; block=True runs the coupled block-GMRES
    comparator (iters = block steps). Returns (x, [Stats per column])."""
    torch = _torch()
    bc, s = _dev_c128(b, H.n)
    if x0 is None:
        x = torch.empty_like(bc)
    else:
        x, s0 = _dev_c128(x0, H.n)
        if s0 != s:
            raise HschurError(HS_EINVAL, "x0 and b differ in columns")
    method = 3 if block else (2 if transformed else (4 if mixed == "refined" else (1 if mixed else 0)))
    opts = SolveOpts(method, restart, tol, max_iters, fixed_iters, inner_steps, inner_tol,
                     0 if x0 is None else 1)
    st = (SolveStats * s)()
    _check(_lib.hs_solve(ctx._h, H._h, P._h if P is not None else None, ctypes.c_void_p(bc.data_ptr()),
                         ctypes.c_void_p(x.data_ptr()), s, ctypes.byref(opts), st), allow_not_converged=True)
    x = x.t()
    stats = [Stats(st[i].iters, bool(st[i].converged), st[i].relres) for i in range(s)]
    return (x.reshape(-1) if b.dim() == 1 else x), stats


def solve_many(ctx: Context, items, restart: int = 30, tol: float = 1e-6, max_iters: int = 0, fixed_iters: int = 0,
               use_x0: bool = False):
    """hs_solve_many: items of (H, P or None, b[, x0]) solved together;
    returns [(x, [Stats per column]) per item]."""
    torch = _torch()
    arr = (SolveItem * len(items))()
    keep, ncols = [], []
    for i, it in enumerate(items):
        H, P, b = it[0], it[1], it[2]
        bc, s = _dev_c128(b, H.n)
        if use_x0:
            x, _ = _dev_c128(it[3], H.n)
        else:
            x = torch.empty_like(bc)
        keep.append((bc, x, b.dim() == 1))
        ncols.append(s)
        arr[i] = SolveItem(H._h.value, P._h.value if P is not None else None, bc.data_ptr(), x.data_ptr(), s)
    opts = SolveOpts(0, restart, tol, max_iters, fixed_iters, 0, 0.0, 1 if use_x0 else 0)
    st = (SolveStats * sum(ncols))()
    _check(_lib.hs_solve_many(ctx._h, len(items), arr, ctypes.byref(opts), st), allow_not_converged=True)
    out, k = [], 0
    for (bc, x, vec), s in zip(keep, ncols):
        xx = x.t()
        out.append(((xx.reshape(-1) if vec else xx), [Stats(st[k + c].iters, bool(st[k + c].converged),
                                                             st[k + c].relres) for c in range(s)]))
        k += s
    return out


class Server:
    """Resident geometries admitted by device footprint and continuous
    batching of right-hand-side columns (hs_server_*): each step runs one
    restart cycle of every geometry with live columns; finished columns leave
    their slots and pending requests join at the cycle boundary."""

    def __init__(self, ctx: Context, budget_bytes: int, slots: int = 32, restart: int = 30,
                 tol: float = 1e-6, max_iters: int = 0):
        self.ctx = ctx
        self._opts = SolveOpts(0, restart, tol, max_iters, 0, 0, 0.0, 0)
        h = ctypes.c_void_p()
        _check(_lib.hs_server_create(ctx._h, int(budget_bytes), int(slots), ctypes.byref(self._opts),
                                     ctypes.byref(h)))
        self._h = h
        self._keep = {}     # request -> (b, x) device buffers, alive until served
        self._geo = []

    @staticmethod
    def clock() -> float:
        return float(load().hs_server_clock())

    def admit(self, H: HMatrix, P: Precond | None) -> int:
        g = ctypes.c_int32()
        _check(_lib.hs_server_admit(self._h, H._h, P._h if P is not None else None, ctypes.byref(g)))
        self._geo.append(H.n)
        return g.value

    def add_geometry(self, points, k: float, self_h: float, leaf_max: int, aca_tol: float = 1e-4,
                     ordering: str | None = "rcm", fill_tol: float = 1e-2):
        """Plan on the host, refuse before allocating if the estimate does not
        fit, else build and set up on the device. Returns (geometry, estimate)."""
        pts = np.ascontiguousarray(points, dtype=np.float64)
        bo = BuildOpts(leaf_max, aca_tol, 0, 0)
        po = PrecondOpts(ORDER[ordering], float(fill_tol), 0, 0, 0) if ordering is not None else None
        est, g = ctypes.c_int64(0), ctypes.c_int32()
        st = _lib.hs_server_add_geometry(self._h, pts.ctypes.data_as(ctypes.c_void_p), pts.shape[0], float(k),
                                         float(self_h), ctypes.byref(bo), ctypes.byref(po) if po is not None else None,
                                         ctypes.byref(est), ctypes.byref(g))
        self.last_estimate = est.value
        _check(st)
        self._geo.append(pts.shape[0])
        return g.value, est.value

    def geometry(self, g: int):
        """(H handle, P handle, bytes charged) of a geometry; the handles are
        borrowed (owned by the server or the caller)."""
        H, P, nb = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        _check(_lib.hs_server_geometry(self._h, int(g), ctypes.byref(H), ctypes.byref(P), ctypes.byref(nb)))
        return H.value, P.value, nb.value

    def submit(self, geometry: int, b, t_arrival: float) -> int:
        torch = _torch()
        bc, s = _dev_c128(b, self._geo[geometry])
        x = torch.empty_like(bc)
        r = ctypes.c_int64()
        _check(_lib.hs_server_submit(self._h, geometry, ctypes.c_void_p(bc.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                     s, float(t_arrival), ctypes.byref(r)))
        self._keep[r.value] = (bc, x, b.dim() == 1)
        return r.value

    def step(self) -> int:
        c = ctypes.c_int32()
        _check(_lib.hs_server_step(self._h, ctypes.byref(c)))
        return c.value

    def pending(self):
        r, c = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.hs_server_pending(self._h, ctypes.byref(r), ctypes.byref(c)))
        return r.value, c.value

    def request(self, r: int) -> dict:
        st = RequestStats()
        _check(_lib.hs_server_request(self._h, r, ctypes.byref(st)))
        return st.as_dict()

    def result(self, r: int):
        """x of a served request (caller order, N or N x ncols)."""
        bc, x, vec = self._keep[r]
        x = x.t()
        return x.reshape(-1) if vec else x

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hs_server_destroy(self._h)
            self._h = None


# C-ABI style aliases
h_build = HMatrix
precond_setup = Precond
