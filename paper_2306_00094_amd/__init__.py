"""Substructuring Schur-complement solver for nonlocal FEM systems on MI355X.

Thin ctypes binding of the C ABI in ``include/dd.h`` (same entry-point
names).  It only marshals arguments: every step of the solve runs in the HIP
library ``_dd.so``.  Importing this package does not require a GPU; loading
the library does, and a missing library raises instead of falling back.

PyTorch is used for device memory and the HIP stream only.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_dd.so")

DD_OK, DD_EINVAL, DD_ENOMEM, DD_ENOTSPD, DD_ENOCONV, DD_EHIP, DD_ESTATE = range(7)
DD_FP64, DD_MIXED = 0, 1
DD_APPLY_AUTO, DD_APPLY_INV, DD_APPLY_TRSM = 0, 1, 2
DD_LAUNCH_AUTO, DD_LAUNCH_KERNELS, DD_LAUNCH_PERSISTENT, DD_LAUNCH_GRAPH = 0, 1, 2, 3

STATUS_NAMES = {0: "DD_OK", 1: "DD_EINVAL", 2: "DD_ENOMEM", 3: "DD_ENOTSPD", 4: "DD_ENOCONV",
                5: "DD_EHIP", 6: "DD_ESTATE"}

EXPORTED = ["dd_default_opts", "dd_footprint", "dd_setup", "dd_factor", "dd_solve",
            "dd_schur_apply", "dd_get_factor", "dd_get_schur_diag", "dd_autotune",
            "dd_set_timing", "dd_get_timing", "dd_batch_begin", "dd_batch_admit",
            "dd_batch_step", "dd_batch_retire", "dd_batch_end", "dd_last_error", "dd_destroy",
            "dd_assemble_2d", "dd_feti_setup", "dd_feti_factor", "dd_feti_solve", "dd_feti_last_error",
            "dd_feti_destroy", "dd_schur_apply_noalloc", "dd_bdd_solve", "dd_method_autotune",
            "dd_method_solve"]
DD_METHOD_AUTO, DD_METHOD_FETI, DD_METHOD_BDD, DD_METHOD_JACOBI = range(4)
DD_SLOT_FREE, DD_SLOT_RUNNING, DD_SLOT_DONE, DD_SLOT_FALLBACK = range(4)
DD_PHASE_KIG, DD_PHASE_INTERIOR, DD_PHASE_GAMMA, DD_PHASE_UPDATE, DD_PHASE_LOOP = range(5)
DD_NPHASES = 5

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class dd_subdomain(ctypes.Structure):
    _fields_ = [("n_i", ctypes.c_int32), ("k_ii", _f64p), ("n_g", ctypes.c_int32),
                ("g_map", _i32p), ("kig_rowptr", _i32p), ("kig_col", _i32p),
                ("kig_val", _f64p), ("i_map", _i32p)]


class dd_problem(ctypes.Structure):
    _fields_ = [("n_dof", ctypes.c_int32), ("n_gamma", ctypes.c_int32),
                ("n_sub", ctypes.c_int32), ("sub", ctypes.POINTER(dd_subdomain)),
                ("gamma_map", _i32p), ("kgg_rowptr", _i32p), ("kgg_col", _i32p),
                ("kgg_val", _f64p)]


class dd_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_it", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("fp64_fallback", ctypes.c_int32),
                ("apply", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("verify", ctypes.c_int32),
                ("gather32", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("reliable", ctypes.c_int32)]


class dd_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("used_fallback", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_resid", ctypes.c_double)]


class dd_tune_result(ctypes.Structure):
    _fields_ = [("apply", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("direction_kernel", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("ms_per_solve", ctypes.c_double), ("candidates", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("three_launch", ctypes.c_int32)]


class dd_feti_sub(ctypes.Structure):
    _fields_ = [("n_g", ctypes.c_int32), ("g_map", _i32p), ("agg_rowptr", _i32p), ("agg_col", _i32p),
                ("agg_val", _f64p), ("kig_rowptr", _i32p), ("kig_col", _i32p), ("kig_val", _f64p),
                ("n_z", ctypes.c_int32), ("z", _f64p)]


class DDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP solver library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP solver library missing: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.dd_default_opts.argtypes = [ctypes.POINTER(dd_solve_opts)]
    lib.dd_default_opts.restype = None
    lib.dd_footprint.argtypes = [ctypes.POINTER(dd_problem), ctypes.c_int, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_size_t)]
    lib.dd_setup.argtypes = [ctypes.POINTER(dd_problem), vp, ctypes.c_int32, ctypes.POINTER(vp)]
    lib.dd_factor.argtypes = [vp, ctypes.c_int]
    lib.dd_solve.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int32, ctypes.c_int32,
                             ctypes.POINTER(dd_solve_opts), ctypes.POINTER(dd_solve_info)]
    lib.dd_schur_apply.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int32, ctypes.c_int32]
    lib.dd_schur_apply_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int32, ctypes.c_int32]
    lib.dd_get_factor.argtypes = [vp, ctypes.c_int, ctypes.c_int32, _f64p]
    lib.dd_get_schur_diag.argtypes = [vp, ctypes.c_int, _f64p]
    lib.dd_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(dd_solve_opts),
                                ctypes.POINTER(dd_tune_result)]
    lib.dd_batch_begin.argtypes = [vp, ctypes.c_int, ctypes.POINTER(dd_solve_opts)]
    lib.dd_batch_admit.argtypes = [vp, _i32p, ctypes.c_int32, vp, ctypes.c_int32]
    lib.dd_batch_step.argtypes = [vp, ctypes.c_int32, _i32p]
    lib.dd_batch_retire.argtypes = [vp, _i32p, ctypes.c_int32, vp, ctypes.c_int32,
                                    ctypes.POINTER(dd_solve_info)]
    lib.dd_batch_end.argtypes = [vp]
    lib.dd_set_timing.argtypes = [vp, ctypes.c_uint32, ctypes.c_int32]
    lib.dd_get_timing.argtypes = [vp, _f64p, ctypes.POINTER(ctypes.c_int64)]
    lib.dd_last_error.argtypes = [vp]
    lib.dd_last_error.restype = ctypes.c_char_p
    lib.dd_destroy.argtypes = [vp]
    lib.dd_destroy.restype = None
    lib.dd_assemble_2d.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp, vp]
    lib.dd_feti_setup.argtypes = [ctypes.POINTER(dd_problem), ctypes.POINTER(dd_feti_sub), vp, ctypes.c_int32,
                                  ctypes.POINTER(vp)]
    lib.dd_feti_factor.argtypes = [vp]
    lib.dd_feti_solve.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                  ctypes.POINTER(dd_solve_info)]
    lib.dd_bdd_solve.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                 ctypes.POINTER(dd_solve_info)]
    lib.dd_method_solve.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_int32, ctypes.POINTER(dd_solve_info)]
    lib.dd_method_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _i32p, _f64p]
    lib.dd_feti_last_error.argtypes = [vp]
    lib.dd_feti_last_error.restype = ctypes.c_char_p
    lib.dd_feti_destroy.argtypes = [vp]
    lib.dd_feti_destroy.restype = None
    for name in ("dd_feti_setup", "dd_feti_factor", "dd_feti_solve", "dd_bdd_solve", "dd_method_solve",
                 "dd_method_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("dd_footprint", "dd_setup", "dd_factor", "dd_solve", "dd_schur_apply",
                 "dd_schur_apply_noalloc", "dd_get_factor", "dd_get_schur_diag", "dd_set_timing", "dd_get_timing",
                 "dd_autotune", "dd_batch_begin", "dd_batch_admit", "dd_batch_step",
                 "dd_batch_retire", "dd_batch_end", "dd_assemble_2d"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


# ----------------------------------------------------------------- marshalling
class _Problem:
    """Holds the ctypes view of a partitioned system (and keeps arrays alive)."""

    def __init__(self, dd):
        self.keep = []

        def i32(a):
            a = np.ascontiguousarray(a, dtype=np.int32)
            self.keep.append(a)
            return a.ctypes.data_as(_i32p)

        def f64(a):
            a = np.ascontiguousarray(a, dtype=np.float64)
            self.keep.append(a)
            return a.ctypes.data_as(_f64p)

        subs = (dd_subdomain * max(1, dd.n_sub))()     # n_sub = 0: undecomposed system
        for k in range(dd.n_sub):
            kig = dd.kig[k].tocsr()
            s = subs[k]
            s.n_i = int(dd.kii[k].shape[0])
            s.k_ii = f64(np.asfortranarray(dd.kii[k]).ravel(order="F"))
            s.n_g = int(len(dd.g_maps[k]))
            s.g_map = i32(dd.g_maps[k])
            s.kig_rowptr = i32(kig.indptr)
            s.kig_col = i32(kig.indices)
            s.kig_val = f64(kig.data)
            s.i_map = i32(dd.i_maps[k])
        self.keep.append(subs)
        kgg = dd.kgg.tocsr()
        self.p = dd_problem(int(dd.n_dof), int(dd.n_gamma), int(dd.n_sub), subs,
                            i32(dd.gamma_map), i32(kgg.indptr), i32(kgg.indices), f64(kgg.data))


def _check(lib, status: int, ctx=None):
    if status != DD_OK:
        msg = lib.dd_last_error(ctx)
        raise DDError(status, msg.decode() if msg else "")


def dd_default_opts(**overrides) -> dd_solve_opts:
    o = dd_solve_opts()
    load_library().dd_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def dd_footprint(dd, prec: int = DD_FP64, max_nrhs: int = 1) -> int:
    lib = load_library()
    pb = _Problem(dd)
    out = ctypes.c_size_t(0)
    _check(lib, lib.dd_footprint(ctypes.byref(pb.p), prec, max_nrhs, ctypes.byref(out)))
    return int(out.value)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    h = getattr(stream, "cuda_stream", stream)
    return ctypes.c_void_p(int(h) if h else 0)


def dd_setup(dd, stream=None, max_nrhs: int = 1) -> ctypes.c_void_p:
    lib = load_library()
    pb = _Problem(dd)
    ctx = ctypes.c_void_p()
    _check(lib, lib.dd_setup(ctypes.byref(pb.p), _stream_handle(stream), max_nrhs,
                             ctypes.byref(ctx)))
    return ctx


def dd_factor(ctx, prec: int = DD_FP64) -> None:
    lib = load_library()
    _check(lib, lib.dd_factor(ctx, prec), ctx)


def _dev_ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(int(t.data_ptr()))


def dd_solve(ctx, prec: int, b, u, nrhs: int, ld: int, opts: dd_solve_opts | None = None,
             raise_on_noconv: bool = True):
    """b, u: torch float64 CUDA tensors holding column-major n_dof x nrhs data
    (e.g. shape (nrhs, ld) row-major).  Returns (status, list of info dicts)."""
    lib = load_library()
    infos = (dd_solve_info * nrhs)()
    st = lib.dd_solve(ctx, prec, _dev_ptr(b), _dev_ptr(u), nrhs, ld,
                      ctypes.byref(opts) if opts is not None else None, infos)
    if st != DD_OK and (st != DD_ENOCONV or raise_on_noconv):
        _check(lib, st, ctx)
    return st, [dict(iters=i.iters, refine_steps=i.refine_steps, used_fallback=i.used_fallback,
                     converged=i.converged, rel_resid=i.rel_resid) for i in infos]


def dd_schur_apply(ctx, prec: int, p, q, nrhs: int, ld: int) -> None:
    lib = load_library()
    _check(lib, lib.dd_schur_apply(ctx, prec, _dev_ptr(p), _dev_ptr(q), nrhs, ld), ctx)


def dd_schur_apply_noalloc(ctx, prec: int, p, q, nrhs: int, ld: int) -> None:
    """dd_schur_apply without any device allocation (work vectors in the
    library's static device array; at most 4 Mi doubles of them)."""
    lib = load_library()
    _check(lib, lib.dd_schur_apply_noalloc(ctx, prec, _dev_ptr(p), _dev_ptr(q), nrhs, ld), ctx)


def dd_get_factor(ctx, prec: int, k: int, n: int) -> np.ndarray:
    lib = load_library()
    out = np.zeros(n * n, dtype=np.float64)
    _check(lib, lib.dd_get_factor(ctx, prec, k, out.ctypes.data_as(_f64p)), ctx)
    return out.reshape(n, n, order="F")


def dd_get_schur_diag(ctx, prec: int, n_gamma: int) -> np.ndarray:
    lib = load_library()
    out = np.zeros(n_gamma, dtype=np.float64)
    _check(lib, lib.dd_get_schur_diag(ctx, prec, out.ctypes.data_as(_f64p)), ctx)
    return out


def dd_autotune(ctx, prec: int, nrhs: int, opts: dd_solve_opts | None = None) -> dict:
    """Time the candidate CG schedules and keep the fastest (used by AUTO solves)."""
    lib = load_library()
    r = dd_tune_result()
    _check(lib, lib.dd_autotune(ctx, prec, nrhs, ctypes.byref(opts) if opts is not None else None,
                                ctypes.byref(r)), ctx)
    return dict(apply=r.apply, launch=r.launch, direction_kernel=r.direction_kernel,
                check_every=r.check_every, ms_per_solve=r.ms_per_solve, candidates=r.candidates,
                inner_tol=r.inner_tol, three_launch=r.three_launch)


def dd_batch_begin(ctx, prec: int, opts: dd_solve_opts | None = None) -> None:
    lib = load_library()
    _check(lib, lib.dd_batch_begin(ctx, prec, ctypes.byref(opts) if opts is not None else None), ctx)


def _i32arr(v):
    a = (ctypes.c_int32 * len(v))(*[int(x) for x in v])
    return a


def dd_batch_admit(ctx, slots, b, ld: int) -> None:
    """b: torch float64 CUDA tensor with len(slots) right-hand sides (column-major, ld)."""
    lib = load_library()
    _check(lib, lib.dd_batch_admit(ctx, _i32arr(slots), len(slots), _dev_ptr(b), ld), ctx)


def dd_batch_step(ctx, iters: int, max_nrhs: int) -> list:
    lib = load_library()
    st = (ctypes.c_int32 * max_nrhs)()
    _check(lib, lib.dd_batch_step(ctx, iters, st), ctx)
    return list(st)


def dd_batch_retire(ctx, slots, u, ld: int) -> list:
    lib = load_library()
    infos = (dd_solve_info * len(slots))()
    _check(lib, lib.dd_batch_retire(ctx, _i32arr(slots), len(slots), _dev_ptr(u), ld, infos), ctx)
    return [dict(iters=i.iters, refine_steps=i.refine_steps, used_fallback=i.used_fallback,
                 converged=i.converged, rel_resid=i.rel_resid) for i in infos]


def dd_batch_end(ctx) -> None:
    lib = load_library()
    _check(lib, lib.dd_batch_end(ctx), ctx)


def dd_assemble_2d(n: int, collar: int, delta: float, kernel: int, phi: float, s: float, R: int,
                   win, stream=None) -> None:
    """Device assembly of the 2D nonlocal stiffness windows into `win` (a
    float64 CUDA tensor of (n-1)^2 rows of (2R+1)^2 values, 4 (2R+1)^2 for the
    peridynamic kernel); launched on `stream` (default: the current one)."""
    lib = load_library()
    W = 2 * R + 1
    need = (n - 1) * (n - 1) * W * W * (4 if kernel == 2 else 1)
    if win.dtype.itemsize != 8 or not win.is_cuda or not win.is_contiguous() or win.numel() != need:
        raise ValueError(f"win must be a contiguous float64 CUDA tensor of {need} values")
    _check(lib, lib.dd_assemble_2d(n, collar, delta, kernel, phi, s, R, ctypes.c_void_p(win.data_ptr()),
                                   _stream_handle(stream)))


def dd_set_timing(ctx, phase_mask: int, reset: bool = True) -> None:
    lib = load_library()
    _check(lib, lib.dd_set_timing(ctx, phase_mask, 1 if reset else 0), ctx)


def dd_get_timing(ctx):
    """Returns (ms per phase, launches per phase) accumulated since the last reset."""
    lib = load_library()
    ms = (ctypes.c_double * DD_NPHASES)()
    n = (ctypes.c_int64 * DD_NPHASES)()
    _check(lib, lib.dd_get_timing(ctx, ms, n), ctx)
    return list(ms), list(n)


def dd_last_error(ctx=None) -> str:
    m = load_library().dd_last_error(ctx)
    return m.decode() if m else ""


def dd_destroy(ctx) -> None:
    if ctx is not None and ctx.value:
        load_library().dd_destroy(ctx)


# --------------------------------------------------------------- convenience
@dataclass
class SolveResult:
    u: object            # torch tensor (nrhs, ld) on the device
    status: int
    info: list


class Solver:
    """Owns one solver context bound to a torch stream."""

    def __init__(self, dd, max_nrhs: int = 1, stream=None):
        import torch
        self.torch = torch
        self.dd = dd
        self.n_dof = int(dd.n_dof)
        self.n_gamma = int(dd.n_gamma)
        self.max_nrhs = max_nrhs
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = dd_setup(dd, self.stream, max_nrhs)

    def factor(self, prec: int = DD_FP64) -> None:
        dd_factor(self.ctx, prec)

    def solve(self, b, prec: int = DD_FP64, opts: dd_solve_opts | None = None, u=None,
              raise_on_noconv: bool = True) -> SolveResult:
        """b: (nrhs, n_dof) float64 CUDA tensor (each row one right-hand side)."""
        torch = self.torch
        nrhs = int(b.shape[0])
        ld = int(b.stride(0)) if nrhs > 1 else int(b.shape[1])
        if b.dtype != torch.float64 or not b.is_cuda or (b.shape[1] > 1 and b.stride(1) != 1):
            raise ValueError("b must be a CUDA float64 tensor with unit inner stride")
        if u is None:
            u = torch.empty((nrhs, ld), dtype=torch.float64, device=b.device)
        st, info = dd_solve(self.ctx, prec, b, u, nrhs, ld, opts, raise_on_noconv)
        return SolveResult(u[:, :self.n_dof], st, info)

    def autotune(self, prec: int = DD_FP64, nrhs: int = 1, opts: dd_solve_opts | None = None) -> dict:
        return dd_autotune(self.ctx, prec, nrhs, opts)

    def schur_apply(self, p, prec: int = DD_FP64):
        torch = self.torch
        p = p.contiguous()
        q = torch.empty_like(p)
        dd_schur_apply(self.ctx, prec, p, q, int(p.shape[0]), int(p.shape[1]))
        return q

    def factor_block(self, k: int, prec: int = DD_FP64) -> np.ndarray:
        return dd_get_factor(self.ctx, prec, k, int(self.dd.kii[k].shape[0]))

    def schur_diag(self, prec: int = DD_FP64) -> np.ndarray:
        return dd_get_schur_diag(self.ctx, prec, self.n_gamma)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None:
            dd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- one-level FETI
def _feti_check(lib, status: int, ctx=None):
    if status != DD_OK:
        msg = lib.dd_feti_last_error(ctx)
        raise DDError(status, msg.decode() if msg else "")


class _FetiSubs:
    """ctypes view of the per-subdomain FETI data (keeps the arrays alive).
    fp: workloads.FetiProblem-like object with g_sets, agg, kig and, per
    floating subdomain, z (empty for the others)."""

    def __init__(self, fp):
        self.keep = []

        def i32(a):
            a = np.ascontiguousarray(a, dtype=np.int32)
            self.keep.append(a)
            return a.ctypes.data_as(_i32p)

        def f64(a):
            a = np.ascontiguousarray(a, dtype=np.float64)
            self.keep.append(a)
            return a.ctypes.data_as(_f64p)

        K = len(fp.g_sets)
        self.subs = (dd_feti_sub * K)()
        for k in range(K):
            agg = fp.agg[k].tocsr()
            kig = fp.kig[k].tocsr()
            z = np.asarray(fp.z[k], dtype=np.float64)
            s = self.subs[k]
            s.n_g = int(len(fp.g_sets[k]))
            s.g_map = i32(fp.g_sets[k])
            s.agg_rowptr, s.agg_col, s.agg_val = i32(agg.indptr), i32(agg.indices), f64(agg.data)
            s.kig_rowptr, s.kig_col, s.kig_val = i32(kig.indptr), i32(kig.indices), f64(kig.data)
            s.n_z = int(z.shape[1]) if fp.floating[k] else 0
            s.z = f64(z.ravel(order="F")) if s.n_z else None


def dd_feti_setup(dd, fp, stream=None, max_nrhs: int = 1):
    lib = load_library()
    pb = _Problem(dd)
    fs = _FetiSubs(fp)
    ctx = ctypes.c_void_p()
    st = lib.dd_feti_setup(ctypes.byref(pb.p), fs.subs, _stream_handle(stream), max_nrhs, ctypes.byref(ctx))
    _feti_check(lib, st, None)
    return ctx


def dd_feti_factor(ctx) -> None:
    lib = load_library()
    _feti_check(lib, lib.dd_feti_factor(ctx), ctx)


def dd_feti_solve(ctx, b, u, nrhs: int, ld: int, tol: float, max_it: int, raise_on_noconv: bool = True):
    lib = load_library()
    info = (dd_solve_info * nrhs)()
    st = lib.dd_feti_solve(ctx, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(u.data_ptr()), nrhs, ld, tol,
                           max_it, info)
    if st != DD_OK and not (st == DD_ENOCONV and not raise_on_noconv):
        _feti_check(lib, st, ctx)
    return st, [dict(iters=i.iters, converged=i.converged, rel_resid=i.rel_resid) for i in info]


def dd_bdd_solve(ctx, b, u, nrhs: int, ld: int, tol: float, max_it: int, raise_on_noconv: bool = True):
    lib = load_library()
    info = (dd_solve_info * nrhs)()
    st = lib.dd_bdd_solve(ctx, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(u.data_ptr()), nrhs, ld, tol,
                          max_it, info)
    if st != DD_OK and not (st == DD_ENOCONV and not raise_on_noconv):
        _feti_check(lib, st, ctx)
    return st, [dict(iters=i.iters, converged=i.converged, rel_resid=i.rel_resid) for i in info]


def dd_method_solve(ctx, method: int, b, u, nrhs: int, ld: int, tol: float, max_it: int,
                    raise_on_noconv: bool = True):
    lib = load_library()
    info = (dd_solve_info * nrhs)()
    st = lib.dd_method_solve(ctx, method, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(u.data_ptr()), nrhs,
                             ld, tol, max_it, info)
    if st != DD_OK and not (st == DD_ENOCONV and not raise_on_noconv):
        _feti_check(lib, st, ctx)
    return st, [dict(iters=i.iters, converged=i.converged, rel_resid=i.rel_resid) for i in info]


def dd_method_autotune(ctx, nrhs: int, tol: float, max_it: int = 1000) -> dict:
    """Time FETI, BDD and Jacobi on a seeded batch; the fastest serves DD_METHOD_AUTO."""
    lib = load_library()
    m = ctypes.c_int32(0)
    ms = (ctypes.c_double * 3)()
    _feti_check(lib, lib.dd_method_autotune(ctx, nrhs, tol, max_it, ctypes.byref(m),
                                            ctypes.cast(ms, _f64p)), ctx)
    return dict(method=int(m.value), ms_feti=ms[0], ms_bdd=ms[1], ms_jacobi=ms[2])


def dd_feti_destroy(ctx) -> None:
    if ctx is not None and ctx.value:
        load_library().dd_feti_destroy(ctx)


class FetiSolver:
    """One-level FETI context (dd_feti_*) bound to a torch stream."""

    def __init__(self, dd, fp, max_nrhs: int = 1, stream=None):
        import torch
        self.torch = torch
        self.n_dof = int(dd.n_dof)
        self.max_nrhs = max_nrhs
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = dd_feti_setup(dd, fp, self.stream, max_nrhs)

    def factor(self) -> None:
        dd_feti_factor(self.ctx)

    def solve(self, b, tol: float = 1e-10, max_it: int = 1000, raise_on_noconv: bool = True) -> SolveResult:
        torch = self.torch
        nrhs = int(b.shape[0])
        ld = int(b.stride(0)) if nrhs > 1 else int(b.shape[1])
        if b.dtype != torch.float64 or not b.is_cuda or (b.shape[1] > 1 and b.stride(1) != 1):
            raise ValueError("b must be a CUDA float64 tensor with unit inner stride")
        u = torch.empty((nrhs, ld), dtype=torch.float64, device=b.device)
        st, info = dd_feti_solve(self.ctx, b, u, nrhs, ld, tol, max_it, raise_on_noconv)
        return SolveResult(u[:, :self.n_dof], st, info)

    def _out(self, b):
        torch = self.torch
        nrhs = int(b.shape[0])
        ld = int(b.stride(0)) if nrhs > 1 else int(b.shape[1])
        if b.dtype != torch.float64 or not b.is_cuda or (b.shape[1] > 1 and b.stride(1) != 1):
            raise ValueError("b must be a CUDA float64 tensor with unit inner stride")
        return nrhs, ld, torch.empty((nrhs, ld), dtype=torch.float64, device=b.device)

    def solve_bdd(self, b, tol: float = 1e-10, max_it: int = 1000, raise_on_noconv: bool = True) -> SolveResult:
        """Primal interface CG with the balancing Neumann-Neumann preconditioner."""
        nrhs, ld, u = self._out(b)
        st, info = dd_bdd_solve(self.ctx, b, u, nrhs, ld, tol, max_it, raise_on_noconv)
        return SolveResult(u[:, :self.n_dof], st, info)

    def solve_method(self, b, method: int = DD_METHOD_AUTO, tol: float = 1e-10, max_it: int = 1000,
                     raise_on_noconv: bool = True) -> SolveResult:
        nrhs, ld, u = self._out(b)
        st, info = dd_method_solve(self.ctx, method, b, u, nrhs, ld, tol, max_it, raise_on_noconv)
        return SolveResult(u[:, :self.n_dof], st, info)

    def autotune(self, nrhs: int, tol: float = 1e-10, max_it: int = 1000) -> dict:
        return dd_method_autotune(self.ctx, nrhs, tol, max_it)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None:
            dd_feti_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
