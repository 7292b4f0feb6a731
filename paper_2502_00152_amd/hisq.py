"""Python binding of libhisq (ctypes).  Argument marshalling only.

Every function here has the name of the C entry point it calls (include/hisq.h)
and takes torch tensors for device buffers; torch supplies memory and the
current stream, the library does all the work.  There is no CPU fallback: if
libhisq.so is missing or no GPU is present, calls raise.

Layouts (see include/hisq.h):
    links          complex128 [4, T, Z, Y, X, 3, 3]  (device)
    full vectors   complex128 [nrhs, T, Z, Y, X, 3]
    parity vectors complex128 [nrhs, 3, Vh]          (Vh = X*Y*Z*T/2)
                   complex64 for the FP32 stencil and FP32 eigenvectors
                   bfloat16 [nrhs, 3, Vh, 2] (real, imaginary) for BF16 storage
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhisq.so")

HISQ_OK = 0
HISQ_ERR_INVALID_ARG = 1
HISQ_ERR_HIP = 2
HISQ_ERR_OOM = 3
HISQ_ERR_NOT_CONVERGED = 4
HISQ_ERR_NAN = 5
HISQ_ERR_BREAKDOWN = 6
HISQ_ERR_UNSUPPORTED = 7
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "HIP", 3: "OOM", 4: "NOT_CONVERGED", 5: "NAN",
                6: "BREAKDOWN", 7: "UNSUPPORTED"}

HISQ_FP64, HISQ_FP32, HISQ_BF16, HISQ_Q16, HISQ_HALF = 0, 1, 2, 3, 4
HISQ_GAUGE_FOLD_PHASES = 1
HISQ_GAUGE_ANTIPERIODIC_T = 2
ABI_VERSION = 10
NOALLOC_SCRATCH_BYTES = 64 << 20  # HISQ_NOALLOC_SCRATCH_BYTES
HISQ_NN_CHANNELS = 8
HISQ_NN_PARAMS = 752
HISQ_NN_NORMALIZE, HISQ_NN_BF16 = 1, 2

# Entry points declared in include/hisq.h (the tests check the library exports them all).
EXPORTS = (
    "hisq_last_error", "hisq_abi_version", "hisq_gauge_create", "hisq_gauge_destroy",
    "hisq_gauge_half_volume", "hisq_spinor_split", "hisq_spinor_merge", "hisq_dslash_eo",
    "hisq_mdagm", "hisq_prepare_source", "hisq_reconstruct_odd", "hisq_cg_solve",
    "hisq_deflate", "hisq_eigensolve", "hisq_set_tuning", "hisq_profile_enable",
    "hisq_profile_read", "hisq_convert_vectors", "hisq_propagator_solve",
    "hisq_autotune_dslash", "hisq_cg_solve_multi", "hisq_nn_create", "hisq_nn_destroy",
    "hisq_nn_set_params", "hisq_nn_get_params", "hisq_nn_apply", "hisq_nn_loss_grad",
    "hisq_nn_adam_step", "hisq_nn_train", "hisq_nn_guess", "hisq_mdagm_noalloc",
)


class HisqError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class CgParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("check_interval", ctypes.c_int), ("sloppy_prec", ctypes.c_int),
                ("reliable_interval", ctypes.c_int), ("reliable_delta", ctypes.c_double),
                ("n_ev", ctypes.c_int), ("evec_prec", ctypes.c_int),
                ("evecs_dev", ctypes.c_void_p), ("evals_host", ctypes.POINTER(ctypes.c_double)),
                ("tol_restart", ctypes.c_double),
                ("two_m_rhs", ctypes.POINTER(ctypes.c_double)), ("parity", ctypes.c_int),
                ("reserved", ctypes.c_int * 7)]


class CgStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("true_residual_checks", ctypes.c_int),
                ("converged", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("redeflations", ctypes.c_int), ("reserved0", ctypes.c_int),
                ("true_residual", ctypes.c_double), ("b_norm", ctypes.c_double)]


class System(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("two_m", ctypes.c_double), ("b_dev", ctypes.c_void_p),
                ("x_dev", ctypes.c_void_p), ("nrhs", ctypes.c_int), ("reserved", ctypes.c_int)]


class PropParams(ctypes.Structure):
    _fields_ = [("cg", CgParams), ("polish_tol", ctypes.c_double),
                ("polish_max_iter", ctypes.c_int), ("reserved", ctypes.c_int * 7)]


class PropStats(ctypes.Structure):
    _fields_ = [("even", CgStats), ("polish", CgStats), ("residual", ctypes.c_double),
                ("residual_even", ctypes.c_double), ("reserved", ctypes.c_double * 2)]


class TuneResult(ctypes.Structure):
    _fields_ = [("rhs_per_thread", ctypes.c_int), ("lanes_per_site", ctypes.c_int),
                ("group_order", ctypes.c_int), ("xcd_remap", ctypes.c_int),
                ("us_best", ctypes.c_double), ("us_default", ctypes.c_double),
                ("shapes_timed", ctypes.c_int), ("march", ctypes.c_int),
                ("blocks_per_cu", ctypes.c_int), ("reserved", ctypes.c_int * 1)]


EIG_PROGRESS = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_double)


class EigParams(ctypes.Structure):
    _fields_ = [("n_kr", ctypes.c_int), ("cheb_degree", ctypes.c_int),
                ("cheb_a", ctypes.c_double), ("cheb_b", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_restarts", ctypes.c_int),
                ("evec_prec", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("progress", EIG_PROGRESS), ("progress_user", ctypes.c_void_p),
                ("block", ctypes.c_int), ("reserved", ctypes.c_int * 7)]


class EigStats(ctypes.Structure):
    _fields_ = [("restarts", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("converged", ctypes.c_int), ("cheb_degree", ctypes.c_int),
                ("cheb_a", ctypes.c_double), ("cheb_b", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("max_residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]


_lib = None


def lib():
    """Load libhisq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2502_00152_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
    sigs = {
        "hisq_last_error": ([], ctypes.c_char_p),
        "hisq_abi_version": ([], I),
        "hisq_gauge_create": ([ctypes.POINTER(P), ctypes.POINTER(I), P, P, D, D, U, P], I),
        "hisq_gauge_destroy": ([P], I),
        "hisq_gauge_half_volume": ([P], ctypes.c_int64),
        "hisq_spinor_split": ([P, P, P, P, I, P], I),
        "hisq_spinor_merge": ([P, P, P, P, I, P], I),
        "hisq_dslash_eo": ([P, I, P, P, I, I, P], I),
        "hisq_mdagm": ([P, D, P, P, I, I, P], I),
        "hisq_mdagm_noalloc": ([P, D, P, P, I, I, P], I),
        "hisq_prepare_source": ([P, D, P, P, P, I, P], I),
        "hisq_reconstruct_odd": ([P, D, P, P, P, I, P], I),
        "hisq_cg_solve": ([P, D, P, P, I, ctypes.POINTER(CgParams), ctypes.POINTER(CgStats),
                           P], I),
        "hisq_deflate": ([P, I, P, I, ctypes.POINTER(D), D, P, P, I, P], I),
        "hisq_eigensolve": ([P, D, I, ctypes.POINTER(EigParams), P, ctypes.POINTER(D),
                             ctypes.POINTER(EigStats), P], I),
        "hisq_set_tuning": ([ctypes.c_char_p, ctypes.c_int64], I),
        "hisq_convert_vectors": ([P, I, P, I, ctypes.c_int64, P], I),
        "hisq_propagator_solve": ([P, D, P, P, I, ctypes.POINTER(PropParams),
                                   ctypes.POINTER(PropStats), P], I),
        "hisq_autotune_dslash": ([P, I, I, I, ctypes.POINTER(TuneResult), P], I),
        "hisq_cg_solve_multi": ([I, ctypes.POINTER(System), ctypes.POINTER(CgParams),
                                 ctypes.POINTER(CgStats), P], I),
        "hisq_nn_create": ([ctypes.POINTER(P), P, ctypes.POINTER(ctypes.c_float)], I),
        "hisq_nn_destroy": ([P], I),
        "hisq_nn_set_params": ([P, ctypes.POINTER(ctypes.c_float)], I),
        "hisq_nn_get_params": ([P, ctypes.POINTER(ctypes.c_float)], I),
        "hisq_nn_apply": ([P, P, P, I, U, P], I),
        "hisq_nn_loss_grad": ([P, P, P, I, U, ctypes.POINTER(D), ctypes.POINTER(D), P], I),
        "hisq_nn_adam_step": ([P, D, D, D, D, P], I),
        "hisq_nn_train": ([P, P, P, I, I, I, D, U, ctypes.POINTER(D), P], I),
        "hisq_nn_guess": ([P, D, P, P, I, U, I, P, I, ctypes.POINTER(D), ctypes.POINTER(I), P],
                          I),
        "hisq_profile_enable": ([I], I),
        "hisq_profile_read": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(D)], I),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    if L.hisq_abi_version() != ABI_VERSION:
        raise RuntimeError("libhisq ABI version mismatch: rebuild the library")
    _lib = L
    return L


def _check(status: int, where: str, ok=(HISQ_OK,)):
    if status not in ok:
        raise HisqError(status, where, lib().hisq_last_error().decode())
    return status


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


_PREC_OF_DTYPE = {"complex128": HISQ_FP64, "complex64": HISQ_FP32, "bfloat16": HISQ_BF16}
_VEC_DTYPES = ("complex128", "complex64", "bfloat16")


def _prec_of(t, name):
    """HISQ_FP64 for complex128 tensors, HISQ_FP32 for complex64, HISQ_BF16 for
    bfloat16 tensors with a trailing (real, imaginary) axis of 2."""
    dt = str(t.dtype).replace("torch.", "")
    if dt not in _PREC_OF_DTYPE:
        raise TypeError(f"{name} must be complex128, complex64 or bfloat16, got {t.dtype}")
    if dt == "bfloat16" and (t.dim() < 1 or t.shape[-1] != 2):
        raise ValueError(f"{name}: a bfloat16 vector needs a trailing axis of 2 (re, im)")
    return _PREC_OF_DTYPE[dt]


def _complex_view_shape(t):
    """Shape of t as complex numbers (drops the (re, im) axis of bfloat16)."""
    return tuple(t.shape[:-1]) if str(t.dtype) == "torch.bfloat16" else tuple(t.shape)


def _ptr(t, name, dtype_ok=("complex128",)):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if str(t.dtype).replace("torch.", "") not in dtype_ok:
        raise TypeError(f"{name} must have dtype {dtype_ok}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ sizes
def vector_bytes(dims, n_vectors: int, single_parity: bool = True, prec: int = HISQ_FP64) -> int:
    """Bytes of n colour-vector fields: 3 complex per site, 8/4/2 bytes per real."""
    V = int(np.prod([int(d) for d in dims]))
    sites = V // 2 if single_parity else V
    real = {HISQ_FP64: 8, HISQ_FP32: 4, HISQ_BF16: 2}[prec]
    return sites * n_vectors * 3 * 2 * real


# ------------------------------------------------------------------ gauge
class Gauge:
    """Owns a hisq_gauge handle."""

    def __init__(self, dims, fat, lng, c_fat=1.0, c_long=1.0,
                 flags=HISQ_GAUGE_FOLD_PHASES | HISQ_GAUGE_ANTIPERIODIC_T, stream=None):
        self.dims = tuple(int(d) for d in dims)
        self.handle = hisq_gauge_create(self.dims, fat, lng, c_fat, c_long, flags, stream)
        self.vh = int(lib().hisq_gauge_half_volume(self.handle))

    def close(self):
        if self.handle:
            hisq_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _h(g):
    return g.handle if isinstance(g, Gauge) else g


def _nrhs(t, vh, name):
    if t.dim() != 3 or t.shape[1] != 3 or t.shape[2] != vh:
        raise ValueError(f"{name} must have shape [nrhs, 3, {vh}], got {tuple(t.shape)}")
    return int(t.shape[0])


def hisq_gauge_create(dims, fat, lng, c_fat, c_long, flags, stream=None):
    X, Y, Z, T = (int(d) for d in dims)
    for t, nm in ((fat, "fat"), (lng, "long")):
        if tuple(t.shape) != (4, T, Z, Y, X, 3, 3):
            raise ValueError(f"{nm} links must have shape [4,T,Z,Y,X,3,3]")
    h = ctypes.c_void_p()
    d = (ctypes.c_int * 4)(X, Y, Z, T)
    _check(lib().hisq_gauge_create(ctypes.byref(h), d, _ptr(fat, "fat"), _ptr(lng, "long"),
                                   float(c_fat), float(c_long), int(flags), _stream(stream)),
           "hisq_gauge_create")
    return h


def hisq_gauge_destroy(handle):
    _check(lib().hisq_gauge_destroy(handle), "hisq_gauge_destroy")


def hisq_spinor_split(g, full, even, odd, stream=None):
    nrhs = int(full.shape[0])
    _check(lib().hisq_spinor_split(_h(g), _ptr(full, "full"),
                                   None if even is None else _ptr(even, "even"),
                                   None if odd is None else _ptr(odd, "odd"), nrhs,
                                   _stream(stream)), "hisq_spinor_split")


def hisq_spinor_merge(g, even, odd, full, stream=None):
    nrhs = int(full.shape[0])
    _check(lib().hisq_spinor_merge(_h(g), None if even is None else _ptr(even, "even"),
                                   None if odd is None else _ptr(odd, "odd"),
                                   _ptr(full, "full"), nrhs, _stream(stream)),
           "hisq_spinor_merge")


def _nrhs_any(t, vh, name):
    shp = _complex_view_shape(t)
    if len(shp) != 3 or shp[1] != 3 or shp[2] != vh:
        raise ValueError(f"{name} must hold [nrhs, 3, {vh}] complex numbers, got {tuple(t.shape)}")
    return int(shp[0])


def _vec_pair(g, inp, out, prec):
    """nrhs and precision of an (in, out) pair; prec defaults to the tensors' dtype."""
    nrhs = _nrhs_any(inp, g.vh, "in")
    if _nrhs_any(out, g.vh, "out") != nrhs:
        raise ValueError("in and out must have the same nrhs")
    if inp.dtype != out.dtype:
        raise TypeError("in and out must have the same dtype")
    p = _prec_of(inp, "in")
    return nrhs, p if prec is None else int(prec)


def hisq_dslash_eo(g, out_parity, inp, out, prec=None, stream=None):
    nrhs, prec = _vec_pair(g, inp, out, prec)
    _check(lib().hisq_dslash_eo(_h(g), int(out_parity), _ptr(inp, "in", _VEC_DTYPES),
                                _ptr(out, "out", _VEC_DTYPES), nrhs, prec, _stream(stream)),
           "hisq_dslash_eo")


def hisq_mdagm(g, two_m, inp, out, prec=None, stream=None):
    nrhs, prec = _vec_pair(g, inp, out, prec)
    _check(lib().hisq_mdagm(_h(g), float(two_m), _ptr(inp, "in", _VEC_DTYPES),
                            _ptr(out, "out", _VEC_DTYPES), nrhs, prec, _stream(stream)),
           "hisq_mdagm")


def hisq_mdagm_noalloc(g, two_m, inp, out, prec=None, stream=None):
    """hisq_mdagm with its temporary in the library's fixed device array (no
    allocation); FP64 or FP32 vectors, at most NOALLOC_SCRATCH_BYTES of temporary."""
    nrhs, prec = _vec_pair(g, inp, out, prec)
    _check(lib().hisq_mdagm_noalloc(_h(g), float(two_m), _ptr(inp, "in", _VEC_DTYPES),
                                    _ptr(out, "out", _VEC_DTYPES), nrhs, prec, _stream(stream)),
           "hisq_mdagm_noalloc")


def hisq_prepare_source(g, two_m, eta_e, eta_o, y_e, stream=None):
    nrhs = _nrhs(eta_e, g.vh, "eta_e")
    for t, nm in ((eta_o, "eta_o"), (y_e, "y_e")):
        if _nrhs(t, g.vh, nm) != nrhs:
            raise ValueError("all vectors must have the same nrhs")
    _check(lib().hisq_prepare_source(_h(g), float(two_m), _ptr(eta_e, "eta_e"),
                                     _ptr(eta_o, "eta_o"), _ptr(y_e, "y_e"), nrhs,
                                     _stream(stream)), "hisq_prepare_source")


def hisq_reconstruct_odd(g, two_m, psi_e, eta_o, psi_o, stream=None):
    nrhs = _nrhs(psi_e, g.vh, "psi_e")
    for t, nm in ((eta_o, "eta_o"), (psi_o, "psi_o")):
        if _nrhs(t, g.vh, nm) != nrhs:
            raise ValueError("all vectors must have the same nrhs")
    _check(lib().hisq_reconstruct_odd(_h(g), float(two_m), _ptr(psi_e, "psi_e"),
                                      _ptr(eta_o, "eta_o"), _ptr(psi_o, "psi_o"), nrhs,
                                      _stream(stream)), "hisq_reconstruct_odd")


@dataclass
class CgResult:
    status: int
    iterations: list
    true_residual: list
    converged: list
    checks: list
    b_norm: list
    reliable_updates: list
    redeflations: list


def hisq_cg_solve(g, two_m, b, x, tol=1e-10, max_iter=100000, check_interval=0,
                  sloppy_prec=HISQ_FP64, stream=None, raise_on_fail=True, reliable_interval=0,
                  reliable_delta=0.0, evecs=None, evals=None, tol_restart=0.0,
                  parity=0) -> CgResult:
    """CG on A x = b.  With sloppy_prec=HISQ_FP32: mixed precision with reliable
    updates; evecs/evals/tol_restart enable re-deflation (evecs complex128 or
    complex64 [n_ev, 3, Vh])."""
    nrhs = _nrhs(b, g.vh, "b")
    if _nrhs(x, g.vh, "x") != nrhs:
        raise ValueError("b and x must have the same nrhs")
    p, keep = _cg_params(tol, max_iter, check_interval, sloppy_prec, reliable_interval,
                         reliable_delta, evecs, evals, tol_restart, parity, g.vh, two_m, nrhs)
    stats = (CgStats * nrhs)()
    st = lib().hisq_cg_solve(_h(g), _scalar_mass(two_m), _ptr(b, "b"), _ptr(x, "x"), nrhs,
                             ctypes.byref(p), stats, _stream(stream))
    if raise_on_fail:
        _check(st, "hisq_cg_solve")
    elif st not in (HISQ_OK, HISQ_ERR_NOT_CONVERGED, HISQ_ERR_NAN, HISQ_ERR_BREAKDOWN):
        _check(st, "hisq_cg_solve")
    del keep  # host arrays kept alive across the call above
    return _cg_result(st, stats)


@dataclass
class PropResult:
    status: int
    even: CgResult
    polish: CgResult
    residual: list
    residual_even: list


def _scalar_mass(two_m):
    return float(np.asarray(two_m, dtype=np.float64).ravel()[0])


def _cg_params(tol, max_iter, check_interval, sloppy_prec, reliable_interval, reliable_delta,
               evecs, evals, tol_restart, parity, vh, two_m=None, nrhs=None):
    """CgParams and the host arrays it points to (keep them alive for the call)."""
    p = CgParams(tol=float(tol), max_iter=int(max_iter), check_interval=int(check_interval),
                 sloppy_prec=int(sloppy_prec), reliable_interval=int(reliable_interval),
                 reliable_delta=float(reliable_delta), tol_restart=float(tol_restart),
                 parity=int(parity))
    keep = []
    if two_m is not None and np.ndim(two_m) > 0:
        ms = np.ascontiguousarray(np.asarray(two_m, dtype=np.float64))
        if ms.shape != (nrhs,):
            raise ValueError("two_m must be a scalar or have one entry per RHS")
        p.two_m_rhs = ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        keep.append(ms)
    ev = None
    if evecs is not None:
        n_ev = _nrhs(evecs, vh, "evecs")
        ev = np.ascontiguousarray(np.asarray(evals, dtype=np.float64))
        if ev.shape != (n_ev,):
            raise ValueError("evals must have one entry per eigenvector")
        p.n_ev = n_ev
        p.evec_prec = _prec_of(evecs, "evecs")
        p.evecs_dev = _ptr(evecs, "evecs", ("complex128", "complex64")).value
        p.evals_host = ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        keep.append(ev)
    return p, keep


def _cg_result(st, stats):
    return CgResult(st, [s.iterations for s in stats], [s.true_residual for s in stats],
                    [bool(s.converged) for s in stats], [s.true_residual_checks for s in stats],
                    [s.b_norm for s in stats], [s.reliable_updates for s in stats],
                    [s.redeflations for s in stats])


def hisq_propagator_solve(g, two_m, eta, psi, tol=1e-10, max_iter=100000, sloppy_prec=HISQ_FP64,
                          reliable_delta=0.0, evecs=None, evals=None, tol_restart=0.0,
                          polish_tol=0.0, polish_max_iter=0, stream=None,
                          raise_on_fail=True) -> PropResult:
    """M psi = eta for full-lattice sources eta [nrhs, T, Z, Y, X, 3] (complex128):
    even solve (FP64 or mixed, optional deflation and re-deflation), odd
    reconstruction, optional odd polish to polish_tol."""
    X, Y, Z, T = g.dims
    nrhs = int(eta.shape[0])
    for t, nm in ((eta, "eta"), (psi, "psi")):
        if tuple(t.shape) != (nrhs, T, Z, Y, X, 3):
            raise ValueError(f"{nm} must have shape [nrhs, T, Z, Y, X, 3]")
    cg, keep = _cg_params(tol, max_iter, 0, sloppy_prec, 0, reliable_delta, evecs, evals,
                          tol_restart, 0, g.vh)
    p = PropParams(cg=cg, polish_tol=float(polish_tol), polish_max_iter=int(polish_max_iter))
    stats = (PropStats * nrhs)()
    st = lib().hisq_propagator_solve(_h(g), float(two_m), _ptr(eta, "eta"), _ptr(psi, "psi"), nrhs,
                                     ctypes.byref(p), stats, _stream(stream))
    del keep  # kept alive across the call above
    if raise_on_fail:
        _check(st, "hisq_propagator_solve")
    elif st not in (HISQ_OK, HISQ_ERR_NOT_CONVERGED, HISQ_ERR_NAN, HISQ_ERR_BREAKDOWN):
        _check(st, "hisq_propagator_solve")
    return PropResult(st, _cg_result(st, [s.even for s in stats]),
                      _cg_result(st, [s.polish for s in stats]),
                      [s.residual for s in stats], [s.residual_even for s in stats])


def hisq_cg_solve_multi(systems, tol=1e-10, max_iter=100000, sloppy_prec=HISQ_FP64,
                        reliable_delta=0.0, stream=None, raise_on_fail=True):
    """Solve independent systems [(gauge, two_m, b, x), ...] concurrently (one
    parameter set for all; two_m a scalar or one mass per RHS); returns one
    CgResult per system."""
    n = len(systems)
    arr = (System * n)()
    prm = (CgParams * n)()
    total, keep = 0, []
    for i, (g, two_m, b, x) in enumerate(systems):
        nr = _nrhs(b, g.vh, "b")
        if _nrhs(x, g.vh, "x") != nr:
            raise ValueError("b and x must have the same nrhs")
        arr[i] = System(g=_h(g), two_m=_scalar_mass(two_m), b_dev=_ptr(b, "b").value,
                        x_dev=_ptr(x, "x").value, nrhs=nr)
        prm[i], k = _cg_params(tol, max_iter, 0, sloppy_prec, 0, reliable_delta, None, None, 0.0,
                               0, g.vh, two_m, nr)
        keep += k
        total += nr
    stats = (CgStats * total)()
    st = lib().hisq_cg_solve_multi(n, arr, prm, stats, _stream(stream))
    del keep
    if raise_on_fail:
        _check(st, "hisq_cg_solve_multi")
    out, k = [], 0
    for i in range(n):
        nr = arr[i].nrhs
        out.append(_cg_result(st, stats[k:k + nr]))
        k += nr
    return out


def hisq_convert_vectors(src, dst, stream=None):
    """dst = src in dst's precision (complex128, complex64 or bfloat16 pairs; the
    same number of complex entries), rounded to nearest even."""
    ps, pd = _prec_of(src, "src"), _prec_of(dst, "dst")
    n = int(np.prod(_complex_view_shape(src)))
    if _complex_view_shape(src) != _complex_view_shape(dst):
        raise ValueError("src and dst must hold the same shape of complex numbers")
    _check(lib().hisq_convert_vectors(_ptr(src, "src", _VEC_DTYPES), ps,
                                      _ptr(dst, "dst", _VEC_DTYPES), pd, n, _stream(stream)),
           "hisq_convert_vectors")


def hisq_deflate(g, evecs, evals, two_m, b, x0, stream=None):
    """x0 = V diag(1/(eps + (2m)^2)) V^H b; evecs complex128 or complex64 (FP32)."""
    n_ev = _nrhs(evecs, g.vh, "evecs")
    nrhs = _nrhs(b, g.vh, "b")
    if _nrhs(x0, g.vh, "x0") != nrhs:
        raise ValueError("b and x0 must have the same nrhs")
    ev = np.ascontiguousarray(np.asarray(evals, dtype=np.float64))
    if ev.shape != (n_ev,):
        raise ValueError("evals must have one entry per eigenvector")
    _check(lib().hisq_deflate(_h(g), n_ev, _ptr(evecs, "evecs", ("complex128", "complex64")),
                              _prec_of(evecs, "evecs"), ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(two_m),
                              _ptr(b, "b"), _ptr(x0, "x0"), nrhs, _stream(stream)),
           "hisq_deflate")


def hisq_eigensolve(g, two_m, n_ev, evecs, n_kr=0, cheb_degree=0, cheb_a=0.0, cheb_b=0.0,
                    tol=1e-10, max_restarts=0, seed=0, stream=None, raise_on_fail=True,
                    progress=None, block=0):
    """progress: optional callable(restart, step, matvecs, seconds), called after
    every Lanczos step (restart -1 = pilot).  evecs complex128, or complex64 for
    single-precision eigenvectors (the solve is FP64 either way).  block: the
    Lanczos block size (0 or 1: one vector per step)."""
    if _nrhs(evecs, g.vh, "evecs") != n_ev:
        raise ValueError("evecs must hold n_ev vectors")
    p = EigParams(n_kr=int(n_kr), cheb_degree=int(cheb_degree), cheb_a=float(cheb_a),
                  cheb_b=float(cheb_b), tol=float(tol), max_restarts=int(max_restarts),
                  seed=int(seed), evec_prec=_prec_of(evecs, "evecs"), block=int(block))
    cb = None
    if progress is not None:
        cb = EIG_PROGRESS(lambda _u, r, j, mv, sec: progress(r, j, mv, sec))
        p.progress = cb
    evals = np.zeros(n_ev, dtype=np.float64)
    stats = EigStats()
    st = lib().hisq_eigensolve(_h(g), float(two_m), int(n_ev), ctypes.byref(p),
                               _ptr(evecs, "evecs", ("complex128", "complex64")),
                               evals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(stats), _stream(stream))
    del cb  # kept alive across the call above
    if raise_on_fail:
        _check(st, "hisq_eigensolve")
    return st, evals, stats


def hisq_autotune_dslash(g, nrhs, prec=HISQ_FP64, reps=0, stream=None) -> TuneResult:
    """Time every half-stencil launch shape for this volume, nrhs and precision
    and keep the fastest for later launches of that size."""
    r = TuneResult()
    _check(lib().hisq_autotune_dslash(_h(g), int(nrhs), int(prec), int(reps), ctypes.byref(r),
                                      _stream(stream)), "hisq_autotune_dslash")
    return r


# ------------------------------------------------------- learned guess
def _params_f32(params):
    if params is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
    if a.size != HISQ_NN_PARAMS:
        raise ValueError(f"network parameters must have {HISQ_NN_PARAMS} entries, got {a.size}")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Network:
    """Owns a hisq_nn handle (the learned initial guess) on a gauge handle."""

    def __init__(self, g, params=None):
        self.gauge = g
        self.handle = hisq_nn_create(g, params)

    def close(self):
        if self.handle:
            hisq_nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _nn(n):
    return n.handle if isinstance(n, Network) else n


def hisq_nn_create(g, params=None):
    a, ptr = _params_f32(params)
    h = ctypes.c_void_p()
    _check(lib().hisq_nn_create(ctypes.byref(h), _h(g), ptr), "hisq_nn_create")
    return h


def hisq_nn_destroy(n):
    _check(lib().hisq_nn_destroy(_nn(n)), "hisq_nn_destroy")


def hisq_nn_set_params(n, params):
    a, ptr = _params_f32(params)
    _check(lib().hisq_nn_set_params(_nn(n), ptr), "hisq_nn_set_params")


def hisq_nn_get_params(n):
    out = np.zeros(HISQ_NN_PARAMS, dtype=np.float32)
    _check(lib().hisq_nn_get_params(_nn(n), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
           "hisq_nn_get_params")
    return out


def _nn_vh(n):
    g = n.gauge if isinstance(n, Network) else None
    return g.vh if isinstance(g, Gauge) else None


def _samples(n, t, name):
    vh = _nn_vh(n)
    if vh is not None:
        return _nrhs(t, vh, name)
    return int(t.shape[0])


def hisq_nn_apply(n, r, out, flags=HISQ_NN_NORMALIZE, stream=None):
    S = _samples(n, r, "r")
    if tuple(out.shape) != tuple(r.shape):
        raise ValueError("out must have the shape of r")
    _check(lib().hisq_nn_apply(_nn(n), _ptr(r, "r"), _ptr(out, "out"), S, int(flags),
                               _stream(stream)), "hisq_nn_apply")


def hisq_nn_loss_grad(n, r, e, flags=HISQ_NN_NORMALIZE, stream=None):
    """(loss, gradient as float64 numpy [752]) of the batch (r, e)."""
    S = _samples(n, r, "r")
    if tuple(e.shape) != tuple(r.shape):
        raise ValueError("e must have the shape of r")
    loss = ctypes.c_double()
    grad = np.zeros(HISQ_NN_PARAMS, dtype=np.float64)
    _check(lib().hisq_nn_loss_grad(_nn(n), _ptr(r, "r"), _ptr(e, "e"), S, int(flags),
                                   ctypes.byref(loss),
                                   grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   _stream(stream)), "hisq_nn_loss_grad")
    return float(loss.value), grad


def hisq_nn_adam_step(n, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().hisq_nn_adam_step(_nn(n), float(lr), float(beta1), float(beta2), float(eps),
                                   _stream(stream)), "hisq_nn_adam_step")


def hisq_nn_train(n, r, e, batch, steps, lr, flags=HISQ_NN_NORMALIZE, stream=None):
    """Adam training over the pairs (r, e); returns the per-step losses."""
    S = _samples(n, r, "r")
    if tuple(e.shape) != tuple(r.shape):
        raise ValueError("e must have the shape of r")
    losses = np.zeros(max(int(steps), 1), dtype=np.float64)
    _check(lib().hisq_nn_train(_nn(n), _ptr(r, "r"), _ptr(e, "e"), S, int(batch), int(steps),
                               float(lr), int(flags),
                               losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               _stream(stream)), "hisq_nn_train")
    return losses[:int(steps)]


def hisq_nn_guess(n, two_m, b, x, flags=HISQ_NN_NORMALIZE, evecs=None, evals=None,
                  stream=None):
    """x += N(b - A x) per RHS where that lowers the residual, projected off the
    deflation space first when evecs (complex128/complex64) and evals (eps_i)
    are given; returns the kept flags."""
    S = _samples(n, b, "b")
    if tuple(x.shape) != tuple(b.shape):
        raise ValueError("x must have the shape of b")
    kept = (ctypes.c_int * S)()
    n_ev, ev_ptr, prec, ev_host = 0, None, HISQ_FP64, None
    if evecs is not None:
        n_ev = int(evecs.shape[0])
        ev_ptr = _ptr(evecs, "evecs", ("complex128", "complex64"))
        prec = _prec_of(evecs, "evecs")
        ev_host = np.ascontiguousarray(np.asarray(evals, dtype=np.float64))
        if ev_host.shape != (n_ev,):
            raise ValueError("evals must have one entry per eigenvector")
    _check(lib().hisq_nn_guess(_nn(n), _scalar_mass(two_m), _ptr(b, "b"), _ptr(x, "x"), S,
                               int(flags), n_ev, ev_ptr, prec,
                               None if ev_host is None
                               else ev_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               kept, _stream(stream)), "hisq_nn_guess")
    return [int(k) for k in kept]


def hisq_set_tuning(key: str, value: int):
    _check(lib().hisq_set_tuning(key.encode(), int(value)), "hisq_set_tuning")


def hisq_profile_enable(on, period: int = 1):
    """Time launches per kernel class: off if not on, else every period-th launch."""
    _check(lib().hisq_profile_enable(int(period) if on else 0), "hisq_profile_enable")


def hisq_profile_read(kernel_class: str):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib().hisq_profile_read(kernel_class.encode(), ctypes.byref(n), ctypes.byref(ms)),
           "hisq_profile_read")
    return int(n.value), float(ms.value)
