"""ctypes binding of liblq (include/lq.h): argument marshalling only.

Every operator and solver runs in the HIP library; this module converts
numpy arrays / torch tensors to pointers and back.  Host arrays (numpy,
complex128, canonical layout) go through the host-pointer entry points;
torch CUDA tensors (complex128 or float64 views, canonical layout) go through
the `_dev` entry points on the tensor's current stream.  If liblq.so is not
built, importing works but every call raises (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LQ_LIB selects another build of the same library (e.g. a layout variant)
LIB_PATH = os.environ.get("LQ_LIB", os.path.join(HERE, "liblq.so"))

LQ_OK, LQ_EINVAL, LQ_ENOMEM, LQ_EDEVICE, LQ_ENOCONV, LQ_EBREAKDOWN, LQ_ENUMERIC, LQ_EBUSY, LQ_ENOTSUP = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
LQ_WILSON, LQ_TM_CLOVER, LQ_HISQ, LQ_OVERLAP = 0, 1, 2, 3
LQ_PREC_RECON12 = 0x100
LQ_MAX_COLUMNS = 65535
(LQ_OP_D, LQ_OP_DDAG, LQ_OP_HOP, LQ_OP_SITE, LQ_OP_SITE_INV, LQ_OP_SCHUR, LQ_OP_HW, LQ_OP_SIGN,
 LQ_OP_NORMAL_EVEN) = range(9)

EXPORTS = [
    "lq_init", "lq_finalize", "lq_last_error", "lq_version", "lq_gauge_load", "lq_gauge_load_dev",
    "lq_hisq_load", "lq_hisq_load_dev", "lq_field_free", "lq_apply", "lq_apply_dev", "lq_apply_noalloc", "lq_solve",
    "lq_solve_dev", "lq_eigs", "lq_mg_setup", "lq_mg_apply", "lq_hw_bounds", "lq_cheb_coeffs", "lq_copy_bandwidth", "lq_profile", "lq_profile_get",
    "lq_profile_bytes",
    "lq_server_create", "lq_server_destroy", "lq_submit", "lq_poll", "lq_wait", "lq_server_stats",
]


class LqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblq error {code}: {msg}")
        self.code = code


class lq_geom(C.Structure):
    _fields_ = [("L", C.c_int32 * 4), ("t_antiperiodic", C.c_int32)]


class lq_action(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_double), ("mu", C.c_double), ("c_sw", C.c_double),
                ("rho", C.c_double), ("cheb_N", C.c_int32), ("cheb_a", C.c_double), ("cheb_b", C.c_double),
                ("cheb_c", C.POINTER(C.c_double)), ("n_lowmodes", C.c_int32)]


class lq_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int32), ("sloppy_bits", C.c_int32),
                ("reliable_delta", C.c_double), ("n_shift", C.c_int32), ("masses", C.POINTER(C.c_double)),
                ("reconstruct_full", C.c_int32), ("recon12", C.c_int32), ("use_initial_guess", C.c_int32),
                ("fault_inject", C.c_int32), ("solver", C.c_int32), ("deflate", C.c_int32)]


class lq_mg_params(C.Structure):
    _fields_ = [("block", C.c_int32 * 4), ("n_vec", C.c_int32), ("setup_passes", C.c_int32),
                ("setup_maxiter", C.c_int32), ("coarse_maxiter", C.c_int32), ("setup_tol", C.c_double),
                ("coarse_tol", C.c_double), ("seed", C.c_uint64), ("null_vecs", C.POINTER(C.c_double)),
                ("nu_post", C.c_int32), ("gcr_kmax", C.c_int32), ("nu_pre", C.c_int32),
                ("reserved", C.c_int32)]


class lq_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("reliable_updates", C.c_int32), ("true_rel_res", C.c_double),
                ("seconds", C.c_double), ("gflops", C.c_double), ("hbm_bytes", C.c_double),
                ("status", C.c_int32), ("n_apply", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib_available() -> bool:
    return os.path.exists(LIB_PATH)


def load():
    """Load liblq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2201_09004_amd.build` "
                           "(the HIP library is required; there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    sig = {
        "lq_init": ([C.c_int, C.POINTER(P)], C.c_int),
        "lq_finalize": ([P], C.c_int),
        "lq_last_error": ([], C.c_char_p),
        "lq_version": ([], C.c_char_p),
        "lq_gauge_load": ([P, C.POINTER(lq_geom), P, C.POINTER(P)], C.c_int),
        "lq_gauge_load_dev": ([P, C.POINTER(lq_geom), P, P, C.POINTER(P)], C.c_int),
        "lq_hisq_load": ([P, C.POINTER(lq_geom), P, P, C.POINTER(P)], C.c_int),
        "lq_hisq_load_dev": ([P, C.POINTER(lq_geom), P, P, P, C.POINTER(P)], C.c_int),
        "lq_field_free": ([P], C.c_int),
        "lq_apply": ([P, C.POINTER(lq_action), P, C.c_int, C.c_int, C.c_int, P, P], C.c_int),
        "lq_apply_dev": ([P, C.POINTER(lq_action), P, C.c_int, C.c_int, C.c_int, P, P, P], C.c_int),
        "lq_apply_noalloc": ([P, C.POINTER(lq_action), P, C.c_int, C.c_int, C.c_int, P, P, P], C.c_int),
        "lq_solve": ([P, C.POINTER(lq_action), P, C.POINTER(lq_params), C.c_int, P, P, C.POINTER(lq_stats)],
                     C.c_int),
        "lq_solve_dev": ([P, C.POINTER(lq_action), P, C.POINTER(lq_params), C.c_int, P, P, C.POINTER(lq_stats),
                          P], C.c_int),
        "lq_hw_bounds": ([P, C.POINTER(lq_action), P, C.c_int, D, D], C.c_int),
        "lq_eigs": ([P, C.POINTER(lq_action), P, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_double, D,
                     C.POINTER(lq_stats)], C.c_int),
        "lq_mg_setup": ([P, C.POINTER(lq_action), P, C.POINTER(lq_mg_params), C.POINTER(lq_stats)], C.c_int),
        "lq_mg_apply": ([P, C.POINTER(lq_action), P, C.c_int, C.c_int, C.c_int, P, P], C.c_int),
        "lq_cheb_coeffs": ([C.c_double, C.c_double, C.c_int, D], C.c_int),
        "lq_copy_bandwidth": ([P, C.c_size_t, C.c_int, D], C.c_int),
        "lq_profile": ([P, C.c_int], C.c_int),
        "lq_profile_get": ([P, C.c_char_p, C.POINTER(C.c_int64), D], C.c_int),
        "lq_profile_bytes": ([P, C.c_char_p, D], C.c_int),
        "lq_server_create": ([P, C.c_size_t, C.c_int, C.POINTER(P)], C.c_int),
        "lq_server_destroy": ([P], C.c_int),
        "lq_submit": ([P, C.POINTER(lq_action), P, C.POINTER(lq_params), C.c_int, P, P, C.POINTER(lq_stats),
                       C.POINTER(C.c_uint64)], C.c_int),
        "lq_poll": ([P, C.c_uint64, C.POINTER(C.c_int)], C.c_int),
        "lq_wait": ([P, C.c_uint64], C.c_int),
        "lq_server_stats": ([P, D, D, D], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(code, ok=(LQ_OK,)):
    if code not in ok:
        raise LqError(code, load().lq_last_error().decode())
    return code


def last_error() -> str:
    return load().lq_last_error().decode()


# ------------------------------------------------------------------ marshalling helpers
def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """Pointer of a C-contiguous complex128 numpy array or CUDA torch tensor."""
    if a is None:
        return None
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(a.data_ptr())
    if not (isinstance(a, np.ndarray) and a.dtype == np.complex128 and a.flags.c_contiguous):
        raise ValueError("host arrays must be C-contiguous complex128")
    return C.c_void_p(a.ctypes.data)


def _stream_of(t):
    import torch
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def geom(L, antiperiodic=True):
    g = lq_geom()
    for k in range(4):
        g.L[k] = int(L[k])
    g.t_antiperiodic = 1 if antiperiodic else 0
    return g


def action(kind, m=0.0, mu=0.0, c_sw=0.0, rho=0.0, cheb_N=0, cheb_a=0.0, cheb_b=0.0, cheb_c=None, n_lowmodes=0):
    a = lq_action(kind=kind, m=m, mu=mu, c_sw=c_sw, rho=rho, cheb_N=cheb_N, cheb_a=cheb_a, cheb_b=cheb_b,
                  n_lowmodes=n_lowmodes)
    if cheb_c is not None:
        arr = np.ascontiguousarray(cheb_c, dtype=np.float64)
        a._keep = arr
        a.cheb_c = arr.ctypes.data_as(C.POINTER(C.c_double))
    return a


def params(tol=1e-10, maxiter=0, sloppy_bits=64, reliable_delta=0.0, masses=None, reconstruct_full=0,
           recon12=0, use_initial_guess=0, fault_inject=0, solver=0, deflate=0):
    p = lq_params(tol=tol, maxiter=maxiter, sloppy_bits=sloppy_bits, reliable_delta=reliable_delta,
                  reconstruct_full=reconstruct_full, recon12=recon12, use_initial_guess=use_initial_guess,
                  fault_inject=fault_inject, solver=solver, deflate=deflate)
    if masses is not None:
        arr = np.ascontiguousarray(masses, dtype=np.float64)
        p._keep = arr
        p.n_shift = len(arr)
        p.masses = arr.ctypes.data_as(C.POINTER(C.c_double))
    return p


# ------------------------------------------------------------------ C-ABI twins
def lq_init(device=0):
    h = C.c_void_p()
    _check(load().lq_init(device, C.byref(h)))
    return h


def lq_finalize(ctx):
    _check(load().lq_finalize(ctx))


def lq_version():
    return load().lq_version().decode()


def lq_gauge_load(ctx, L, U, antiperiodic=True):
    g = geom(L, antiperiodic)
    h = C.c_void_p()
    if _is_torch(U):
        _check(load().lq_gauge_load_dev(ctx, C.byref(g), _ptr(U), _stream_of(U), C.byref(h)))
    else:
        _check(load().lq_gauge_load(ctx, C.byref(g), _ptr(np.ascontiguousarray(U)), C.byref(h)))
    return h


def lq_hisq_load(ctx, L, fat, lng, antiperiodic=True):
    g = geom(L, antiperiodic)
    h = C.c_void_p()
    if _is_torch(fat):
        _check(load().lq_hisq_load_dev(ctx, C.byref(g), _ptr(fat), _ptr(lng), _stream_of(fat), C.byref(h)))
    else:
        _check(load().lq_hisq_load(ctx, C.byref(g), _ptr(np.ascontiguousarray(fat)),
                                   _ptr(np.ascontiguousarray(lng)), C.byref(h)))
    return h


def lq_field_free(field):
    _check(load().lq_field_free(field))


def lq_apply(ctx, act, field, op, prec_bits, inp, out=None):
    """Apply op once to the leading-dimension columns of `inp` (numpy or CUDA tensor)."""
    n_rhs = inp.shape[0]
    if _is_torch(inp):
        import torch
        out = torch.empty_like(inp) if out is None else out
        _check(load().lq_apply_dev(ctx, C.byref(act), field, op, prec_bits, n_rhs, _ptr(inp), _ptr(out),
                                   _stream_of(inp)))
        return out
    inp = np.ascontiguousarray(inp)
    out = np.empty_like(inp) if out is None else out
    _check(load().lq_apply(ctx, C.byref(act), field, op, prec_bits, n_rhs, _ptr(inp), _ptr(out)))
    return out


def lq_apply_noalloc(ctx, act, field, op, prec_bits, inp, out):
    """lq_apply_noalloc on CUDA tensors `inp` and `out` (same shape); enqueued
    on the current stream of `inp`'s device, not synchronised."""
    _check(load().lq_apply_noalloc(ctx, C.byref(act), field, op, prec_bits, inp.shape[0], _ptr(inp), _ptr(out),
                                   _stream_of(inp)))
    return out


def lq_solve(ctx, act, field, prm, b, x=None):
    """Solve D x = b for the columns of b; returns (x, stats dict).

    For HISQ or overlap with several masses x has a leading n_shift axis.  A non-converged
    solve (LQ_ENOCONV) still returns x and stats with stats['status'] set.
    """
    n_rhs = b.shape[0]
    nsh = prm.n_shift if prm.n_shift > 1 else 1
    shape = ((nsh,) if nsh > 1 else ()) + tuple(b.shape)
    st = lq_stats()
    if _is_torch(b):
        import torch
        if x is None:
            x = torch.zeros(shape, dtype=b.dtype, device=b.device)
        code = load().lq_solve_dev(ctx, C.byref(act), field, C.byref(prm), n_rhs, _ptr(b), _ptr(x), C.byref(st),
                                   _stream_of(b))
    else:
        b = np.ascontiguousarray(b)
        if x is None:
            x = np.zeros(shape, dtype=np.complex128)
        code = load().lq_solve(ctx, C.byref(act), field, C.byref(prm), n_rhs, _ptr(b), _ptr(x), C.byref(st))
    _check(code, ok=(LQ_OK, LQ_ENOCONV))
    return x, st.as_dict()


LQ_EIG_HW, LQ_EIG_OVERLAP = 0, 1


def lq_eigs(ctx, act, field, which, nev, tol=1e-10, max_restarts=0, filter_degree=0, filter_cut=0.0):
    """Low modes kept resident with the field; returns (eigenvalues, stats dict).
    LQ_ENOCONV (modes stored, a residual above tol) is returned in stats['status']."""
    n = nev * (2 if which == LQ_EIG_OVERLAP else 1)
    ev = np.zeros(n)
    st = lq_stats()
    code = load().lq_eigs(ctx, C.byref(act), field, which, nev, tol, max_restarts, filter_degree, filter_cut,
                          ev.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st))
    _check(code, ok=(LQ_OK, LQ_ENOCONV))
    return ev, st.as_dict()


LQ_MG_RESTRICT, LQ_MG_PROLONG, LQ_MG_COARSE = 0, 1, 2


def mg_params(block=(4, 4, 4, 4), n_vec=30, setup_passes=0, setup_maxiter=0, setup_tol=0.0, coarse_tol=0.0,
              coarse_maxiter=0, nu_post=0, gcr_kmax=0, seed=1, null_vecs=None, nu_pre=0):
    p = lq_mg_params(n_vec=n_vec, setup_passes=setup_passes, setup_maxiter=setup_maxiter,
                     coarse_maxiter=coarse_maxiter, setup_tol=setup_tol, coarse_tol=coarse_tol, seed=seed,
                     nu_post=nu_post, gcr_kmax=gcr_kmax, nu_pre=nu_pre)
    p.block[:] = list(block)
    if null_vecs is not None:
        arr = np.ascontiguousarray(null_vecs, dtype=np.complex128)
        p._keep = arr
        p.null_vecs = arr.ctypes.data_as(C.POINTER(C.c_double))
    return p


def lq_mg_setup(ctx, act, field, mp):
    """Multigrid hierarchy for (field, act), kept with the field; returns the stats dict."""
    st = lq_stats()
    _check(load().lq_mg_setup(ctx, C.byref(act), field, C.byref(mp), C.byref(st)))
    return st.as_dict()


def lq_mg_apply(ctx, act, field, op, prec_bits, inp, out_shape):
    """Restriction, prolongation or coarse operator of the stored hierarchy on host arrays."""
    inp = np.ascontiguousarray(inp, dtype=np.complex128)
    out = np.zeros(out_shape, dtype=np.complex128)
    _check(load().lq_mg_apply(ctx, C.byref(act), field, op, prec_bits, inp.shape[0], _ptr(inp), _ptr(out)))
    return out


def lq_hw_bounds(ctx, act, field, iters=200):
    lo, hi = C.c_double(), C.c_double()
    _check(load().lq_hw_bounds(ctx, C.byref(act), field, iters, C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def lq_cheb_coeffs(a, b, N):
    c = np.zeros(N + 1)
    _check(load().lq_cheb_coeffs(a, b, N, c.ctypes.data_as(C.POINTER(C.c_double))))
    return c


def lq_copy_bandwidth(ctx, nbytes, reps=20):
    g = C.c_double()
    _check(load().lq_copy_bandwidth(ctx, C.c_size_t(int(nbytes)), reps, C.byref(g)))
    return g.value


def lq_profile(ctx, enable=True):
    _check(load().lq_profile(ctx, 1 if enable else 0))


def lq_profile_get(ctx, name):
    n, ms = C.c_int64(), C.c_double()
    _check(load().lq_profile_get(ctx, name.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def lq_profile_bytes(ctx, name):
    b = C.c_double()
    _check(load().lq_profile_bytes(ctx, name.encode(), C.byref(b)))
    return b.value


def lq_server_create(ctx, hbm_budget, max_cols):
    h = C.c_void_p()
    _check(load().lq_server_create(ctx, C.c_size_t(int(hbm_budget)), max_cols, C.byref(h)))
    return h


def lq_server_destroy(srv):
    _check(load().lq_server_destroy(srv))


def lq_submit(srv, act, field, prm, b, x, stats=None):
    """Queue a solve; b, x: host complex128 arrays kept alive by the caller until done."""
    t = C.c_uint64()
    st = stats if stats is not None else None
    _check(load().lq_submit(srv, C.byref(act), field, C.byref(prm), b.shape[0], _ptr(b), _ptr(x),
                            C.byref(st) if st is not None else None, C.byref(t)))
    return t.value


def lq_poll(srv, ticket):
    d = C.c_int()
    _check(load().lq_poll(srv, ticket, C.byref(d)))
    return bool(d.value)


def lq_wait(srv, ticket):
    return _check(load().lq_wait(srv, ticket), ok=(LQ_OK, LQ_ENOCONV))


def lq_server_stats(srv):
    p50, p99, sps = C.c_double(), C.c_double(), C.c_double()
    _check(load().lq_server_stats(srv, C.byref(p50), C.byref(p99), C.byref(sps)))
    return p50.value, p99.value, sps.value
