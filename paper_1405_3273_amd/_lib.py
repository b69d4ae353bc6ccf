"""ctypes binding of libgf2 (the C ABI declared in include/gf2.h).

Argument marshalling only: every step runs in the HIP library.  Device
arrays are passed as torch tensors (their data pointers); torch is used for
device memory and the stream, nothing else.  Importing this module does not
load the library; the first call does, and raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgf2.so")
_lib = None

GF2_OK = 0
GF2_EINVAL = -1
GF2_EHIP = -2
GF2_ENOMEM = -3
GF2_ENOCONV = -4
GF2_EBRACKET = -5
GF2_ENONFINITE = -6
GF2_ESTATE = -7

GF2_PREC_FP64 = 0
GF2_PREC_FP32 = 1
GF2_PREC_BF16X3 = 2
GF2_PREC_BF16X6 = 3
GF2_PREC_BF16MIX = 4
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "bf16mix": 4}

GF2_TAU2IW = 0
GF2_IW2TAU = 1

GF2_DYSON_TRACE = 0
GF2_DYSON_FULL = 1
GF2_DYSON_ENERGY = 2

GF2_MU_BISECT = 0
GF2_MU_ILLINOIS = 1
GF2_MU_SECANT = 2

EXPORTED = ("gf2_ctx_create", "gf2_ctx_destroy", "gf2_last_error", "gf2_set_system",
            "gf2_sigma_tau", "gf2_fourier", "gf2_dyson", "gf2_fock", "gf2_density_fock",
            "gf2_iterate", "gf2_iterate_batched", "gf2_natural_occupations", "gf2_set_tau_grid",
            "gf2_profile_enable", "gf2_profile_read", "gf2_dyson_noalloc",
            "gf2_set_df_factors", "gf2_sigma_tau_df")

GF2_KC_SIGMA_GEMM = 0
GF2_KC_SIGMA_SPLITK = 1
GF2_KC_DYSON = 2
GF2_KC_T2I_EXPAND = 3
GF2_KC_I2T_FOLD = 4
GF2_KC_FOCK = 5
GF2_KC_SIGMA_S23 = 6
GF2_KC_OCCUPATIONS = 7
GF2_KC_SIGMA_DF = 8
GF2_KC_COUNT = 9
KERNEL_CLASSES = ("sigma_gemm", "sigma_splitk", "dyson", "t2i_expand", "i2t_fold", "fock",
                  "sigma_s23", "occupations", "sigma_df")


class Gf2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libgf2 error {code}: {msg}")
        self.code = code


class gf2_dims(C.Structure):
    _fields_ = [("n", C.c_int), ("nelec", C.c_int), ("ntau", C.c_int), ("niw", C.c_int),
                ("beta", C.c_double)]


class gf2_params(C.Structure):
    _fields_ = [("tol_mu", C.c_double), ("tol_N", C.c_double), ("tol_P", C.c_double),
                ("tol_E", C.c_double), ("max_inner", C.c_int), ("max_bisect", C.c_int),
                ("mu_halfwidth", C.c_double), ("damp_P", C.c_double), ("mix_depth", C.c_int),
                ("damp_Sigma", C.c_double), ("mu_method", C.c_int), ("prec", C.c_int),
                ("tol_N_rel", C.c_double), ("sigma_df", C.c_int)]


class gf2_state(C.Structure):
    _fields_ = [("mu", C.c_double), ("F", C.c_void_p), ("P", C.c_void_p),
                ("G_tau", C.c_void_p), ("Sigma_tau", C.c_void_p), ("iteration", C.c_int),
                ("has_P", C.c_int), ("energy", C.c_double)]


class gf2_report(C.Structure):
    _fields_ = [("energy", C.c_double), ("e1b", C.c_double), ("e2b", C.c_double),
                ("dE", C.c_double), ("dP", C.c_double), ("mu", C.c_double),
                ("n_inner", C.c_int), ("n_eval", C.c_int), ("ms_sigma", C.c_double),
                ("ms_fourier", C.c_double), ("ms_inner", C.c_double), ("ms_total", C.c_double)]


def lib_path() -> str:
    return _LIB_PATH


def load(path: str = None):
    """Load libgf2.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libgf2.so not found at {p}; build it with "
                           "`python -m paper_1405_3273_amd.build`")
    L = C.CDLL(p)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    dp = C.POINTER(C.c_double)
    sig = {
        "gf2_ctx_create": ([C.POINTER(vp), i, vp], i),
        "gf2_ctx_destroy": ([vp], i),
        "gf2_last_error": ([], C.c_char_p),
        "gf2_set_system": ([vp, i, vp, vp, vp], i),
        "gf2_sigma_tau": ([vp, C.POINTER(gf2_dims), i, vp, vp], i),
        "gf2_set_df_factors": ([vp, i, vp], i),
        "gf2_sigma_tau_df": ([vp, C.POINTER(gf2_dims), i, vp, vp], i),
        "gf2_fourier": ([vp, C.POINTER(gf2_dims), i, vp, vp, vp, vp], i),
        "gf2_dyson": ([vp, C.POINTER(gf2_dims), i, d, vp, vp, vp, vp, vp, dp], i),
        "gf2_dyson_noalloc": ([vp, C.POINTER(gf2_dims), i, d, vp, vp, vp, vp, vp, dp], i),
        "gf2_fock": ([vp, vp, vp], i),
        "gf2_natural_occupations": ([vp, vp, vp], i),
        "gf2_set_tau_grid": ([vp, i, vp], i),
        "gf2_density_fock": ([vp, C.POINTER(gf2_dims), C.POINTER(gf2_params), vp, vp, vp, dp, vp,
                              vp, vp, dp], i),
        "gf2_iterate": ([vp, C.POINTER(gf2_dims), C.POINTER(gf2_params), C.POINTER(gf2_state),
                         C.POINTER(gf2_report)], i),
        "gf2_iterate_batched": ([C.POINTER(vp), i, C.POINTER(gf2_dims), C.POINTER(gf2_params),
                                 C.POINTER(gf2_state), C.POINTER(gf2_report)], i),
        "gf2_profile_enable": ([vp, i], i),
        "gf2_profile_read": ([vp, i, dp, C.POINTER(C.c_longlong), dp], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _lib = L
    return L


def _check(code: int):
    if code != GF2_OK:
        msg = load().gf2_last_error().decode(errors="replace")
        raise Gf2Error(code, msg)


def _ptr(t):
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libgf2 takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libgf2 takes contiguous tensors")
    return C.c_void_p(t.data_ptr())


def make_dims(n, nelec, ntau, niw, beta) -> gf2_dims:
    return gf2_dims(int(n), int(nelec), int(ntau), int(niw), float(beta))


def make_params(tol_mu=1e-12, tol_N=1e-10, tol_P=1e-10, tol_E=1e-11, max_inner=100,
                max_bisect=200, mu_halfwidth=0.5, damp_P=0.3, mix_depth=8, damp_Sigma=0.0,
                mu_method="secant", prec="fp32", tol_N_rel=0.0, sigma_df=False) -> gf2_params:
    mm = {"bisect": GF2_MU_BISECT, "illinois": GF2_MU_ILLINOIS, "secant": GF2_MU_SECANT}[mu_method]
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    return gf2_params(tol_mu, tol_N, tol_P, tol_E, max_inner, max_bisect, mu_halfwidth, damp_P,
                      mix_depth, damp_Sigma, mm, pr, float(tol_N_rel), 1 if sigma_df else 0)


# ---------------------------------------------------------------------------
# thin wrappers with the C names

def gf2_ctx_create(device: int = 0, stream=None):
    import torch
    L = load()
    h = C.c_void_p()
    s = stream if stream is not None else torch.cuda.current_stream(device).cuda_stream
    _check(L.gf2_ctx_create(C.byref(h), int(device), C.c_void_p(s)))
    return h


def gf2_ctx_destroy(ctx):
    _check(load().gf2_ctx_destroy(ctx))


def gf2_last_error() -> str:
    return load().gf2_last_error().decode(errors="replace")


def gf2_set_system(ctx, S, h, v):
    _check(load().gf2_set_system(ctx, int(S.shape[0]), _ptr(S), _ptr(h), _ptr(v)))


def gf2_sigma_tau(ctx, dims: gf2_dims, prec, G_tau, Sigma_tau):
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    _check(load().gf2_sigma_tau(ctx, C.byref(dims), pr, _ptr(G_tau), _ptr(Sigma_tau)))


def gf2_set_df_factors(ctx, B):
    """B: device [naux][n][n] FP64 density-fitting factors."""
    _check(load().gf2_set_df_factors(ctx, int(B.shape[0]), _ptr(B)))


def gf2_sigma_tau_df(ctx, dims: gf2_dims, prec, G_tau, Sigma_tau):
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    _check(load().gf2_sigma_tau_df(ctx, C.byref(dims), pr, _ptr(G_tau), _ptr(Sigma_tau)))


def gf2_fourier(ctx, dims: gf2_dims, direction, inp, moments, out, moment1_out=None):
    _check(load().gf2_fourier(ctx, C.byref(dims), int(direction), _ptr(inp), _ptr(moments),
                              _ptr(out), _ptr(moment1_out)))


def gf2_dyson(ctx, dims: gf2_dims, mode, mu, F, Sigma_iw=None, Sigma1=None, G_iw=None, P=None):
    out = (C.c_double * 2)()
    _check(load().gf2_dyson(ctx, C.byref(dims), int(mode), float(mu), _ptr(F), _ptr(Sigma_iw),
                            _ptr(Sigma1), _ptr(G_iw), _ptr(P), out))
    return out[0], out[1]


def gf2_dyson_noalloc(ctx, dims: gf2_dims, mode, mu, F, Sigma_iw=None, Sigma1=None, G_iw=None,
                      P=None):
    """gf2_dyson on the library's fixed per-GPU workspace (allocates nothing)."""
    out = (C.c_double * 2)()
    _check(load().gf2_dyson_noalloc(ctx, C.byref(dims), int(mode), float(mu), _ptr(F),
                                    _ptr(Sigma_iw), _ptr(Sigma1), _ptr(G_iw), _ptr(P), out))
    return out[0], out[1]


def gf2_fock(ctx, P, F):
    _check(load().gf2_fock(ctx, _ptr(P), _ptr(F)))


def gf2_natural_occupations(ctx, P, occ):
    _check(load().gf2_natural_occupations(ctx, _ptr(P), _ptr(occ)))


def gf2_set_tau_grid(ctx, tau):
    """tau: device FP64 tensor of grid points, or None for the uniform grid."""
    _check(load().gf2_set_tau_grid(ctx, 0 if tau is None else int(tau.numel()), _ptr(tau)))


def gf2_density_fock(ctx, dims: gf2_dims, params: gf2_params, F_in, Sigma_iw, Sigma1, mu,
                     P_out, F_out=None, G_iw_out=None):
    m = C.c_double(mu)
    out = (C.c_double * 4)()
    _check(load().gf2_density_fock(ctx, C.byref(dims), C.byref(params), _ptr(F_in),
                                   _ptr(Sigma_iw), _ptr(Sigma1), C.byref(m), _ptr(P_out),
                                   _ptr(F_out), _ptr(G_iw_out), out))
    return m.value, {"trPS": out[0], "e1b": out[1], "e2b": out[2], "n_eval": int(out[3])}


def gf2_iterate(ctx, dims: gf2_dims, params: gf2_params, state: gf2_state) -> gf2_report:
    rep = gf2_report()
    _check(load().gf2_iterate(ctx, C.byref(dims), C.byref(params), C.byref(state), C.byref(rep)))
    return rep


def gf2_iterate_batched(ctxs, dims, params: gf2_params, states):
    """ctxs, dims, states: sequences of equal length; states are updated in place."""
    n = len(ctxs)
    if not (len(dims) == len(states) == n):
        raise ValueError("gf2_iterate_batched: ctxs, dims and states differ in length")
    c_arr = (C.c_void_p * n)(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    d_arr = (gf2_dims * n)(*dims)
    s_arr = (gf2_state * n)(*states)
    r_arr = (gf2_report * n)()
    code = load().gf2_iterate_batched(c_arr, n, d_arr, C.byref(params), s_arr, r_arr)
    for k in range(n):   # copy the updated states back
        C.memmove(C.addressof(states[k]), C.addressof(s_arr[k]), C.sizeof(gf2_state))
    _check(code)
    return [r_arr[k] for k in range(n)]


def gf2_profile_enable(ctx, on: bool = True):
    _check(load().gf2_profile_enable(ctx, 1 if on else 0))


def gf2_profile_read(ctx) -> dict:
    """{class name: (total ms, launches, total work)} for every kernel class."""
    n = GF2_KC_COUNT
    ms = (C.c_double * n)()
    cnt = (C.c_longlong * n)()
    work = (C.c_double * n)()
    _check(load().gf2_profile_read(ctx, n, ms, cnt, work))
    return {KERNEL_CLASSES[k]: (ms[k], int(cnt[k]), work[k]) for k in range(n)}
