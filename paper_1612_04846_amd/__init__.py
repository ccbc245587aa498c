"""Python binding of libbura.so: argument marshalling only.

Every step of the solve runs in the HIP library (see include/bura.h).  The
functions below carry the C names; device buffers are torch CUDA tensors
(float64, contiguous) whose data pointers are handed to the library, and the
current torch stream is used unless another is given.  If the library has not
been built this module raises on import -- there is no fallback path.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbura.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bura.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libbura.so is not built: run `python paper_1612_04846_amd/build.py` "
        "(hipcc --offload-arch=gfx950) first"
    )

_lib = ctypes.CDLL(LIB_PATH)

BURA_OK = 0
BURA_PENDING = 1
BURA_EINVAL = -1
BURA_EUNSUPPORTED = -2
BURA_EREMEZ = -3
BURA_ENOCONV = -4
BURA_ENOMEM = -5
BURA_EDEVICE = -6
BURA_ENAN = -7
BURA_EBUSY = -8
BURA_ETOOBIG = -9
BURA_STATIC_SCRATCH_BYTES = 64 << 20
BURA_FP64 = 0
BURA_MIXED = 1
BURA_BATCHED = 0
BURA_PER_POLE = 1
BURA_MAX_TERMS = 64
BURA_TILE_VARIANTS = 5
# bura_opts_t.variant bits: alternative code paths of the same steps
BURA_VARIANT_UNFUSED = 1
BURA_VARIANT_NO_FOLDXR = 2
BURA_VARIANT_FOLD_SCALARS = 4
BURA_VARIANT_NO_GRAPH = 8


class bura_grid_t(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int),
        ("coeff", ctypes.POINTER(ctypes.c_double)),
        ("lambda_upper", ctypes.c_double),
        ("rhs_unscaled", ctypes.c_int),
    ]


class bura_opts_t(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("schedule", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("max_outer", ctypes.c_int),
        ("nrhs_max", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("nu_pre", ctypes.c_int),
        ("nu_post", ctypes.c_int),
        ("omega", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("hbm_budget", ctypes.c_size_t),
        ("autotune", ctypes.c_int),
        ("err_tol", ctypes.c_double),
        ("variant", ctypes.c_int),
    ]


class bura_report_t(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("nterms", ctypes.c_int),
        ("E", ctypes.c_double),
        ("iters", ctypes.c_int * BURA_MAX_TERMS),
        ("outer", ctypes.c_int * BURA_MAX_TERMS),
        ("relres", ctypes.c_double * BURA_MAX_TERMS),
        ("seconds", ctypes.c_double),
        ("err_bound", ctypes.c_double),
    ]


class bura_request_t(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int),
        ("alpha", ctypes.c_double),
        ("k", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("precision", ctypes.c_int),
    ]


class bura_server_stats_t(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_longlong),
        ("completed", ctypes.c_longlong),
        ("failed", ctypes.c_longlong),
        ("batches", ctypes.c_longlong),
        ("plans_created", ctypes.c_longlong),
        ("plans_evicted", ctypes.c_longlong),
        ("unknown_pole_solves", ctypes.c_double),
        ("p50_latency_s", ctypes.c_double),
        ("p99_latency_s", ctypes.c_double),
        ("mean_batch", ctypes.c_double),
        ("resident_bytes", ctypes.c_size_t),
        ("joined_running", ctypes.c_longlong),
    ]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_DP = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "bura_opts_default": (_I, [ctypes.POINTER(bura_opts_t)]),
    "bura_coefficients": (_I, [_D, _I, _I, _DP, _DP, _DP]),
    "bura_plan_create": (_I, [ctypes.POINTER(bura_grid_t), _D, _I, _I, ctypes.POINTER(bura_opts_t), ctypes.POINTER(_P)]),
    "bura_plan_create_rational": (_I, [ctypes.POINTER(bura_grid_t), _I, _DP, _DP, ctypes.POINTER(bura_opts_t),
                                       ctypes.POINTER(_P)]),
    "bura_plan_create_multi": (_I, [ctypes.POINTER(bura_grid_t), _I, _DP, _I, ctypes.POINTER(_I),
                                    ctypes.POINTER(bura_opts_t), ctypes.POINTER(_P)]),
    "bura_plan_create_rational_multi": (_I, [ctypes.POINTER(bura_grid_t), _I, ctypes.POINTER(_I), _DP, _DP,
                                             ctypes.POINTER(bura_opts_t), ctypes.POINTER(_P)]),
    "bura_sinc_coefficients": (_I, [_D, _D, _D, _I, _DP, _DP, ctypes.POINTER(_I)]),
    "bura_sinc_kprime": (_I, [_D, _D, _DP]),
    "bura_zeros": (_I, [_D, _I, _I, _DP, _DP]),
    "bura_plan_create_multistep": (_I, [ctypes.POINTER(bura_grid_t), _I, _DP, ctypes.POINTER(_I),
                                        ctypes.POINTER(bura_opts_t), ctypes.POINTER(_P)]),
    "bura_plan_create_product": (_I, [ctypes.POINTER(bura_grid_t), _D, _I, _I, ctypes.POINTER(bura_opts_t),
                                      ctypes.POINTER(_P)]),
    "bura_plan_create_sinc": (_I, [ctypes.POINTER(bura_grid_t), _I, _DP, _DP, ctypes.POINTER(bura_opts_t),
                                   ctypes.POINTER(_P)]),
    "bura_plan_create_slots": (_I, [ctypes.POINTER(bura_grid_t), _I, ctypes.POINTER(bura_opts_t), ctypes.POINTER(_P)]),
    "bura_solve_slots": (_I, [_P, _P, _P, _I, ctypes.POINTER(_I), _DP, _DP, _DP, ctypes.POINTER(bura_report_t)]),
    "bura_submit_slots": (_I, [_P, _P, _P, _I, ctypes.POINTER(_I), _DP, _DP, _DP, ctypes.POINTER(ctypes.c_uint64)]),
    "bura_plan_outputs": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "bura_solve": (_I, [_P, _P, _P, _I, ctypes.POINTER(bura_report_t)]),
    "bura_submit": (_I, [_P, _P, _P, _I, _D, ctypes.POINTER(ctypes.c_uint64)]),
    "bura_poll": (_I, [ctypes.c_uint64, ctypes.POINTER(bura_report_t)]),
    "bura_wait": (_I, [ctypes.c_uint64, ctypes.POINTER(bura_report_t)]),
    "bura_plan_coeffs": (_I, [_P, ctypes.POINTER(_I), _DP, _DP, _DP]),
    "bura_plan_info": (_I, [_P, _DP, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_size_t)]),
    "bura_plan_apply": (_I, [_P, _D, _P, _P, _I]),
    "bura_plan_profile": (_I, [_P, _I]),
    "bura_plan_kernel_stats": (_I, [_P, _I, ctypes.POINTER(ctypes.c_longlong), _DP, _DP]),
    "bura_plan_tiles": (_I, [_P, ctypes.POINTER(_I), _I, ctypes.POINTER(_I)]),
    "bura_plan_set_tiles": (_I, [_P, ctypes.POINTER(_I), _I]),
    "bura_plan_destroy": (None, [_P]),
    "bura_solve_static": (_I, [ctypes.POINTER(bura_grid_t), _I, _DP, _DP, ctypes.POINTER(bura_opts_t), _P, _P, _I,
                               ctypes.POINTER(bura_report_t)]),
    "bura_strerror": (ctypes.c_char_p, [_I]),
    "bura_device_copy": (_I, [_P, _P, ctypes.c_size_t, _P]),
    "bura_server_create": (_I, [ctypes.c_size_t, _I, _I, ctypes.POINTER(_P)]),
    "bura_server_submit": (_I, [_P, ctypes.POINTER(bura_request_t), _P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "bura_server_poll": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(bura_report_t)]),
    "bura_server_wait": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(bura_report_t)]),
    "bura_server_stats": (_I, [_P, ctypes.POINTER(bura_server_stats_t)]),
    "bura_server_reset_latency": (_I, [_P]),
    "bura_server_destroy": (None, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class BuraError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {bura_strerror(code)} ({code})")


def bura_strerror(code: int) -> str:
    return _lib.bura_strerror(code).decode()


def _check(code: int, where: str, ok=(BURA_OK,)):
    if code not in ok:
        raise BuraError(code, where)
    return code


def exported_symbols():
    """Names of the functions declared in include/bura.h that the library exports."""
    return {n for n in _SIGS if hasattr(_lib, n)}


# --------------------------------------------------------------------------
# thin wrappers with the C names
# --------------------------------------------------------------------------

def bura_opts_default(**overrides) -> bura_opts_t:
    o = bura_opts_t()
    _check(_lib.bura_opts_default(ctypes.byref(o)), "bura_opts_default")
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def bura_coefficients(alpha: float, k: int, beta: int = 1):
    """(c, d, E) of the (k,k) BURA of t^(1-alpha), computed by the library's host code.
    beta = 2: the (k+1,k) 2-BURA; c then has k+2 entries, c[k+1] = c_{0,2}."""
    c = (ctypes.c_double * (k + 2))()
    d = (ctypes.c_double * (k + 1))()
    E = ctypes.c_double()
    _check(_lib.bura_coefficients(alpha, beta, k, c, d, ctypes.byref(E)), "bura_coefficients")
    return list(c)[: k + 1 + (beta == 2)], list(d), E.value


def _grid(dim, n, coeff=None, lambda_upper=0.0, rhs_unscaled=0):
    g = bura_grid_t()
    g.dim = dim
    g.n = n
    g.rhs_unscaled = rhs_unscaled
    keep = None
    if coeff is not None:
        import numpy as np
        keep = np.ascontiguousarray(coeff, dtype=np.float64)
        if keep.size != (n + 2) ** dim:
            raise ValueError("coeff must hold (n+2)^dim nodal values")
        g.coeff = keep.ctypes.data_as(_DP)
    g.lambda_upper = lambda_upper
    return g, keep


def _stream_ptr(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def bura_plan_create(dim: int, n: int, alpha: float, k: int, opts: Optional[bura_opts_t] = None,
                     coeff=None, lambda_upper: float = 0.0, beta: int = 1, rhs_unscaled: int = 0):
    g, _keep = _grid(dim, n, coeff, lambda_upper, rhs_unscaled)
    o = opts if opts is not None else bura_opts_default()
    h = _P()
    _check(_lib.bura_plan_create(ctypes.byref(g), alpha, beta, k, ctypes.byref(o), ctypes.byref(h)),
           "bura_plan_create")
    return h


def bura_plan_create_multi(dim: int, n: int, alphas: Sequence[float], ks: Sequence[int],
                           opts: Optional[bura_opts_t] = None, coeff=None, lambda_upper: float = 0.0, beta: int = 1, rhs_unscaled: int = 0):
    g, _keep = _grid(dim, n, coeff, lambda_upper, rhs_unscaled)
    o = opts if opts is not None else bura_opts_default()
    m = len(alphas)
    a = (ctypes.c_double * m)(*alphas)
    k = (ctypes.c_int * m)(*ks)
    h = _P()
    _check(_lib.bura_plan_create_multi(ctypes.byref(g), m, a, beta, k, ctypes.byref(o), ctypes.byref(h)),
           "bura_plan_create_multi")
    return h


def bura_plan_outputs(plan):
    n = ctypes.c_int()
    tb = (ctypes.c_int * (BURA_MAX_TERMS + 1))()
    _check(_lib.bura_plan_outputs(plan, ctypes.byref(n), tb), "bura_plan_outputs")
    return n.value, list(tb)[: n.value + 1]


def bura_plan_create_rational(dim: int, n: int, weights: Sequence[float], shifts: Sequence[float],
                              opts: Optional[bura_opts_t] = None, coeff=None, lambda_upper: float = 0.0):
    g, _keep = _grid(dim, n, coeff, lambda_upper)
    o = opts if opts is not None else bura_opts_default()
    m = len(weights)
    w = (ctypes.c_double * m)(*weights)
    s = (ctypes.c_double * m)(*shifts)
    h = _P()
    _check(_lib.bura_plan_create_rational(ctypes.byref(g), m, w, s, ctypes.byref(o), ctypes.byref(h)),
           "bura_plan_create_rational")
    return h


def bura_solve_static(dim: int, n: int, weights: Sequence[float], shifts: Sequence[float], f: torch.Tensor,
                      u: torch.Tensor, opts: Optional[bura_opts_t] = None, coeff=None, lambda_upper: float = 0.0,
                      ok=(BURA_OK,)) -> bura_report_t:
    """The allocation-free one-shot solve: f, u are [nrhs][N] float64 CUDA tensors."""
    g, _keep = _grid(dim, n, coeff, lambda_upper)
    o = opts if opts is not None else bura_opts_default()
    m = len(weights)
    w = (ctypes.c_double * m)(*weights)
    s = (ctypes.c_double * m)(*shifts)
    nrhs = f.shape[0] if f.dim() == 2 else 1
    rep = bura_report_t()
    code = _lib.bura_solve_static(ctypes.byref(g), m, w, s, ctypes.byref(o), _devptr(f, "f"), _devptr(u, "u"), nrhs,
                                  ctypes.byref(rep))
    rep.status = code
    _check(code, "bura_solve_static", ok)
    return rep


def bura_plan_create_slots(dim: int, n: int, max_terms: int, opts: Optional[bura_opts_t] = None, coeff=None,
                           lambda_upper: float = 0.0):
    g, _keep = _grid(dim, n, coeff, lambda_upper)
    o = opts if opts is not None else bura_opts_default()
    h = _P()
    _check(_lib.bura_plan_create_slots(ctypes.byref(g), max_terms, ctypes.byref(o), ctypes.byref(h)),
           "bura_plan_create_slots")
    return h


def _slot_arrays(max_terms, terms, tols):
    """terms: per rhs a (weights, shifts) pair -> the C arrays of bura_solve_slots."""
    nr = len(terms)
    nt = (ctypes.c_int * nr)(*[len(w) for w, _ in terms])
    w = (ctypes.c_double * (nr * max_terms))()
    s = (ctypes.c_double * (nr * max_terms))()
    for r, (wr, sr) in enumerate(terms):
        if len(wr) != len(sr) or len(wr) > max_terms:
            raise ValueError("each rhs needs equally many weights and shifts, at most max_terms")
        for j, (a, b) in enumerate(zip(wr, sr)):
            w[r * max_terms + j] = a
            s[r * max_terms + j] = b
    t = (ctypes.c_double * nr)(*tols) if tols is not None else None
    return nt, w, s, t


def bura_solve_slots(plan, max_terms: int, f: torch.Tensor, u: torch.Tensor, terms, tols=None,
                     ok=(BURA_OK,)) -> bura_report_t:
    """terms[r] = (weights, shifts) of right-hand side r; tols[r] its tolerance (None: the plan's)."""
    nt, w, s, t = _slot_arrays(max_terms, terms, tols)
    rep = bura_report_t()
    code = _lib.bura_solve_slots(plan, _devptr(f, "f"), _devptr(u, "u"), len(terms), nt, w, s, t, ctypes.byref(rep))
    rep.status = code
    _check(code, "bura_solve_slots", ok)
    return rep


def bura_submit_slots(plan, max_terms: int, f: torch.Tensor, u: torch.Tensor, terms, tols=None) -> int:
    """Queue a slot solve; returns its ticket (see bura_poll / bura_wait)."""
    nt, w, s, t = _slot_arrays(max_terms, terms, tols)
    tk = ctypes.c_uint64()
    _check(_lib.bura_submit_slots(plan, _devptr(f, "f"), _devptr(u, "u"), len(terms), nt, w, s, t,
                                  ctypes.byref(tk)), "bura_submit_slots")
    return tk.value


def bura_plan_create_rational_multi(dim: int, n: int, nterms: Sequence[int], weights: Sequence[float],
                                    shifts: Sequence[float], opts: Optional[bura_opts_t] = None, coeff=None,
                                    lambda_upper: float = 0.0):
    g, _keep = _grid(dim, n, coeff, lambda_upper)
    o = opts if opts is not None else bura_opts_default()
    m = len(weights)
    nt = (ctypes.c_int * len(nterms))(*nterms)
    w = (ctypes.c_double * m)(*weights)
    s = (ctypes.c_double * m)(*shifts)
    h = _P()
    _check(_lib.bura_plan_create_rational_multi(ctypes.byref(g), len(nterms), nt, w, s, ctypes.byref(o),
                                                ctypes.byref(h)), "bura_plan_create_rational_multi")
    return h


def sinc_kprime(alpha: float, kq: float) -> float:
    """The quadrature step k' for a nominal number of systems k_Q = pi^2/(4 alpha (1-alpha) k'^2)."""
    kp = ctypes.c_double()
    _check(_lib.bura_sinc_kprime(alpha, kq, ctypes.byref(kp)), "bura_sinc_kprime")
    return kp.value


def bura_sinc_coefficients(alpha: float, kprime: float, scale: float = 1.0):
    """(weights, shifts) of the sinc quadrature applied to scale * A, for A (host only)."""
    cnt = ctypes.c_int()
    w = (ctypes.c_double * BURA_MAX_TERMS)()
    s = (ctypes.c_double * BURA_MAX_TERMS)()
    code = _lib.bura_sinc_coefficients(alpha, kprime, scale, BURA_MAX_TERMS, w, s, ctypes.byref(cnt))
    if code == BURA_EINVAL and cnt.value > BURA_MAX_TERMS:
        w = (ctypes.c_double * cnt.value)()
        s = (ctypes.c_double * cnt.value)()
        code = _lib.bura_sinc_coefficients(alpha, kprime, scale, cnt.value, w, s, ctypes.byref(cnt))
    _check(code, "bura_sinc_coefficients")
    return list(w)[: cnt.value], list(s)[: cnt.value]


def bura_zeros(alpha: float, k: int, beta: int = 1):
    """(zeta_1 > ... > zeta_k, C) of the (k,k) BURA: r(t) = C prod (t - zeta_j)/(t - d_j) (host only)."""
    z = (ctypes.c_double * k)()
    C = ctypes.c_double()
    _check(_lib.bura_zeros(alpha, beta, k, z, ctypes.byref(C)), "bura_zeros")
    return list(z), C.value


def bura_plan_create_multistep(dim: int, n: int, alphas: Sequence[float], ks: Sequence[int],
                               opts: Optional[bura_opts_t] = None, coeff=None, lambda_upper: float = 0.0, rhs_unscaled: int = 0):
    g, _keep = _grid(dim, n, coeff, lambda_upper, rhs_unscaled)
    o = opts if opts is not None else bura_opts_default()
    m = len(alphas)
    a = (ctypes.c_double * m)(*alphas)
    k = (ctypes.c_int * m)(*ks)
    h = _P()
    _check(_lib.bura_plan_create_multistep(ctypes.byref(g), m, a, k, ctypes.byref(o), ctypes.byref(h)),
           "bura_plan_create_multistep")
    return h


def bura_plan_create_product(dim: int, n: int, alpha: float, k: int, opts: Optional[bura_opts_t] = None,
                             coeff=None, lambda_upper: float = 0.0, beta: int = 1, rhs_unscaled: int = 0):
    g, _keep = _grid(dim, n, coeff, lambda_upper, rhs_unscaled)
    o = opts if opts is not None else bura_opts_default()
    h = _P()
    _check(_lib.bura_plan_create_product(ctypes.byref(g), alpha, beta, k, ctypes.byref(o), ctypes.byref(h)),
           "bura_plan_create_product")
    return h


def bura_plan_create_sinc(dim: int, n: int, alphas: Sequence[float], kprimes: Sequence[float],
                          opts: Optional[bura_opts_t] = None, coeff=None, lambda_upper: float = 0.0, rhs_unscaled: int = 0):
    g, _keep = _grid(dim, n, coeff, lambda_upper, rhs_unscaled)
    o = opts if opts is not None else bura_opts_default()
    m = len(alphas)
    a = (ctypes.c_double * m)(*alphas)
    kp = (ctypes.c_double * m)(*kprimes)
    h = _P()
    _check(_lib.bura_plan_create_sinc(ctypes.byref(g), m, a, kp, ctypes.byref(o), ctypes.byref(h)),
           "bura_plan_create_sinc")
    return h


def _devptr(t: torch.Tensor, what: str):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def bura_solve(plan, f: torch.Tensor, u: torch.Tensor, nrhs: int, ok=(BURA_OK,)) -> bura_report_t:
    rep = bura_report_t()
    code = _lib.bura_solve(plan, _devptr(f, "f"), _devptr(u, "u"), nrhs, ctypes.byref(rep))
    rep.status = code
    _check(code, "bura_solve", ok)
    return rep


def bura_submit(plan, f: torch.Tensor, u: torch.Tensor, nrhs: int, tol: float = 0.0) -> int:
    """Queue a solve (tol > 0 overrides the plan's tolerance for it); returns its ticket."""
    tk = ctypes.c_uint64()
    _check(_lib.bura_submit(plan, _devptr(f, "f"), _devptr(u, "u"), nrhs, tol, ctypes.byref(tk)), "bura_submit")
    return tk.value


def bura_poll(ticket: int):
    """(status, report) of a ticket; BURA_PENDING while it runs, then the ticket is released."""
    rep = bura_report_t()
    code = _lib.bura_poll(ticket, ctypes.byref(rep))
    return code, rep


def bura_wait(ticket: int):
    rep = bura_report_t()
    code = _lib.bura_wait(ticket, ctypes.byref(rep))
    return code, rep


def bura_plan_coeffs(plan):
    n = ctypes.c_int()
    c = (ctypes.c_double * BURA_MAX_TERMS)()
    d = (ctypes.c_double * BURA_MAX_TERMS)()
    E = ctypes.c_double()
    _check(_lib.bura_plan_coeffs(plan, ctypes.byref(n), c, d, ctypes.byref(E)), "bura_plan_coeffs")
    return list(c)[: n.value], list(d)[: n.value], E.value


def bura_plan_info(plan):
    lam = ctypes.c_double()
    nl = ctypes.c_int()
    nb = ctypes.c_size_t()
    _check(_lib.bura_plan_info(plan, ctypes.byref(lam), ctypes.byref(nl), ctypes.byref(nb)), "bura_plan_info")
    return lam.value, nl.value, nb.value


def bura_plan_apply(plan, shift: float, x: torch.Tensor, y: torch.Tensor, nvec: int):
    _check(_lib.bura_plan_apply(plan, shift, _devptr(x, "x"), _devptr(y, "y"), nvec), "bura_plan_apply")


KERNEL_CLASSES = ["smooth_fine", "smooth_coarse", "restrict", "prolong", "coarse_lds", "spmv", "update_xr",
                  "update_p", "residual64", "combine", "other", "down_fine", "up_fine", "down_fine_plain",
                  "smooth_fine_rup"]


def bura_plan_profile(plan, enable):
    """enable: False/0 off, True/1 all classes timed, or the C bitmask (1 << (class + 1))."""
    _check(_lib.bura_plan_profile(plan, int(enable)), "bura_plan_profile")


def bura_plan_kernel_stats(plan, kclass: int):
    """(launches, total_ms, algorithmic_bytes) of one kernel class."""
    n = ctypes.c_longlong()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(_lib.bura_plan_kernel_stats(plan, kclass, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)),
           "bura_plan_kernel_stats")
    return n.value, ms.value, by.value


def bura_plan_tiles(plan):
    """Tile-shape variants in use: [stencil product, down_0, up_0, down_1, up_1, ...]."""
    n = ctypes.c_int()
    _check(_lib.bura_plan_tiles(plan, None, 0, ctypes.byref(n)), "bura_plan_tiles")
    if n.value == 0:
        return []
    buf = (ctypes.c_int * n.value)()
    _check(_lib.bura_plan_tiles(plan, buf, n.value, ctypes.byref(n)), "bura_plan_tiles")
    return list(buf)


def bura_plan_set_tiles(plan, variants):
    v = list(variants)
    buf = (ctypes.c_int * len(v))(*v)
    _check(_lib.bura_plan_set_tiles(plan, buf, len(v)), "bura_plan_set_tiles")


def bura_device_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    """dst = src with the library's streaming copy kernel (counter calibration)."""
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("contiguous CUDA tensors expected")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _check(_lib.bura_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                 _stream_ptr(stream)), "bura_device_copy")


def bura_plan_destroy(plan):
    if plan:
        _lib.bura_plan_destroy(plan)


# --------------------------------------------------------------------------
# convenience object
# --------------------------------------------------------------------------

@dataclass
class SolveResult:
    u: torch.Tensor
    report: bura_report_t


class Plan:
    """Owns a plan handle; ``solve(f)`` returns A^-alpha f for a batch f of shape (nrhs, n, ..., n)."""

    def __init__(self, dim, n, alpha=None, k=None, *, weights=None, shifts=None, nterms=None, kprime=None,
                 form="fractions", beta=1, coeff=None, precision=BURA_MIXED, schedule=BURA_BATCHED, tol=1e-12,
                 nrhs_max=1, stream=None, rhs_unscaled=0, **opt):
        """alpha (one value or a list) with k poles: the BURA; alpha with kprime
        (one value or lists): the sinc quadrature of step k'; weights/shifts
        (with nterms per output for several outputs): a caller-given form.
        form="multistep" (alpha and k lists: the steps, in order) or
        form="product" (one alpha): the sequential forms.  beta=2: the (k+1,k)
        2-BURA of t^(2-alpha)."""
        self.dim, self.n = dim, n
        o = bura_opts_default(precision=precision, schedule=schedule, tol=tol, nrhs_max=nrhs_max, **opt)
        o.stream = _stream_ptr(stream).value if torch.cuda.is_available() else None
        self.opts = o
        self.handle = None
        self.nout = 1
        if form == "multistep":
            al = list(alpha)
            ks = list(k) if isinstance(k, (list, tuple)) else [k] * len(al)
            self.handle = bura_plan_create_multistep(dim, n, al, ks, o, coeff=coeff, rhs_unscaled=rhs_unscaled)
        elif form == "product":
            self.handle = bura_plan_create_product(dim, n, alpha, k, o, coeff=coeff, rhs_unscaled=rhs_unscaled)
        elif form != "fractions":
            raise ValueError("form must be 'fractions', 'multistep' or 'product'")
        elif weights is not None and nterms is not None:
            self.handle = bura_plan_create_rational_multi(dim, n, nterms, weights, shifts, o, coeff=coeff)
            self.nout = len(nterms)
        elif weights is not None:
            self.handle = bura_plan_create_rational(dim, n, weights, shifts, o, coeff=coeff)
        elif kprime is not None:
            al = list(alpha) if isinstance(alpha, (list, tuple)) else [alpha]
            kp = list(kprime) if isinstance(kprime, (list, tuple)) else [kprime] * len(al)
            self.handle = bura_plan_create_sinc(dim, n, al, kp, o, coeff=coeff, rhs_unscaled=rhs_unscaled)
            self.nout = len(al) if isinstance(alpha, (list, tuple)) else 1
        elif isinstance(alpha, (list, tuple)):
            ks = list(k) if isinstance(k, (list, tuple)) else [k] * len(alpha)
            self.handle = bura_plan_create_multi(dim, n, list(alpha), ks, o, coeff=coeff, rhs_unscaled=rhs_unscaled)
            self.nout = len(alpha)
        else:
            self.handle = bura_plan_create(dim, n, alpha, k, o, coeff=coeff, beta=beta,
                                           rhs_unscaled=rhs_unscaled)

    @property
    def coeffs(self):
        return bura_plan_coeffs(self.handle)

    @property
    def info(self):
        return bura_plan_info(self.handle)

    @property
    def tiles(self):
        return bura_plan_tiles(self.handle)

    @tiles.setter
    def tiles(self, variants):
        bura_plan_set_tiles(self.handle, variants)

    def solve(self, f: torch.Tensor, u: Optional[torch.Tensor] = None, ok=(BURA_OK,)) -> SolveResult:
        f = f.contiguous()
        nrhs = f.shape[0] if f.dim() == self.dim + 1 else 1
        if u is None:
            u = torch.empty_like(f) if self.nout == 1 else torch.empty((self.nout,) + tuple(f.shape),
                                                                         dtype=f.dtype, device=f.device)
        rep = bura_solve(self.handle, f, u, nrhs, ok)
        return SolveResult(u, rep)

    def apply(self, x: torch.Tensor, shift: float = 0.0) -> torch.Tensor:
        x = x.contiguous()
        y = torch.empty_like(x)
        nvec = x.shape[0] if x.dim() == self.dim + 1 else 1
        bura_plan_apply(self.handle, shift, x, y, nvec)
        return y

    def close(self):
        if self.handle:
            bura_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# request server
# --------------------------------------------------------------------------

def bura_server_create(hbm_budget: int = 0, max_concurrent: int = 4, max_group: int = 4):
    h = _P()
    _check(_lib.bura_server_create(hbm_budget, max_concurrent, max_group, ctypes.byref(h)), "bura_server_create")
    return h


def bura_server_submit(server, dim, n, alpha, k, f: torch.Tensor, u: torch.Tensor, tol=1e-10,
                       precision=BURA_MIXED) -> int:
    q = bura_request_t(dim, n, alpha, k, tol, precision)
    t = ctypes.c_uint64()
    _check(_lib.bura_server_submit(server, ctypes.byref(q), _devptr(f, "f"), _devptr(u, "u"), ctypes.byref(t)),
           "bura_server_submit")
    return t.value


def bura_server_poll(server, ticket: int):
    rep = bura_report_t()
    code = _lib.bura_server_poll(server, ticket, ctypes.byref(rep))
    return code, rep


def bura_server_wait(server, ticket: int):
    rep = bura_report_t()
    code = _lib.bura_server_wait(server, ticket, ctypes.byref(rep))
    return code, rep


def bura_server_reset_latency(server):
    _check(_lib.bura_server_reset_latency(server), "bura_server_reset_latency")


def bura_server_stats(server) -> dict:
    st = bura_server_stats_t()
    _check(_lib.bura_server_stats(server, ctypes.byref(st)), "bura_server_stats")
    return {name: getattr(st, name) for name, _ in bura_server_stats_t._fields_}


def bura_server_destroy(server):
    if server:
        _lib.bura_server_destroy(server)
