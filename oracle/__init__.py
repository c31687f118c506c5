"""ctypes shim over the FP64 CPU oracle of ATSFFT (arXiv:1908.02461).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library; the product path never
imports it.  The oracle's arithmetic lives in ``oracle.c``; this module only
marshals numpy arrays.  Each wrapper names the paper passage its C function
follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

PHASE_PROBE, PHASE_LOC, PHASE_EST = 0, 1, 2
OK, TRUNCATED, PROBE_NOT_CONVERGED, PROBE_SATURATED, EMPTY, RETRIED = 0, 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C99, -O2)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"], cwd=_HERE
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


class _Params(C.Structure):
    _fields_ = [
        ("ndim", C.c_int),
        ("n", C.c_int64),
        ("B0", C.c_int64),
        ("B_max", C.c_int64),
        ("alpha_probe", C.c_int),
        ("alpha", C.c_int),
        ("L_loc", C.c_int),
        ("L_est", C.c_int),
        ("T_vote", C.c_int),
        ("P_max", C.c_int),
        ("d", C.c_int),
        ("gamma", C.c_int),
        ("delta", C.c_double),
        ("q", C.c_double),
        ("noise_rate", C.c_double),
        ("rho", C.c_double),
        ("seed", C.c_uint64),
        ("signal", C.c_uint32),
        ("fixed_B", C.c_int64),
        ("fixed_k", C.c_int64),
        ("max_out", C.c_int64),
        ("res_tol", C.c_double),
        ("res_retries", C.c_int),
    ]


_MAXP = 64
_MAXL = 64


class _Result(C.Structure):
    _fields_ = [
        ("status", C.c_int),
        ("khat", C.c_int64),
        ("B_star", C.c_int64),
        ("count", C.c_int64),
        ("n_probe", C.c_int),
        ("probe_B", C.c_int64 * _MAXP),
        ("probe_k", C.c_int64 * _MAXP),
        ("probe_T", C.c_double * _MAXP),
        ("probe_decision", C.c_int * _MAXP),
        ("T_loc", C.c_double * _MAXL),
        ("J_count", C.c_int64 * _MAXL),
        ("yhat", C.POINTER(C.c_double)),
        ("yhat_stride", C.c_int64),
        ("J", C.POINTER(C.c_uint8)),
        ("locs", C.POINTER(C.c_int64)),
        ("vals", C.POINTER(C.c_double)),
        ("est", C.POINTER(C.c_double)),
        ("res_ratio", C.c_double),
        ("retries", C.c_int),
    ]


class _ProbeState(C.Structure):
    _fields_ = [
        ("B", C.c_int64),
        ("k_prev", C.c_int64),
        ("visited", C.c_uint64),
        ("iter", C.c_int),
        ("done", C.c_int),
        ("status", C.c_int),
        ("B_star", C.c_int64),
        ("khat", C.c_int64),
    ]


_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_U8 = C.POINTER(C.c_uint8)
_I32 = C.POINTER(C.c_int32)


def _declare(L):
    L.or_splitmix64_at.restype = C.c_uint64
    L.or_splitmix64_at.argtypes = [C.c_uint64, C.c_uint64]
    L.or_draw_word.restype = C.c_uint64
    L.or_draw_word.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int]
    L.or_draw.restype = None
    L.or_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int, C.c_int64, _I64, _I64, _I64]
    L.or_inverse_mod.restype = C.c_int64
    L.or_inverse_mod.argtypes = [C.c_int64, C.c_int64]
    for name in ("or_dft_naive", "or_fft", "or_fft2", "or_idft_naive"):
        getattr(L, name).restype = None
        getattr(L, name).argtypes = [C.c_int64, _D, _D]
    L.or_window_len.restype = C.c_int64
    L.or_window_len.argtypes = [C.c_int64, C.c_int64, C.c_int]
    L.or_window_taps.restype = None
    L.or_window_taps.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, _D]
    L.or_window_hat.restype = C.c_double
    L.or_window_hat.argtypes = [C.c_int64, C.c_int64, _D, C.c_int64, _D]
    L.or_hash_bucket.restype = C.c_int64
    L.or_hash_bucket.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int64]
    L.or_hash_offset.restype = C.c_int64
    L.or_hash_offset.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int64]
    L.or_hash_1d.restype = None
    L.or_hash_1d.argtypes = [C.c_int64, _D, C.c_int64, C.c_int64, C.c_int64, C.c_int64, _D, _D]
    L.or_hash_2d.restype = None
    L.or_hash_2d.argtypes = [C.c_int64, _D, _I64, _I64, C.c_int64, C.c_int64, _D, _D]
    L.or_threshold.restype = C.c_double
    L.or_threshold.argtypes = [_D, C.c_int64, C.c_double, C.c_double, C.c_double]
    L.or_local_max_1d.restype = C.c_int64
    L.or_local_max_1d.argtypes = [_D, C.c_int64, C.c_double]
    L.or_local_max_2d.restype = C.c_int64
    L.or_local_max_2d.argtypes = [_D, C.c_int64, C.c_double]
    L.or_rule.restype = C.c_int
    L.or_rule.argtypes = [C.c_int64, C.c_int64]
    L.or_topnum.restype = C.c_int64
    L.or_topnum.argtypes = [_D, C.c_int64, C.c_double, C.c_int64, _U8]
    L.or_vote_hist.restype = None
    L.or_vote_hist.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_int, _I64, _U8, _I32]
    L.or_median.restype = C.c_double
    L.or_median.argtypes = [_D, C.c_int]
    L.or_l1_error.restype = C.c_double
    L.or_l1_error.argtypes = [C.c_int64, _D, C.c_int64, _I64, _D, C.c_int64]
    L.or_default_params.restype = None
    L.or_default_params.argtypes = [C.POINTER(_Params), C.c_int, C.c_int64]
    L.or_residual_reach.restype = C.c_int
    L.or_residual_reach.argtypes = [C.c_int, C.c_double]
    L.or_residual.restype = None
    L.or_residual.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_int64, _D, C.c_int, C.c_int, _I64, _I64, _D,
                              C.c_int64, _I64, _D, _D, _D]
    L.or_probe_init.restype = None
    L.or_probe_init.argtypes = [C.POINTER(_Params), C.POINTER(_ProbeState)]
    L.or_probe_step.restype = C.c_int
    L.or_probe_step.argtypes = [C.POINTER(_Params), C.POINTER(_ProbeState), C.c_int64]
    L.or_atsfft.restype = C.c_int
    L.or_atsfft.argtypes = [C.POINTER(_Params), _D, C.POINTER(_Result)]


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


# ---- draws (Definition 1; counter-based SplitMix64) ----

def splitmix64_at(seed: int, index: int) -> int:
    return int(lib().or_splitmix64_at(seed & (2**64 - 1), index & (2**64 - 1)))


def draw_word(seed, signal, phase, it, axis) -> int:
    return int(lib().or_draw_word(seed & (2**64 - 1), signal, phase, it, axis))


def draw(seed, signal, phase, it, axis, n):
    s, t, si = C.c_int64(), C.c_int64(), C.c_int64()
    lib().or_draw(seed & (2**64 - 1), signal, phase, it, axis, n, C.byref(s), C.byref(t), C.byref(si))
    return s.value, t.value, si.value


def inverse_mod(a, n) -> int:
    return int(lib().or_inverse_mod(a, n))


# ---- DFT display ----

def _xform(name, x):
    x = _c128(x)
    out = np.empty_like(x)
    getattr(lib(), name)(x.shape[0] if name != "or_fft2" else x.shape[0], _dp(x), _dp(out))
    return out


def dft_naive(x):
    return _xform("or_dft_naive", x)


def idft_naive(X):
    return _xform("or_idft_naive", X)


def fft(x):
    return _xform("or_fft", x)


def fft2(x):
    x = _c128(x)
    assert x.ndim == 2 and x.shape[0] == x.shape[1]
    out = np.empty_like(x)
    lib().or_fft2(x.shape[0], _dp(x), _dp(out))
    return out


# ---- window (Sec. II-A-2) ----

def window_len(n, B, alpha) -> int:
    return int(lib().or_window_len(n, B, alpha))


def window_taps(n, B, w, delta) -> np.ndarray:
    G = np.empty(w, dtype=np.float64)
    lib().or_window_taps(n, B, w, delta, _dp(G))
    return G


def window_hat(n, w, G, q, with_imag=False):
    G = np.ascontiguousarray(G, dtype=np.float64)
    im = C.c_double()
    re = lib().or_window_hat(n, w, _dp(G), int(q), C.byref(im))
    return (re, im.value) if with_imag else re


# ---- hash (Sec. II-A-3) ----

def hash_bucket(n, B, sigma, f) -> int:
    return int(lib().or_hash_bucket(n, B, sigma, f))


def hash_offset(n, B, sigma, f) -> int:
    return int(lib().or_hash_offset(n, B, sigma, f))


def hash_1d(x, sigma, tau, B, w, G):
    x = _c128(x)
    G = np.ascontiguousarray(G, dtype=np.float64)
    out = np.empty(B, dtype=np.complex128)
    lib().or_hash_1d(x.shape[0], _dp(x), sigma, tau, B, w, _dp(G), _dp(out))
    return out


def hash_2d(x, sigma, tau, B, w, G):
    x = _c128(x)
    G = np.ascontiguousarray(G, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.int64)
    t = np.asarray(tau, dtype=np.int64)
    out = np.empty((B, B), dtype=np.complex128)
    lib().or_hash_2d(x.shape[0], _dp(x), s.ctypes.data_as(_I64), t.ctypes.data_as(_I64), B, w,
                     _dp(G), _dp(out))
    return out


# ---- selection (Sec. III-A, Algorithms 1 and 2) ----

def threshold(m, q=0.1, noise_rate=0.01, rho=1e-6) -> float:
    m = np.ascontiguousarray(m, dtype=np.float64).ravel()
    return float(lib().or_threshold(_dp(m), m.size, q, noise_rate, rho))


def local_max_1d(m, T) -> int:
    m = np.ascontiguousarray(m, dtype=np.float64)
    return int(lib().or_local_max_1d(_dp(m), m.size, T))


def local_max_2d(m, T) -> int:
    m = np.ascontiguousarray(m, dtype=np.float64)
    return int(lib().or_local_max_2d(_dp(m), m.shape[0], T))


def rule(k_prev, k_cur) -> int:
    return int(lib().or_rule(k_prev, k_cur))


def topnum(m, T, num):
    m = np.ascontiguousarray(m, dtype=np.float64).ravel()
    J = np.zeros(m.size, dtype=np.uint8)
    c = lib().or_topnum(_dp(m), m.size, T, num, J.ctypes.data_as(_U8))
    return J.astype(bool), int(c)


def vote_hist(ndim, n, B, sigma_inv, J):
    """sigma_inv: [L] (1D) or [L][2] (2D); J: [L][B^ndim] flags."""
    si = np.ascontiguousarray(sigma_inv, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.uint8)
    L = J.shape[0]
    votes = np.zeros(n if ndim == 1 else n * n, dtype=np.int32)
    lib().or_vote_hist(ndim, n, B, L, si.ctypes.data_as(_I64), J.ctypes.data_as(_U8),
                       votes.ctypes.data_as(_I32))
    return votes


def residual_reach(alpha, delta) -> int:
    return int(lib().or_residual_reach(alpha, delta))


def residual(ndim, n, B, w, G, sigma, tau, yhat, locs, vals, reach):
    """Residual test (an addition to the method): E_res, E_tot of the loops'
    bucket DFTs yhat [L][B^ndim] against the model of the located values, with
    per-loop draws sigma, tau [L] (1D) or [L][2] (2D), the model reaching
    `reach` buckets to each side of a frequency's own."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    s = np.ascontiguousarray(sigma, dtype=np.int64)
    t = np.ascontiguousarray(tau, dtype=np.int64)
    y = _c128(yhat)
    L = y.shape[0]
    locs = np.ascontiguousarray(locs, dtype=np.int64)
    vals = _c128(vals)
    er, et = C.c_double(), C.c_double()
    lib().or_residual(ndim, n, B, w, _dp(G), reach, L, s.ctypes.data_as(_I64), t.ctypes.data_as(_I64), _dp(y),
                      locs.size, locs.ctypes.data_as(_I64), _dp(vals), C.byref(er), C.byref(et))
    return er.value, et.value


def median(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return float(lib().or_median(_dp(v), v.size))


def l1_error(Xtrue, locs, vals, k) -> float:
    Xtrue = _c128(Xtrue).ravel()
    locs = np.ascontiguousarray(locs, dtype=np.int64)
    vals = _c128(vals)
    return float(lib().or_l1_error(Xtrue.size, _dp(Xtrue), locs.size, locs.ctypes.data_as(_I64),
                                   _dp(vals), k))


# ---- Algorithm 2 ----

@dataclass
class Params:
    ndim: int = 1
    n: int = 1 << 14
    B0: int = 32
    B_max: int = 512
    alpha_probe: int = 16
    alpha: int = 32
    L_loc: int = 9
    L_est: int = 9
    T_vote: int = 5
    P_max: int = 12
    d: int = 2
    gamma: int = 32
    delta: float = 1e-8
    q: float = 0.1
    noise_rate: float = 0.01
    rho: float = 1e-6
    seed: int = 0
    signal: int = 0
    fixed_B: int = 0
    fixed_k: int = 0
    max_out: int = 4096
    res_tol: float = 0.0
    res_retries: int = 1

    @staticmethod
    def defaults(ndim: int, n: int, **kw) -> "Params":
        p = _Params()
        lib().or_default_params(C.byref(p), ndim, n)
        out = Params(**{f.name: getattr(p, f.name) for f in fields(Params)})
        for k, v in kw.items():
            setattr(out, k, v)
        return out

    def _c(self) -> _Params:
        p = _Params()
        for f in fields(Params):
            setattr(p, f.name, getattr(self, f.name))
        return p


def probe_run(p: "Params", count_at) -> dict:
    """Drive the oracle's probe (or_probe_init / or_probe_step, the iteration
    of Algorithm 2) with given local-maximum counts instead of hashing:
    count_at maps a bucket count B (per axis) to the count k of the iteration
    hashed at B (a dict or a callable)."""
    get = count_at if callable(count_at) else count_at.__getitem__
    pc = p._c()
    s = _ProbeState()
    L = lib()
    L.or_probe_init(C.byref(pc), C.byref(s))
    Bs, ks, decs = [], [], []
    while not s.done:
        B = int(s.B)
        k = int(get(B))
        Bs.append(B)
        ks.append(k)
        decs.append(int(L.or_probe_step(C.byref(pc), C.byref(s), k)))
    return dict(probe_B=Bs, probe_k=ks, probe_decision=decs, B_star=int(s.B_star), khat=int(s.khat),
                status=int(s.status), n_probe=int(s.iter))


def atsfft(x, p: Params, trace: bool = True) -> dict:
    """Run the oracle's Algorithm 2 on x (1D length n, or N x N)."""
    x = _c128(x)
    lib()
    B = p.fixed_B if p.fixed_B > 0 else p.B_max
    if p.res_tol > 0:
        B = max(B, p.B_max)
    cnt = B if p.ndim == 1 else B * B
    L = p.L_loc + p.L_est
    r = _Result()
    yhat = J = est = None
    if trace:
        yhat = np.zeros((L, cnt), dtype=np.complex128)
        J = np.zeros((p.L_loc, cnt), dtype=np.uint8)
        est = np.zeros((p.max_out, p.L_est), dtype=np.complex128)
        r.yhat = yhat.ctypes.data_as(_D)
        r.J = J.ctypes.data_as(_U8)
        r.est = est.ctypes.data_as(_D)
    r.yhat_stride = cnt
    locs = np.zeros(p.max_out, dtype=np.int64)
    vals = np.zeros(p.max_out, dtype=np.complex128)
    r.locs = locs.ctypes.data_as(_I64)
    r.vals = vals.ctypes.data_as(_D)
    pc = p._c()
    rc = lib().or_atsfft(C.byref(pc), _dp(x), C.byref(r))
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    count = int(r.count)
    kept = min(count, p.max_out) if not (r.status & TRUNCATED) else 0
    out = {
        "status": int(r.status),
        "khat": int(r.khat),
        "B_star": int(r.B_star),
        "count": count,
        "locs": locs[:kept].copy(),
        "vals": vals[:kept].copy(),
        "probe_B": [int(r.probe_B[i]) for i in range(r.n_probe)],
        "probe_k": [int(r.probe_k[i]) for i in range(r.n_probe)],
        "probe_T": [float(r.probe_T[i]) for i in range(r.n_probe)],
        "probe_decision": [int(r.probe_decision[i]) for i in range(r.n_probe)],
        "T_loc": [float(r.T_loc[i]) for i in range(p.L_loc)],
        "J_count": [int(r.J_count[i]) for i in range(p.L_loc)],
        "res_ratio": float(r.res_ratio),
        "retries": int(r.retries),
    }
    if trace and not (r.status & EMPTY):
        c = int(r.B_star) if p.ndim == 1 else int(r.B_star) ** 2
        out["yhat"] = yhat[:, :c].copy()
        out["J"] = J[:, :c].astype(bool)
        out["est"] = est[:kept].copy()
    return out
