"""Plain FP64 CPU oracle for sparse COO MTTKRP / CP-ALS (arXiv 1809.09175, Phipps & Kolda).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with
the HIP library (``paper_1809_09175_amd``); the two meet only through seeded input arrays.

The arithmetic lives in ``oracle.c`` (single-threaded C, FP64, built with -ffp-contract=off so
every product and sum is rounded exactly as written).  This module only marshals numpy arrays.

Functions and what pins them (tests/test_oracle_pins.py):
  mttkrp        eq. (mttkrp), Sec. 3  -- brute force (dense unfolding x explicit Khatri-Rao),
                                          rank-1 closed form, d=2 sparse-times-dense product,
                                          linearity / duplicate splitting / order invariance
  perm          Sec. 6 (stable sort)   -- numpy stable argsort, bijection, sortedness
  model_values  eq. (CP), Sec. 3        -- dense Kruskal tensor built with einsum
  fit           eq. (CP), Sec. 3        -- brute-force residual over every cell of a tiny tensor
  cp_als_mode   Sec. 3 (textbook ALS)  -- normal-equation optimality, independent lstsq ALS,
                                          exact low-rank recovery, monotone fit
  gcp_poisson   Sec. 8 (future work: generalized CP) -- central finite differences, dense loss
  gcp           the same with Bernoulli-logit and Gaussian losses -- finite differences, dense
                loss, Gaussian gradient = 2 (model - data) MTTKRP closed form
  bf16_rne      rounding of FP32 to BF16 -- torch's CPU conversion on sampled and boundary bits
  bf16_rne_f64  rounding of FP64 to BF16 in one step -- bf16_rne on every FP64 value that is an
                FP32, exact rational arithmetic (fractions) on random and tie-adjacent values
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {0: "ok", -1: "invalid argument", -2: "index out of range", -4: "singular Gram"}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, single-threaded, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.oracle_bf16_rne.restype = ctypes.c_uint16
        _lib.oracle_bf16_rne.argtypes = [ctypes.c_uint32]
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc):
    if rc != 0:
        raise OracleError(f"oracle returned {rc} ({ERRORS.get(rc, '?')})")


class _T:
    """Validated, FP64/int32-contiguous copies of a COO tensor's arrays."""

    def __init__(self, subs, vals, dims):
        self.subs = np.ascontiguousarray(subs, dtype=np.int32)
        if self.subs.ndim != 2:
            raise ValueError("subs must be P x d")
        self.P, self.d = self.subs.shape
        self.dims = np.ascontiguousarray(dims, dtype=np.int64)
        if self.dims.shape != (self.d,):
            raise ValueError("dims must have d entries")
        self.vals = None if vals is None else np.ascontiguousarray(vals, dtype=np.float64)
        if self.vals is not None and self.vals.shape != (self.P,):
            raise ValueError("vals must have P entries")

    def head(self):
        return (ctypes.c_int(self.d), _p(self.dims), ctypes.c_int64(self.P), _p(self.subs))


def _factor_array(factors, dims, R):
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
    for m, f in enumerate(fs):
        if f.shape != (dims[m], R):
            raise ValueError(f"factor {m} has shape {f.shape}, expected {(dims[m], R)}")
    arr = (ctypes.c_void_p * len(fs))(*[f.ctypes.data for f in fs])
    return fs, arr


def mttkrp(subs, vals, dims, factors, n, lam=None):
    t = _T(subs, vals, dims)
    R = int(np.asarray(factors[0]).shape[1])
    fs, arr = _factor_array(factors, t.dims, R)
    lam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    V = np.empty((int(t.dims[n]), R), dtype=np.float64)
    _check(_load().oracle_mttkrp(*t.head(), _p(t.vals), ctypes.c_int(n), ctypes.c_int(R), arr,
                                 _p(lam), _p(V)))
    return V


def perm(subs, dims, n):
    t = _T(subs, None, dims)
    p = np.empty(t.P, dtype=np.int32)
    k = np.empty(t.P, dtype=np.int32)
    _check(_load().oracle_perm(*t.head(), ctypes.c_int(n), _p(p), _p(k)))
    return p, k


def model_values(subs, dims, factors, lam=None):
    t = _T(subs, None, dims)
    R = int(np.asarray(factors[0]).shape[1])
    fs, arr = _factor_array(factors, t.dims, R)
    lam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    m = np.empty(t.P, dtype=np.float64)
    _check(_load().oracle_model_values(*t.head(), ctypes.c_int(R), arr, _p(lam), _p(m)))
    return m


def gram(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    G = np.empty((A.shape[1], A.shape[1]), dtype=np.float64)
    _check(_load().oracle_gram(ctypes.c_int64(A.shape[0]), ctypes.c_int(A.shape[1]), _p(A), _p(G)))
    return G


def cp_als_mode(subs, vals, dims, factors, lam, grams, n):
    """One ALS mode update.  Returns new (factors, lam, grams); inputs are not modified."""
    t = _T(subs, vals, dims)
    R = int(np.asarray(factors[0]).shape[1])
    fs = [np.array(f, dtype=np.float64, order="C", copy=True) for f in factors]
    arr = (ctypes.c_void_p * t.d)(*[f.ctypes.data for f in fs])
    lam = np.array(lam, dtype=np.float64, copy=True)
    G = np.array(grams, dtype=np.float64, order="C", copy=True).reshape(t.d, R, R)
    _check(_load().oracle_cp_als_mode(*t.head(), _p(t.vals), ctypes.c_int(n), ctypes.c_int(R),
                                      arr, _p(lam), _p(G)))
    return fs, lam, G


def cp_als_sweep(subs, vals, dims, factors, lam, grams):
    t = _T(subs, vals, dims)
    R = int(np.asarray(factors[0]).shape[1])
    fs = [np.array(f, dtype=np.float64, order="C", copy=True) for f in factors]
    arr = (ctypes.c_void_p * t.d)(*[f.ctypes.data for f in fs])
    lam = np.array(lam, dtype=np.float64, copy=True)
    G = np.array(grams, dtype=np.float64, order="C", copy=True).reshape(t.d, R, R)
    _check(_load().oracle_cp_als_sweep(*t.head(), _p(t.vals), ctypes.c_int(R), arr, _p(lam),
                                       _p(G)))
    return fs, lam, G


def fit(subs, vals, dims, factors, lam=None, return_parts=False):
    t = _T(subs, vals, dims)
    R = int(np.asarray(factors[0]).shape[1])
    fs, arr = _factor_array(factors, t.dims, R)
    lam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    f = ctypes.c_double()
    parts = np.empty(3, dtype=np.float64)
    _check(_load().oracle_fit(*t.head(), _p(t.vals), ctypes.c_int(R), arr, _p(lam),
                              ctypes.byref(f), _p(parts)))
    return (f.value, parts) if return_parts else f.value


def gcp_poisson(subs, vals, dims, factors, w=None, grads=True):
    t = _T(subs, vals, dims)
    R = int(np.asarray(factors[0]).shape[1])
    fs, arr = _factor_array(factors, t.dims, R)
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    loss = ctypes.c_double()
    gs = None
    garr = None
    if grads:
        gs = [np.empty((int(t.dims[m]), R), dtype=np.float64) for m in range(t.d)]
        garr = (ctypes.c_void_p * t.d)(*[g.ctypes.data for g in gs])
    _check(_load().oracle_gcp_poisson(*t.head(), _p(t.vals), _p(w), ctypes.c_int(R), arr,
                                      ctypes.byref(loss), garr))
    return (loss.value, gs) if grads else loss.value


GCP_LOSSES = {"poisson": 0, "bernoulli": 1, "gaussian": 2, "gamma": 3}


def gcp(subs, vals, dims, factors, loss="poisson", w=None, grads=True):
    """Generalized CP loss (poisson: exp(m) - x m; bernoulli: log(1+exp(m)) - x m; gaussian:
    (x - m)^2; gamma: x / m + log m for m > 0) over the stored entries, and its gradient (an
    MTTKRP per mode)."""
    t = _T(subs, vals, dims)
    R = int(np.asarray(factors[0]).shape[1])
    fs, arr = _factor_array(factors, t.dims, R)
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    out = ctypes.c_double()
    gs = None
    garr = None
    if grads:
        gs = [np.empty((int(t.dims[m]), R), dtype=np.float64) for m in range(t.d)]
        garr = (ctypes.c_void_p * t.d)(*[g.ctypes.data for g in gs])
    _check(_load().oracle_gcp(*t.head(), _p(t.vals), _p(w), ctypes.c_int(R), arr,
                              ctypes.c_int(GCP_LOSSES[loss]), ctypes.byref(out), garr))
    return (out.value, gs) if grads else out.value


def philox4x64(ctr, key):
    """Philox4x64-10 block: four uint64 words from a 4-word counter and a 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    if c.shape != (4,) or k.shape != (2,):
        raise ValueError("counter must have 4 words, key 2")
    out = np.empty(4, dtype=np.uint64)
    _load().oracle_philox4x64(_p(c), _p(k), _p(out))
    return out


def gcp_sample(subs, vals, dims, seed, it, s_nz, s_z):
    """Stratified GCP-SGD sample of iteration `it`: (subs (s_nz+s_z) x d, vals, weights)."""
    t = _T(subs, vals, dims)
    n = int(s_nz) + int(s_z)
    os_ = np.empty((n, t.d), dtype=np.int32)
    ov = np.empty(n, dtype=np.float64)
    ow = np.empty(n, dtype=np.float64)
    _check(_load().oracle_gcp_sample(*t.head(), _p(t.vals), ctypes.c_uint64(int(seed)),
                                     ctypes.c_int64(int(it)), ctypes.c_int64(int(s_nz)),
                                     ctypes.c_int64(int(s_z)), _p(os_), _p(ov), _p(ow)))
    return os_, ov, ow


def adam(x, g, m, v, lr, beta1, beta2, eps, t, lower=-np.inf):
    """One Adam step in place on FP64 arrays x, m, v (g read)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, g, m, v)]
    for a in (x, m, v):
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
            raise ValueError("x, m, v must be contiguous float64 arrays (updated in place)")
    _check(_load().oracle_adam(ctypes.c_int64(x.size), _p(x), _p(arrs[1]), _p(m), _p(v),
                               ctypes.c_double(lr), ctypes.c_double(beta1),
                               ctypes.c_double(beta2), ctypes.c_double(eps),
                               ctypes.c_int64(int(t)), ctypes.c_double(lower)))


def bf16_rne(x):
    """FP32 array (or its uint32 bit patterns) -> uint16 BF16 bit patterns."""
    a = np.ascontiguousarray(x)
    bits = a.view(np.uint32) if a.dtype == np.float32 else np.ascontiguousarray(a, np.uint32)
    out = np.empty(bits.shape, dtype=np.uint16)
    _check(_load().oracle_bf16_rne_array(ctypes.c_int64(bits.size), _p(bits), _p(out)))
    return out


def bf16_rne_f64(x):
    """FP64 array -> uint16 BF16 bit patterns, rounded once (no FP32 step)."""
    a = np.ascontiguousarray(x, np.float64)
    out = np.empty(a.shape, dtype=np.uint16)
    _check(_load().oracle_bf16_rne_f64_array(ctypes.c_int64(a.size), _p(a), _p(out)))
    return out


def _swap_library(path):
    """Load another build of oracle.c in place of the default one (used by the mutation tests,
    which compile deliberately broken copies to show the pins catch them).  Returns the
    previous handle; pass it back to restore."""
    global _lib
    prev = _load()
    _lib = ctypes.CDLL(path)
    _lib.oracle_bf16_rne.restype = ctypes.c_uint16
    _lib.oracle_bf16_rne.argtypes = [ctypes.c_uint32]
    return prev


def _restore_library(handle):
    global _lib
    _lib = handle
