"""MI355X-native sparse COO tensor MTTKRP and CP-ALS (arXiv 1809.09175, Phipps & Kolda).

Thin Python layer over libspt.so: torch supplies device memory and streams, every computation
runs in the library's HIP kernels.  Nothing here computes MTTKRP, sorts or solves on the host.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (ALGO_ATOMIC, ALGO_AUTO, ALGO_PERMUTED, ALGO_PERMUTED_COPY, ALGO_PRIVATIZED,
                   SPT_BF16, SPT_F32, SPT_F64, SptError, SptTune, SptUnavailable)

__all__ = ["SparseTensor", "mttkrp", "CPState", "cp_als", "model_values", "GCPLoss",
           "GCPPoissonLoss",
           "default_tune", "autotune", "Batch", "to_bf16", "stream_triad", "SptError",
           "SptUnavailable",
           "ALGO_AUTO", "ALGO_ATOMIC", "ALGO_PERMUTED", "dtype_code"]

COPY_ORDERS = {"storage": 0, "second_mode": 1}

_ALGOS = {"auto": ALGO_AUTO, "atomic": ALGO_ATOMIC, "permuted": ALGO_PERMUTED,
          "permuted_copy": ALGO_PERMUTED_COPY, "privatized": ALGO_PRIVATIZED,
          ALGO_AUTO: ALGO_AUTO, ALGO_ATOMIC: ALGO_ATOMIC, ALGO_PERMUTED: ALGO_PERMUTED,
          ALGO_PERMUTED_COPY: ALGO_PERMUTED_COPY, ALGO_PRIVATIZED: ALGO_PRIVATIZED}
_ALGO_NAMES = {ALGO_AUTO: "auto", ALGO_ATOMIC: "atomic", ALGO_PERMUTED: "permuted",
               ALGO_PERMUTED_COPY: "permuted_copy", ALGO_PRIVATIZED: "privatized"}


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def dtype_code(t) -> int:
    """spt dtype of a factor tensor: float64, float32, or bfloat16 (BF16 bit patterns)."""
    dt = t.dtype if isinstance(t, torch.Tensor) else t
    if dt == torch.float64:
        return SPT_F64
    if dt == torch.float32:
        return SPT_F32
    if dt == torch.bfloat16:
        return SPT_BF16
    raise TypeError(f"unsupported factor dtype {dt}")


def _dev_check(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA (HIP) tensor")


def _tune(algo="auto", lanes=0, cols=0, chunk=0, deterministic=False, lds_kib=0):
    return SptTune(_ALGOS[algo], int(lanes), int(cols), int(chunk),
                   _lib.TUNE_DETERMINISTIC if deterministic else 0, int(lds_kib))


class SparseTensor:
    """COO tensor held by libspt: packed entry records plus per-mode permutations.

    subs: (P, d) int32 CUDA tensor of 0-based subscripts; vals: (P,) float32/float64 CUDA tensor.
    The library packs them into a workspace this object owns (a torch uint8 buffer)."""

    def __init__(self, subs: torch.Tensor, vals: torch.Tensor, dims, stream=None):
        lib = _lib.load()
        _dev_check(subs, "subs")
        _dev_check(vals, "vals")
        if subs.dtype != torch.int32 or subs.dim() != 2:
            raise ValueError("subs must be a (P, d) int32 tensor")
        if vals.dtype not in (torch.float32, torch.float64) or vals.shape != (subs.shape[0],):
            raise ValueError("vals must be (P,) float32 or float64")
        self.d = int(subs.shape[1])
        self.dims = tuple(int(x) for x in dims)
        if len(self.dims) != self.d:
            raise ValueError("dims must have d entries")
        self.nnz = int(subs.shape[0])
        self.device = subs.device
        self.vdtype = SPT_F64 if vals.dtype == torch.float64 else SPT_F32
        self.vals_dtype = vals.dtype
        dims_arr = (ctypes.c_int64 * self.d)(*self.dims)
        nbytes = lib.spt_tensor_workspace_bytes(self.d, dims_arr, self.nnz, self.vdtype)
        if nbytes == 0:
            raise ValueError("unsupported tensor shape (order must be 2..5, dims < 2^31)")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib.spt_tensor_create(ctypes.byref(h), self.d, dims_arr, self.nnz,
                                             ctypes.c_void_p(subs.data_ptr()),
                                             ctypes.c_void_p(vals.data_ptr()), self.vdtype,
                                             ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                             _stream(stream)), "spt_tensor_create")
        self._h = h
        self._keep = (subs, vals)   # alive until the packing work has run

    @classmethod
    def from_host(cls, subs, vals, dims, chunk: int = 1 << 23, device="cuda", stream=None):
        """Builds the tensor from host arrays (numpy or CPU torch tensors; (P, d) int32
        subscripts, (P,) float32/float64 values) in chunks of `chunk` entries (a multiple of
        8192): each chunk is copied to the device on a copy stream of its own while the previous
        chunk is packed (spt_tensor_append, which also counts the first radix digit of every
        mode).  The copies run asynchronously from pinned host memory (torch's pin_memory());
        from pageable memory each copy is staged by the runtime and overlaps less."""
        if chunk <= 0 or chunk % 8192:
            raise ValueError("chunk must be a positive multiple of 8192")
        subs = torch.as_tensor(subs)
        vals = torch.as_tensor(vals)
        if subs.dtype != torch.int32 or subs.dim() != 2 or subs.device.type != "cpu":
            raise ValueError("subs must be a (P, d) int32 host array")
        if vals.dtype not in (torch.float32, torch.float64) or vals.shape != (subs.shape[0],) \
                or vals.device.type != "cpu":
            raise ValueError("vals must be (P,) float32 or float64 host values")
        self = cls.__new__(cls)
        lib = _lib.load()
        self.d = int(subs.shape[1])
        self.dims = tuple(int(x) for x in dims)
        if len(self.dims) != self.d:
            raise ValueError("dims must have d entries")
        self.nnz = int(subs.shape[0])
        self.device = torch.device(device)
        self.vdtype = SPT_F64 if vals.dtype == torch.float64 else SPT_F32
        self.vals_dtype = vals.dtype
        dims_arr = (ctypes.c_int64 * self.d)(*self.dims)
        nbytes = lib.spt_tensor_workspace_bytes(self.d, dims_arr, self.nnz, self.vdtype)
        if nbytes == 0:
            raise ValueError("unsupported tensor shape (order must be 2..5, dims < 2^31)")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        subs_d = torch.empty(subs.shape, dtype=torch.int32, device=self.device)
        vals_d = torch.empty(vals.shape, dtype=vals.dtype, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            compute = stream if stream is not None else torch.cuda.current_stream()
            _lib.check(lib.spt_tensor_create_begin(ctypes.byref(h), self.d, dims_arr, self.nnz,
                                                   self.vdtype,
                                                   ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                                   _stream(compute)), "spt_tensor_create_begin")
            self._h = h
            copy = torch.cuda.Stream(device=self.device)
            copy.wait_stream(compute)   # the device buffers come from the compute stream
            for a in range(0, self.nnz, chunk):
                b = min(self.nnz, a + chunk)
                with torch.cuda.stream(copy):
                    subs_d[a:b].copy_(subs[a:b], non_blocking=True)
                    vals_d[a:b].copy_(vals[a:b], non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(copy)
                compute.wait_event(ev)
                _lib.check(lib.spt_tensor_append(
                    h, a, b - a, ctypes.c_void_p(subs_d[a:b].data_ptr()),
                    ctypes.c_void_p(vals_d[a:b].data_ptr()), _stream(compute)), "spt_tensor_append")
            subs_d.record_stream(compute)
            vals_d.record_stream(compute)
        self._keep = (subs_d, vals_d, subs, vals)   # alive until the packing work has run
        return self

    @property
    def handle(self):
        return self._h

    def permute(self, mode: int = -1, stream=None):
        _lib.check(_lib.load().spt_tensor_permute(self._h, int(mode), _stream(stream)),
                   "spt_tensor_permute")
        return self

    def sort_copy(self, mode: int = -1, order: str = "auto", stream=None):
        """Build mode-sorted copies of the records (needs permute(mode) first); the permuted
        MTTKRP then streams records instead of gathering them.  Within a row the entries follow
        `order`: "second_mode" (increasing subscript of the other mode with the most rows, which
        must be permuted too; better cache reuse of the gathered factor rows), "storage", or
        "auto" (second_mode where that mode is permuted, else storage).  Costs one record array
        (16 or 32 bytes per entry) per mode, plus 4 bytes per entry for the second-mode order."""
        lib = _lib.load()
        orders = ("second_mode", "storage") if order == "auto" else (order,)
        for k, name in enumerate(orders):
            o = COPY_ORDERS[name]
            nbytes = lib.spt_tensor_sorted_copy_bytes(self._h, int(mode), o)
            buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            rc = lib.spt_tensor_sort_copy(self._h, int(mode), o, ctypes.c_void_p(buf.data_ptr()),
                                          nbytes, _stream(stream))
            # the state check precedes any launch, so "auto" can retry in storage order
            if rc == -7 and k + 1 < len(orders):
                continue
            _lib.check(rc, "spt_tensor_sort_copy")
            break
        if not hasattr(self, "_copies"):
            self._copies = {}
        self._copies[int(mode)] = buf
        return self

    def validate(self, stream=None):
        bad = ctypes.c_int64(-1)
        rc = _lib.load().spt_tensor_validate(self._h, ctypes.byref(bad), _stream(stream))
        if rc != 0:
            raise SptError(rc, f"validate (first bad entry {bad.value})")
        self._keep = None
        return self

    def status(self, stream=None) -> int:
        return _lib.load().spt_tensor_status(self._h, _stream(stream))

    def perm(self, mode: int):
        """(perm, skey) of a permuted mode, as int32 views into the workspace."""
        p = ctypes.c_void_p()
        k = ctypes.c_void_p()
        _lib.check(_lib.load().spt_tensor_perm(self._h, int(mode), ctypes.byref(p),
                                               ctypes.byref(k)), "spt_tensor_perm")
        base = self.ws.data_ptr()
        n = self.nnz
        out = []
        for q in (p.value, k.value):
            off = (q or base) - base
            out.append(self.ws[off:off + 4 * n].view(torch.int32))
        return out[0], out[1]

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().spt_tensor_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_tune(X: SparseTensor, mode: int, R: int, fdtype, algo="auto") -> dict:
    t = SptTune()
    _lib.check(_lib.load().spt_mttkrp_default_tune(X.handle, int(mode), int(R),
                                                   dtype_code(fdtype), _ALGOS[algo],
                                                   ctypes.byref(t)), "default_tune")
    return {"algo": _ALGO_NAMES[t.algo], "lanes": t.lanes_per_nnz, "cols": t.cols_per_lane,
            "chunk": t.nnz_per_wave}


def _factor_ptrs(factors, skip=-1):
    ptrs = []
    for m, f in enumerate(factors):
        if m == skip and f is None:
            ptrs.append(None)
            continue
        _dev_check(f, f"factor {m}")
        ptrs.append(f.data_ptr())
    return _lib.ptr_array(ptrs)


def mttkrp(X: SparseTensor, factors, mode: int, lam=None, algo="auto", lanes=0, cols=0,
           chunk=0, vals=None, out=None, deterministic=False, lds_kib=0, stream=None):
    """Mode-`mode` MTTKRP (eq. (mttkrp)).  factors: d CUDA tensors (I_m, R) of one dtype
    (float64, float32 or bfloat16); lam: optional (R,) float64.  Returns V (I_n, R): float64
    for float64 factors, float32 otherwise."""
    lib = _lib.load()
    ref = factors[0] if factors[0] is not None else factors[1]
    R = int(ref.shape[1])
    fd = dtype_code(ref)
    vdt = torch.float64 if fd == SPT_F64 else torch.float32
    if out is None:
        out = torch.empty((X.dims[mode], R), dtype=vdt, device=X.device)
    _dev_check(out, "out")
    if lam is not None:
        _dev_check(lam, "lam")
        if lam.dtype != torch.float64:
            raise ValueError("lam must be float64")
    if vals is not None:
        _dev_check(vals, "vals")
    tune = _tune(algo, lanes, cols, chunk, deterministic, lds_kib)
    _lib.check(lib.spt_mttkrp(X.handle, int(mode), R, _factor_ptrs(factors, mode), fd,
                              ctypes.c_void_p(lam.data_ptr()) if lam is not None else None,
                              ctypes.c_void_p(vals.data_ptr()) if vals is not None else None,
                              ctypes.c_void_p(out.data_ptr()), ctypes.byref(tune),
                              _stream(stream)), "spt_mttkrp")
    return out


def to_bf16(x: torch.Tensor, stream=None) -> torch.Tensor:
    """FP32 or FP64 -> BF16 (round to nearest even; FP64 in a single rounding) with the
    library's kernels."""
    _dev_check(x, "x")
    if x.dtype not in (torch.float32, torch.float64):
        raise ValueError("x must be float32 or float64")
    x = x.contiguous()
    out = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    name = "spt_f32_to_bf16" if x.dtype == torch.float32 else "spt_f64_to_bf16"
    _lib.check(getattr(_lib.load(), name)(ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), x.numel(),
                                          _stream(stream)), name)
    return out


def stream_triad(a, b, c, s=3.0, stream=None):
    _lib.check(_lib.load().spt_stream_triad(ctypes.c_void_p(a.data_ptr()),
                                            ctypes.c_void_p(b.data_ptr()),
                                            ctypes.c_void_p(c.data_ptr()), float(s), a.numel(),
                                            _stream(stream)), "spt_stream_triad")


# ------------------------------------------------------------------------------------ CP-ALS

class CPState:
    """Kruskal tensor state of CP-ALS: factors (d CUDA tensors, I_m x R, float64/float32/
    bfloat16), weights lam (R float64) and the Gram matrices (d x R x R float64)."""

    def __init__(self, X: SparseTensor, factors, stream=None):
        lib = _lib.load()
        self.X = X
        self.factors = [f.contiguous() for f in factors]
        for f in self.factors:
            _dev_check(f, "factor")
        self.R = int(self.factors[0].shape[1])
        self.fdtype = dtype_code(self.factors[0])
        dev = X.device
        self.lam = torch.ones(self.R, dtype=torch.float64, device=dev)
        self.grams = torch.empty((X.d, self.R, self.R), dtype=torch.float64, device=dev)
        nbytes = lib.spt_cp_workspace_bytes(X.handle, self.R)
        if nbytes == 0:
            raise SptError(_lib.SPT_EUNSUPPORTED, "spt_cp_workspace_bytes (R must be <= 256)")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._last_mode = None  # mode whose MTTKRP the workspace holds (for the fast fit)
        for m, f in enumerate(self.factors):
            _lib.check(lib.spt_cp_gram(int(f.shape[0]), self.R, ctypes.c_void_p(f.data_ptr()),
                                       self.fdtype,
                                       ctypes.c_void_p(self.grams[m].data_ptr()),
                                       ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                       _stream(stream)), "spt_cp_gram")

    def _fptrs(self):
        return _lib.ptr_array([f.data_ptr() for f in self.factors])

    def mode_update(self, n: int, algo="auto", lanes=0, cols=0, chunk=0, stream=None):
        tune = _tune(algo, lanes, cols, chunk)
        _lib.check(_lib.load().spt_cp_als_mode(
            self.X.handle, int(n), self.R, self._fptrs(), self.fdtype,
            ctypes.c_void_p(self.lam.data_ptr()), ctypes.c_void_p(self.grams.data_ptr()),
            ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), ctypes.byref(tune),
            _stream(stream)), "spt_cp_als_mode")
        self._last_mode = int(n)

    def solution(self) -> torch.Tensor:
        """The FP64 solution rows (I_n x R, before normalisation and storage rounding) of the
        last mode update, as a view into the workspace (valid until the next call using it)."""
        if self._last_mode is None:
            raise SptError(_lib.SPT_ESTATE, "CPState.solution: no mode update yet")
        y = ctypes.c_void_p()
        _lib.check(_lib.load().spt_cp_solution(self.X.handle, self.R,
                                                ctypes.c_void_p(self.ws.data_ptr()),
                                                self.ws.numel(), ctypes.byref(y)),
                   "spt_cp_solution")
        off = y.value - self.ws.data_ptr()
        I = int(self.X.dims[self._last_mode])
        return self.ws[off:off + I * self.R * 8].view(torch.float64).view(I, self.R)

    def sweep(self, algo="auto", stream=None):
        tune = _tune(algo)
        _lib.check(_lib.load().spt_cp_als_sweep(
            self.X.handle, self.R, self._fptrs(), self.fdtype,
            ctypes.c_void_p(self.lam.data_ptr()), ctypes.c_void_p(self.grams.data_ptr()),
            ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), ctypes.byref(tune),
            _stream(stream)), "spt_cp_als_sweep")
        self._last_mode = self.X.d - 1

    def fit(self, return_parts=False, source="entries", stream=None):
        """Synchronising: fit of the current model.  source="entries": <X,M> from every stored
        entry's model value (FP64).  source="mttkrp": from the MTTKRP of the last mode update
        (an I_n x R inner product, no pass over the entries; valid while the factors, weights
        and Grams are the ones that update left)."""
        f = ctypes.c_double()
        parts = (ctypes.c_double * 3)()
        lib = _lib.load()
        common = (self._fptrs(), self.fdtype, ctypes.c_void_p(self.lam.data_ptr()),
                  ctypes.c_void_p(self.grams.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                  self.ws.numel(), ctypes.byref(f), parts, _stream(stream))
        if source == "entries":
            _lib.check(lib.spt_cp_fit(self.X.handle, self.R, *common), "spt_cp_fit")
        elif source == "mttkrp":
            if self._last_mode is None:
                raise ValueError("fit(source='mttkrp') needs a mode update first")
            _lib.check(lib.spt_cp_fit_after_mode(self.X.handle, self._last_mode, self.R, *common),
                       "spt_cp_fit_after_mode")
        else:
            raise ValueError(f"unknown fit source {source!r}")
        return (f.value, list(parts)) if return_parts else f.value


def cp_als(X: SparseTensor, factors, iters=10, algo="auto", tol=None, fit="mttkrp"):
    """Run CP-ALS sweeps from the given initial factors (updated in place).  Returns the state
    and the fit after every sweep, computed from the last mode's MTTKRP (fit="mttkrp", no pass
    over the entries) or from the stored entries (fit="entries")."""
    st = CPState(X, factors)
    fits = []
    for _ in range(iters):
        st.sweep(algo)
        fits.append(st.fit(source=fit))
        if tol is not None and len(fits) > 1 and abs(fits[-1] - fits[-2]) < tol:
            break
    return st, fits


def model_values(X: SparseTensor, factors, lam=None, stream=None):
    fd = dtype_code(factors[0])
    out = torch.empty(X.nnz, dtype=torch.float64 if fd == SPT_F64 else torch.float32,
                      device=X.device)
    _lib.check(_lib.load().spt_model_values(
        X.handle, int(factors[0].shape[1]), _factor_ptrs(factors), fd,
        ctypes.c_void_p(lam.data_ptr()) if lam is not None else None,
        ctypes.c_void_p(out.data_ptr()), _stream(stream)), "spt_model_values")
    return out


# ----------------------------------------------------------------------- generalized CP (GCP)

class GCPLoss(torch.autograd.Function):
    """Generalized CP loss sum_i w_i f(x_i, m_i) over the tensor's stored entries (nonzeros and
    sampled zeros), m_i = sum_j prod_m A^(m)(l_im, j), with f one of
      "poisson"   exp(m) - x m         (count data, log link)
      "bernoulli" log(1 + exp(m)) - x m (binary data, logit link)
      "gaussian"  (x - m)^2
      "gamma"     x / m + log m         (positive data; nonnegative factors, m > 0)
    Forward and backward run in libspt; the gradient is one MTTKRP per mode of the derivative
    tensor y_i = w_i df/dm(x_i, m_i).  With unit weights (w None) and every mode permuted, the
    forward runs the fused passes (spt_gcp_fused: loss and gradients in one sorted-order pass
    per mode) and the backward only scales the stored gradients by the upstream gradient;
    otherwise the forward computes the model values and loss and the backward the derivative
    tensor and its MTTKRPs.  Setting GCPLoss.use_fused = False forces the second form.

    Usage: loss = GCPLoss.apply(X, w, "bernoulli", *factors)   (w may be None)."""

    use_fused = True

    @staticmethod
    def forward(ctx, X, w, loss_kind, *factors):
        lib = _lib.load()
        fd = dtype_code(factors[0])
        if fd == SPT_BF16:
            raise TypeError("GCP factors must be float32 or float64")
        kind = _lib.GCP_LOSSES[loss_kind]
        R = int(factors[0].shape[1])
        vdt = torch.float64 if fd == SPT_F64 else torch.float32
        facs = [f.detach().contiguous() for f in factors]
        ctx.fused_grads = None
        if GCPLoss.use_fused and w is None:
            loss = torch.empty((), dtype=torch.float64, device=X.device)
            grads = [torch.empty_like(f) for f in facs]
            rc = lib.spt_gcp_fused(X.handle, R, _factor_ptrs(facs), fd, kind,
                                   ctypes.c_void_p(loss.data_ptr()),
                                   _lib.ptr_array([t.data_ptr() for t in grads]), None, None,
                                   _stream())
            if rc == 0:
                ctx.fused_grads = grads
                ctx.fd = fd
                return loss
            if rc != _lib.SPT_ESTATE:
                _lib.check(rc, "spt_gcp_fused")
        m = torch.empty(X.nnz, dtype=vdt, device=X.device)
        loss = torch.empty((), dtype=torch.float64, device=X.device)
        ws = torch.empty(32768, dtype=torch.uint8, device=X.device)
        _lib.check(lib.spt_gcp_forward(
            X.handle, R, _factor_ptrs(facs), fd, kind,
            ctypes.c_void_p(w.data_ptr()) if w is not None else None,
            ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "spt_gcp_forward")
        ctx.X = X
        ctx.w = w
        ctx.fd = fd
        ctx.kind = kind
        ctx.save_for_backward(m, *facs)
        return loss

    @staticmethod
    def backward(ctx, gout):
        if ctx.fused_grads is not None:
            g = gout.detach().to(torch.float64).contiguous()
            out = []
            for t in ctx.fused_grads:
                o = torch.empty_like(t)
                _lib.check(_lib.load().spt_scale_values(
                    ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(o.data_ptr()), t.numel(),
                    ctx.fd, ctypes.c_void_p(g.data_ptr()), _stream()), "spt_scale_values")
                out.append(o)
            return (None, None, None, *out)
        m, *facs = ctx.saved_tensors
        X = ctx.X
        R = int(facs[0].shape[1])
        g = gout.detach().to(torch.float64).contiguous()
        y = torch.empty_like(m)
        grads = [torch.empty_like(f) for f in facs]
        _lib.check(_lib.load().spt_gcp_backward(
            X.handle, R, _factor_ptrs(facs), ctx.fd, ctx.kind,
            ctypes.c_void_p(ctx.w.data_ptr()) if ctx.w is not None else None,
            ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(g.data_ptr()),
            ctypes.c_void_p(y.data_ptr()), _lib.ptr_array([t.data_ptr() for t in grads]), None,
            _stream()), "spt_gcp_backward")
        return (None, None, None, *grads)


class GCPPoissonLoss(torch.autograd.Function):
    """The Poisson (log link) case of GCPLoss.  Usage: GCPPoissonLoss.apply(X, w, *factors)."""

    @staticmethod
    def forward(ctx, X, w, *factors):
        return GCPLoss.forward(ctx, X, w, "poisson", *factors)

    @staticmethod
    def backward(ctx, gout):
        g = GCPLoss.backward(ctx, gout)
        return (g[0], g[1], *g[3:])


# ------------------------------------------------------------------ stochastic generalized CP

def gcp_sample(X: SparseTensor, seed: int, it: int, s_nz: int, s_z: int, dtype=torch.float32,
               stream=None):
    """Iteration `it`'s stratified sample drawn on the device (spt_gcp_sample): subscripts
    ((s_nz + s_z) x d int32), values and weights (dtype)."""
    n = int(s_nz) + int(s_z)
    subs = torch.empty((n, X.d), dtype=torch.int32, device=X.device)
    vals = torch.empty(n, dtype=dtype, device=X.device)
    w = torch.empty(n, dtype=dtype, device=X.device)
    _lib.check(_lib.load().spt_gcp_sample(
        X.handle, int(seed), int(it), int(s_nz), int(s_z), ctypes.c_void_p(subs.data_ptr()),
        ctypes.c_void_p(vals.data_ptr()), ctypes.c_void_p(w.data_ptr()), dtype_code(vals),
        _stream(stream)), "spt_gcp_sample")
    return subs, vals, w


def adam_step(x, g, m, v, t, lr, betas=(0.9, 0.999), eps=1e-8, lower=float("-inf"),
              stream=None):
    """One Adam step on CUDA tensors (spt_adam_step); x, m, v updated in place."""
    for a in (x, g, m, v):
        _dev_check(a, "adam operand")
    _lib.check(_lib.load().spt_adam_step(
        ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(g.data_ptr()),
        ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), x.numel(), dtype_code(x),
        float(lr), float(betas[0]), float(betas[1]), float(eps), int(t), float(lower),
        _stream(stream)), "spt_adam_step")


def gcp_sgd(X: SparseTensor, factors, loss="poisson", iters=100, samples=(1 << 16, 1 << 16),
            lr=1e-3, seed=0, lower=None, betas=(0.9, 0.999), eps=1e-8, start=1):
    """Stochastic generalized CP (GCP-SGD with Adam).  Every iteration draws a stratified sample
    of s_nz stored entries and s_z uniform cells on the device, evaluates the weighted sample
    loss and its gradient (spt_gcp_forward / spt_gcp_backward over the sample), and takes an Adam
    step on every factor.  factors: d CUDA float32/float64 tensors, updated in place.  lower:
    elementwise lower bound of the factors (default 0 for the Gamma loss, else none).  Returns
    the sample-loss estimates of every iteration (a CPU float64 tensor)."""
    lib = _lib.load()
    fd = dtype_code(factors[0])
    if fd == SPT_BF16:
        raise TypeError("GCP-SGD factors must be float32 or float64")
    kind = _lib.GCP_LOSSES[loss]
    if lower is None:
        lower = 0.0 if loss == "gamma" else float("-inf")
    s_nz, s_z = (int(samples[0]), int(samples[1]))
    dt = factors[0].dtype
    R = int(factors[0].shape[1])
    mom = [torch.zeros_like(f) for f in factors]
    vel = [torch.zeros_like(f) for f in factors]
    grads = [torch.empty_like(f) for f in factors]
    losses = torch.empty(iters, dtype=torch.float64, device=X.device)
    ws = torch.empty(32768, dtype=torch.uint8, device=X.device)
    ptrs = _factor_ptrs(factors)
    gptrs = _lib.ptr_array([g.data_ptr() for g in grads])
    for k in range(iters):
        t = start + k
        subs, vals, w = gcp_sample(X, seed, t, s_nz, s_z, dtype=dt)
        S = SparseTensor(subs, vals, X.dims)
        m = torch.empty(s_nz + s_z, dtype=dt, device=X.device)
        y = torch.empty_like(m)
        _lib.check(lib.spt_gcp_forward(S.handle, R, ptrs, fd, kind, ctypes.c_void_p(w.data_ptr()),
                                       ctypes.c_void_p(m.data_ptr()),
                                       ctypes.c_void_p(losses[k:].data_ptr()),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
                   "spt_gcp_forward")
        _lib.check(lib.spt_gcp_backward(S.handle, R, ptrs, fd, kind, ctypes.c_void_p(w.data_ptr()),
                                        ctypes.c_void_p(m.data_ptr()), None,
                                        ctypes.c_void_p(y.data_ptr()), gptrs, None, _stream()),
                   "spt_gcp_backward")
        for f, g, a, b in zip(factors, grads, mom, vel):
            adam_step(f, g, a, b, t, lr, betas, eps, lower)
        S.close()
    return losses.cpu()


# ------------------------------------------------------------------ autotuner and batching

def autotune(X: SparseTensor, factors, mode: int, batch=False, algos=("atomic", "permuted"),
             reps=0, out=None, stream=None):
    """Time the library default and every compiled launch configuration of this MTTKRP on the
    device (median of `reps` single launches each; 0 = the library's default count); returns
    the fastest as a dict(algo, lanes, cols, chunk, ms)."""
    lib = _lib.load()
    ref = factors[0] if factors[0] is not None else factors[1]
    R = int(ref.shape[1])
    fd = dtype_code(ref)
    if out is None:
        out = torch.empty((X.dims[mode], R), dtype=torch.float64 if fd == SPT_F64 else torch.float32,
                          device=X.device)
    flags = (_lib.TUNE_BATCH_CONFIGS if batch else 0)
    if "atomic" not in algos:
        flags |= _lib.TUNE_NO_ATOMIC
    if "permuted" not in algos:
        flags |= _lib.TUNE_NO_PERMUTED
    best = SptTune()
    ms = ctypes.c_float()
    _lib.check(lib.spt_mttkrp_autotune(X.handle, int(mode), R, _factor_ptrs(factors, mode), fd,
                                       ctypes.c_void_p(out.data_ptr()), flags, int(reps),
                                       ctypes.byref(best), ctypes.byref(ms), _stream(stream)),
               "spt_mttkrp_autotune")
    return {"algo": _ALGO_NAMES[best.algo], "lanes": best.lanes_per_nnz,
            "cols": best.cols_per_lane, "chunk": best.nnz_per_wave, "ms": ms.value}


class Batch:
    """Many MTTKRPs in one persistent kernel replayed from a HIP graph.

    items: list of dicts with keys X (SparseTensor), mode, factors, out (float32 CUDA tensor),
    and optional tune (dict as returned by autotune(batch=True))."""

    def __init__(self, items, stream=None):
        lib = _lib.load()
        n = len(items)
        self.items = items
        fd = dtype_code(items[0]["factors"][0])
        self._factor_arrays = [_factor_ptrs(it["factors"]) for it in items]
        tensors = (ctypes.c_void_p * n)(*[it["X"].handle.value for it in items])
        modes = (ctypes.c_int * n)(*[int(it["mode"]) for it in items])
        ranks = (ctypes.c_int * n)(*[int(it["factors"][0].shape[1]) for it in items])
        facs = (ctypes.c_void_p * n)(*[ctypes.cast(a, ctypes.c_void_p).value
                                       for a in self._factor_arrays])
        outs = (ctypes.c_void_p * n)(*[it["out"].data_ptr() for it in items])
        tunes = (SptTune * n)()
        for i, it in enumerate(items):
            t = it.get("tune") or {}
            tunes[i] = _tune(t.get("algo", "auto"), t.get("lanes", 0), t.get("cols", 0),
                             t.get("chunk", 0))
        nbytes = lib.spt_batch_workspace_bytes(n)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=items[0]["out"].device)
        h = ctypes.c_void_p()
        _lib.check(lib.spt_batch_create(ctypes.byref(h), n, tensors, modes, ranks, facs, fd, outs,
                                        tunes, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                        _stream(stream)), "spt_batch_create")
        self._h = h

    def launch(self, stream=None):
        _lib.check(_lib.load().spt_batch_launch(self._h, _stream(stream)), "spt_batch_launch")

    def info(self):
        u = ctypes.c_int64()
        sm = ctypes.c_int()
        _lib.check(_lib.load().spt_batch_info(self._h, ctypes.byref(u), ctypes.byref(sm)),
                   "spt_batch_info")
        return {"units": u.value, "smem": sm.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().spt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
