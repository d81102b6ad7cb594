"""GPU parity of the CP-ALS update, the fit, model values and the GCP Poisson loss/gradient
against the FP64 CPU oracle, through the C ABI.

Tolerances.  FP64 CP-ALS: a relative perturbation of 1e-15 in the factors of the 100 x 80 x 60
workload stays below 4e-15 after 10 sweeps (the Hadamard Gram products there have condition
numbers 8..35), so FP64 factors, weights and Grams are held to 1e-11 and the fit to 1e-12.
FP32 storage: one mode update maps the MTTKRP error (<= 1e-6 measured) through Gamma^-1, so
factors are held to max(1e-5, 1e-6 cond(Gamma)).  BF16 storage adds one rounding of 2^-9."""
import ctypes
import itertools
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1809_09175_amd import datagen

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (nb if nb > 0 else 1.0)


def _dev_tensor(X, dtype):
    import paper_1809_09175_amd as spt
    subs = torch.from_numpy(np.ascontiguousarray(X.subs, np.int32)).cuda()
    vals = torch.from_numpy(np.ascontiguousarray(X.vals).astype(dtype)).cuda()
    T = spt.SparseTensor(subs, vals, X.dims)
    T.validate()
    return T


def _np(t):
    return t.float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 \
        else t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("algo", ["atomic", "permuted", "permuted_copy"])
def test_cpals_small_fp64_ten_sweeps(gpu, algo):
    import paper_1809_09175_amd as spt
    X, A = datagen.cpals_small()
    T = _dev_tensor(X, np.float64)
    T.permute()
    if algo == "permuted_copy":
        T.sort_copy()  # the MTTKRPs then read the sorted record copies
    st = spt.CPState(T, [torch.from_numpy(a.copy()).cuda() for a in A])
    Ao = [a.copy() for a in A]
    lo = np.ones(16)
    Go = np.stack([oracle.gram(a) for a in Ao])
    assert _relerr(st.grams.cpu().numpy(), Go) < 1e-13
    for it in range(10):
        _log(f"cpals sweep {it} {algo}")
        st.sweep(algo)
        f_gpu, parts = st.fit(return_parts=True)
        Ao, lo, Go = oracle.cp_als_sweep(X.subs, X.vals, X.dims, Ao, lo, Go)
        f_ref, parts_ref = oracle.fit(X.subs, X.vals, X.dims, Ao, lo, return_parts=True)
        for m in range(3):
            assert _relerr(_np(st.factors[m]), Ao[m]) < 1e-11, (it, m)
        assert _relerr(st.lam.cpu().numpy(), lo) < 1e-11
        assert _relerr(st.grams.cpu().numpy(), Go) < 1e-11
        assert abs(f_gpu - f_ref) < 1e-12, (it, f_gpu, f_ref)
        assert np.allclose(parts, parts_ref, rtol=1e-12)


def _skewed4_small():
    X = datagen.skewed_tensor((2000, 500, 100, 365), 60_000, (1.2, 1.2, 0.0, 0.0), seed=3,
                              distinct=True)
    return X


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_cp_mode_update_low_precision(gpu, kind):
    import paper_1809_09175_amd as spt
    X = _skewed4_small()
    R = 32
    T = _dev_tensor(X, np.float32)
    T.permute()
    A32 = datagen.factors(X.dims, R, seed=8, dtype=np.float32)
    dev = [torch.from_numpy(a.copy()).cuda() for a in A32]
    if kind == "bf16":
        dev = [spt.to_bf16(a) for a in dev]
    st = spt.CPState(T, dev)
    for n in range(4):
        # the oracle starts from exactly the values the GPU holds before this mode update
        Ain = [_np(f) for f in st.factors]
        lin = st.lam.cpu().numpy()
        Gin = st.grams.cpu().numpy()
        assert _relerr(Gin, np.stack([a.T @ a for a in Ain])) < 1e-12
        _log(f"mode update {kind} n={n}")
        st.mode_update(n)
        Ao, lo, Go = oracle.cp_als_mode(X.subs, X.vals, X.dims, Ain, lin, Gin, n)
        Gam = np.ones((R, R))
        for m in range(4):
            if m != n:
                Gam *= Gin[m]
        cond = np.linalg.cond(Gam)
        tol = max(1e-5, 1e-6 * cond)
        if kind == "bf16":
            tol += 2.0 ** -8
        assert _relerr(_np(st.factors[n]), Ao[n]) < tol, (n, cond)
        assert _relerr(st.lam.cpu().numpy(), lo) < tol
        # the Gram is of the stored (rounded) factor, in FP64
        stored = _np(st.factors[n])
        assert _relerr(st.grams[n].cpu().numpy(), stored.T @ stored) < 1e-12
        # the stored factor is the FP64 solution over lambda, rounded once to the storage type:
        # bit-exact against numpy's FP64 -> FP32 conversion / the oracle's FP64 -> BF16 rounding
        Y = st.solution().cpu().numpy()
        lam = st.lam.cpu().numpy()
        a = np.where(lam > 0, Y / np.where(lam > 0, lam, 1.0), Y)
        if kind == "bf16":
            bits = st.factors[n].view(torch.int16).cpu().numpy().view(np.uint16)
            assert np.array_equal(bits, oracle.bf16_rne_f64(a)), n
        else:
            assert np.array_equal(st.factors[n].cpu().numpy(), a.astype(np.float32)), n


@pytest.mark.parametrize("R", [5, 20, 40, 64, 96, 98, 128, 200, 256])
def test_cp_mode_update_fp64_ranks(gpu, R):
    """FP64 mode updates at ranks off the 16/32/64 grid (padded Cholesky, solve and Gram tiles),
    at 64 (the largest of the one-wavefront Cholesky) and above it up to 256 (blocked Cholesky
    and inverse in one workgroup, Gamma padded to a multiple of 16 at 98 and 200; the row solves
    as one product with the inverse and the Gram in 128 x 128 tiles, partial at 96, 98 and 200),
    against the oracle's mode update from the same state."""
    import paper_1809_09175_amd as spt
    X = _skewed4_small()
    X.vals = X.vals.astype(np.float64)
    T = _dev_tensor(X, np.float64)
    T.permute()
    A = datagen.factors(X.dims, R, seed=R, dtype=np.float64)
    st = spt.CPState(T, [torch.from_numpy(a.copy()).cuda() for a in A])
    for n in range(4):
        Ain = [_np(f) for f in st.factors]
        lin = st.lam.cpu().numpy()
        Gin = st.grams.cpu().numpy()
        _log(f"fp64 mode update R={R} n={n}")
        st.mode_update(n)
        Ao, lo, Go = oracle.cp_als_mode(X.subs, X.vals, X.dims, Ain, lin, Gin, n)
        Gam = np.ones((R, R))
        for m in range(4):
            if m != n:
                Gam *= Gin[m]
        tol = 1e-13 * max(1.0, np.linalg.cond(Gam))
        assert _relerr(_np(st.factors[n]), Ao[n]) < tol, (n, np.linalg.cond(Gam))
        assert _relerr(st.lam.cpu().numpy(), lo) < tol
        assert _relerr(st.grams[n].cpu().numpy(), Go[n]) < 1e-12


@pytest.mark.parametrize("copy_mode", [None, 0, 2])
def test_fit_matches_oracle_fp32_factors(gpu, copy_mode):
    """Fit from FP32 factors over the stored entries; a permuted mode with a sorted record copy
    (mode 0 or 2) present leaves it unchanged."""
    import paper_1809_09175_amd as spt
    X = _skewed4_small()
    R = 16
    T = _dev_tensor(X, np.float32)
    if copy_mode is not None:
        T.permute(copy_mode)
        T.sort_copy(copy_mode)
    A32 = datagen.factors(X.dims, R, seed=9, dtype=np.float32)
    st = spt.CPState(T, [torch.from_numpy(a).cuda() for a in A32])
    st.lam = torch.linspace(0.5, 2.0, R, dtype=torch.float64, device="cuda")
    f, parts = st.fit(return_parts=True)
    f_ref, parts_ref = oracle.fit(X.subs, X.vals, X.dims, [a.astype(np.float64) for a in A32],
                                  st.lam.cpu().numpy(), return_parts=True)
    assert abs(f - f_ref) < 1e-12 * max(1.0, abs(f_ref))
    assert np.allclose(parts, parts_ref, rtol=1e-12)


@pytest.mark.parametrize("fit", ["mttkrp", "entries"])
def test_cp_als_driver(gpu, fit):
    """cp_als: factors updated in place, one fit per sweep from either source matching the
    oracle's sweeps, and the tolerance stop ending the run early once the fit settles."""
    import paper_1809_09175_amd as spt
    X, A = datagen.cpals_small()
    T = _dev_tensor(X, np.float64)
    T.permute()
    facs = [torch.from_numpy(a.copy()).cuda() for a in A]
    st, fits = spt.cp_als(T, facs, iters=5, fit=fit)
    assert len(fits) == 5
    Ao, lo = [a.copy() for a in A], np.ones(16)
    Go = np.stack([oracle.gram(a) for a in Ao])
    for it in range(5):
        Ao, lo, Go = oracle.cp_als_sweep(X.subs, X.vals, X.dims, Ao, lo, Go)
        assert abs(fits[it] - oracle.fit(X.subs, X.vals, X.dims, Ao, lo)) < 1e-12, it
    for m in range(3):
        assert facs[m].data_ptr() == st.factors[m].data_ptr()  # updated in place
        assert _relerr(_np(facs[m]), Ao[m]) < 1e-11
    _, fits2 = spt.cp_als(T, [torch.from_numpy(a.copy()).cuda() for a in A], iters=200,
                          fit=fit, tol=1e-3)
    assert 2 <= len(fits2) < 200
    assert abs(fits2[-1] - fits2[-2]) < 1e-3


def test_fit_after_mode_fp64_matches_oracle(gpu):
    """The fit from the last mode's MTTKRP (no pass over the entries) equals the oracle's fit
    from the entries, every sweep of an FP64 run, and the entry-pass fit of the same state; also
    right after a single update of a middle mode, and with ||X||^2 served from the handle."""
    import paper_1809_09175_amd as spt
    X, A = datagen.cpals_small()
    T = _dev_tensor(X, np.float64)
    T.permute()
    st = spt.CPState(T, [torch.from_numpy(a.copy()).cuda() for a in A])
    with pytest.raises(ValueError):
        st.fit(source="mttkrp")
    Ao = [a.copy() for a in A]
    lo = np.ones(16)
    Go = np.stack([oracle.gram(a) for a in Ao])
    for it in range(6):
        _log(f"fit after mode, sweep {it}")
        st.sweep()
        f_fast, p_fast = st.fit(return_parts=True, source="mttkrp")
        f_ent, p_ent = st.fit(return_parts=True)
        Ao, lo, Go = oracle.cp_als_sweep(X.subs, X.vals, X.dims, Ao, lo, Go)
        f_ref, p_ref = oracle.fit(X.subs, X.vals, X.dims, Ao, lo, return_parts=True)
        assert abs(f_fast - f_ref) < 1e-12, (it, f_fast, f_ref)
        assert abs(f_fast - f_ent) < 1e-12
        assert np.allclose(p_fast, p_ref, rtol=1e-11)
    st.mode_update(1)
    Ao, lo, Go = oracle.cp_als_mode(X.subs, X.vals, X.dims, Ao, lo, Go, 1)
    f_ref = oracle.fit(X.subs, X.vals, X.dims, Ao, lo)
    assert abs(st.fit(source="mttkrp") - f_ref) < 1e-12


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_fit_after_mode_low_precision(gpu, kind):
    """FP32 / BF16 factors: the MTTKRP-based fit agrees with the FP64 entry-pass fit of the
    same state to the FP32 accumulation of V (4-way tensor, R = 16, both after a sweep and
    after the update of mode 2)."""
    import paper_1809_09175_amd as spt
    X = _skewed4_small()
    T = _dev_tensor(X, np.float32)
    T.permute()
    T.sort_copy()
    A32 = datagen.factors(X.dims, 16, seed=4, dtype=np.float32)
    facs = [torch.from_numpy(a).cuda() for a in A32]
    if kind == "bf16":
        facs = [spt.to_bf16(f) for f in facs]
    st = spt.CPState(T, facs)
    for step in range(3):
        _log(f"fit after mode {kind} step {step}")
        if step < 2:
            st.sweep()
        else:
            st.mode_update(2)
        f_fast = st.fit(source="mttkrp")
        f_ent = st.fit()
        assert abs(f_fast - f_ent) < 1e-5, (step, f_fast, f_ent)


def test_fit_rank_one_many_entries(gpu):
    """R = 1 with 5e6 entries: the entry-pass fit's 2 x ~600 block partials exceed the R x R
    Gram partial area of R = 1, which the workspace now sizes for both; both fits against the
    oracle."""
    import paper_1809_09175_amd as spt
    rng = np.random.default_rng(12)
    dims = (3000, 2000, 1000)
    P = 5_000_000
    subs = np.stack([rng.integers(0, I, size=P) for I in dims], 1).astype(np.int32)
    vals = rng.random(P)
    T = spt.SparseTensor(torch.from_numpy(subs).cuda(), torch.from_numpy(vals).cuda(), dims)
    T.permute()
    A = [rng.random((I, 1)) for I in dims]
    st = spt.CPState(T, [torch.from_numpy(a.copy()).cuda() for a in A])
    st.mode_update(0)
    Ao = [a.copy() for a in A]
    Go = np.stack([oracle.gram(a) for a in Ao])
    Ao, lo, Go = oracle.cp_als_mode(subs, vals, dims, Ao, np.ones(1), Go, 0)
    f_ref = oracle.fit(subs, vals, dims, Ao, lo)
    assert abs(st.fit() - f_ref) < 1e-11
    assert abs(st.fit(source="mttkrp") - f_ref) < 1e-11


@pytest.mark.parametrize("R", [24, 96, 98, 128, 200, 256])
def test_model_values(gpu, R):
    """Model values of every stored entry, including the wide lane layouts above 64 columns."""
    import paper_1809_09175_amd as spt
    X = _skewed4_small()
    A = datagen.factors(X.dims, R, seed=1, dtype=np.float64)
    X.vals = X.vals.astype(np.float64)
    T = _dev_tensor(X, np.float64)
    lam = np.linspace(1.0, 2.0, R)
    m = spt.model_values(T, [torch.from_numpy(a).cuda() for a in A],
                         torch.from_numpy(lam).cuda())
    assert _relerr(m.cpu().numpy(), oracle.model_values(X.subs, X.dims, A, lam)) < 1e-13


@pytest.mark.parametrize("kind", ["f64", "f32", "bf16"])
def test_large_rank_mode_update_fit_and_loss(gpu, kind):
    """R = 128: a CP-ALS mode update against the oracle from the same state (FP32 and BF16
    factors at the tolerance of their MTTKRP mapped through Gamma^-1, as for R <= 64), the
    stored factor bit-exact against the FP64 solution rounded once, the entry-pass and
    allocation-free fits and the generalized-CP (Poisson) loss against the oracle."""
    import ctypes
    import paper_1809_09175_amd as spt
    from paper_1809_09175_amd import _lib
    X = _skewed4_small()
    R = 128
    vdt = np.float64 if kind == "f64" else np.float32
    X.vals = X.vals.astype(vdt)
    T = _dev_tensor(X, vdt)
    T.permute()
    A = datagen.factors(X.dims, R, seed=12, dtype=vdt)
    dev = [torch.from_numpy(a.copy()).cuda() for a in A]
    if kind == "bf16":
        dev = [spt.to_bf16(a) for a in dev]
    st = spt.CPState(T, dev)
    Ain = [_np(f) for f in st.factors]
    Gin = st.grams.cpu().numpy()
    assert _relerr(Gin, np.stack([a.T @ a for a in Ain])) < 1e-12
    st.mode_update(1)
    Ao, lo, Go = oracle.cp_als_mode(X.subs, X.vals, X.dims, Ain, np.ones(R), Gin, 1)
    Gam = Gin[0] * Gin[2] * Gin[3]
    cond = np.linalg.cond(Gam)
    tol = 1e-13 * max(1.0, cond) if kind == "f64" else max(1e-5, 1e-6 * cond)
    if kind == "bf16":
        tol += 2.0 ** -8
    assert _relerr(_np(st.factors[1]), Ao[1]) < tol, cond
    assert _relerr(st.lam.cpu().numpy(), lo) < tol
    stored = _np(st.factors[1])
    assert _relerr(st.grams[1].cpu().numpy(), stored.T @ stored) < 1e-12
    Y = st.solution().cpu().numpy()
    lam = st.lam.cpu().numpy()
    a = np.where(lam > 0, Y / np.where(lam > 0, lam, 1.0), Y)
    if kind == "bf16":
        bits = st.factors[1].view(torch.int16).cpu().numpy().view(np.uint16)
        assert np.array_equal(bits, oracle.bf16_rne_f64(a))
    else:
        assert np.array_equal(st.factors[1].cpu().numpy(), a.astype(vdt))
    # fits of the updated state (from the stored entries, with and without a workspace)
    Acur = [_np(f) for f in st.factors]
    f_ref = oracle.fit(X.subs, X.vals, X.dims, Acur, lam)
    f = st.fit()
    assert abs(f - f_ref) < 1e-12 * max(1.0, abs(f_ref))
    fna = ctypes.c_double()
    parts = (ctypes.c_double * 3)()
    assert _lib.load().spt_cp_fit_noalloc(T.handle, R, st._fptrs(), st.fdtype,
                                          ctypes.c_void_p(st.lam.data_ptr()),
                                          ctypes.c_void_p(st.grams.data_ptr()),
                                          ctypes.byref(fna), parts, None) == 0
    assert fna.value == f
    if kind == "bf16":
        return
    # generalized-CP loss at R = 128 (unfused forward), small factors so exp(m) stays moderate
    facs = [torch.from_numpy((a * 0.05).astype(vdt)).cuda().requires_grad_(True) for a in A]
    loss = spt.GCPPoissonLoss.apply(T, torch.ones(X.nnz, dtype=facs[0].dtype, device="cuda"),
                                    *facs)
    loss_ref = oracle.gcp_poisson(X.subs, X.vals, X.dims,
                                  [(a * 0.05).astype(vdt).astype(np.float64) for a in A],
                                  grads=False)
    assert abs(loss.item() - loss_ref) < (1e-12 if kind == "f64" else 1e-5) * abs(loss_ref)


def test_singular_gram_reported(gpu):
    import paper_1809_09175_amd as spt
    from paper_1809_09175_amd import SptError
    dims = (4, 3, 3)
    cells = np.array(list(itertools.product(*[range(I) for I in dims])), dtype=np.int32)
    X = datagen.CooTensor(cells, np.ones(len(cells)), dims)
    T = _dev_tensor(X, np.float64)
    st = spt.CPState(T, [torch.ones(I, 2, dtype=torch.float64, device="cuda") for I in dims])
    st.mode_update(0)
    with pytest.raises(SptError) as e:
        st.fit()
    assert e.value.code == -4
    assert T.status() == 0          # the status was cleared once reported


def test_exact_low_rank_recovery(gpu):
    import paper_1809_09175_amd as spt
    rng = np.random.default_rng(31)
    dims = (12, 10, 8)
    R = 3
    Tr = [rng.standard_normal((I, R)) for I in dims]
    Xd = np.einsum("ir,jr,kr->ijk", *Tr)
    cells = np.array(list(itertools.product(*[range(I) for I in dims])), dtype=np.int32)
    X = datagen.CooTensor(cells, Xd[cells[:, 0], cells[:, 1], cells[:, 2]], dims)
    T = _dev_tensor(X, np.float64)
    T.permute()
    A0 = [t + 1e-2 * rng.standard_normal(t.shape) for t in Tr]
    st = spt.CPState(T, [torch.from_numpy(a).cuda() for a in A0])
    prev = -1.0
    for it in range(300):
        st.sweep()
        if it % 10 == 9:
            A = [_np(f) for f in st.factors]
            M = np.einsum("r,ir,jr,kr->ijk", st.lam.cpu().numpy(), *A)
            fit = 1.0 - np.linalg.norm(Xd - M) / np.linalg.norm(Xd)
            if fit > 1.0 - 1e-10 and abs(fit - prev) < 1e-15:
                break
            prev = fit
    assert fit > 1.0 - 1e-10


# -------------------------------------------------------------------------------------- GCP

def _gcp_case(dtype):
    X, A = datagen.gcp_counts(scale=2e-4, dims=(200, 100, 50), R=8)
    X.vals = X.vals.astype(dtype)
    A = [a.astype(dtype) for a in A]
    return X, A


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_gcp_poisson_forward_backward(gpu, kind):
    import paper_1809_09175_amd as spt
    dt = np.float64 if kind == "f64" else np.float32
    X, A = _gcp_case(dt)
    T = _dev_tensor(X, dt)
    T.permute()
    rng = np.random.default_rng(2)
    w = (rng.random(X.nnz) + 0.5).astype(dt)
    wd = torch.from_numpy(w).cuda()
    facs = [torch.from_numpy(a).cuda().requires_grad_(True) for a in A]
    loss = spt.GCPPoissonLoss.apply(T, wd, *facs)
    (3.0 * loss).backward()
    loss_ref, g_ref = oracle.gcp_poisson(X.subs, X.vals, X.dims, [a.astype(np.float64) for a in A],
                                         w.astype(np.float64))
    tol = 1e-12 if kind == "f64" else 1e-5
    assert abs(loss.item() - loss_ref) < tol * abs(loss_ref)
    gtol = 1e-12 if kind == "f64" else 1e-4
    for n in range(3):
        assert _relerr(facs[n].grad.cpu().numpy(), 3.0 * g_ref[n]) < gtol, n


def test_gcp_gradcheck_fp64(gpu):
    import paper_1809_09175_amd as spt
    X, A = datagen.gcp_counts(scale=6e-7, dims=(9, 7, 5), R=3)
    X.vals = X.vals.astype(np.float64)
    T = _dev_tensor(X, np.float64)
    facs = tuple(torch.from_numpy(a.astype(np.float64)).cuda().requires_grad_(True) for a in A)
    assert torch.autograd.gradcheck(lambda *f: spt.GCPPoissonLoss.apply(T, None, *f), facs,
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("loss", ["bernoulli", "gaussian", "poisson", "gamma"])
@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("copies", [False, True])
def test_gcp_general_losses(gpu, loss, kind, copies):
    """Weighted losses (the unfused forward and backward; with copies, the backward's MTTKRPs
    read the derivative values through the second-mode copy's order array)."""
    import paper_1809_09175_amd as spt
    dt = np.float64 if kind == "f64" else np.float32
    X, A = _gcp_case(dt)
    if loss == "bernoulli":
        X.vals = (X.vals > 0).astype(dt)
    T = _dev_tensor(X, dt)
    T.permute()
    if copies:
        T.sort_copy(order="second_mode")
    rng = np.random.default_rng(4)
    w = (rng.random(X.nnz) + 0.5).astype(dt)
    shift = 0.05 if loss == "gamma" else -0.2  # the Gamma model is a positive mean
    facs = [torch.from_numpy(a + shift).cuda().requires_grad_(True) for a in A]
    L = spt.GCPLoss.apply(T, torch.from_numpy(w).cuda(), loss, *facs)
    (0.5 * L).backward()
    L_ref, g_ref = oracle.gcp(X.subs, X.vals, X.dims, [a.astype(np.float64) + shift for a in A],
                              loss, w.astype(np.float64))
    tol, gtol = (1e-12, 1e-12) if kind == "f64" else (1e-5, 1e-4)
    assert abs(L.item() - L_ref) < tol * abs(L_ref)
    for n in range(3):
        assert _relerr(facs[n].grad.cpu().numpy(), 0.5 * g_ref[n]) < gtol, n


# ----------------------------------------------------------------------- fused GCP passes

def _fused_case(dt, d, P, seed, R=6):
    dims = (60, 45, 30, 20)[:d]
    rng = np.random.default_rng(seed)
    lin = rng.choice(int(np.prod(dims)), size=P, replace=False)
    subs = np.stack(np.unravel_index(lin, dims), axis=1).astype(np.int32)
    vals = rng.poisson(1.0, size=P).astype(dt)
    scale = 0.6 * (6.0 / R) ** (1.0 / d)   # keeps the model values of order one at any rank
    A = [(rng.random((I, R)) * scale + 0.02 * scale).astype(dt) for I in dims]
    return subs, vals, dims, A


@pytest.mark.parametrize("R", [96, 128, 256])
@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_gcp_fused_and_unfused_large_rank(gpu, kind, R):
    """Poisson GCP loss and gradients above 64 columns (wide lane layouts of the fused passes
    and of the unfused model pass) against the FP64 oracle, fused against unfused."""
    import paper_1809_09175_amd as spt
    dt = np.float64 if kind == "f64" else np.float32
    subs, vals, dims, A = _fused_case(dt, 3, 5003, seed=R, R=R)
    T = spt.SparseTensor(torch.from_numpy(subs).cuda(), torch.from_numpy(vals).cuda(), dims)
    T.permute()
    T.sort_copy()
    L_ref, g_ref = oracle.gcp(subs, vals, dims, [a.astype(np.float64) for a in A], "poisson")
    tol, gtol = (1e-12, 1e-12) if kind == "f64" else (1e-5, 1e-4)
    for fused in (True, False):
        spt.GCPLoss.use_fused = fused
        try:
            facs = [torch.from_numpy(a).cuda().requires_grad_(True) for a in A]
            L = spt.GCPLoss.apply(T, None, "poisson", *facs)
            L.backward()
            torch.cuda.synchronize()
        finally:
            spt.GCPLoss.use_fused = True
        assert abs(L.item() - L_ref) < tol * abs(L_ref), (fused, L.item(), L_ref)
        for n in range(3):
            assert _relerr(facs[n].grad.cpu().numpy(), g_ref[n]) < gtol, (fused, n)


@pytest.mark.parametrize("loss", ["poisson", "bernoulli", "gaussian", "gamma"])
@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("d,copies", [(3, False), (3, True), (4, True)])
def test_gcp_fused_matches_oracle_and_unfused(gpu, loss, kind, d, copies):
    """Fused loss-and-gradient passes (unit weights, permuted tensor) against the FP64 oracle,
    and against the unfused forward/backward on the same factors."""
    import paper_1809_09175_amd as spt
    dt = np.float64 if kind == "f64" else np.float32
    subs, vals, dims, A = _fused_case(dt, d, 5003, seed=d * 10 + len(loss))
    if loss == "bernoulli":
        vals = (vals > 0).astype(dt)
    T = spt.SparseTensor(torch.from_numpy(subs).cuda(), torch.from_numpy(vals).cuda(), dims)
    T.permute()
    if copies:
        T.sort_copy()
    L_ref, g_ref = oracle.gcp(subs, vals, dims, [a.astype(np.float64) for a in A], loss)
    tol, gtol = (1e-12, 1e-12) if kind == "f64" else (1e-5, 1e-4)
    results = []
    for fused in (True, False):
        spt.GCPLoss.use_fused = fused
        try:
            facs = [torch.from_numpy(a).cuda().requires_grad_(True) for a in A]
            L = spt.GCPLoss.apply(T, None, loss, *facs)
            (0.5 * L).backward()
            torch.cuda.synchronize()
        finally:
            spt.GCPLoss.use_fused = True
        assert abs(L.item() - L_ref) < tol * abs(L_ref), fused
        for n in range(d):
            assert _relerr(facs[n].grad.cpu().numpy(), 0.5 * g_ref[n]) < gtol, (fused, n)
        results.append((L.item(), [f.grad.cpu().numpy() for f in facs]))
    assert abs(results[0][0] - results[1][0]) < tol * abs(L_ref)
    for n in range(d):
        assert _relerr(results[0][1][n], results[1][1][n]) < gtol, n


def test_gcp_fused_gradcheck_fp64(gpu):
    import paper_1809_09175_amd as spt
    X, A = datagen.gcp_counts(scale=6e-7, dims=(9, 7, 5), R=3)
    X.vals = X.vals.astype(np.float64)
    T = _dev_tensor(X, np.float64)
    T.permute()
    facs = tuple(torch.from_numpy(a.astype(np.float64)).cuda().requires_grad_(True) for a in A)
    assert torch.autograd.gradcheck(lambda *f: spt.GCPPoissonLoss.apply(T, None, *f), facs,
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


def test_gcp_fused_abi_edges(gpu):
    """Through the C ABI: a tune with 64-entry wave chunks (the loss pass lengthens them so its
    partials fit the tensor's scratch), ragged tiny tensors, the upstream scale, and the
    refusal of an unpermuted tensor."""
    import paper_1809_09175_amd as spt
    from paper_1809_09175_amd import _lib
    lib = _lib.load()
    for P, chunk in ((1, 0), (63, 0), (65, 64), (600_001, 64)):
        dims = (700, 900, 1100)
        rng = np.random.default_rng(P)
        lin = np.unique(rng.integers(0, int(np.prod(dims)), size=P + P // 8 + 16))[:P]
        assert lin.size == P
        lin = lin[rng.permutation(P)]
        subs = np.stack(np.unravel_index(lin, dims), axis=1).astype(np.int32)
        vals = rng.poisson(1.5, size=P).astype(np.float32)
        A = [(rng.random((I, 8)) * 0.5).astype(np.float32) for I in dims]
        T = spt.SparseTensor(torch.from_numpy(subs).cuda(), torch.from_numpy(vals).cuda(), dims)
        facs = [torch.from_numpy(a).cuda() for a in A]
        grads = [torch.empty_like(f) for f in facs]
        loss = torch.empty((), dtype=torch.float64, device="cuda")
        g = torch.tensor(2.0, dtype=torch.float64, device="cuda")
        tune = spt._tune("auto", 0, 0, chunk)
        args = (T.handle, 8, spt._factor_ptrs(facs), _lib.SPT_F32, 0,
                ctypes.c_void_p(loss.data_ptr()), _lib.ptr_array([t.data_ptr() for t in grads]),
                ctypes.c_void_p(g.data_ptr()), ctypes.byref(tune), None)
        assert lib.spt_gcp_fused(*args) == _lib.SPT_ESTATE
        T.permute()
        assert lib.spt_gcp_fused(*args) == 0
        torch.cuda.synchronize()
        L_ref, g_ref = oracle.gcp(subs, vals, dims, [a.astype(np.float64) for a in A])
        assert abs(loss.item() - L_ref) < 1e-5 * abs(L_ref), P
        for n in range(3):
            assert _relerr(grads[n].cpu().numpy(), 2.0 * g_ref[n]) < 1e-4, (P, n)
