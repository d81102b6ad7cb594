"""Pins for the FP64 CPU oracle: each check is an independent route to the same number
(brute force, closed forms, textbook library routines, invariants), never the oracle's own
formula typed again.  CPU only."""
import itertools
import math

import numpy as np
import pytest

import oracle


def _rand_coo(rng, dims, P, dup=True, vals="normal"):
    subs = np.stack([rng.integers(0, I, size=P) for I in dims], axis=1).astype(np.int32)
    if dup and P >= 4:
        subs[P // 2] = subs[0]          # force repeated coordinates
        subs[P // 2 + 1] = subs[1]
    v = rng.standard_normal(P) if vals == "normal" else rng.random(P)
    return subs, v


def _dense(subs, vals, dims):
    X = np.zeros(dims)
    np.add.at(X, tuple(subs[:, m] for m in range(len(dims))), vals)
    return X


def _unfold(X, n):
    """Mode-n unfolding: rows = mode n, columns = remaining modes in increasing order, the
    last one varying fastest."""
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def _khatri_rao(mats):
    """Column-wise Kronecker product, first matrix's index slowest (matches _unfold)."""
    R = mats[0].shape[1]
    cols = []
    for j in range(R):
        c = np.ones(1)
        for M in mats:
            c = np.kron(c, M[:, j])
        cols.append(c)
    return np.stack(cols, axis=1)


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ------------------------------------------------------------------------------------- MTTKRP

@pytest.mark.parametrize("dims", [(4, 5, 6), (3, 2, 5, 4), (6, 1, 3), (2, 3, 2, 2, 3)])
@pytest.mark.parametrize("R", [1, 3, 7])
def test_mttkrp_brute_force(dims, R):
    rng = np.random.default_rng(sum(dims) * 10 + R)
    subs, vals = _rand_coo(rng, dims, 40)
    A = [rng.standard_normal((I, R)) for I in dims]
    lam = rng.standard_normal(R)
    X = _dense(subs, vals, dims)
    for n in range(len(dims)):
        others = [A[m] for m in range(len(dims)) if m != n]
        ref = _unfold(X, n) @ _khatri_rao(others) @ np.diag(lam)
        got = oracle.mttkrp(subs, vals, dims, A, n, lam)
        assert _relerr(got, ref) < 1e-13
        got1 = oracle.mttkrp(subs, vals, dims, A, n)         # lambda omitted = ones
        ref1 = _unfold(X, n) @ _khatri_rao(others)
        assert _relerr(got1, ref1) < 1e-13


def test_mttkrp_rank1_closed_form():
    rng = np.random.default_rng(7)
    dims = (5, 4, 3)
    a, b, c = (rng.random(I) + 0.5 for I in dims)
    cells = np.array(list(itertools.product(*[range(I) for I in dims])), dtype=np.int32)
    vals = a[cells[:, 0]] * b[cells[:, 1]] * c[cells[:, 2]]
    R = 4
    A = [rng.standard_normal((I, R)) for I in dims]
    lam = rng.random(R) + 0.1
    vecs = (a, b, c)
    for n in range(3):
        got = oracle.mttkrp(cells, vals, dims, A, n, lam)
        ref = np.outer(vecs[n], lam)
        for m in range(3):
            if m != n:
                ref = ref * (vecs[m] @ A[m])[None, :]
        assert _relerr(got, ref) < 1e-13


def test_mttkrp_two_way_is_sparse_matrix_product():
    rng = np.random.default_rng(3)
    dims = (7, 9)
    subs, vals = _rand_coo(rng, dims, 30)
    A = [rng.standard_normal((I, 5)) for I in dims]
    X = _dense(subs, vals, dims)
    assert _relerr(oracle.mttkrp(subs, vals, dims, A, 0), X @ A[1]) < 1e-14
    assert _relerr(oracle.mttkrp(subs, vals, dims, A, 1), X.T @ A[0]) < 1e-14


def test_mttkrp_linear_duplicates_and_order():
    rng = np.random.default_rng(11)
    dims = (6, 5, 4)
    subs, x = _rand_coo(rng, dims, 50)
    y = rng.standard_normal(50)
    A = [rng.standard_normal((I, 3)) for I in dims]
    for n in range(3):
        vx = oracle.mttkrp(subs, x, dims, A, n)
        vy = oracle.mttkrp(subs, y, dims, A, n)
        vxy = oracle.mttkrp(subs, 2.0 * x - 0.5 * y, dims, A, n)
        assert _relerr(vxy, 2.0 * vx - 0.5 * vy) < 1e-13
        split = oracle.mttkrp(np.concatenate([subs, subs]), np.concatenate([x, x]) * 0.5,
                              dims, A, n)
        assert _relerr(split, vx) < 1e-14
        p = rng.permutation(50)
        assert _relerr(oracle.mttkrp(subs[p], x[p], dims, A, n), vx) < 1e-14


def test_mttkrp_empty_and_errors():
    dims = (3, 4, 5)
    A = [np.ones((I, 2)) for I in dims]
    V = oracle.mttkrp(np.zeros((0, 3), np.int32), np.zeros(0), dims, A, 1)
    assert V.shape == (4, 2) and not V.any()
    with pytest.raises(oracle.OracleError):
        oracle.mttkrp(np.array([[0, 4, 0]], np.int32), np.ones(1), dims, A, 0)
    with pytest.raises(oracle.OracleError):
        oracle.mttkrp(np.array([[0, -1, 0]], np.int32), np.ones(1), dims, A, 0)


# ----------------------------------------------------------------------------------- permutation

@pytest.mark.parametrize("I", [1, 3, 17, 1000])
def test_perm_matches_stable_argsort(I):
    rng = np.random.default_rng(I)
    dims = (I, 5, 9)
    subs = np.stack([rng.integers(0, D, size=5000) for D in dims], axis=1).astype(np.int32)
    for n in range(3):
        p, k = oracle.perm(subs, dims, n)
        ref = np.argsort(subs[:, n], kind="stable")
        assert np.array_equal(p, ref)
        assert np.array_equal(k, subs[ref, n])
        assert np.array_equal(np.sort(p), np.arange(5000))   # bijection
        assert np.all(np.diff(k) >= 0)                        # keys non-decreasing
        # stability: equal keys appear in storage order
        same = np.diff(k) == 0
        assert np.all(np.diff(p)[same] > 0)


# ------------------------------------------------------------------------- model, fit, gram

def test_model_values_and_gram_match_dense():
    rng = np.random.default_rng(5)
    dims = (4, 3, 5)
    R = 3
    A = [rng.standard_normal((I, R)) for I in dims]
    lam = rng.random(R)
    M = np.einsum("r,ir,jr,kr->ijk", lam, *A)
    cells = np.array(list(itertools.product(*[range(I) for I in dims])), dtype=np.int32)
    m = oracle.model_values(cells, dims, A, lam)
    assert _relerr(m, M[cells[:, 0], cells[:, 1], cells[:, 2]]) < 1e-14
    assert _relerr(oracle.gram(A[0]), A[0].T @ A[0]) < 1e-15


def test_fit_matches_brute_force_residual():
    rng = np.random.default_rng(9)
    dims = (6, 5, 4)
    cells = rng.choice(int(np.prod(dims)), size=60, replace=False)
    subs = np.stack(np.unravel_index(cells, dims), axis=1).astype(np.int32)
    vals = rng.random(60)
    R = 2
    A = [rng.random((I, R)) for I in dims]
    lam = rng.random(R)
    X = _dense(subs, vals, dims)
    M = np.einsum("r,ir,jr,kr->ijk", lam, *A)
    ref = 1.0 - np.linalg.norm(X - M) / np.linalg.norm(X)
    f, parts = oracle.fit(subs, vals, dims, A, lam, return_parts=True)
    assert abs(f - ref) < 1e-12
    assert abs(parts[0] - np.sum(X * X)) < 1e-12 * parts[0]
    assert abs(parts[1] - np.sum(X * M)) < 1e-12 * abs(parts[1])
    assert abs(parts[2] - np.sum(M * M)) < 1e-12 * parts[2]


# ----------------------------------------------------------------------------------- CP-ALS

def _state(A):
    lam = np.ones(A[0].shape[1])
    G = np.stack([a.T @ a for a in A])
    return lam, G


def test_cp_als_mode_solves_normal_equations_and_matches_lstsq():
    rng = np.random.default_rng(21)
    dims = (7, 6, 5)
    cells = rng.choice(int(np.prod(dims)), size=120, replace=False)
    subs = np.stack(np.unravel_index(cells, dims), axis=1).astype(np.int32)
    vals = rng.random(120)
    R = 3
    A = [rng.random((I, R)) for I in dims]
    lam, G = _state(A)
    X = _dense(subs, vals, dims)
    for n in range(3):
        A2, lam2, G2 = oracle.cp_als_mode(subs, vals, dims, A, lam, G, n)
        others = [A[m] for m in range(3) if m != n]
        KR = _khatri_rao(others)
        # independent route: dense least squares  min || X_(n) - B KR^T ||
        B = np.linalg.lstsq(KR, _unfold(X, n).T, rcond=None)[0].T
        nrm = np.linalg.norm(B, axis=0)
        assert _relerr(lam2, nrm) < 1e-10
        assert _relerr(A2[n], B / nrm) < 1e-10
        assert np.allclose(np.linalg.norm(A2[n], axis=0), 1.0, atol=1e-14)
        assert _relerr(G2[n], A2[n].T @ A2[n]) < 1e-14
        for m in range(3):                 # other modes untouched
            if m != n:
                assert np.array_equal(A2[m], A[m]) and np.array_equal(G2[m], G[m])


def _dense_fit(X, A, lam):
    M = np.einsum("r,ir,jr,kr->ijk", lam, *A)
    return 1.0 - np.linalg.norm(X - M) / np.linalg.norm(X)


@pytest.mark.parametrize("start", ["near", "random"])
def test_cp_als_recovers_exact_low_rank(start):
    rng = np.random.default_rng(31)
    dims = (12, 10, 8)
    R = 3
    T = [rng.standard_normal((I, R)) for I in dims]
    X = np.einsum("ir,jr,kr->ijk", *T)
    cells = np.array(list(itertools.product(*[range(I) for I in dims])), dtype=np.int32)
    vals = X[cells[:, 0], cells[:, 1], cells[:, 2]]
    if start == "near":
        A = [t + 1e-2 * rng.standard_normal(t.shape) for t in T]
    else:
        A = [rng.standard_normal(t.shape) for t in T]
    lam, G = _state(A)
    prev = -np.inf
    fit = None
    for it in range(2000):
        A, lam, G = oracle.cp_als_sweep(cells, vals, dims, A, lam, G)
        fit = _dense_fit(X, A, lam)
        assert fit >= prev - 1e-12, f"fit decreased at sweep {it}: {prev} -> {fit}"
        if fit - prev < 1e-15 and fit > 1 - 1e-10:
            break
        prev = fit
    assert fit > 1.0 - 1e-10


def test_cp_als_singular_gram_reported():
    dims = (4, 3, 3)
    cells = np.array(list(itertools.product(*[range(I) for I in dims])), dtype=np.int32)
    vals = np.ones(len(cells))
    A = [np.ones((I, 2)) for I in dims]      # two identical columns: Gamma is rank one
    lam, G = _state(A)
    with pytest.raises(oracle.OracleError, match="singular"):
        oracle.cp_als_mode(cells, vals, dims, A, lam, G, 0)


# -------------------------------------------------------------------------------------- GCP

def test_gcp_poisson_loss_dense_and_gradient_finite_differences():
    rng = np.random.default_rng(41)
    dims = (5, 4, 3)
    cells = rng.choice(int(np.prod(dims)), size=30, replace=False)
    subs = np.stack(np.unravel_index(cells, dims), axis=1).astype(np.int32)
    vals = rng.poisson(2.0, size=30).astype(np.float64)
    w = rng.random(30) + 0.5
    R = 2
    A = [0.5 * rng.random((I, R)) for I in dims]
    loss, grads = oracle.gcp_poisson(subs, vals, dims, A, w)
    M = np.einsum("ir,jr,kr->ijk", *A)[subs[:, 0], subs[:, 1], subs[:, 2]]
    assert abs(loss - np.sum(w * (np.exp(M) - vals * M))) < 1e-12 * abs(loss)
    for n in range(3):
        for (k, j) in [(0, 0), (dims[n] - 1, 1), (1, 0)]:
            h = 1e-6 * max(1.0, abs(A[n][k, j]))
            Ap = [a.copy() for a in A]
            Am = [a.copy() for a in A]
            Ap[n][k, j] += h
            Am[n][k, j] -= h
            fd = (oracle.gcp_poisson(subs, vals, dims, Ap, w, grads=False)
                  - oracle.gcp_poisson(subs, vals, dims, Am, w, grads=False)) / (2 * h)
            assert abs(fd - grads[n][k, j]) < 1e-7 * max(1.0, abs(fd))


# ------------------------------------------------------------------------------------- BF16

def _torch_bf16_bits(bits):
    import torch
    t = torch.from_numpy(bits.view(np.float32).copy()).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def test_bf16_rne_matches_torch_on_samples_and_boundaries():
    rng = np.random.default_rng(51)
    rnd = rng.integers(0, 1 << 32, size=1 << 21, dtype=np.uint64).astype(np.uint32)
    hi = np.arange(0, 1 << 16, dtype=np.uint32) << 16
    edges = np.concatenate([hi | 0x8000, hi | 0x7FFF, hi | 0x8001, hi, hi | 0xFFFF])
    bits = np.concatenate([rnd, edges])
    f = bits.view(np.float32)
    finite = ~np.isnan(f)
    got = oracle.bf16_rne(bits)
    ref = _torch_bf16_bits(bits)
    assert np.array_equal(got[finite], ref[finite])
    nan_bits = bits[~finite]
    g = got[~finite]
    assert np.all((g & 0x7F80) == 0x7F80) and np.all(g & 0x0040)      # still NaN, quiet
    assert np.array_equal(g >> 15, (nan_bits >> 31).astype(np.uint16))  # sign kept
    # ties go to the even neighbour: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7
    assert oracle.bf16_rne(np.array([0x3F808000], np.uint32))[0] == 0x3F80
    assert oracle.bf16_rne(np.array([0x3F818000], np.uint32))[0] == 0x3F82
    # largest finite FP32 rounds to infinity; the largest finite BF16 stays
    assert oracle.bf16_rne(np.array([0x7F7FFFFF], np.uint32))[0] == 0x7F80
    assert oracle.bf16_rne(np.array([0x7F7F0000], np.uint32))[0] == 0x7F7F


def _bf16_table():
    """Every finite non-negative BF16 value as a double, indexed by its bit pattern
    (0x0000 .. 0x7f7f), followed by 2^128, the value that stands for infinity when rounding."""
    bits = (np.arange(0, 0x7F80, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)
    return np.concatenate([bits, [2.0 ** 128]])


def _bf16_nearest_exact(values):
    """Nearest BF16 pattern to each finite double by exact rational arithmetic over the table of
    all BF16 values: the two neighbours come from a search in the table, the distances are
    Fractions, a tie picks the even pattern."""
    from fractions import Fraction
    table = _bf16_table()
    out = []
    for v in values:
        a = abs(float(v))
        sign = 0x8000 if np.signbit(v) else 0
        if a >= 2.0 ** 128:
            out.append(sign | 0x7F80)
            continue
        i = int(np.searchsorted(table, a, side="right")) - 1
        if table[i] == a:
            out.append(sign | i)
            continue
        dlo = Fraction(a) - Fraction(float(table[i]))
        dhi = Fraction(float(table[i + 1])) - Fraction(a)
        k = i if dlo < dhi else i + 1 if dhi < dlo else (i if i % 2 == 0 else i + 1)
        out.append(sign | k)
    return np.array(out, dtype=np.uint16)


def _bf16_f64_cases(rng, n_random=6000):
    """Random doubles over the whole BF16 range (subnormals and overflow included), values at
    and one double-ulp beside every kind of BF16 midpoint, and the special values."""
    e = rng.integers(-150, 130, size=n_random)
    rnd = rng.random(n_random) * np.ldexp(1.0, e) * np.where(rng.random(n_random) < 0.5, -1, 1)
    table = _bf16_table()
    idx = rng.integers(0, 0x7F7F, size=3000)
    mids = (table[idx] + table[idx + 1]) / 2          # exact: one more bit than BF16 carries
    near = np.concatenate([mids, np.nextafter(mids, np.inf), np.nextafter(mids, -np.inf)])
    special = np.array([0.0, -0.0, np.inf, -np.inf, 2.0 ** 128, np.finfo(np.float64).max,
                        float(np.finfo(np.float32).max), 2.0 ** -134, 2.0 ** -133, 2.0 ** -150,
                        5e-324, 1.0 + 2.0 ** -8 + 2.0 ** -30, 1.0 + 2.0 ** -8])
    return np.concatenate([rnd, near, -near[:500], special])


def test_bf16_rne_f64_matches_exact_rounding_and_fp32_rounding():
    rng = np.random.default_rng(52)
    # 1. every double that is an FP32 value rounds as the FP32 rounding does
    bits = rng.integers(0, 1 << 32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    f = bits.view(np.float32)
    finite = ~np.isnan(f)
    assert np.array_equal(oracle.bf16_rne_f64(f[finite].astype(np.float64)),
                          oracle.bf16_rne(bits[finite]))
    # 2. exact rational rounding over the table of every BF16 value
    v = _bf16_f64_cases(rng)
    assert np.array_equal(oracle.bf16_rne_f64(v), _bf16_nearest_exact(v))
    # 3. one rounding, not two: 1 + 2^-8 + 2^-30 lies above the midpoint 1 + 2^-8, to which an
    # FP32 step would round it first (and the tie would then go down to 1)
    x = np.array([1.0 + 2.0 ** -8 + 2.0 ** -30])
    assert oracle.bf16_rne_f64(x)[0] == 0x3F81
    assert oracle.bf16_rne(x.astype(np.float32))[0] == 0x3F80
    # 4. NaN: quiet, sign kept
    nan = np.array([np.nan, -np.nan, np.frombuffer(np.uint64(0x7FF0000000000001).tobytes(), np.float64)[0]])
    got = oracle.bf16_rne_f64(nan)
    assert list(got) == [0x7FC0, 0xFFC0, 0x7FC0]


@pytest.mark.parametrize("loss", ["poisson", "bernoulli", "gaussian", "gamma"])
def test_gcp_losses_dense_and_finite_differences(loss):
    rng = np.random.default_rng(43)
    dims = (5, 4, 3)
    cells = rng.choice(int(np.prod(dims)), size=30, replace=False)
    subs = np.stack(np.unravel_index(cells, dims), axis=1).astype(np.int32)
    vals = (rng.random(30) < 0.5).astype(np.float64) if loss == "bernoulli" else rng.random(30) * 3
    w = rng.random(30) + 0.5
    R = 2
    # the Gamma model is a positive mean: nonnegative factors, kept away from m = 0
    A = [rng.random((I, R)) + (0.2 if loss == "gamma" else -0.3) for I in dims]
    L, grads = oracle.gcp(subs, vals, dims, A, loss, w)
    M = np.einsum("ir,jr,kr->ijk", *A)[subs[:, 0], subs[:, 1], subs[:, 2]]
    f = {"poisson": lambda: np.exp(M) - vals * M,
         "bernoulli": lambda: np.logaddexp(0.0, M) - vals * M,
         "gaussian": lambda: (vals - M) ** 2,
         "gamma": lambda: vals / (M + 1e-10) + np.log(M + 1e-10)}[loss]()
    assert abs(L - np.sum(w * f)) < 1e-12 * abs(L)
    if loss == "gaussian":
        # d/dA of sum w (x - m)^2 = MTTKRP of 2 w (m - x): check against a dense route
        Y = np.zeros(dims)
        np.add.at(Y, (subs[:, 0], subs[:, 1], subs[:, 2]), 2 * w * (M - vals))
        ref0 = np.einsum("ijk,jr,kr->ir", Y, A[1], A[2])
        assert np.linalg.norm(grads[0] - ref0) < 1e-12 * np.linalg.norm(ref0)
    for n in range(3):
        for (k, j) in [(0, 0), (dims[n] - 1, 1)]:
            h = 1e-6
            Ap = [a.copy() for a in A]
            Am = [a.copy() for a in A]
            Ap[n][k, j] += h
            Am[n][k, j] -= h
            fd = (oracle.gcp(subs, vals, dims, Ap, loss, w, grads=False)
                  - oracle.gcp(subs, vals, dims, Am, loss, w, grads=False)) / (2 * h)
            assert abs(fd - grads[n][k, j]) < 1e-7 * max(1.0, abs(fd))


# ------------------------------------------------------------------ stochastic generalized CP

def test_philox_matches_numpy_philox():
    """The oracle's Philox4x64-10 block equals numpy's independent implementation of the
    published generator (numpy advances its counter before each block)."""
    for key, ctr in [((5, 0), (1, 0, 0, 0)), ((2**63 + 11, 77), (9, 3, 1, 0)),
                     ((0, 0), (2**40, 2**33, 1, 1)), ((123456789, 0), (65537, 0, 0, 5))]:
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array((ctr[0] - 1,) + ctr[1:], dtype=np.uint64))
        assert list(oracle.philox4x64(ctr, key)) == list(bg.random_raw(4)), (key, ctr)


def test_gcp_sample_is_unbiased_and_uniform():
    """Stratified sample: every nonzero sample is a stored entry (value and subscripts), zero
    samples are uniform cells with value 0, and the weighted sample loss is an unbiased estimate
    of the loss over every cell of the tensor (mean over many iterations within 4 standard
    errors of the dense value)."""
    rng = np.random.default_rng(3)
    dims = (6, 5, 4)
    cells = rng.choice(120, size=25, replace=False)
    subs = np.stack(np.unravel_index(cells, dims), axis=1).astype(np.int32)
    vals = rng.random(25) * 3 + 0.5
    A = [rng.random((I, 2)) * 0.5 for I in dims]
    dense = np.einsum("ir,jr,kr->ijk", *A)
    X = np.zeros(dims)
    X[tuple(subs.T)] = vals
    full = np.sum(np.exp(dense) - X * dense)          # Poisson loss over every cell
    est = []
    counts_nz = np.zeros(25)
    counts_z = np.zeros(dims)
    key_rows = {tuple(r): i for i, r in enumerate(subs)}
    for it in range(400):
        s, v, w = oracle.gcp_sample(subs, vals, dims, 99, it, 16, 32)
        for k in range(16):
            i = key_rows[tuple(s[k])]
            assert v[k] == vals[i]
            counts_nz[i] += 1
        assert np.all(v[16:] == 0.0)
        np.add.at(counts_z, tuple(s[16:].T), 1)
        m = dense[tuple(s.T)]
        est.append(np.sum(w * (np.exp(m) - v * m)))
    assert np.allclose(w[:16], 25 / 16) and np.allclose(w[16:], (120 - 25) / 32)
    est = np.array(est)
    assert abs(est.mean() - full) < 4 * est.std() / np.sqrt(len(est))
    # uniformity: chi-square statistics far below what a wrong mapping would give
    e_nz = counts_nz.sum() / 25
    assert np.sum((counts_nz - e_nz) ** 2 / e_nz) < 25 + 6 * np.sqrt(2 * 25)
    e_z = counts_z.sum() / 120
    assert np.sum((counts_z - e_z) ** 2 / e_z) < 120 + 6 * np.sqrt(2 * 120)
    # deterministic per (seed, iteration); another iteration draws another sample
    a = oracle.gcp_sample(subs, vals, dims, 99, 7, 16, 32)[0]
    assert np.array_equal(a, oracle.gcp_sample(subs, vals, dims, 99, 7, 16, 32)[0])
    assert not np.array_equal(a, oracle.gcp_sample(subs, vals, dims, 99, 8, 16, 32)[0])


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2 at every
    step, so x_t = x_0 - t lr g / (|g| + eps); the lower bound clamps."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    x = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in range(1, 31):
        oracle.adam(x, g, m, v, lr, 0.9, 0.999, eps, t)
        ref = 1.0 - t * lr * g / (np.abs(g) + eps)
        assert np.allclose(x, ref, rtol=0, atol=1e-12), t
    x = np.array([0.005, 1.0])
    m = np.zeros(2)
    v = np.zeros(2)
    oracle.adam(x, np.array([1.0, 1.0]), m, v, 0.01, 0.9, 0.999, 1e-8, 1, lower=0.0)
    assert x[0] == 0.0 and abs(x[1] - 0.99) < 1e-9
