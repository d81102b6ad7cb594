"""GPU parity of the permutation build and both MTTKRP kernels against the FP64 CPU oracle,
through the C ABI.  Tolerances (relative Frobenius error of V): 1e-12 for FP64, 1e-5 for FP32,
2e-2 for BF16 factors against the unrounded FP64 factors."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1809_09175_amd import datagen

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


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


def _factors(dims, R, seed, kind):
    A64 = datagen.factors(dims, R, seed, np.float64)
    if kind == "f64":
        dev = [torch.from_numpy(a).cuda() for a in A64]
        ref = A64
    elif kind == "f32":
        a32 = [a.astype(np.float32) for a in A64]
        dev = [torch.from_numpy(a).cuda() for a in a32]
        ref = [a.astype(np.float64) for a in a32]
    else:
        a32 = [a.astype(np.float32) for a in A64]
        import paper_1809_09175_amd as spt
        dev = [spt.to_bf16(torch.from_numpy(a).cuda()) for a in a32]   # the library's rounding
        ref = [a.astype(np.float64) for a in a32]          # unrounded factors
    return dev, ref


def _small(kind, dims, nnz, skew, seed):
    X = datagen.skewed_tensor(dims, nnz, skew, seed)
    if kind == "f64":
        X.vals = X.vals.astype(np.float64)
    return X


# --------------------------------------------------------------------------------- permutation

@pytest.mark.parametrize("dims,nnz,skew", [
    ((1, 7, 300), 1000, (0.0, 1.1, 1.1)),
    ((200, 3000, 70000), 50_001, (1.1, 1.1, 0.0)),
    ((2, 5_000_000, 17), 200_003, (0.0, 1.2, 0.0)),
    ((65536, 256, 257), 131_072, (0.0, 0.0, 0.0)),
])
def test_permutation_bit_exact(gpu, dims, nnz, skew):
    _log(f"perm dims={dims} nnz={nnz}")
    X = datagen.skewed_tensor(dims, nnz, skew, seed=nnz)
    T = _dev_tensor(X, np.float32)
    T.permute()
    torch.cuda.synchronize()
    for n in range(3):
        p_ref, k_ref = oracle.perm(X.subs, X.dims, n)
        p, k = T.perm(n)
        assert np.array_equal(p.cpu().numpy(), p_ref)
        assert np.array_equal(k.cpu().numpy(), k_ref)


@pytest.mark.parametrize("vdt,d,pinned,chunk", [(np.float32, 3, True, 16384),
                                                (np.float32, 3, False, 8192),
                                                (np.float64, 4, True, 24576)])
def test_chunked_ingest_matches_whole(gpu, vdt, d, pinned, chunk):
    """A tensor ingested chunk by chunk from host memory (copies on their own stream overlapping
    the packing, first radix digit counted while packing) has the same permutations (bit-exact,
    against the oracle) and the same deterministic MTTKRP, bit for bit, as one packed whole; a
    ragged last chunk."""
    import paper_1809_09175_amd as spt
    dims = (700, 5000, 90, 40)[:d]
    X = datagen.skewed_tensor(dims, 5 * 8192 + 1237, (1.1,) * d, seed=17)
    X.vals = X.vals.astype(vdt)
    T1 = _dev_tensor(X, vdt)
    hs, hv = torch.from_numpy(X.subs), torch.from_numpy(X.vals)
    if pinned:
        hs, hv = hs.pin_memory(), hv.pin_memory()
    T2 = spt.SparseTensor.from_host(hs, hv, X.dims, chunk=chunk)
    T2.validate()
    for T in (T1, T2):
        T.permute()
    torch.cuda.synchronize()
    kind = "f64" if vdt == np.float64 else "f32"
    dev, _ = _factors(dims, 16, seed=3, kind=kind)
    for n in range(d):
        p_ref, k_ref = oracle.perm(X.subs, X.dims, n)
        for T in (T1, T2):
            p, k = T.perm(n)
            assert np.array_equal(p.cpu().numpy(), p_ref), n
            assert np.array_equal(k.cpu().numpy(), k_ref), n
        a = spt.mttkrp(T1, dev, n, algo="permuted", deterministic=True)
        b = spt.mttkrp(T2, dev, n, algo="permuted", deterministic=True)
        torch.cuda.synchronize()
        assert torch.equal(a, b), n


def test_chunked_ingest_errors(gpu):
    """Appends out of order or off the 8192-entry grid are refused; calls that read the entries
    wait for the last chunk; a bad subscript in a later chunk is reported with its global
    index."""
    import ctypes
    import paper_1809_09175_amd as spt
    from paper_1809_09175_amd import _lib
    lib = _lib.load()
    P = 3 * 8192 + 5
    dims = (50, 60, 70)
    X = datagen.skewed_tensor(dims, P, (0.0, 0.0, 0.0), seed=2)
    X.subs[2 * 8192 + 3, 1] = 60          # out of range, in the last chunk
    subs = torch.from_numpy(X.subs).cuda()
    vals = torch.from_numpy(X.vals).cuda()
    dims_arr = (ctypes.c_int64 * 3)(*dims)
    nbytes = lib.spt_tensor_workspace_bytes(3, dims_arr, P, 1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    assert lib.spt_tensor_create_begin(ctypes.byref(h), 3, dims_arr, P, 1,
                                       ctypes.c_void_p(ws.data_ptr()), nbytes, None) == 0

    def app(first, count):
        return lib.spt_tensor_append(h, first, count,
                                     ctypes.c_void_p(subs[first:].data_ptr()),
                                     ctypes.c_void_p(vals[first:].data_ptr()), None)
    assert app(100, 8192) == -1            # off the grid
    assert app(0, 5000) == -1              # short chunk that does not end the tensor
    assert app(8192, 8192) == -7           # out of order
    assert app(0, 8192) == 0
    assert lib.spt_tensor_permute(h, -1, None) == -7   # entries still missing
    assert app(8192, 2 * 8192 + 5) == 0
    bad = ctypes.c_int64()
    assert lib.spt_tensor_validate(h, ctypes.byref(bad), None) == -2
    assert bad.value == 2 * 8192 + 3
    assert lib.spt_tensor_destroy(h) == 0


def test_permutation_empty(gpu):
    X = datagen.CooTensor(np.zeros((0, 3), np.int32), np.zeros(0, np.float32), (4, 5, 6))
    T = _dev_tensor(X, np.float32)
    T.permute()
    torch.cuda.synchronize()
    assert T.perm(0)[0].numel() == 0


# ------------------------------------------------------------------------------------- MTTKRP

CASES = [
    # (kind, dims, nnz, skew, R)
    ("f32", (500, 400, 30), 100_000, (1.1, 1.1, 1.1), 32),
    ("f32", (500, 400, 30), 77_777, (1.1, 1.1, 1.1), 16),
    ("f32", (3000, 20, 9), 50_001, (1.2, 0.0, 1.1), 64),
    ("f32", (100, 90, 80), 20_000, (0.0, 0.0, 0.0), 7),
    ("f32", (50, 60, 70, 8), 40_000, (1.2, 1.2, 0.0, 0.0), 32),
    ("f32", (40, 30, 20, 10, 5), 30_000, (1.1, 0.0, 0.0, 0.0, 0.0), 24),
    ("f32", (300, 200), 10_000, (1.1, 1.1), 48),
    ("f32", (1000, 1000, 1000), 60_000, (1.1, 1.1, 1.1), 128),
    ("f32", (1000, 1000, 1000), 30_000, (1.1, 1.1, 1.1), 98),
    ("f32", (200, 150, 100), 30_000, (1.1, 1.1, 1.1), 256),
    ("f64", (100, 80, 60), 10_000, (0.0, 0.0, 0.0), 16),
    ("f64", (500, 400, 30), 50_000, (1.1, 1.1, 1.1), 32),
    ("f64", (60, 50, 40, 30), 20_000, (1.1, 0.0, 1.1, 0.0), 64),
    ("bf16", (500, 400, 30), 100_000, (1.1, 1.1, 1.1), 32),
    ("bf16", (3000, 20, 9), 50_001, (1.2, 0.0, 1.1), 64),
    ("bf16", (100, 90, 80), 20_000, (0.0, 0.0, 0.0), 9),
    ("bf16", (1000, 1000, 1000), 60_000, (1.1, 1.1, 1.1), 128),
    ("bf16", (1000, 1000, 1000), 30_000, (1.1, 1.1, 1.1), 72),
    # the smallest ranks: one column (most lanes of a group idle), two, three
    ("f32", (500, 400, 30), 30_001, (1.1, 1.1, 1.1), 1),
    ("bf16", (500, 400, 30), 30_001, (1.1, 1.1, 1.1), 2),
    ("f64", (300, 200, 100), 20_000, (1.1, 0.0, 0.0), 3),
]


@pytest.mark.parametrize("algo", ["atomic", "permuted", "permuted_copy"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-d{len(c[1])}-R{c[4]}-P{c[2]}" for c in CASES])
def test_mttkrp_parity(gpu, case, algo):
    """Every case against the oracle: the atomic kernel, the permuted kernel gathering through
    the permutation, and the permuted kernel over mode-sorted record copies (second-mode order
    within rows, the default), at a short and a long wave chunk."""
    import paper_1809_09175_amd as spt
    kind, dims, nnz, skew, R = case
    _log(f"mttkrp {kind} dims={dims} nnz={nnz} R={R} algo={algo}")
    X = _small(kind, dims, nnz, skew, seed=nnz + R)
    T = _dev_tensor(X, np.float64 if kind == "f64" else np.float32)
    T.permute()
    if algo == "permuted_copy":
        T.sort_copy()
    dev, ref = _factors(dims, R, seed=R, kind=kind)
    lam = np.linspace(0.5, 1.5, R)
    lam_d = torch.from_numpy(lam).cuda()
    for n in range(len(dims)):
        V_ref = oracle.mttkrp(X.subs, X.vals, dims, ref, n, lam)
        for chunk in (64, 2048):
            V = spt.mttkrp(T, dev, n, lam=lam_d, algo=algo, chunk=chunk)
            torch.cuda.synchronize()
            err = _relerr(V.cpu().numpy(), V_ref)
            assert err < TOL[kind], (n, chunk, err)


def _configs_for(R, kind):
    out = []
    for lanes, cols in [(4, 4), (4, 8), (8, 1), (8, 2), (8, 4), (8, 8), (16, 1), (16, 2),
                        (16, 4), (16, 8), (32, 1), (32, 2), (32, 4), (32, 8), (64, 1), (64, 2),
                        (64, 4)]:
        if lanes * cols >= R and R % cols == 0:
            out.append((lanes, cols))
    return out


@pytest.mark.parametrize("kind,R", [("f32", 16), ("f32", 32), ("bf16", 32), ("f64", 16)])
def test_mttkrp_every_lane_config(gpu, kind, R):
    import paper_1809_09175_amd as spt
    dims = (700, 500, 40)
    X = _small(kind, dims, 65_537, (1.1, 1.1, 1.1), seed=5)
    T = _dev_tensor(X, np.float64 if kind == "f64" else np.float32)
    T.permute()
    dev, ref = _factors(dims, R, seed=3, kind=kind)
    for n in range(3):
        V_ref = oracle.mttkrp(X.subs, X.vals, dims, ref, n)
        for lanes, cols in _configs_for(R, kind):
            for algo in ("atomic", "permuted"):
                _log(f"cfg {kind} R={R} n={n} lanes={lanes} cols={cols} {algo}")
                V = spt.mttkrp(T, dev, n, algo=algo, lanes=lanes, cols=cols, chunk=512)
                torch.cuda.synchronize()
                assert _relerr(V.cpu().numpy(), V_ref) < TOL[kind], (lanes, cols, algo)


def test_bf16_against_rounded_factors_is_fp32_tight(gpu):
    """With the factors the kernel actually sees (BF16 values widened exactly), only FP32
    accumulation separates kernel and oracle."""
    import paper_1809_09175_amd as spt
    dims = (500, 400, 30)
    X = _small("bf16", dims, 100_000, (1.1, 1.1, 1.1), seed=9)
    T = _dev_tensor(X, np.float32)
    T.permute()
    dev, _ = _factors(dims, 32, seed=4, kind="bf16")
    rounded = [d.float().cpu().numpy().astype(np.float64) for d in dev]
    for n in range(3):
        V_ref = oracle.mttkrp(X.subs, X.vals, dims, rounded, n)
        for algo in ("atomic", "permuted"):
            V = spt.mttkrp(T, dev, n, algo=algo)
            torch.cuda.synchronize()
            assert _relerr(V.cpu().numpy(), V_ref) < 1e-5


def test_mttkrp_edge_cases(gpu):
    import paper_1809_09175_amd as spt
    # empty tensor -> zeros
    X = datagen.CooTensor(np.zeros((0, 3), np.int32), np.zeros(0, np.float32), (4, 5, 6))
    T = _dev_tensor(X, np.float32)
    T.permute()
    dev, _ = _factors(X.dims, 8, 1, "f32")
    for algo in ("atomic", "permuted"):
        V = spt.mttkrp(T, dev, 1, algo=algo)
        torch.cuda.synchronize()
        assert V.shape == (5, 8) and not V.cpu().numpy().any()
    for order in ("storage", "second_mode"):
        T.sort_copy(order=order)  # zero bytes: a null workspace is accepted
        V = spt.mttkrp(T, dev, 1, algo="permuted_copy")
        torch.cuda.synchronize()
        assert V.shape == (5, 8) and not V.cpu().numpy().any()
    # a single entry, a mode of length one, replacement values
    X = datagen.CooTensor(np.array([[3, 0, 2]], np.int32), np.array([2.5], np.float32), (4, 1, 6))
    T = _dev_tensor(X, np.float32)
    T.permute()
    dev, ref = _factors(X.dims, 8, 2, "f32")
    y = torch.tensor([-1.0], device="cuda")
    for n in range(3):
        for algo in ("atomic", "permuted"):
            V = spt.mttkrp(T, dev, n, algo=algo)
            V2 = spt.mttkrp(T, dev, n, algo=algo, vals=y)
            torch.cuda.synchronize()
            assert _relerr(V.cpu().numpy(), oracle.mttkrp(X.subs, X.vals, X.dims, ref, n)) < 1e-6
            assert _relerr(V2.cpu().numpy(), oracle.mttkrp(X.subs, [-1.0], X.dims, ref, n)) < 1e-6


def test_errors_reported(gpu):
    import paper_1809_09175_amd as spt
    from paper_1809_09175_amd import SptError
    X = datagen.CooTensor(np.array([[0, 0, 0], [1, 7, 0]], np.int32),
                          np.ones(2, np.float32), (2, 5, 3))
    subs = torch.from_numpy(X.subs).cuda()
    vals = torch.from_numpy(X.vals).cuda()
    T = spt.SparseTensor(subs, vals, X.dims)
    with pytest.raises(SptError) as e:
        T.validate()
    assert e.value.code == -2 and "first bad entry 1" in str(e.value)
    X = datagen.CooTensor(np.array([[0, 0, 0]], np.int32), np.ones(1, np.float32), (2, 5, 3))
    T = _dev_tensor(X, np.float32)
    dev, _ = _factors(X.dims, 4, 1, "f32")
    with pytest.raises(SptError) as e:
        spt.mttkrp(T, dev, 0, algo="permuted")
    assert e.value.code == -7
    with pytest.raises(SptError) as e:
        spt.mttkrp(T, dev, 3, out=torch.empty(4, 4, device="cuda"))   # mode >= d
    assert e.value.code == -1
    with pytest.raises(SptError) as e:
        spt.mttkrp(T, [torch.empty(2, 300, device="cuda")] * 3, 0)     # R > 256
    assert e.value.code == -1
    dev64, _ = _factors(X.dims, 4, 1, "f64")
    with pytest.raises(SptError) as e:
        spt.mttkrp(T, dev64, 0)
    assert e.value.code == -6


def test_factor_matrices_of_4_gib_are_rejected(gpu):
    """Factor rows are addressed with 32-bit byte offsets: every call that gathers from a factor
    matrix of 4 GiB or more refuses it on the host (SPT_EUNSUPPORTED) before anything is
    enqueued.  Mode 1 has 2^24 rows, so R = 64 FP32 (or R = 128 BF16) makes A^(1) exactly 4 GiB;
    the factor pointers are small placeholders that no kernel ever reads."""
    import ctypes
    from paper_1809_09175_amd import _lib
    lib = _lib.load()
    X = datagen.CooTensor(np.array([[0, 5, 1], [3, (1 << 24) - 1, 2]], np.int32),
                          np.ones(2, np.float32), (4, 1 << 24, 3))
    T = _dev_tensor(X, np.float32)
    T.permute()
    buf = torch.zeros(1 << 16, device="cuda")
    p = buf.data_ptr()
    facs = _lib.ptr_array([p, p, p])
    out = ctypes.c_void_p(p)
    fit = ctypes.c_double()
    loss = ctypes.c_double()
    for R, fdt in ((64, _lib.SPT_F32), (128, _lib.SPT_BF16)):
        for n in (0, 2):
            for algo in (_lib.ALGO_ATOMIC, _lib.ALGO_PERMUTED):
                tune = _lib.SptTune(algo, 0, 0, 0, 0, 0)
                assert lib.spt_mttkrp(T.handle, n, R, facs, fdt, None, None, out,
                                      ctypes.byref(tune), None) == _lib.SPT_EUNSUPPORTED, (R, n)
    R, fdt = 64, _lib.SPT_F32
    assert lib.spt_cp_fit(T.handle, R, facs, fdt, out, out, out, 1 << 18, ctypes.byref(fit),
                          None, None) == _lib.SPT_EUNSUPPORTED
    assert lib.spt_model_values(T.handle, R, facs, fdt, None, out, None) == _lib.SPT_EUNSUPPORTED
    assert lib.spt_gcp_forward(T.handle, R, facs, fdt, 0, None, out, ctypes.byref(loss), out,
                               1 << 18, None) == _lib.SPT_EUNSUPPORTED
    assert lib.spt_gcp_fused(T.handle, R, facs, fdt, 0, ctypes.byref(loss),
                             _lib.ptr_array([p, p, p]), out, None, None) == _lib.SPT_EUNSUPPORTED
    # one row fewer fits: the same calls at R = 63 pass the extent check (not run here)
    assert (1 << 24) * 63 * 4 < (1 << 32) <= (1 << 24) * 64 * 4
    torch.cuda.synchronize()


# ------------------------------------------------------------------ full-size sampled parity

def _sampled_rows(X, n, rows):
    mask = np.isin(X.subs[:, n], rows)
    return X.subs[mask], X.vals[mask]


@pytest.fixture(scope="module")
def powerlaw3_full(gpu):
    """The 1e8-entry power-law tensor, generated once for the module: host arrays and a device
    tensor with FP32 values (permutations and second-mode record copies, as the benchmark
    builds them)."""
    _log("powerlaw3 full size: generating")
    X = datagen.powerlaw3()
    T = _dev_tensor(X, np.float32)
    T.permute()
    T.sort_copy()
    torch.cuda.synchronize()
    yield X, T
    del T
    torch.cuda.empty_cache()


# every configuration the benchmark line reports for this tensor: the ranks of its per-rank
# table (three algorithms each), the BF16-factor leg and the FP64 (the paper's arithmetic) leg
POWERLAW3_CASES = [
    ("f32", 16, ("atomic", "permuted", "permuted_copy", "auto")),
    ("f32", 32, ("atomic", "permuted", "permuted_copy", "auto")),
    ("f32", 64, ("atomic", "permuted", "permuted_copy", "auto")),
    ("f32", 128, ("auto",)),   # the MTTKRP of the CP-ALS sweep at R = 128 (32 x 4 layout)
    ("bf16", 16, ("auto",)),
    ("bf16", 32, ("auto",)),
    ("bf16", 64, ("auto",)),
    ("f64", 32, ("permuted", "auto")),
]


@pytest.mark.slow
@pytest.mark.parametrize("kind,R,algos", POWERLAW3_CASES,
                         ids=[f"{k}-R{r}" for k, r, _ in POWERLAW3_CASES])
def test_powerlaw3_full_size_sampled(gpu, powerlaw3_full, kind, R, algos):
    """The 1e8-entry power-law tensor in the benchmark's launch configurations (default layouts
    and chunks; "auto" is the timed path, the traversal over mode-sorted record copies):
    selected rows of V (the hottest row of each mode and a ragged set of random rows) against
    the oracle on exactly the entries that feed them, at the tolerance of the factor type (BF16
    against the unrounded factors).  FP64 uses a tensor with FP64 values (32-byte records)."""
    import paper_1809_09175_amd as spt
    X, T = powerlaw3_full
    if kind == "f64":
        _log("powerlaw3 full size: FP64-valued tensor")
        T = _dev_tensor(X, np.float64)
        T.permute()
        T.sort_copy()
    dev, ref = _factors(X.dims, R, seed=7, kind=kind)
    rng = np.random.default_rng(R)
    for n in range(3):
        counts = np.bincount(X.subs[:, n], minlength=X.dims[n])
        hot = int(np.argmax(counts))
        rows = np.unique(np.concatenate([[hot], rng.integers(0, X.dims[n], size=40)]))
        s, v = _sampled_rows(X, n, rows)
        _log(f"powerlaw3 {kind} R={R} n={n}: oracle on {len(v)} entries")
        V_ref = oracle.mttkrp(s, v, X.dims, ref, n)[rows]
        for algo in algos:
            _log(f"powerlaw3 {kind} R={R} n={n} {algo}")
            V = spt.mttkrp(T, dev, n, algo=algo)
            torch.cuda.synchronize()
            got = V[torch.from_numpy(rows).cuda()].cpu().numpy()
            assert _relerr(got, V_ref) < TOL[kind], (n, algo)
            # the hot row alone (the FP32 accuracy risk: 12.7% of all entries)
            assert _relerr(got[rows == hot], V_ref[rows == hot]) < TOL[kind], (n, algo)
    if kind == "f64":
        del T
        torch.cuda.empty_cache()


@pytest.mark.parametrize("kind,R,d", [("f32", 32, 3), ("f32", 16, 4), ("bf16", 32, 3), ("f64", 16, 3)])
def test_sorted_copy_matches_gathered(gpu, kind, R, d):
    """The storage-ordered record copy changes where records are read from, not the traversal:
    both kernels sum every row in the same order, so they agree to the rounding of the (at most
    two per wave chunk) boundary atomics, whose order is not fixed.  The second-mode copy sums
    each row in another order, so it agrees to rounding.  With and without replacement values
    (read through the copy's own order array), and every result matches the oracle."""
    import paper_1809_09175_amd as spt
    dims = (900, 700, 60, 30)[:d]
    X = _small(kind, dims, 70_001, (1.1,) * d, seed=77)
    T = _dev_tensor(X, np.float64 if kind == "f64" else np.float32)
    T.permute()
    dev, ref = _factors(dims, R, seed=5, kind=kind)
    vdt = np.float64 if kind == "f64" else np.float32
    yh = np.random.default_rng(1).standard_normal(X.nnz).astype(vdt)
    y = torch.from_numpy(yh).cuda()
    for order in ("storage", "second_mode"):
        T.sort_copy(order=order)
        for n in range(d):
            assert spt.default_tune(T, n, R, dev[0].dtype)["algo"] == "permuted_copy"
            for vals in (None, y):
                _log(f"sorted copy {kind} d={d} order={order} n={n} vals={vals is not None}")
                a = spt.mttkrp(T, dev, n, algo="permuted", vals=vals)
                b = spt.mttkrp(T, dev, n, algo="permuted_copy", vals=vals)
                torch.cuda.synchronize()
                if order == "storage":
                    tight = 1e-14 if kind == "f64" else 1e-6
                else:
                    tight = 1e-13 if kind == "f64" else 1e-5
                assert _relerr(a.cpu().numpy(), b.cpu().numpy().astype(np.float64)) < tight, n
                if vals is not None:
                    V_y = oracle.mttkrp(X.subs, yh.astype(np.float64), dims, ref, n)
                    assert _relerr(b.cpu().numpy(), V_y) < TOL[kind], (order, n)
            V_ref = oracle.mttkrp(X.subs, X.vals, dims, ref, n)
            assert _relerr(spt.mttkrp(T, dev, n).cpu().numpy(), V_ref) < TOL[kind]
    # re-permuting a mode drops its copy; the permuted-copy kernel then reports the state error
    from paper_1809_09175_amd import SptError
    T.permute(0)
    with pytest.raises(SptError) as e:
        spt.mttkrp(T, dev, 0, algo="permuted_copy")
    assert e.value.code == -7


@pytest.mark.parametrize("vdt,d,dims", [(np.float32, 3, (900, 700, 60)),
                                        (np.float32, 4, (50, 700, 700, 9)),
                                        (np.float64, 3, (5, 1, 3000)),
                                        (np.float64, 2, (1, 400))])
def test_second_mode_copy_order_is_exact(gpu, vdt, d, dims):
    """The second-mode copy of mode n holds the records ordered by (mode-n subscript, mode-m
    subscript, storage position), m the other mode with the most rows (lowest index among
    equals): bit-exact against a lexicographic sort on the host, record words included, for
    every mode at once (the copies laid back to back) and for one mode alone.  Covers a mode of
    size one (no radix pass: the order is perm_m itself) and duplicate coordinates."""
    import paper_1809_09175_amd as spt
    rng = np.random.default_rng(31)
    P = 40_003
    subs = np.stack([np.minimum(rng.zipf(1.3, size=P) - 1, I - 1) for I in dims], 1).astype(np.int32)
    subs[P // 2:P // 2 + 100] = subs[:100]  # duplicate coordinates
    vals = rng.standard_normal(P).astype(vdt)
    T = spt.SparseTensor(torch.from_numpy(subs).cuda(), torch.from_numpy(vals).cuda(), dims)
    T.permute()
    rw = 4 if d * 4 + vals.itemsize <= 16 else 8
    expect_rec = np.zeros((P, rw), np.int32)
    expect_rec[:, :d] = subs
    if vdt == np.float64:
        expect_rec[:, rw - 2:] = vals.view(np.int32).reshape(P, 2)
    else:
        expect_rec[:, rw - 1] = vals.view(np.int32)
    one = -(-P * rw * 4 // 256) * 256 + -(-P * 4 // 256) * 256
    for mode in (-1, d - 1):
        _log(f"second-mode copy order d={d} dims={dims} mode={mode}")
        T.sort_copy(mode, order="second_mode")
        torch.cuda.synchronize()
        buf = T._copies[mode].cpu().numpy()
        modes = range(d) if mode == -1 else [mode]
        assert buf.size == one * len(modes)
        for k, n in enumerate(modes):
            others = [m for m in range(d) if m != n]
            m2 = max(others, key=lambda m: (dims[m], -m))
            order = np.lexsort((np.arange(P), subs[:, m2], subs[:, n]))
            got = buf[k * one:k * one + P * rw * 4].view(np.int32).reshape(P, rw)
            assert np.array_equal(got, expect_rec[order]), (mode, n)
            qbase = k * one + -(-P * rw * 4 // 256) * 256
            q = buf[qbase:qbase + P * 4].view(np.int32)
            assert np.array_equal(q, order.astype(np.int32)), (mode, n)
    # the second mode must be permuted too
    T2 = spt.SparseTensor(torch.from_numpy(subs).cuda(), torch.from_numpy(vals).cuda(), dims)
    T2.permute(0)
    from paper_1809_09175_amd import SptError
    with pytest.raises(SptError) as e:
        T2.sort_copy(0, order="second_mode")
    assert e.value.code == -7
    T2.sort_copy(0, order="storage")


@pytest.mark.parametrize("kind,R,chunk", [("f32", 32, 64), ("f32", 16, 0), ("bf16", 32, 256),
                                          ("f64", 16, 64), ("f64", 256, 64)])
def test_deterministic_permuted_is_reproducible_and_atomic_free(gpu, kind, R, chunk):
    """Deterministic mode: chunk-boundary rows go to scratch slots summed in sorted order, so
    two runs give bit-identical V; matches the oracle and the atomic-boundary kernel."""
    import paper_1809_09175_amd as spt
    dims = (600, 500, 40)
    X = _small(kind, dims, 80_003, (1.1, 1.1, 1.1), seed=19)
    T = _dev_tensor(X, np.float64 if kind == "f64" else np.float32)
    T.permute()
    T.sort_copy(1)
    dev, ref = _factors(dims, R, seed=7, kind=kind)
    lam = torch.from_numpy(np.linspace(0.5, 2.0, R)).cuda()
    y = torch.from_numpy(np.random.default_rng(3).standard_normal(X.nnz).astype(
        np.float64 if kind == "f64" else np.float32)).cuda()
    for n in range(3):
        V_ref = oracle.mttkrp(X.subs, X.vals, dims, ref, n, lam.cpu().numpy())
        for vals in (None, y):
            a = spt.mttkrp(T, dev, n, lam=lam, vals=vals, chunk=chunk, deterministic=True)
            b = spt.mttkrp(T, dev, n, lam=lam, vals=vals, chunk=chunk, deterministic=True)
            c = spt.mttkrp(T, dev, n, lam=lam, vals=vals, chunk=chunk)
            torch.cuda.synchronize()
            assert torch.equal(a, b), n
            tight = 1e-14 if kind == "f64" else 1e-6
            assert _relerr(a.cpu().numpy(), c.cpu().numpy().astype(np.float64)) < tight
            if vals is None:
                assert _relerr(a.cpu().numpy(), V_ref) < TOL[kind]


def test_privatized_short_mode(gpu):
    """Privatised output for short modes (whole V in one workgroup's LDS): parity, and the
    eligibility check rejects long modes."""
    import paper_1809_09175_amd as spt
    from paper_1809_09175_amd import SptError
    dims = (5000, 365, 40, 7)
    X = _small("f32", dims, 120_007, (1.2, 0.0, 1.1, 0.0), seed=23)
    T = _dev_tensor(X, np.float32)
    for R in (8, 16, 32):
        dev, ref = _factors(dims, R, seed=R, kind="f32")
        for n in (1, 2, 3):
            V = spt.mttkrp(T, dev, n, algo="privatized")
            torch.cuda.synchronize()
            assert _relerr(V.cpu().numpy(), oracle.mttkrp(X.subs, X.vals, dims, ref, n)) < 1e-5
        with pytest.raises(SptError) as e:
            spt.mttkrp(T, dev, 0, algo="privatized")
        assert e.value.code == -6


@pytest.mark.parametrize("kind", ["f32", "f64"])
def test_atomic_sorted_tile_edges(gpu, kind):
    """The atomic kernel sorts tiles of entries by output row: entry counts around the tile size
    (a single entry, one short tile, exactly one tile, one entry past it, several tiles and a
    tail), a tensor whose entries all share one output row (one run across every lane group,
    wavefront and tile), every output row distinct, layouts with several columns per lane and
    short and long workgroup ranges, against the oracle.  FP64 values take 32-byte records
    (smaller tiles)."""
    import paper_1809_09175_amd as spt
    dims = (6000, 50, 40)
    dtype = np.float64 if kind == "f64" else np.float32
    for P in (1, 511, 1024, 1025, 4097):
        for pattern in ("one_row", "distinct", "skewed"):
            X = _small(kind, dims, P, (1.2, 0.0, 0.0), seed=P)
            if pattern == "one_row":
                X.subs[:, 0] = 7
            elif pattern == "distinct":
                X.subs[:, 0] = np.random.default_rng(P).permutation(dims[0])[:P]
            T = _dev_tensor(X, dtype)
            for R, lanes, cols, chunk in ((8, 0, 0, 0), (32, 8, 4, 64), (16, 16, 1, 1024),
                                          (24, 8, 4, 4096)):
                if R % max(cols, 1):
                    continue
                dev, ref = _factors(dims, R, seed=R, kind=kind)
                for n in range(3):
                    _log(f"atomic tiles {kind} P={P} {pattern} R={R} {lanes}x{cols} chunk={chunk} n={n}")
                    V = spt.mttkrp(T, dev, n, algo="atomic", lanes=lanes, cols=cols, chunk=chunk)
                    torch.cuda.synchronize()
                    assert _relerr(V.cpu().numpy(),
                                   oracle.mttkrp(X.subs, X.vals, dims, ref, n)) < TOL[kind], \
                        (P, pattern, R, lanes, cols, chunk, n)


def test_atomic_heavy_row_accuracy(gpu):
    """Rows holding a large share of the entries (Zipf exponent 1.1 over 200000 rows, the
    hottest about a tenth of 8e6 entries), in several lane layouts: the heavy rows' FP32 sums
    (one pre-summed term per sorted tile) stay within the FP32 tolerance."""
    import paper_1809_09175_amd as spt
    dims = (200_000, 3000, 5000)
    X = datagen.skewed_tensor(dims, 8_000_000, (1.1, 0.0, 0.0), seed=41)
    T = _dev_tensor(X, np.float32)
    R = 32
    dev, ref = _factors(dims, R, seed=5, kind="f32")
    counts = np.bincount(X.subs[:, 0], minlength=dims[0])
    heavy = np.argsort(counts)[-6:]
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([heavy, rng.integers(0, dims[0], size=30)]))
    s, v = _sampled_rows(X, 0, rows)
    V_ref = oracle.mttkrp(s, v, dims, ref, 0)[rows]
    hot = rows == heavy[-1]
    for lanes, cols in ((0, 0), (8, 4), (16, 2)):
        _log(f"heavy rows {lanes}x{cols}")
        V = spt.mttkrp(T, dev, 0, algo="atomic", lanes=lanes, cols=cols)
        torch.cuda.synchronize()
        got = V[torch.from_numpy(rows).cuda()].cpu().numpy()
        assert _relerr(got[hot], V_ref[hot]) < TOL["f32"], (lanes, cols)
        assert _relerr(got, V_ref) < TOL["f32"], (lanes, cols)
