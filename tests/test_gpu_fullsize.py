"""Parity at the full workload sizes, in the launch configuration the benchmark times (default
layouts, mode-sorted record copies, the "auto" algorithm).  What the oracle can compute row by
row is compared row by row: the rows of V (or of a gradient) fed by the entries whose mode-n
subscript is one of the selected rows.  Selected rows: the heaviest row of each mode plus a
ragged set of random rows.  The GCP loss is compared whole."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1809_09175_amd import datagen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (nb if nb > 0 else 1.0)


def _rows(X, n, count, seed):
    counts = np.bincount(X.subs[:, n], minlength=X.dims[n])
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[int(np.argmax(counts))],
                                     rng.integers(0, X.dims[n], size=count)]))


def _entries_of(X, n, rows):
    mask = np.isin(X.subs[:, n], rows)
    return X.subs[mask], X.vals[mask]


def _device_tensor(X):
    import paper_1809_09175_amd as spt
    T = spt.SparseTensor(torch.from_numpy(X.subs).cuda(), torch.from_numpy(X.vals).cuda(), X.dims)
    T.validate()
    T.permute()
    T.sort_copy()
    return T


def test_skewed4_full_size_bf16_and_fp32(gpu):
    """4-way 1e6 x 1e5 x 1e4 x 365 tensor, 5e7 entries, R = 32: FP32 factors to 1e-5, BF16
    factors to 2e-2 against the oracle on the unrounded factors, every mode."""
    import paper_1809_09175_amd as spt
    _log("skewed4 full size: generating")
    X = datagen.skewed4()
    T = _device_tensor(X)
    R = 32
    a32 = [a.astype(np.float32) for a in datagen.factors(X.dims, R, 11, np.float64)]
    ref = [a.astype(np.float64) for a in a32]
    dev32 = [torch.from_numpy(a).cuda() for a in a32]
    devbf = [spt.to_bf16(t) for t in dev32]
    for n in range(X.d):
        rows = _rows(X, n, 30, seed=n)
        s, v = _entries_of(X, n, rows)
        V_ref = oracle.mttkrp(s, v, X.dims, ref, n)[rows]
        for name, dev, tol in (("f32", dev32, 1e-5), ("bf16", devbf, 2e-2)):
            _log(f"skewed4 mode {n} {name}")
            V = spt.mttkrp(T, dev, n)
            torch.cuda.synchronize()
            got = V[torch.from_numpy(rows).cuda()].cpu().numpy()
            assert _relerr(got, V_ref) < tol, (n, name)


def test_gcp_counts_full_size(gpu):
    """Count tensor 2e5 x 1e5 x 5e3 with 5e7 nonzeros and 5e7 sampled zeros, R = 32, Poisson
    log link: the whole loss against the oracle's FP64 loss, and selected gradient rows of every
    mode against the oracle's gradient over the entries that feed them."""
    import paper_1809_09175_amd as spt
    _log("gcp_counts full size: generating")
    X, A = datagen.gcp_counts(R=32)
    T = _device_tensor(X)
    facs = [torch.from_numpy(a).cuda().requires_grad_(True) for a in A]
    loss = spt.GCPPoissonLoss.apply(T, None, *facs)
    loss.backward()
    torch.cuda.synchronize()
    ref = [a.astype(np.float64) for a in A]
    _log("gcp_counts: oracle loss")
    loss_ref = oracle.gcp(X.subs, X.vals, X.dims, ref, grads=False)
    assert abs(loss.item() - loss_ref) < 1e-5 * abs(loss_ref)
    for n in range(X.d):
        rows = _rows(X, n, 20, seed=10 + n)
        s, v = _entries_of(X, n, rows)
        _, g_ref = oracle.gcp(s, v, X.dims, ref)
        got = facs[n].grad[torch.from_numpy(rows).cuda()].cpu().numpy()
        assert _relerr(got, g_ref[n][rows]) < 1e-4, n


def test_batch64_full_size(gpu):
    """All 64 tensors x 3 modes in one graph-replayed persistent launch with autotuned
    per-product layouts: every output against the oracle, on two replays."""
    import paper_1809_09175_amd as spt
    _log("batch64 full size: generating")
    Xs = datagen.batch64()
    items, refs, keep = [], [], []
    for t, X in enumerate(Xs):
        T = _device_tensor(X)
        R = X.meta["R"]
        a32 = [a.astype(np.float32) for a in datagen.factors(X.dims, R, 400 + t, np.float64)]
        dev = [torch.from_numpy(a).cuda() for a in a32]
        keep.append((T, dev))
        for n in range(3):
            out = torch.empty((X.dims[n], R), device="cuda")
            tune = spt.autotune(T, dev, n, batch=True, reps=1, out=out)
            items.append({"X": T, "mode": n, "factors": dev, "out": out, "tune": tune})
            refs.append(oracle.mttkrp(X.subs, X.vals, X.dims, [a.astype(np.float64) for a in a32], n))
    B = spt.Batch(items)
    for rep in range(2):
        for it in items:
            it["out"].fill_(float("nan"))
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for i, (it, ref) in enumerate(zip(items, refs)):
            got = it["out"].cpu().numpy()
            assert np.isfinite(got).all(), (rep, i)
            assert _relerr(got, ref) < 1e-5, (rep, i, it["tune"])
    B.close()


def test_max_entry_count(gpu):
    """2^31 - 1 entries, the most that int32 subscripts and permutations allow, so that every
    index computation of packing, sorting, the sorted copy and the traversals is exercised at
    its limit (about 180 GB of device memory).  Each mode's permutation is checked on the device
    against its definition (keys non-decreasing, each key the subscript of the entry it names,
    equal keys in increasing storage position, every position exactly once); MTTKRP rows (16
    random rows per mode, about 1,000-2,000 entries each) against the oracle on exactly the
    entries that feed them, for the atomic and gather traversals and, on mode 0, the
    second-mode sorted copy."""
    import paper_1809_09175_amd as spt
    _log("max entries: drawing 2^31 - 1 entries on the device")
    subs, vals, dims = datagen.max_entries()
    P = subs.shape[0]
    T = spt.SparseTensor(subs, vals, dims)
    T.validate()
    T.permute()
    torch.cuda.synchronize()
    step = 1 << 28
    for n in range(3):
        _log(f"max entries: permutation of mode {n}")
        p, k = T.perm(n)
        seen = torch.zeros(P, dtype=torch.bool, device="cuda")
        for a in range(0, P, step):
            b = min(P, a + step + 1)  # one element of overlap for the adjacent-pair checks
            pa = p[a:b].long()
            ka = k[a:b]
            assert bool((ka[1:] >= ka[:-1]).all()), (n, a)
            eq = ka[1:] == ka[:-1]
            assert bool((pa[1:][eq] > pa[:-1][eq]).all()), (n, a)
            assert torch.equal(subs[pa, n], ka), (n, a)
            seen[pa] = True
            del pa, ka, eq
        assert bool(seen.all()), n
        del seen
    R = 16
    a32 = [a.astype(np.float32) for a in datagen.factors(dims, R, 61, np.float64)]
    ref = [a.astype(np.float64) for a in a32]
    dev = [torch.from_numpy(a).cuda() for a in a32]
    _log("max entries: second-mode sorted copy of mode 0")
    T.sort_copy(0)
    rng = np.random.default_rng(62)
    for n in range(3):
        rows = np.unique(rng.integers(0, dims[n], size=16))
        rows_t = torch.from_numpy(rows.astype(np.int32)).cuda()
        idx = torch.cat([torch.nonzero(torch.isin(subs[a:a + step, n], rows_t)).flatten() + a
                         for a in range(0, P, step)])
        s_h = subs[idx].cpu().numpy()
        v_h = vals[idx].cpu().numpy()
        _log(f"max entries: mode {n}, oracle on {len(v_h)} entries")
        V_ref = oracle.mttkrp(s_h, v_h, dims, ref, n)[rows]
        for algo in ["atomic", "permuted"] + (["permuted_copy"] if n == 0 else []):
            _log(f"max entries: mode {n} {algo}")
            V = spt.mttkrp(T, dev, n, algo=algo)
            torch.cuda.synchronize()
            got = V[torch.from_numpy(rows).cuda()].cpu().numpy()
            assert _relerr(got, V_ref) < 1e-5, (n, algo)
            del V
    del T, subs, vals
    torch.cuda.empty_cache()


def test_max_mode_length(gpu):
    """A mode of 2^31 - 1 rows (the int32 limit): 31-bit keys take four radix passes, and V
    (2^31 - 1 rows x R) is addressed beyond 32-bit element offsets.  The permutation against a
    host stable sort, and the rows of V the entries feed against the oracle evaluated with the
    used rows renumbered densely (V's rows are independent, so this changes no arithmetic), for
    the atomic, gather and sorted-copy traversals; rows no entry feeds stay zero."""
    import paper_1809_09175_amd as spt
    rng = np.random.default_rng(71)
    I0 = (1 << 31) - 1
    dims = (I0, 5, 3)
    P = 1_000_003
    subs = np.stack([rng.integers(0, I0, size=P), rng.integers(0, 5, size=P),
                     rng.integers(0, 3, size=P)], 1).astype(np.int32)
    subs[:3, 0] = [I0 - 1, 0, I0 - 1]          # the first and the last row
    vals = rng.random(P).astype(np.float32)
    T = spt.SparseTensor(torch.from_numpy(subs).cuda(), torch.from_numpy(vals).cuda(), dims)
    T.validate()
    T.permute()
    p, k = T.perm(0)
    ref_order = np.argsort(subs[:, 0], kind="stable")
    assert np.array_equal(p.cpu().numpy(), ref_order)
    assert np.array_equal(k.cpu().numpy(), subs[ref_order, 0])
    T.sort_copy(0)
    R = 2
    a32 = [a.astype(np.float32) for a in datagen.factors((1, 5, 3), R, 72, np.float64)]
    dev = [None, torch.from_numpy(a32[1]).cuda(), torch.from_numpy(a32[2]).cuda()]  # A^(0) unread
    used, dense = np.unique(subs[:, 0], return_inverse=True)
    s_dense = subs.copy()
    s_dense[:, 0] = dense
    V_ref = oracle.mttkrp(s_dense, vals, (len(used), 5, 3), [np.zeros((len(used), R))] +
                          [a.astype(np.float64) for a in a32[1:]], 0)
    pick = np.unique(np.concatenate([[0, len(used) - 1], rng.integers(0, len(used), 2000)]))
    rows_t = torch.from_numpy(used[pick].astype(np.int64)).cuda()
    unused = [1, I0 - 2]
    assert not np.isin(unused, used).any()
    for algo in ("atomic", "permuted", "permuted_copy"):
        _log(f"max mode length: {algo}")
        V = spt.mttkrp(T, dev, 0, algo=algo)
        torch.cuda.synchronize()
        assert V.shape == (I0, R)
        got = V[rows_t].cpu().numpy()
        assert _relerr(got, V_ref[pick]) < 1e-5, algo
        assert float(V[torch.tensor(unused, device="cuda")].abs().max()) == 0.0, algo
        del V
        torch.cuda.empty_cache()
