"""GPU parity of the autotuner's choices and of the batched, graph-replayed MTTKRP against
the FP64 CPU oracle (FP32 1e-5; BF16 factors 1e-5 against the widened BF16 values)."""
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


def _small_batch(count=12):
    return datagen.batch64(count=count, nnz_range=(2e3, 6e4), dim_range=(200, 4000))


def _prep(Xs, bf16=False):
    import paper_1809_09175_amd as spt
    items = []
    for t, X in enumerate(Xs):
        T = spt.SparseTensor(torch.from_numpy(X.subs).cuda(), torch.from_numpy(X.vals).cuda(), X.dims)
        T.validate()
        T.permute()
        R = X.meta["R"]
        A = datagen.factors(X.dims, R, seed=100 + t, dtype=np.float32)
        dev = [torch.from_numpy(a).cuda() for a in A]
        if bf16:
            dev = [spt.to_bf16(a) for a in dev]
        ref = [d.float().cpu().numpy().astype(np.float64) for d in dev]
        items.append((X, T, dev, ref))
    return items


def test_autotune_choice_is_a_valid_fast_config(gpu):
    import paper_1809_09175_amd as spt
    X = datagen.skewed_tensor((3000, 2000, 500), 200_000, (1.1, 1.1, 1.1), seed=4)
    T = spt.SparseTensor(torch.from_numpy(X.subs).cuda(), torch.from_numpy(X.vals).cuda(), X.dims)
    T.permute()
    A = datagen.factors(X.dims, 32, seed=1, dtype=np.float32)
    dev = [torch.from_numpy(a).cuda() for a in A]
    for n in range(3):
        best = spt.autotune(T, dev, n)
        _log(f"autotune mode {n}: {best}")
        assert best["lanes"] * best["cols"] >= 32 and 32 % best["cols"] == 0
        assert best["chunk"] % 64 == 0 and best["chunk"] >= 64 and best["ms"] > 0
        V = spt.mttkrp(T, dev, n, algo=best["algo"], lanes=best["lanes"], cols=best["cols"],
                       chunk=best["chunk"])
        torch.cuda.synchronize()
        ref = oracle.mttkrp(X.subs, X.vals, X.dims, [a.astype(np.float64) for a in A], n)
        assert _relerr(V.cpu().numpy(), ref) < 1e-5
        bb = spt.autotune(T, dev, n, batch=True)
        from paper_1809_09175_amd import _lib
        algo = {"atomic": 1, "permuted": 2}[bb["algo"]]
        assert _lib.load().spt_batch_supported_tune(3, 1, algo, bb["lanes"], bb["cols"]) == 1


def _median_ms(spt, T, dev, n, out, reps=15, **kw):
    spt.mttkrp(T, dev, n, out=out, **kw)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        spt.mttkrp(T, dev, n, out=out, **kw)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def test_autotune_never_loses_to_the_default(gpu):
    """The tuner's candidates include the library default (with the chunk its launch uses), so
    its choice is at least as fast as the default, re-timed independently (5% for timing
    noise), on a 2e6-entry tensor with and without sorted record copies."""
    import paper_1809_09175_amd as spt
    X = datagen.skewed_tensor((60_000, 40_000, 3000), 2_000_000, (1.1, 1.1, 1.1), seed=6)
    T = spt.SparseTensor(torch.from_numpy(X.subs).cuda(), torch.from_numpy(X.vals).cuda(), X.dims)
    T.permute()
    for copies in (False, True):
        if copies:
            T.sort_copy()
        for R in (16, 32):
            dev = [torch.from_numpy(a).cuda() for a in datagen.factors(X.dims, R, 2, np.float32)]
            for n in range(3):
                out = torch.empty((X.dims[n], R), device="cuda")
                best = spt.autotune(T, dev, n, out=out)
                kw = {k: best[k] for k in ("algo", "lanes", "cols", "chunk")}
                t_default = _median_ms(spt, T, dev, n, out)
                t_tuned = _median_ms(spt, T, dev, n, out, **kw)
                _log(f"autotune copies={copies} R={R} n={n}: {best} default {t_default:.4f} ms "
                     f"tuned {t_tuned:.4f} ms")
                assert t_tuned <= 1.05 * t_default, (copies, R, n, best, t_default, t_tuned)


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("tuned", [False, True])
def test_batched_graph_replays_match_oracle(gpu, bf16, tuned):
    import paper_1809_09175_amd as spt
    prepared = _prep(_small_batch(), bf16=bf16)
    items = []
    refs = []
    for (X, T, dev, ref) in prepared:
        for n in range(3):
            out = torch.full((X.dims[n], X.meta["R"]), float("nan"), device="cuda")
            tune = spt.autotune(T, dev, n, batch=True, reps=1) if tuned else None
            if not tuned:
                tune = {"algo": "permuted" if n % 2 == 0 else "atomic", "lanes": 8, "cols": 4}
            items.append({"X": T, "mode": n, "factors": dev, "out": out, "tune": tune})
            refs.append(oracle.mttkrp(X.subs, X.vals, X.dims, ref, n))
    B = spt.Batch(items)
    _log(f"batch of {len(items)} products: {B.info()}")
    for rep in range(3):
        for it in items:                     # eager work between replays: poison the outputs
            it["out"].fill_(float("nan"))
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for it, ref in zip(items, refs):
            got = it["out"].cpu().numpy()
            assert np.isfinite(got).all()
            assert _relerr(got, ref) < 1e-5, (rep, it["mode"], it["tune"])
    B.close()


def test_batch_rejects_unsupported_layout(gpu):
    import paper_1809_09175_amd as spt
    from paper_1809_09175_amd import SptError
    (X, T, dev, ref), = _prep(_small_batch(1))
    out = torch.empty((X.dims[0], X.meta["R"]), device="cuda")
    with pytest.raises(SptError) as e:
        spt.Batch([{"X": T, "mode": 0, "factors": dev, "out": out,
                    "tune": {"algo": "permuted", "lanes": 64, "cols": 1}}])
    assert e.value.code == -6
