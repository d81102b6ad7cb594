"""Host-side pieces of bench.py: the FP64 row evaluation behind its accuracy figure agrees with
the oracle, the model-byte formula gives the per-entry figures of the paper's bandwidth model
(Sec. 7.1, typed per operand), and a run on more than one GPU is refused with a message."""
import subprocess
import sys
from pathlib import Path

import numpy as np

import bench
import oracle

ROOT = Path(__file__).resolve().parent.parent


def test_sampled_rows_match_oracle():
    rng = np.random.default_rng(0)
    dims = (50, 40, 30, 7)
    P = 20_000
    subs = np.stack([rng.integers(0, I, P) for I in dims], 1).astype(np.int32)
    vals = rng.random(P).astype(np.float32)
    A = [rng.random((I, 8)) for I in dims]
    for n in range(4):
        rows = np.unique(rng.integers(0, dims[n], 5))
        mask = np.isin(subs[:, n], rows)
        got = bench._rows_fp64(subs[mask], vals[mask], A, n, rows, chunk=777)
        ref = oracle.mttkrp(subs[mask], vals[mask].astype(np.float64), dims, A, n)[rows]
        assert np.allclose(got, ref, rtol=1e-14, atol=0), n


def test_model_bytes_per_entry():
    # value + d subscripts + (d-1) gathered rows + one output row, FP32 (16 + 12R at d = 3)
    for R in (16, 32, 64):
        assert bench.model_bytes(3, R) == 16 + 12 * R
    assert bench.model_bytes(3, 32, s_f=2) == 16 + 2 * 32 * 2 + 4 * 32


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
