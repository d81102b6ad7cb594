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


def test_compulsory_bytes_counts_each_touched_row_once():
    # 3-way tensor: mode 0 touches rows {0, 2}, mode 1 {1}, mode 2 {0, 1, 3}
    from types import SimpleNamespace
    subs = np.array([[0, 1, 0], [2, 1, 1], [2, 1, 3], [0, 1, 3]], np.int32)
    X = SimpleNamespace(subs=subs, dims=(4, 2, 5), d=3)
    t = bench.touched_rows(X)
    assert t == [2, 1, 3]
    R = 8
    # records (16 B) + perm (4 B) per entry, other modes' touched rows read once (FP32), the
    # output's touched rows written once (FP32)
    got = bench.compulsory_bytes(t, 0, R, 16, 4, 4, 4, P=4)
    assert got == 4 * 20 + (1 + 3) * R * 4 + 2 * R * 4


def _write_csv(path, header, rows):
    import csv
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        for r in rows:
            w.writerow(r)


def test_profile_summary_legs_and_calibration(tmp_path):
    """The rocprofv3 summary assigns the permuted kernel's first grid to the sorted-copy leg and
    its second to the gather leg, and calibrates the counters with the triad."""
    perm = ("void spt::k_mttkrp_perm<3, 8, 4, float, float, float>(HIP_vector_type<int, 4u> "
            "const*, int)")
    atom = "void spt::k_mttkrp_atomic<3, 32, 1, float, float, float>(long)"
    triad = "spt::k_triad(HIP_vector_type<float, 4u>*, float)"
    disp = [(1, triad, 16777216, 0, 600_000), (2, perm, 1000, 1_000_000, 2_000_000),
            (3, perm, 5000, 3_000_000, 6_000_000), (4, atom, 7000, 7_000_000, 17_000_000)]
    hdr = ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp",
           "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    _write_csv(tmp_path / "prof_trace" / "run_kernel_trace.csv", hdr,
               [["KERNEL_DISPATCH", i, k, a, b, g, 1, 1] for i, k, g, a, b in disp])
    chdr = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    fetch = {1: 1048576.0, 2: 100.0, 3: 300.0, 4: 50.0}   # triad: half of the 2 GiB read
    write = {1: 1048576.0, 2: 10.0, 3: 20.0, 4: 700.0}
    _write_csv(tmp_path / "prof_fetch" / "run_counter_collection.csv", chdr,
               [[i, g, k, "FETCH_SIZE", fetch[i]] for i, k, g, _, _ in disp])
    _write_csv(tmp_path / "prof_write" / "run_counter_collection.csv", chdr,
               [[i, g, k, "WRITE_SIZE", write[i]] for i, k, g, _, _ in disp])
    md, ctr = bench.summarize_profile(str(tmp_path))
    kv = dict(l.split(" = ", 1) for l in ctr.splitlines() if " = " in l)
    assert kv["copy.grid"] == "1000" and kv["gather.grid"] == "5000"
    assert float(kv["copy.hbm_bytes_per_dispatch"]) == (100 * 2 + 10) * 1024
    assert float(kv["gather.hbm_bytes_per_dispatch"]) == (300 * 2 + 20) * 1024
    assert float(kv["atomic.hbm_bytes_per_dispatch"]) == (50 * 2 + 700) * 1024
    assert "| `spt::k_mttkrp_perm<3, 8, 4, float, float, float>` | copy | 1000 | 1 | 1000.0 |" in md
