"""Benchmark: all-mode MTTKRP on the 1e8-entry power-law tensor (500,000 x 500,000 x 20,000,
Zipf(1.1) subscripts per mode, FP32 values and factors) on one MI355X.

One step = one MTTKRP of every mode (zero V, then the permuted-traversal kernel over the
mode-sorted record copies, built beforehand like the permutations), R = 32.  The metric is
effective GB/s under the paper's bandwidth model (bytes per entry = value + d subscripts + (d-1)
gathered factor rows + one output row), the same byte count for every kernel so effective GB/s
is proportional to 1/time.  Also reported: the gather and atomic kernels, R = 16 and 64, the
permutation and copy build costs against one CP-ALS iteration, a STREAM-style triad, BF16
factors, the 64-tensor batch, the generalized-CP passes, the dominant kernel's roofline
fraction, and the FP64 CPU oracle timed on a bounded sample of the same tensor.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def model_bytes(d, R, s_val=4, s_idx=4, s_f=4, s_out=4):
    """Bytes per entry of the paper's MTTKRP bandwidth model (Sec. 7.1), typed per operand."""
    return s_val + d * s_idx + (d - 1) * R * s_f + R * s_out


def kernel_source_hash():
    """Hash of the sources the MTTKRP kernels are compiled from (not the host launch code)."""
    h = hashlib.sha256()
    for f in ("mttkrp_kernels.h", "mttkrp_f32.hip", "spt_internal.h"):
        with open(os.path.join(ROOT, "paper_1809_09175_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


COUNTERS_FILE = os.path.join(ROOT, "profiles", "mttkrp_powerlaw3_R32_counters.txt")


def read_counters():
    """HBM traffic per dispatch of the MTTKRP kernels, from the committed rocprofv3 counter
    summary: {variant: {"kernel": name, "grid": workgroups, "bytes": calibrated bytes}}.  Empty
    when absent or taken from a different kernel source."""
    if not os.path.exists(COUNTERS_FILE):
        return {}
    kv = {}
    for line in open(COUNTERS_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return {}
    out = {}
    for k, v in kv.items():
        if "." not in k:
            continue
        var, field = k.split(".", 1)
        out.setdefault(var, {})[field] = v
    res = {}
    for var, f in out.items():
        try:
            res[var] = {"kernel": f["kernel"], "grid": int(f["grid"]),
                        "bytes": float(f["hbm_bytes_per_dispatch"])}
        except (KeyError, ValueError):
            continue
    return res


def touched_rows(X):
    """Rows of each mode that hold at least one entry."""
    return [int(np.count_nonzero(np.bincount(X.subs[:, m], minlength=X.dims[m])))
            for m in range(X.d)]


def compulsory_bytes(touched, n, R, rec_bytes, s_f, s_out, extra_per_entry, P):
    """Unique bytes one mode-n MTTKRP must move: every record once (plus per-entry index
    arrays the traversal reads, e.g. the permutation), every touched row of the other factor
    matrices once, and every touched row of V written once."""
    b = P * (rec_bytes + extra_per_entry)
    for m, t in enumerate(touched):
        b += t * R * (s_out if m == n else s_f)
    return b


def _rows_fp64(subs, vals, factors, n, rows, chunk=1 << 20):
    """Rows `rows` of the mode-n MTTKRP (eq. (mttkrp)) in FP64 with numpy, from the entries
    whose mode-n subscript is one of them (a measurement-side check of the accuracy figure)."""
    pos = {int(r): k for k, r in enumerate(rows)}
    out = np.zeros((len(rows), factors[0].shape[1]))
    lookup = np.full(int(rows.max()) + 1, -1, np.int64)
    lookup[rows] = [pos[int(r)] for r in rows]
    for c0 in range(0, len(vals), chunk):
        s, v = subs[c0:c0 + chunk], vals[c0:c0 + chunk].astype(np.float64)
        t = v[:, None] * np.ones((1, out.shape[1]))
        for m in range(len(factors)):
            if m != n:
                t = t * factors[m][s[:, m]]
        np.add.at(out, lookup[s[:, n]], t)
    return out


def _sampled_rel_errors(X, dev_outs, ref_factors, rows_per_mode=20, seed=0):
    """Relative error of selected output rows (each mode's hottest row plus random rows)
    against an FP64 evaluation on exactly the entries that feed them."""
    rng = np.random.default_rng(seed)
    errs = []
    for n in range(X.d):
        counts = np.bincount(X.subs[:, n], minlength=X.dims[n])
        rows = np.unique(np.concatenate([[int(np.argmax(counts))],
                                         rng.integers(0, X.dims[n], size=rows_per_mode)]))
        mask = np.isin(X.subs[:, n], rows)
        ref = _rows_fp64(X.subs[mask], X.vals[mask], ref_factors, n, rows)
        got = dev_outs[n][rows].astype(np.float64)
        errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    return max(errs)


def bench_skewed4_bf16(spt, datagen, torch, dev, R=32, steps=10, warmup=2):
    """BF16 vs FP32 factors on the 4-way skewed tensor, all modes, permuted kernel."""
    t0 = time.time()
    X = datagen.skewed4()
    log(f"generated skewed4 ({X.nnz} entries) in {time.time() - t0:.1f}s")
    T = spt.SparseTensor(torch.from_numpy(X.subs).to(dev), torch.from_numpy(X.vals).to(dev), X.dims)
    T.validate()
    T.permute()
    T.sort_copy()
    A32 = [torch.from_numpy(a).to(dev) for a in datagen.factors(X.dims, R, seed=3, dtype=np.float32)]
    A16 = [spt.to_bf16(a) for a in A32]
    outs = [torch.empty((I, R), dtype=torch.float32, device=dev) for I in X.dims]
    res = {}
    for name, A in (("fp32", A32), ("bf16", A16)):
        for _ in range(warmup):
            for n in range(X.d):
                spt.mttkrp(T, A, n, out=outs[n])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            for n in range(X.d):
                spt.mttkrp(T, A, n, out=outs[n])
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ref = [a.cpu().numpy().astype(np.float64) for a in A32]
        err = _sampled_rel_errors(X, [o.cpu().numpy() for o in outs], ref)
        sbytes = 2 if name == "bf16" else 4
        gbs = X.nnz * model_bytes(X.d, R, s_f=sbytes) * X.d / (ms * 1e-3) / 1e9
        res[name] = {"ms_all_modes": round(ms, 3), "model_gbs": round(gbs, 1),
                     "max_rel_err_vs_fp64_sampled_rows": err}
        log(f"skewed4 {name}: {ms:.3f} ms all modes, sampled rel err {err:.2e}")
    res["bf16_speedup"] = round(res["fp32"]["ms_all_modes"] / res["bf16"]["ms_all_modes"], 3)
    del T
    return res


def bench_batch64(spt, datagen, torch, dev, reps=10):
    """64 uneven 3-way tensors x 3 modes: separate default launches vs separate tuned launches
    vs one batched persistent kernel replayed from a HIP graph (tuned per product)."""
    t0 = time.time()
    Xs = datagen.batch64()
    log(f"generated batch64 ({sum(x.nnz for x in Xs)} entries) in {time.time() - t0:.1f}s")
    items = []
    for t, X in enumerate(Xs):
        T = spt.SparseTensor(torch.from_numpy(X.subs).to(dev), torch.from_numpy(X.vals).to(dev),
                             X.dims)
        T.permute()
        T.sort_copy()
        R = X.meta["R"]
        A = [torch.from_numpy(a).to(dev) for a in datagen.factors(X.dims, R, seed=400 + t,
                                                                  dtype=np.float32)]
        for n in range(3):
            items.append({"X": T, "mode": n, "factors": A,
                          "out": torch.empty((X.dims[n], R), dtype=torch.float32, device=dev),
                          "nnz": X.nnz, "R": R})
    torch.cuda.synchronize()

    def run_separate(tuned):
        for it in items:
            kw = {}
            if tuned:
                kw = {k: it["tune"][k] for k in ("algo", "lanes", "cols", "chunk")}
            spt.mttkrp(it["X"], it["factors"], it["mode"], out=it["out"], **kw)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    plain_ms = timed(lambda: run_separate(False))
    # separate launches: tuned over every configuration (the library default included)
    for it in items:
        it["tune"] = spt.autotune(it["X"], it["factors"], it["mode"], out=it["out"])
    tuned_ms = timed(lambda: run_separate(True))
    # the batch: tuned over the configurations the batched kernel holds
    t0 = time.time()
    for it in items:
        it["tune"] = spt.autotune(it["X"], it["factors"], it["mode"], batch=True, out=it["out"])
    tune_s = time.time() - t0
    B = spt.Batch([{k: it[k] for k in ("X", "mode", "factors", "out", "tune")} for it in items])
    batch_ms = timed(B.launch)
    Bd = spt.Batch([{k: it[k] for k in ("X", "mode", "factors", "out")} for it in items])
    batch_default_ms = timed(Bd.launch)
    Bd.close()
    model = sum(it["nnz"] * model_bytes(3, it["R"]) for it in items)
    algos = {}
    for it in items:
        key = f"{it['tune']['algo']}:{it['tune']['lanes']}x{it['tune']['cols']}"
        algos[key] = algos.get(key, 0) + 1
    res = {"products": len(items), "entries_total": int(sum(x.nnz for x in Xs)),
           "separate_default_ms": round(plain_ms, 3), "separate_tuned_ms": round(tuned_ms, 3),
           "batched_graph_ms": round(batch_ms, 3),
           "batched_graph_default_layouts_ms": round(batch_default_ms, 3),
           "batched_speedup_vs_separate_default": round(plain_ms / batch_ms, 3),
           "batched_speedup_vs_separate_tuned": round(tuned_ms / batch_ms, 3),
           "batched_model_gbs": round(model / (batch_ms * 1e-3) / 1e9, 1),
           "autotune_s": round(tune_s, 1), "tuned_layouts": algos}
    log(f"batch64: separate {plain_ms:.3f} ms, tuned {tuned_ms:.3f} ms, batched {batch_ms:.3f} ms")
    B.close()
    return res


def bench_shard_share(spt, torch, T, X, dev, R, shards=8):
    """The kernel at one GPU's share of a row-owning split over `shards` GPUs: for each mode n,
    the first 1/shards of the entries in mode-n order (a contiguous range of output rows) as a
    tensor of its own, with the full factor matrices; MTTKRP time of that mode on it."""
    out = []
    subs_all = None
    for n in range(X.d):
        perm, _ = T.perm(n)
        q = perm[: X.nnz // shards].long()
        if subs_all is None:
            subs_all = torch.from_numpy(X.subs).to(dev)
            vals_all = torch.from_numpy(X.vals).to(dev)
        S = spt.SparseTensor(subs_all[q].contiguous(), vals_all[q].contiguous(), X.dims)
        S.permute(n)
        S.sort_copy(n)
        A = [torch.rand(I, R, device=dev) for I in X.dims]
        V = torch.empty(X.dims[n], R, device=dev)
        spt.mttkrp(S, A, n, out=V)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            spt.mttkrp(S, A, n, out=V)
        e1.record()
        torch.cuda.synchronize()
        out.append(round(e0.elapsed_time(e1) / 10, 3))
        S.close()
        del S, q
    del subs_all, vals_all
    torch.cuda.empty_cache()
    return {"entries_per_shard": X.nnz // shards, "rank": R, "mttkrp_ms_per_mode": out}


def bench_ingest(spt, torch, X, dev, chunk=1 << 23, reps=2):
    """Host arrays in pinned memory to a permuted tensor (every mode): one whole copy, then
    packing and the sort, against chunked ingest, where chunk k+1 is copied while chunk k is
    packed and its first radix digit counted.  Wall-clock time of the second of `reps` runs of
    each (the first warms the allocator), synchronised at both ends."""
    hs = torch.from_numpy(X.subs).pin_memory()
    hv = torch.from_numpy(X.vals).pin_memory()

    def serial():
        subs = hs.to(dev, non_blocking=True)
        vals = hv.to(dev, non_blocking=True)
        T = spt.SparseTensor(subs, vals, X.dims)
        T.permute()
        return T

    def overlapped():
        T = spt.SparseTensor.from_host(hs, hv, X.dims, chunk=chunk)
        T.permute()
        return T

    res = {}
    for name, fn in (("whole_copy_then_pack_ms", serial), ("chunked_overlap_ms", overlapped)):
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            T = fn()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            T.close()
            del T
        res[name] = round(ms, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d_s = hs.to(dev, non_blocking=True)
    d_v = hv.to(dev, non_blocking=True)
    torch.cuda.synchronize()
    res["pinned_h2d_only_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    del d_s, d_v, hs, hv
    torch.cuda.empty_cache()
    res["chunk_entries"] = chunk
    res["overlap_gain_ms"] = round(res["whole_copy_then_pack_ms"] - res["chunked_overlap_ms"], 2)
    log(f"ingest to permuted: whole copy then pack {res['whole_copy_then_pack_ms']} ms, "
        f"chunked overlap {res['chunked_overlap_ms']} ms (copy alone {res['pinned_h2d_only_ms']} ms)")
    return res


def bench_gcp(spt, datagen, torch, dev, R=32, steps=3):
    """Generalized CP (Poisson log link) forward + backward on the count tensor: 5e7 nonzeros
    plus 5e7 sampled zeros; the backward is one MTTKRP per mode of the derivative tensor."""
    t0 = time.time()
    X, A = datagen.gcp_counts(R=R)
    log(f"generated gcp_counts ({X.nnz} entries) in {time.time() - t0:.1f}s")
    T = spt.SparseTensor(torch.from_numpy(X.subs).to(dev), torch.from_numpy(X.vals).to(dev), X.dims)
    T.validate()
    T.permute()
    T.sort_copy()
    facs = [torch.from_numpy(a).to(dev).requires_grad_(True) for a in A]

    def step():
        for f in facs:
            f.grad = None
        loss = spt.GCPPoissonLoss.apply(T, None, *facs)
        loss.backward()
        return loss

    step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        loss = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    per_entry = (16 + X.d * R * 4 + 4) + X.d * model_bytes(X.d, R)
    res = {"entries": X.nnz, "rank": R, "ms_fwd_bwd": round(ms, 3),
           "model_gbs": round(X.nnz * per_entry / (ms * 1e-3) / 1e9, 1),
           "loss": float(loss.item())}
    log(f"gcp fwd+bwd {ms:.3f} ms")
    del T, facs
    return res


# ------------------------------------------------------------------------------------------
# rocprofv3 summaries (python3 bench.py --summarize-profile DIR): DIR holds prof_trace/ (a
# --kernel-trace --stats run of bench.py --profile) and, optionally, prof_fetch/ and prof_write/
# (--pmc FETCH_SIZE and --pmc WRITE_SIZE runs of the same command)
# ------------------------------------------------------------------------------------------

PROFILE_CMD = ("cd /tmp && export TMPDIR=/tmp && R=<repository root> && OUT=<output directory>; "
               "rocprofv3 --kernel-trace --stats -f csv -d $OUT/prof_trace -o run -- "
               "python3 $R/bench.py --profile; then, each in a run of its own: "
               "rocprofv3 --pmc FETCH_SIZE -f csv -d $OUT/prof_fetch -o run -- "
               "python3 $R/bench.py --profile; "
               "rocprofv3 --pmc WRITE_SIZE -f csv -d $OUT/prof_write -o run -- "
               "python3 $R/bench.py --profile; then, from the repository root: "
               "python3 bench.py --summarize-profile $OUT")
TRIAD_READ_BYTES = 2 * (1 << 28) * 4   # the --profile triad reads b and c (2^28 floats each)
TRIAD_WRITE_BYTES = (1 << 28) * 4      # and writes a


def _short_kernel(name):
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    depth, out = 0, []
    for ch in name:  # drop the argument list, keep the template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out)


def _read_csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(dirpath, suffix):
    for root, _, files in os.walk(dirpath):
        for f in sorted(files):
            if f.endswith(suffix):
                return os.path.join(root, f)
    return None


def _profile_variants(groups):
    """Benchmark leg of each (kernel, grid) group, from the order --profile runs them in: the
    first FP32 permuted-kernel group is the sorted-copy leg, the second the gather leg."""
    legs = {}
    perm32 = [k for k in sorted(groups, key=lambda k: groups[k]["first"])
              if k[0].startswith("spt::k_mttkrp_perm<3,") and k[0].endswith("float, float, float>")]
    if perm32:
        legs[perm32[0]] = "copy"
    if len(perm32) > 1:
        legs[perm32[1]] = "gather"
    for k in groups:
        if k[0].startswith("spt::k_mttkrp_atomic<3,") and k[0].endswith("float, float, float>"):
            legs[k] = "atomic"
        if k[0].startswith("spt::k_mttkrp_perm<3,") and k[0].endswith("double, double, double>"):
            legs[k] = "copy_f64"
    return legs


def summarize_profile(dirpath):
    """Markdown summary and counter file text of a profiled --profile run."""
    trace = _read_csv(_find(os.path.join(dirpath, "prof_trace"), "kernel_trace.csv"))
    groups = {}
    for r in trace:
        key = (_short_kernel(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) *
               int(r["Grid_Size_Z"]))
        g = groups.setdefault(key, {"dur": [], "first": int(r["Dispatch_Id"])})
        g["dur"].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    total = sum(sum(g["dur"]) for g in groups.values())
    legs = _profile_variants(groups)
    lines = ["# rocprofv3 summary: MTTKRP kernels on powerlaw3 (1e8 entries), R = 32", "",
             "Command (run from the repository root on the GPU box):", "", "```", PROFILE_CMD,
             "```", "",
             "The profiled run (`bench.py --profile`) times each R = 32 leg after its own warm-up "
             "launches: sorted copies (3 warm-up + 5 timed steps of three modes), gather (2 + 2), "
             "atomic (2 + 2), FP64 sorted copies (3 + 2), then one triad (the counter "
             "calibration kernel). Durations in microseconds per dispatch; grid in work-items.",
             "", "| kernel | leg | grid | calls | median | mean | min | max | % time |",
             "|---|---|---|---|---|---|---|---|---|"]
    for key in sorted(groups, key=lambda k: -sum(groups[k]["dur"])):
        d = np.array(groups[key]["dur"])
        lines.append(f"| `{key[0]}` | {legs.get(key, '')} | {key[1]} | {len(d)} | "
                     f"{np.median(d):.1f} | {d.mean():.1f} | {d.min():.1f} | {d.max():.1f} | "
                     f"{100 * d.sum() / total:.2f} |")
    counters_txt = None
    fpath = _find(os.path.join(dirpath, "prof_fetch"), "counter_collection.csv")
    wpath = _find(os.path.join(dirpath, "prof_write"), "counter_collection.csv")
    if fpath and wpath:
        vals = {}
        for name, path in (("FETCH_SIZE", fpath), ("WRITE_SIZE", wpath)):
            for r in _read_csv(path):
                if r["Counter_Name"] != name:
                    continue
                key = (_short_kernel(r["Kernel_Name"]), int(r["Grid_Size"]))
                vals.setdefault(key, {}).setdefault(name, []).append(float(r["Counter_Value"]))
        tri = [k for k in vals if k[0] == "spt::k_triad"]
        if not tri:
            raise SystemExit("no triad dispatch in the counter runs: cannot calibrate")
        ff = TRIAD_READ_BYTES / 1024 / np.mean(vals[tri[0]]["FETCH_SIZE"])
        wf = TRIAD_WRITE_BYTES / 1024 / np.mean(vals[tri[0]]["WRITE_SIZE"])
        lines += ["", "## HBM traffic per dispatch (FETCH_SIZE, then WRITE_SIZE, separate runs)",
                  "", f"Calibration: the triad reads {TRIAD_READ_BYTES} and writes "
                  f"{TRIAD_WRITE_BYTES} bytes; FETCH_SIZE reports "
                  f"{np.mean(vals[tri[0]]['FETCH_SIZE']):.0f} KiB (bytes = KiB x 1024 x "
                  f"{ff:.4f}), WRITE_SIZE {np.mean(vals[tri[0]]['WRITE_SIZE']):.0f} KiB "
                  f"(x {wf:.4f}).", "",
                  "| kernel | leg | grid | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | "
                  "GB read | GB written |", "|---|---|---|---|---|---|---|---|"]
        clines = ["# HBM bytes per dispatch of the MTTKRP legs of bench.py --profile "
                  "(powerlaw3, 1e8 entries, R = 32), calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE",
                  "# command: " + PROFILE_CMD,
                  f"# calibration from the triad: fetch x{ff:.4f}, write x{wf:.4f}",
                  f"kernel_source_hash = {kernel_source_hash()}"]
        ctr_legs = _profile_variants({k: {"first": min(groups.get(k, {"first": 1 << 62})["first"],
                                                       1 << 62)} for k in vals})
        for key in sorted(vals, key=lambda k: -np.mean(vals[k].get("FETCH_SIZE", [0]))):
            fk = np.mean(vals[key].get("FETCH_SIZE", [np.nan]))
            wk = np.mean(vals[key].get("WRITE_SIZE", [np.nan]))
            rb, wb = fk * 1024 * ff, wk * 1024 * wf
            leg = ctr_legs.get(key, "")
            lines.append(f"| `{key[0]}` | {leg} | {key[1]} | "
                         f"{len(vals[key].get('FETCH_SIZE', []))} | {fk:.0f} | {wk:.0f} | "
                         f"{rb / 1e9:.3f} | {wb / 1e9:.3f} |")
            if leg:
                clines += [f"{leg}.kernel = {key[0]}", f"{leg}.grid = {key[1]}",
                           f"{leg}.fetch_kib_per_dispatch = {fk:.1f}",
                           f"{leg}.write_kib_per_dispatch = {wk:.1f}",
                           f"{leg}.hbm_bytes_per_dispatch = {rb + wb:.0f}"]
        counters_txt = "\n".join(clines) + "\n"
    return "\n".join(lines) + "\n", counters_txt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--quick", action="store_true", help="skip the extra workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="write the rocprofv3 summaries of a profiled --profile run (DIR holds "
                         "prof_trace/, prof_fetch/, prof_write/) into profiles/ and exit")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: the R=32 legs only (sorted copies 3 warm-up "
                         "+ 5 timed steps, gather, atomic, FP64 sorted copies), plus one triad "
                         "over 3 x 1 GiB (the counter calibration kernel)")
    args = ap.parse_args()
    if args.summarize_profile:
        md, ctr = summarize_profile(args.summarize_profile)
        with open(os.path.join(ROOT, "profiles", "mttkrp_powerlaw3_R32.md"), "w") as fh:
            fh.write(md)
        if ctr is not None:
            with open(COUNTERS_FILE, "w") as fh:
                fh.write(ctr)
        print(md)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    sys.path.insert(0, ROOT)
    import paper_1809_09175_amd as spt
    from paper_1809_09175_amd import datagen

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    X = datagen.powerlaw3()
    log(f"generated powerlaw3 ({X.nnz} entries) in {time.time() - t0:.1f}s")
    # ingest: host (pageable numpy) -> device copies, then packing into records
    torch.empty(1, device=dev)
    torch.cuda.synchronize()
    t0 = time.time()
    subs = torch.from_numpy(X.subs).to(dev)
    vals = torch.from_numpy(X.vals).to(dev)
    torch.cuda.synchronize()
    h2d_ms = (time.time() - t0) * 1e3
    t0 = time.time()
    T = spt.SparseTensor(subs, vals, X.dims)
    T.validate()
    pack_ms = (time.time() - t0) * 1e3
    del subs, vals

    def timed(fn, reps=1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    # permutation build (excluded from MTTKRP time, reported against a CP-ALS sweep)
    T.permute()
    torch.cuda.synchronize()
    sort_ms = timed(lambda: T.permute())
    log(f"permutation build, all modes: {sort_ms:.2f} ms")

    d = X.d
    P = X.nnz

    def factors_for(R, dtype=np.float32):
        return [torch.from_numpy(a).to(dev) for a in datagen.factors(X.dims, R, seed=7, dtype=dtype)]

    def run_modes(R, algo, A, outs, events=None):
        for n in range(d):
            if events is not None:
                events[n][0].record(stream)
            spt.mttkrp(T, A, n, algo=algo, out=outs[n])
            if events is not None:
                events[n][1].record(stream)

    def measure(R, algo, steps, warmup, A=None):
        A = A if A is not None else factors_for(R)
        outs = [torch.empty((I, R), dtype=torch.float32, device=dev) for I in X.dims]
        for _ in range(warmup):
            run_modes(R, algo, A, outs)
        torch.cuda.synchronize()
        per_mode = np.zeros(d)
        ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
               for _ in range(d)] for _ in range(steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for k in range(steps):
            run_modes(R, algo, A, outs, ev[k])
        g1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        total_ms = g0.elapsed_time(g1)
        for k in range(steps):
            for n in range(d):
                per_mode[n] += ev[k][n][0].elapsed_time(ev[k][n][1])
        per_mode /= steps
        ms_step = total_ms / steps
        gbs = P * model_bytes(d, R) * d / (ms_step * 1e-3) / 1e9
        return {"ms_per_step": ms_step, "gbs": gbs, "per_mode_ms": per_mode.tolist(),
                "wall_s": wall}

    R = args.rank
    # mode-sorted record copies: built once, like the permutations
    T.sort_copy()
    torch.cuda.synchronize()
    copy_ms = timed(lambda: T.sort_copy())
    log(f"sorted record copies, all modes: {copy_ms:.2f} ms")
    if args.profile:
        args.steps, args.warmup, args.quick, args.no_cpu = 5, 3, True, True
        n = 1 << 28
        a = torch.empty(n, dtype=torch.float32, device=dev)
        b = torch.rand(n, dtype=torch.float32, device=dev)
        c = torch.rand(n, dtype=torch.float32, device=dev)
        spt.stream_triad(a, b, c)
        torch.cuda.synchronize()
        del a, b, c
    main_res = measure(R, "permuted_copy", args.steps, args.warmup)
    log(f"R={R} permuted (sorted copies): {main_res['ms_per_step']:.3f} ms/step, {main_res['gbs']:.0f} GB/s")
    gather_res = measure(R, "permuted", max(2, args.steps // 2), min(args.warmup, 2))
    log(f"R={R} permuted (gather): {gather_res['ms_per_step']:.3f} ms/step, {gather_res['gbs']:.0f} GB/s")
    atomic_res = measure(R, "atomic", max(2, args.steps // 2), 2)
    log(f"R={R} atomic:   {atomic_res['ms_per_step']:.3f} ms/step, {atomic_res['gbs']:.0f} GB/s")
    touched = touched_rows(X)
    # the paper's arithmetic (Sec. 7: FP64 values and factors): the same tensor with FP64
    # values (32-byte records), FP64 factors and V, sorted copies, all modes
    T64 = spt.SparseTensor(torch.from_numpy(X.subs).to(dev),
                           torch.from_numpy(X.vals.astype(np.float64)).to(dev), X.dims)
    T64.validate()
    T64.permute()
    T64.sort_copy()
    A64 = factors_for(R, np.float64)
    outs64 = [torch.empty((I, R), dtype=torch.float64, device=dev) for I in X.dims]
    for _ in range(args.warmup):
        for n in range(d):
            spt.mttkrp(T64, A64, n, out=outs64[n])
    ev64 = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in range(d)]
    f64_mode_ms = np.zeros(d)
    f64_steps = max(2, args.steps // 2)
    torch.cuda.synchronize()
    for _ in range(f64_steps):
        for n in range(d):
            ev64[n][0].record(stream)
            spt.mttkrp(T64, A64, n, out=outs64[n])
            ev64[n][1].record(stream)
        torch.cuda.synchronize()
        f64_mode_ms += [ev64[n][0].elapsed_time(ev64[n][1]) for n in range(d)]
    f64_mode_ms /= f64_steps
    f64_ms = float(f64_mode_ms.sum())
    f64_model = P * model_bytes(d, R, s_val=8, s_f=8, s_out=8) * d
    f64_res = {"ms_per_step": round(f64_ms, 3),
               "model_gbs": round(f64_model / (f64_ms * 1e-3) / 1e9, 1),
               "per_mode_ms": [round(x, 4) for x in f64_mode_ms]}
    log(f"R={R} FP64 permuted (sorted copies): {f64_ms:.3f} ms/step")
    del T64, A64, outs64
    torch.cuda.empty_cache()

    extras = {}
    per_rank = {}
    if not args.quick:
        for r in (16, 32, 64):
            if r == R:
                per_rank[str(r)] = {"permuted_copy_gbs": round(main_res["gbs"], 1),
                                    "permuted_gbs": round(gather_res["gbs"], 1),
                                    "atomic_gbs": round(atomic_res["gbs"], 1),
                                    "permuted_copy_ms": round(main_res["ms_per_step"], 3),
                                    "permuted_ms": round(gather_res["ms_per_step"], 3),
                                    "atomic_ms": round(atomic_res["ms_per_step"], 3)}
                continue
            pc = measure(r, "permuted_copy", 5, 1)
            p = measure(r, "permuted", 5, 1)
            a = measure(r, "atomic", 3, 1)
            b = measure(r, "permuted_copy", 5, 2, A=[spt.to_bf16(x) for x in factors_for(r)])
            per_rank[str(r)] = {"permuted_copy_gbs": round(pc["gbs"], 1),
                                "permuted_gbs": round(p["gbs"], 1), "atomic_gbs": round(a["gbs"], 1),
                                "permuted_copy_ms": round(pc["ms_per_step"], 3),
                                "permuted_ms": round(p["ms_per_step"], 3),
                                "atomic_ms": round(a["ms_per_step"], 3),
                                "bf16_permuted_copy_ms": round(b["ms_per_step"], 3),
                                "bf16_speedup": round(pc["ms_per_step"] / b["ms_per_step"], 3)}
            log(f"R={r}: permuted copy {pc['gbs']:.0f}, gather {p['gbs']:.0f}, atomic {a['gbs']:.0f} GB/s")
        # BF16 factors on the same tensor
        A32 = factors_for(R)
        A16 = [spt.to_bf16(a) for a in A32]
        # same step and warmup counts as the FP32 figure it is compared with
        b16 = measure(R, "permuted_copy", args.steps, max(args.warmup, 2), A=A16)
        extras["bf16_factors_same_tensor"] = {
            "ms_per_step": round(b16["ms_per_step"], 3),
            "speedup_vs_fp32": round(main_res["ms_per_step"] / b16["ms_per_step"], 3)}
        log(f"BF16 factors: {b16['ms_per_step']:.3f} ms/step")
        if str(R) in per_rank:
            per_rank[str(R)]["bf16_permuted_copy_ms"] = round(b16["ms_per_step"], 3)
            per_rank[str(R)]["bf16_speedup"] = extras["bf16_factors_same_tensor"]["speedup_vs_fp32"]
        # one CP-ALS sweep (FP32 factors, permuted MTTKRP) and the fit
        st = spt.CPState(T, factors_for(R))
        st.sweep()
        torch.cuda.synchronize()
        sweep_ms = timed(lambda: st.sweep(), reps=3)
        t_fit = time.perf_counter()
        st.fit()
        fit_ms = (time.perf_counter() - t_fit) * 1e3
        st.fit(source="mttkrp")  # the handle's first call also sums ||X||^2
        t_fit = time.perf_counter()
        st.fit(source="mttkrp")
        fast_fit_ms = (time.perf_counter() - t_fit) * 1e3
        extras["cp_als_sweep_ms"] = round(sweep_ms, 3)
        extras["cp_fit_ms"] = round(fit_ms, 3)
        extras["cp_fit_from_mttkrp_ms"] = round(fast_fit_ms, 3)
        # one iteration as cp_als runs it: a sweep and the fit from the last mode's MTTKRP
        iter_ms = sweep_ms + fast_fit_ms
        extras["cp_als_iteration_ms"] = round(iter_ms, 3)
        extras["sort_ms_all_modes"] = round(sort_ms, 3)
        extras["sorted_copy_ms_all_modes"] = round(copy_ms, 3)
        extras["ingest_h2d_ms"] = round(h2d_ms, 1)
        extras["ingest_pack_validate_ms"] = round(pack_ms, 1)
        extras["ingest_to_permuted"] = bench_ingest(spt, torch, X, dev)
        # memory side of the trade: one record array per mode beside the records themselves
        lib = spt._lib.load()
        extras["sorted_copy_bytes_all_modes"] = int(lib.spt_tensor_sorted_copy_bytes(T.handle, -1, 1))
        extras["tensor_workspace_bytes"] = int(T.ws.numel())
        extras["one_gpu_share_of_8"] = bench_shard_share(spt, torch, T, X, dev, R, shards=8)
        extras["sort_over_cp_als_iteration"] = round(sort_ms / iter_ms, 3)
        extras["sort_and_copy_over_cp_als_iteration"] = round((sort_ms + copy_ms) / iter_ms, 3)
        log(f"CP-ALS sweep {sweep_ms:.2f} ms, fit {fit_ms:.2f} ms (from the MTTKRP {fast_fit_ms:.2f} ms)")
        del st
        # the rank of the paper's CP-ALS experiment (Sec. 7.1): R = 128, FP32 factors
        st = spt.CPState(T, factors_for(128))
        st.sweep()
        torch.cuda.synchronize()
        extras["cp_als_sweep_ms_R128"] = round(timed(lambda: st.sweep(), reps=2), 3)
        log(f"CP-ALS sweep at R = 128: {extras['cp_als_sweep_ms_R128']:.2f} ms")
        del st
        # STREAM-style triad on 3 x 1 GiB
        n = 1 << 28
        a = torch.empty(n, dtype=torch.float32, device=dev)
        b = torch.rand(n, dtype=torch.float32, device=dev)
        c = torch.rand(n, dtype=torch.float32, device=dev)
        spt.stream_triad(a, b, c)
        tri_ms = timed(lambda: spt.stream_triad(a, b, c), reps=10)
        triad_gbs = 3 * 4 * n / (tri_ms * 1e-3) / 1e9
        extras["stream_triad_gbs"] = round(triad_gbs, 1)
        extras["pct_of_measured_stream"] = round(100.0 * main_res["gbs"] / triad_gbs, 1)
        del a, b, c
        log(f"triad {triad_gbs:.0f} GB/s")
        extras["skewed4_bf16_vs_fp32"] = bench_skewed4_bf16(spt, datagen, torch, dev)
        extras["batch64"] = bench_batch64(spt, datagen, torch, dev)
        extras["gcp_poisson"] = bench_gcp(spt, datagen, torch, dev)

    # roofline of the dominant kernel (the permuted MTTKRP over sorted copies) and of the other
    # two traversals; per launch = one mode.  Three byte counts per launch: the paper's model
    # (the metric; factor rows counted at every use, so it exceeds the HBM peak when they hit in
    # cache), the HBM bytes rocprofv3's counters saw (calibrated), and the compulsory bytes.
    counters = read_counters()
    dtune = spt.default_tune(T, 0, R, torch.float32, algo="permuted_copy")
    kname = f"spt::k_mttkrp_perm<3, {dtune['lanes']}, {dtune['cols']}, float, float, float>"

    def kernel_roofline(variant, res, rec_bytes, extra, s_val=4, s_f=4, s_out=4):
        avg_ms = float(np.mean(res["per_mode_ms"]))
        model = P * model_bytes(d, R, s_val=s_val, s_f=s_f, s_out=s_out)
        comp = float(np.mean([compulsory_bytes(touched, n, R, rec_bytes, s_f, s_out, extra, P)
                              for n in range(d)]))
        c = counters.get(variant)
        r = {"avg_launch_ms": round(avg_ms, 4),
             "model_bytes": model, "model_gbs": round(model / (avg_ms * 1e-3) / 1e9, 1),
             "compulsory_bytes": round(comp),
             "compulsory_gbs": round(comp / (avg_ms * 1e-3) / 1e9, 1),
             "compulsory_frac": round(comp / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "counter_bytes": None, "counter_gbs": None, "counter_frac": None,
             "counter_over_compulsory": None}
        if c is not None:
            r["kernel"] = c["kernel"]
            r["counter_bytes"] = c["bytes"]
            r["counter_gbs"] = round(c["bytes"] / (avg_ms * 1e-3) / 1e9, 1)
            r["counter_frac"] = round(c["bytes"] / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            r["counter_over_compulsory"] = round(c["bytes"] / comp, 3)
        return r

    kr = {"permuted_copy": kernel_roofline("copy", main_res, 16, 0),
          "permuted_gather": kernel_roofline("gather", gather_res, 16, 4),
          "atomic": kernel_roofline("atomic", atomic_res, 16, 0),
          "permuted_copy_f64": kernel_roofline("copy_f64", f64_res, 32, 0, 8, 8, 8)}
    dom = kr["permuted_copy"]
    have = dom["counter_bytes"] is not None
    # achieved = HBM bytes per launch (calibrated counters) over the live average launch time;
    # without current counters, the compulsory bytes (a lower bound) stand in and say so
    achieved = dom["counter_gbs"] if have else dom["compulsory_gbs"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": dom["counter_bytes"],
                "bytes_basis": "rocprofv3 FETCH_SIZE/WRITE_SIZE per launch, calibrated" if have
                               else "compulsory bytes (counters absent for this kernel source)",
                "kernel": kname + " reading the sorted record copies",
                "avg_launch_ms": dom["avg_launch_ms"],
                "model_bytes_per_launch": dom["model_bytes"], "model_gbs": dom["model_gbs"],
                "compulsory_bytes_per_launch": dom["compulsory_bytes"],
                "compulsory_frac": dom["compulsory_frac"],
                "traffic_over_compulsory": dom["counter_over_compulsory"],
                "kernels": kr}

    cpu = None
    if not args.no_cpu:
        import oracle
        S = 40_000_000
        A = [a.astype(np.float64) for a in datagen.factors(X.dims, R, seed=7, dtype=np.float32)]
        sub_s, sub_v = X.subs[:S], X.vals[:S]
        t = time.perf_counter()
        for n in range(d):
            oracle.mttkrp(sub_s, sub_v, X.dims, A, n)
        cpu_s = time.perf_counter() - t
        model = "unknown CPU"
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        cpu = {"value": round(S * model_bytes(d, R) * d / cpu_s / 1e9, 3), "unit": "GB/s",
               "cores": 1, "kind": "oracle",
               "host": f"1 of {os.cpu_count()} logical CPUs, {model}",
               "sample": f"first {S} of {P} entries of the same tensor, all {d} modes, R={R}, "
                         f"FP64 single-threaded ({cpu_s:.1f} s)"}
        log(f"CPU oracle: {cpu['value']} GB/s effective on the sample")

    out = {
        "metric": "MTTKRP effective HBM GB/s (% of peak), permuted vs atomic; BF16/batched vs FP32 speedup",
        "value": round(main_res["gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "powerlaw3: 3-way 500000x500000x20000, 1e8 entries, Zipf(1.1) "
                               "per mode, FP32 values and factors, all-mode MTTKRP",
                   "rank": R, "algo": "permuted traversal over mode-sorted record copies",
                   "nnz": P},
        "pct_of_hbm_peak": round(100.0 * main_res["gbs"] / HBM_PEAK_GBS, 1),
        "gflops": round(P * d * (d + 1) * R / (main_res["ms_per_step"] * 1e-3) / 1e9, 1),
        "permuted_gather": {"gbs": round(gather_res["gbs"], 1),
                            "ms_per_step": round(gather_res["ms_per_step"], 4),
                            "note": "same traversal gathering each record through the permutation"},
        "atomic": {"gbs": round(atomic_res["gbs"], 1), "ms_per_step": round(atomic_res["ms_per_step"], 4),
                   "permuted_speedup": round(atomic_res["ms_per_step"] / main_res["ms_per_step"], 3),
                   "permuted_gather_speedup": round(atomic_res["ms_per_step"] / gather_res["ms_per_step"], 3)},
        "per_mode_ms": [round(x, 4) for x in main_res["per_mode_ms"]],
        "fp64": dict(f64_res, note="FP64 values (32-byte records), factors and V, as in the "
                                   "paper's experiments; permuted traversal over sorted copies"),
        "per_rank": per_rank,
        "extras": extras,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
