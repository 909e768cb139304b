#!/usr/bin/env python3
"""PbP-QLP benchmark on one MI355X: ms per factorization, plain FP32 versus
the mixed-precision plan, with each result's error against the FP64 oracle.

Workload (default): the 16384 x 16384 FP32 planted-spectrum matrix
(U, V from QR of seeded Gaussian 16384 x 512 panels, sigma_i = 1/i for
i <= 512, plus 1e-6 N(0,1)), k = 200, p = 20 (l = 220), q = 2.  A step is one
whole factorization (sketch, 2q power passes with re-orthonormalization,
projection, QR of B^T, QR of R^T, Q Qt) on the resident matrix.

    python bench.py [--steps K] [--warmup W] [--cpu-baseline full|none]
    python bench.py --workload c3|c4|c5|tables|sparse [--steps K] [--warmup W]

Prints one JSON line on stdout; progress goes to stderr.

Timing: `value` is the wall-clock time of K factorizations with tracing off,
between device synchronizations.  The same K factorizations are then run again
with a HIP event pair around every kernel the library launches (on the
library's stream); these give the per-kernel table, the kernel with the most
time per factorization and its roofline (algorithmic bytes or flops per launch
over its mean event-timed duration).  A plain 1 GiB device copy is timed
beside it as a measured HBM peak.

--workload c3 is the tall low-rank-plus-noise matrix: 200000 x 4096 FP32,
X Y^T with X, Y entries N(0, 1/64) (rank 64) plus 1e-3 N(0,1), k = 64, p = 16,
q = 1; the FP16 plan (every pass on FP16 matrix cores, FP32 accumulation)
against the FP32 plan on the same matrix, each against the FP64 oracle.

--workload c4 measures the batched form instead: 1024 FP32 matrices,
m ~ U[256, 4096], n ~ U[256, 2048], rank r ~ U[8, 64] with sigma_i = exp(-i/r)
plus 1e-5 N(0,1) (generated on the GPU from seeded generators, U and V from
QR of Gaussian panels), k = r, p = 8, q = 1; one graph launch for the whole
batch against one pbpqlp_factor call per matrix, with a sample of problems
checked against the FP64 oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2.json")
STREAM_SRC = os.path.join(ROOT, "paper_2103_07245_amd", "csrc", "stream_gemm.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# MI355X published peaks: HBM3E bandwidth and dense matrix-core rates
PEAK = {"hbm": 8000.0, "mfma_bf16": 2500.0, "mfma_fp16": 2500.0, "mfma_fp32": 157.3, "mfma_fp64": 78.6}


def run_plan(B, torch, A_dev, w, plan, steps, warmup):
    """Time one precision plan on the resident matrix.

    Region 1 (the `value`): `steps` factorizations with tracing off, bracketed
    by device synchronizations.  Region 2: the same `steps` factorizations with
    a HIP event pair around every kernel the library launches (on its stream),
    which gives the per-kernel durations and the dominant kernel."""
    f = B.Factorizer(w.A.shape[0], w.A.shape[1], w.k, w.p, w.q, torch.float32, plan, A_dev.device)
    for _ in range(warmup):
        f(A_dev, w.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f(A_dev, w.seed)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    B.trace_reset()
    B.trace_enable(2)
    t0 = time.perf_counter()
    for _ in range(steps):
        f(A_dev, w.seed)
    torch.cuda.synchronize()
    ms_traced = (time.perf_counter() - t0) * 1e3 / steps
    B.trace_enable(0)
    recs = B.trace_records()
    B.trace_reset()
    Q, L, P = (x.cpu().numpy() for x in (f.Q, f.L, f.P))
    return dict(ms=ms, ms_traced=ms_traced, kernels=kernel_table(recs, steps), Q=Q, L=L, P=P,
                info=f.info())


def kernel_bound(name):
    """Resource that bounds a kernel of the library: the streaming products
    in 16-bit modes (and split-BF16x3) stream A from HBM; in FP32/FP64 they are
    matrix-core bound; the Gram is an FP64 matrix-core product; the Cholesky
    is the latency of its pivot chain (reported against FP64 rate)."""
    if name.startswith(("k1_", "k2_")):
        mode = name[3:]
        if mode == "f32":
            return "mfma", "mfma_fp32"
        if mode == "f64":
            return "mfma", "mfma_fp64"
        return "hbm", "hbm"
    if name.startswith(("gram", "chol", "r2r1")):
        return "mfma", "mfma_fp64"
    return "hbm", "hbm"


def kernel_table(recs, steps):
    tab = {}
    for name, by, fl, ms in recs:
        t = tab.setdefault(name, {"launches": 0, "ms": 0.0, "bytes": by, "flops": fl})
        t["launches"] += 1
        t["ms"] += ms
    for name, t in tab.items():
        t["ms_per_step"] = t["ms"] / steps
        t["avg_ms"] = t["ms"] / t["launches"]
        t["gbs"] = t["bytes"] / (t["avg_ms"] * 1e-3) / 1e9
        t["tflops"] = t["flops"] / (t["avg_ms"] * 1e-3) / 1e12
        bound, peak = kernel_bound(name)
        t["bound"], t["peak_key"] = bound, peak
        t["frac"] = (t["gbs"] if bound == "hbm" else t["tflops"]) / PEAK[peak]
    return tab


def copy_peak(torch, dev, reps=10):
    """Measured HBM peak of a plain device copy (1 GiB read + 1 GiB written),
    HIP events around each copy, best of `reps`."""
    src = torch.empty(2 ** 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2 * 2 ** 30 / (best * 1e-3) / 1e9


def roofline_of(tab, steps, traffic_file=TRAFFIC_FILE):
    """Roofline object for the kernel with the most time per step."""
    dom_name, dom = max(tab.items(), key=lambda kv: kv[1]["ms_per_step"])
    bound, peak_key = dom["bound"], dom["peak_key"]
    hbm = bound == "hbm"
    achieved = dom["gbs"] if hbm else dom["tflops"]
    traffic = None
    if os.path.exists(traffic_file):
        try:
            tr = json.load(open(traffic_file))
            if tr.get("stream_gemm_sha") == _sha(STREAM_SRC) and dom_name in tr.get("kernels", {}):
                traffic = tr["kernels"][dom_name]["hbm_bytes_per_launch"]
        except Exception:
            traffic = None
    return {"bound": bound, "kernel": dom_name, "achieved": round(achieved, 1 if hbm else 2),
            "peak": PEAK[peak_key], "unit": "GB/s" if hbm else "TFLOP/s",
            "frac": round(achieved / PEAK[peak_key], 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": dom["bytes"], "algorithmic_flops_per_launch": dom["flops"],
            "avg_launch_ms": round(dom["avg_ms"], 5), "launches_per_step": dom["launches"] / steps,
            "ms_per_step": round(dom["ms_per_step"], 4)}


# ---------------------------------------------------------------------------
# Summaries of rocprofv3 output (run separately; see profiles/):
#   python bench.py --summarize-counters FETCH_DIR WRITE_DIR [MFMA_DIR]
# reads the counter-collection CSVs of rocprofv3 --pmc runs of this bench and
# writes profiles/traffic_c2.json (HBM bytes per launch of each streaming
# kernel, calibrated on the 1 GiB copy the runs include) and prints a
# markdown table; MFMA_DIR (a run with SQ_INSTS_VALU_MFMA_MOPS_* counters)
# adds the matrix-core flops each kernel executed.
# ---------------------------------------------------------------------------
MODE_NAMES = {0: "f64", 1: "f32", 2: "bf16", 3: "fp16", 4: "bf16x3"}


def trace_name(kernel):
    """Bench trace name (k1_bf16, ...) of a streaming kernel's rocprofv3 name."""
    import re
    m = re.search(r"stream_k1_kernel<(\d+),", kernel)
    if m:
        return "k1_" + MODE_NAMES[int(m.group(1))]
    m = re.search(r"stream_kernel<(\d+), *\d+, *(true|false),", kernel)
    if m:
        return ("k2_" if m.group(2) == "true" else "k1_") + MODE_NAMES[int(m.group(1))]
    if "copyBuffer" in kernel:
        return "copy"
    return None


def read_counters(d):
    """{(trace name, counter): [values per dispatch]} from rocprofv3 CSVs under d."""
    import csv
    import glob
    out = {}
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    for fn in files:
        with open(fn) as f:
            for row in csv.DictReader(f):
                name = trace_name(row.get("Kernel_Name", ""))
                if name is None:
                    continue
                out.setdefault((name, row["Counter_Name"]), []).append(float(row["Counter_Value"]))
    return out


def summarize_counters(fetch_dir, write_dir, mfma_dir=None):
    fc, wc = read_counters(fetch_dir), read_counters(write_dir)
    copy_bytes = 2 ** 30
    ff = copy_bytes / (1024 * max(fc[("copy", "FETCH_SIZE")]))
    wf = copy_bytes / (1024 * max(wc[("copy", "WRITE_SIZE")]))
    kernels = {}
    for (name, ctr), vals in fc.items():
        if name == "copy" or ctr != "FETCH_SIZE":
            continue
        wv = wc.get((name, "WRITE_SIZE"), [0.0])
        fb = sum(vals) / len(vals) * 1024 * ff
        wb = sum(wv) / len(wv) * 1024 * wf
        kernels[name] = {"fetch_bytes": fb, "write_bytes": wb, "hbm_bytes_per_launch": fb + wb,
                         "dispatches": [len(vals), len(wv)]}
    mfma = read_counters(mfma_dir) if mfma_dir else {}
    for (name, ctr), vals in mfma.items():
        if name in kernels and ctr.startswith("SQ_INSTS_VALU_MFMA_MOPS"):
            # counted in units of 512 floating-point operations
            kernels[name].setdefault("mfma_flops_per_launch", 0.0)
            kernels[name]["mfma_flops_per_launch"] += sum(vals) / len(vals) * 512
    out = {"workload": "16384x16384 fp32, l=220 (C2)", "stream_gemm_sha": _sha(STREAM_SRC),
           "method": "rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE (KiB per dispatch), each scaled by "
                     "the factor that makes the 1 GiB device copy read/write exactly 1 GiB",
           "calibration": {"copy_bytes": copy_bytes, "fetch_factor": ff, "write_factor": wf},
           "kernels": kernels}
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print("| kernel | HBM fetch (GB) | HBM write (GB) | HBM total (GB) | matrix-core GFLOP |")
    print("|---|---:|---:|---:|---:|")
    for k, v in sorted(kernels.items()):
        mf = v.get("mfma_flops_per_launch")
        print(f"| `{k}` | {v['fetch_bytes'] / 1e9:.4f} | {v['write_bytes'] / 1e9:.4f} | "
              f"{v['hbm_bytes_per_launch'] / 1e9:.4f} | {mf / 1e9 if mf else float('nan'):.1f} |")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-baseline", choices=["full", "none"], default="full",
                    help="time the FP64 oracle on one factorization of the same matrix")
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5", "tables", "sparse"], default="c2")
    ap.add_argument("--sparse-m", type=int, default=2_000_000)
    ap.add_argument("--sparse-n", type=int, default=1_000_000)
    ap.add_argument("--sparse-nnz-row", type=int, default=20)
    ap.add_argument("--tables-n", default="", help="tables: comma-separated orders n (default: the paper's)")
    ap.add_argument("--model", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                    "paper_2103_07245_amd", "weights", "qk_mlp.bin"),
                    help="c5: trained q/k network")
    ap.add_argument("--plan", default=None,
                    help="precision plan: c4 batch (default mixed; the per-matrix baseline is always the "
                         "plain FP32 method), c5 (default native)")
    ap.add_argument("--count", type=int, default=1024, help="c4 batch size")
    ap.add_argument("--skip-per-matrix", action="store_true", help="c4: skip the per-matrix timing")
    ap.add_argument("--no-tune", action="store_true", help="c4: use the built-in batch plan, not the autotuner's")
    ap.add_argument("--host-resident", action="store_true",
                    help="c2/c3: also time the factorization with A in pinned host memory")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (for counter calibration)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="FETCH_DIR WRITE_DIR [MFMA_DIR]: summarize rocprofv3 --pmc runs of this bench")
    args = ap.parse_args()
    if args.summarize_counters:
        return summarize_counters(*args.summarize_counters)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2103_07245_amd import pbpqlp as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    B.library()
    if args.workload == "c4":
        return bench_c4(args, torch, np, synth, B, dev)
    if args.workload == "c5":
        return bench_c5(args, torch, np, synth, B, dev)
    if args.workload == "tables":
        return bench_tables(args, torch, np, synth, B, dev)
    if args.workload == "sparse":
        return bench_sparse(args, torch, np, synth, B, dev)

    return bench_single(args, torch, np, synth, B, dev)


# single-matrix workloads: (generator, flagship plan, baseline plan, description)
SINGLE = {
    "c2": ("config2", "mixed", "native",
           "16384x16384 fp32, sigma_i=1/i (i<=512) + 1e-6 N(0,1), k=200 p=20 q=2",
           "sketch bf16, power bf16, projection split-bf16x3; FP64 Grams and l x l factors", "bf16"),
    "c3": ("config3", "fp16", "native",
           "200000x4096 fp32, X Y^T (rank 64, N(0,1/64) entries) + 1e-3 N(0,1), k=64 p=16 q=1",
           "sketch, power and projection fp16 MFMA with FP32 accumulation; FP64 Grams and l x l factors",
           "fp16"),
}


def bench_single(args, torch, np, synth, B, dev):
    gen, flag_plan, base_plan, desc, plan_desc, flag_dtype = SINGLE[args.workload]
    t = time.time()
    w = getattr(synth, gen)()
    m, n, l, q = w.A.shape[0], w.A.shape[1], w.l, w.q
    log(f"generated {m}x{n} FP32 workload in {time.time() - t:.1f}s")
    A_dev = torch.from_numpy(w.A).to(dev)
    torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.empty(2 ** 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("ran 1 GiB calibration copy")
    copy_gbs = copy_peak(torch, dev)
    log(f"plain 1 GiB device copy: {copy_gbs:.1f} GB/s (read + write)")

    results = {}
    for plan in (base_plan, flag_plan):
        r = run_plan(B, torch, A_dev, w, plan, args.steps, args.warmup)
        results[plan] = r
        log(f"plan {plan}: {r['ms']:.3f} ms/factorization ({r['ms_traced']:.3f} ms with every kernel traced)")

    # errors against the FP64 oracle on the same stored matrix (host, FP64)
    from oracle import rel_residual
    for plan, r in results.items():
        r["resid"] = rel_residual(w.A, r["Q"], r["L"], r["P"])
        r["orth_q"] = float(np.abs(r["Q"].astype(np.float64).T @ r["Q"].astype(np.float64) - np.eye(l)).max())
        r["orth_p"] = float(np.abs(r["P"].astype(np.float64).T @ r["P"].astype(np.float64) - np.eye(l)).max())
        log(f"plan {plan}: residual {r['resid']:.6e}")

    cpu = None
    r_oracle = None
    if args.cpu_baseline == "full":
        from oracle import pbpqlp as oracle_pbpqlp
        try:
            import threadpoolctl
            threads = max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) or 1
        except Exception:
            threads = os.cpu_count() or 1
        log(f"timing the FP64 oracle on {threads} threads ...")
        t0 = time.perf_counter()
        ref = oracle_pbpqlp(w.A, w.k, w.p, w.q, w.seed)
        t_or = time.perf_counter() - t0
        r_oracle = rel_residual(w.A, ref.Q, ref.L, ref.P)
        log(f"oracle: {t_or:.1f}s, residual {r_oracle:.6e}")
        cpu = {"value": t_or * 1e3, "unit": "ms/factorization", "cores": int(threads), "kind": "oracle",
               "sample": f"one whole factorization of the same {m}x{n} matrix (k={w.k}, p={w.p}, q={q}) "
                         "by the FP64 oracle: numpy/OpenBLAS products with A, Householder QR"}

    host = None
    if args.host_resident:
        # the same factorization with A left in pinned host memory: every pass
        # streams A over PCIe in row panels (not the timed `value`)
        Ah = torch.from_numpy(w.A).pin_memory()
        for _ in range(1):
            B.factor_host(Ah, w.k, w.p, w.q, w.seed, plan=flag_plan)
        torch.cuda.synchronize()
        hs = max(1, min(args.steps, 5))
        t0 = time.perf_counter()
        for _ in range(hs):
            Qh, Lh, Ph, _ = B.factor_host(Ah, w.k, w.p, w.q, w.seed, plan=flag_plan)
        torch.cuda.synchronize()
        ms_h = (time.perf_counter() - t0) * 1e3 / hs
        r_h = rel_residual(w.A, *(x.cpu().numpy() for x in (Qh, Lh, Ph)))
        host = {"ms": round(ms_h, 3), "steps": hs, "plan": flag_plan,
                "pcie_gbs": round((2 * q + 2) * m * n * 4 / (ms_h * 1e-3) / 1e9, 2), "resid": r_h,
                "note": "A in pinned host memory, 2q+2 passes streamed in ~256 MiB row panels"}
        log(f"host-resident A: {ms_h:.2f} ms/factorization ({host['pcie_gbs']} GB/s of A), residual {r_h:.6e}")
        del Ah

    flag = results[flag_plan]
    base = results[base_plan]
    roofline = roofline_of(flag["kernels"], args.steps)
    roofline["copy_kernel_gbs"] = round(copy_gbs, 1)
    if roofline["unit"] == "GB/s":
        roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4)

    passes = 2 * q + 2
    flops = passes * 2.0 * m * n * l
    a_bytes = passes * m * n * 4

    def summary(r):
        ks = r["kernels"]
        stream_ms = sum(v["ms_per_step"] for k, v in ks.items() if k.startswith(("k1_", "k2_")))
        d = {"ms": round(r["ms"], 4), "ms_traced": round(r["ms_traced"], 4),
             "tflops": round(flops / (r["ms"] * 1e-3) / 1e12, 2),
             "hbm_frac_whole_step": round(a_bytes / (r["ms"] * 1e-3) / (PEAK["hbm"] * 1e9), 4),
             "streaming_share": round(stream_ms / r["ms_traced"], 4),
             "resid": r["resid"], "orth_err_q": r["orth_q"], "orth_err_p": r["orth_p"],
             "kernels": {k: {"ms_per_step": round(v["ms_per_step"], 4), "launches": v["launches"] // args.steps,
                             "avg_us": round(v["avg_ms"] * 1e3, 1), "gbs": round(v["gbs"], 1),
                             "tflops": round(v["tflops"], 2), "bound": v["bound"], "frac": round(v["frac"], 4)}
                         for k, v in sorted(ks.items(), key=lambda kv: -kv[1]["ms_per_step"])}}
        if r_oracle is not None:
            d["err_vs_fp64_oracle"] = abs(r["resid"] - r_oracle)
        return d

    line = {
        "metric": "PbP-QLP ms/factorization + %HBM roofline, mixed vs FP32 at stated err vs FP64",
        "value": round(flag["ms"], 4),
        "unit": "ms/factorization",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(flag["ms"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": flag_dtype,
        "data": "synthetic",
        "config": {"workload": desc, "m": m, "n": n, "k": w.k, "p": w.p, "q": q, "plan": flag_plan,
                   "plan_passes": plan_desc},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "oracle_resid": r_oracle,
        "host_resident": host,
        flag_plan: summary(flag),
        "fp32": summary(base),
        f"speedup_{flag_plan}_vs_fp32": round(base["ms"] / flag["ms"], 3),
        "hbm_floor_ms": round(a_bytes / (PEAK["hbm"] * 1e9) * 1e3, 4),
        "algorithmic_tflop_per_factorization": flops / 1e12,
    }
    print(json.dumps(line), flush=True)


# The paper's PbP-QLP runtimes (seconds; MATLAB, FP64, on a 4-core 1.8 GHz
# Intel Core i7 with 8 GB of memory), Section V-A Tables I-III:
# PAPER_SECONDS[d/n][q] = times for n = 5000, 10000, 15000, 20000, 25000.
PAPER_SECONDS = {
    0.04: {0: [0.29, 2.2, 7.1, 16.0, 31.6], 1: [0.53, 4.1, 12.7, 28.7, 56.6], 2: [0.81, 5.9, 18.6, 41.4, 81.7]},
    0.2: {0: [2.1, 15.4, 48.7, 160, 319], 1: [3.3, 24.1, 77.5, 248, 496], 2: [4.3, 33.4, 107, 332, 654]},
    0.3: {0: [3.5, 25.9, 95.0, 285, 601], 1: [5.2, 38.7, 146, 402, 896], 2: [7.0, 51.5, 197, 530, 1201]},
}
TABLE_N = [5000, 10000, 15000, 20000, 25000]


def bench_tables(args, torch, np, synth, B, dev):
    """The paper's runtime experiment (square dense matrices of order n,
    d = 0.04 n, 0.2 n, 0.3 n, q = 0, 1, 2) on the GPU, FP64 as in the paper and
    FP32: seconds per factorization with l = d (k = d, p = 0).  The
    distribution of the singular values does not affect the run time, so A
    is a seeded Gaussian matrix generated on the GPU."""
    ns = [int(x) for x in args.tables_n.split(",")] if args.tables_n else TABLE_N
    rows = []
    t_all = time.time()
    for n in ns:
        gen = torch.Generator(device=dev)
        gen.manual_seed(synth.seed_a(6, n))
        A64 = torch.randn(n, n, generator=gen, device=dev, dtype=torch.float64)
        A32 = A64.float()
        for frac in (0.04, 0.2, 0.3):
            d = int(round(frac * n))
            for q in (0, 1, 2):
                rec = {"n": n, "d": d, "q": q}
                for name, A in (("fp64", A64), ("fp32", A32)):
                    f = B.Factorizer(n, n, d, 0, q, A.dtype, "native", dev)
                    f(A, 1)
                    torch.cuda.synchronize()
                    reps = 2
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        f(A, 1)
                    torch.cuda.synchronize()
                    rec[name + "_s"] = (time.perf_counter() - t0) / reps
                    rec[name + "_resid_est"] = f.info().resid_rel_est
                    del f
                if n in TABLE_N:
                    rec["paper_s"] = PAPER_SECONDS[frac][q][TABLE_N.index(n)]
                    rec["fp64_speedup_vs_paper"] = round(rec["paper_s"] / rec["fp64_s"], 1)
                rows.append(rec)
                log(f"n={n} d={d} q={q}: fp64 {rec['fp64_s'] * 1e3:.1f} ms, fp32 {rec['fp32_s'] * 1e3:.1f} ms"
                    + (f" (paper {rec['paper_s']} s)" if "paper_s" in rec else ""))
        del A64, A32
        torch.cuda.empty_cache()
    big = rows[-1]
    line = {
        "metric": "PbP-QLP seconds per factorization on the paper's runtime shapes (Tables I-III), FP64",
        "value": round(big["fp64_s"], 4), "unit": "s/factorization", "n_gpus": 1, "steps": 2, "warmup": 1,
        "ms_per_step": round(big["fp64_s"] * 1e3, 2), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"square Gaussian n x n, d = 0.04n/0.2n/0.3n, q = 0..2; value: n = {big['n']}, "
                               f"d = {big['d']}, q = {big['q']}", "k": "d", "p": 0},
        "rows": rows, "wall_s": round(time.time() - t_all, 1),
        "paper_hardware": "MATLAB, 4-core Intel Core i7 at 1.8 GHz, 8 GB (Section V)",
    }
    print(json.dumps(line), flush=True)


def bench_sparse(args, torch, np, synth, B, dev):
    """Sparse A in CSR (Section IV-E, O(z d) per product): m x n FP32 with a
    fixed number of nonzeros per row whose column indices follow a power law
    (P(j) proportional to (j + 1)^-0.8: a few nearly dense columns), N(0,1)
    values, generated on the GPU from a seeded generator; k = 64, p = 16,
    q = 1.  A step is one whole factorization including the stable transpose
    of the structure."""
    m, n, per_row = args.sparse_m, args.sparse_n, args.sparse_nnz_row
    k, p, q = 64, 16, 1
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.seed_a(7, 0))
    nnz = m * per_row
    u = torch.rand(nnz, generator=gen, device=dev, dtype=torch.float64)
    cols = torch.clamp((n * u ** (1.0 / 0.2)).long(), max=n - 1)      # inverse CDF of ~ (j/n)^0.2
    rows = torch.arange(m, device=dev).repeat_interleave(per_row)
    key = rows * n + cols
    key = torch.unique(key)                                             # sorted, duplicates dropped
    rows, cols = key // n, key % n
    nnz = key.numel()
    rowptr = torch.zeros(m + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(torch.bincount(rows, minlength=m), 0)
    colind = cols.to(torch.int32).contiguous()
    vals = torch.randn(nnz, generator=gen, device=dev, dtype=torch.float32)
    del u, key, rows, cols
    torch.cuda.synchronize()
    log(f"sparse {m}x{n}, nnz {nnz} ({nnz / m:.1f} per row)")
    for _ in range(args.warmup):
        B.factor_csr(rowptr, colind, vals, (m, n), k, p, q, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Q, L, P, info = B.factor_csr(rowptr, colind, vals, (m, n), k, p, q, 1)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    B.trace_reset()
    B.trace_enable(2)
    for _ in range(args.steps):
        B.factor_csr(rowptr, colind, vals, (m, n), k, p, q, 1)
    torch.cuda.synchronize()
    B.trace_enable(0)
    tab = kernel_table(B.trace_records(), args.steps)
    B.trace_reset()
    roofline = roofline_of(tab, args.steps)
    line = {
        "metric": "PbP-QLP ms/factorization of a sparse CSR matrix (FP32, power-law columns)",
        "value": round(ms, 3), "unit": "ms/factorization", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"CSR {m}x{n}, {per_row} nonzeros per row drawn with P(j) ~ (j+1)^-0.8, N(0,1) "
                               f"values, k={k} p={p} q={q}", "nnz": nnz},
        "roofline": roofline, "resid_est": info.resid_rel_est,
        "kernels": {k_: {"ms_per_step": round(v["ms_per_step"], 4), "launches": v["launches"] // args.steps,
                         "gbs": round(v["gbs"], 1)} for k_, v in sorted(tab.items(), key=lambda kv: -kv[1]["ms_per_step"])},
    }
    print(json.dumps(line), flush=True)


def bench_c4(args, torch, np, synth, B, dev):
    """Batched uneven sizes: one graph launch per batch (mixed plan by default:
    BF16 sketch and power passes, split-BF16x3 projection) against the plain
    FP32 method called once per matrix; the FP32 batch is timed beside it."""
    plan = args.plan or "mixed"
    shapes = synth.config4_shapes(args.count)
    t = time.time()
    gen = torch.Generator(device=dev)
    mats, ks, ps, qs, seeds = [], [], [], [], []
    for b, (m, n, r) in enumerate(shapes):
        gen.manual_seed(synth.seed_a(4, b))
        U = torch.linalg.qr(torch.randn(m, r, generator=gen, device=dev, dtype=torch.float64))[0]
        V = torch.linalg.qr(torch.randn(n, r, generator=gen, device=dev, dtype=torch.float64))[0]
        sig = torch.exp(-torch.arange(1, r + 1, device=dev, dtype=torch.float64) / r)
        A = (U * sig) @ V.T + 1e-5 * torch.randn(m, n, generator=gen, device=dev, dtype=torch.float64)
        mats.append(A.float().contiguous())
        ks.append(r); ps.append(8); qs.append(1); seeds.append(synth.seed_omega(4, b))
    torch.cuda.synchronize()
    log(f"generated {len(mats)} matrices on the GPU in {time.time() - t:.1f}s")
    abytes = sum((2 * q + 2) * a.shape[0] * a.shape[1] * 4 for a, q in zip(mats, qs))

    tuned = None
    if not args.no_tune:
        # the project autotuner picks the batch's Gram plan for this shape class
        t = time.time()
        probe_bt = B.Batch(mats, ks, ps, qs, seeds, plan=plan)
        tuned = probe_bt.tune()
        probe_bt.close()
        del probe_bt
        log(f"autotuned the batch plan in {time.time() - t:.1f}s: {tuned}")
    t = time.time()
    bt = B.Batch(mats, ks, ps, qs, seeds, plan=plan)
    torch.cuda.synchronize()
    log(f"planned the batch in {time.time() - t:.1f}s: {bt.stats()}, problem 0 plan {bt.problem_plan(0)}")

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms_batch = timed(bt.run, args.steps, args.warmup)
    log(f"batched (graph): {ms_batch:.3f} ms per batch")
    bt.use_graph(False)
    ms_direct = timed(bt.run, max(1, args.steps // 2), 1)
    bt.use_graph(True)
    log(f"batched (grouped launches, no graph): {ms_direct:.3f} ms per batch")

    ms_batch_fp32 = None
    if plan != "native":
        bt32 = B.Batch(mats, ks, ps, qs, seeds, plan="native")
        ms_batch_fp32 = timed(bt32.run, max(1, args.steps // 2), 1)
        bt32.close()
        del bt32
        log(f"batched FP32 plan (graph): {ms_batch_fp32:.3f} ms per batch")

    # the plain FP32 method, one pbpqlp_factor call per matrix with its own
    # automatic plan
    facs = [B.Factorizer(a.shape[0], a.shape[1], k, p, q, torch.float32, "native", dev)
            for a, k, p, q in zip(mats, ks, ps, qs)]

    def per_matrix():
        for f, a, s_ in zip(facs, mats, seeds):
            f(a, s_)

    ms_single = None
    if not args.skip_per_matrix:
        ms_single = timed(per_matrix, max(1, args.steps // 4), 1)
        log(f"per-matrix calls, plain FP32: {ms_single:.3f} ms per batch")

    # sample against the FP64 oracle and against the per-matrix results
    from oracle import pbpqlp as oracle_pbpqlp, rel_residual
    bt.run()
    torch.cuda.synchronize()
    errs = []
    for i in (0, len(mats) // 3, 2 * len(mats) // 3, len(mats) - 1):
        A64 = mats[i].double().cpu().numpy()
        ref = oracle_pbpqlp(A64, ks[i], ps[i], qs[i], seeds[i])
        r_ref = rel_residual(A64, ref.Q, ref.L, ref.P)
        r = rel_residual(A64, *(x.cpu().numpy().astype(np.float64) for x in (bt.Q[i], bt.L[i], bt.P[i])))
        errs.append(abs(r - r_ref))
        # pbpqlp_factor with the plan the batch chose reproduces it bit for bit
        split_k, gram_wg = bt.problem_plan(i)
        f1 = B.Factorizer(mats[i].shape[0], mats[i].shape[1], ks[i], ps[i], qs[i], torch.float32,
                          plan, dev, split_k=split_k, gram_wg=gram_wg)
        same = all(torch.equal(x, y) for x, y in zip((bt.Q[i], bt.L[i], bt.P[i]), f1(mats[i], seeds[i])))
        if not same:
            log(f"problem {i}: batched and per-matrix results differ")
    line = {
        "metric": "PbP-QLP batched factorizations: ms per batch of 1024 uneven FP32 matrices",
        "value": round(ms_batch, 3), "unit": "ms/batch", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_batch, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if plan == "native" else "bf16",
        "data": "synthetic",
        "config": {"workload": f"{len(mats)} FP32 matrices m~U[256,4096] n~U[256,2048] r~U[8,64], "
                               "sigma_i=exp(-i/r) + 1e-5 N(0,1), k=r p=8 q=1", "plan": plan},
        "per_matrix_fp32_ms": round(ms_single, 3) if ms_single else None,
        "batched_fp32_ms": round(ms_batch_fp32, 3) if ms_batch_fp32 else None,
        "grouped_no_graph_ms": round(ms_direct, 3),
        "speedup_vs_per_matrix_fp32": round(ms_single / ms_batch, 2) if ms_single else None,
        "launches_per_batch": bt.stats()["launches"],
        "autotuned_plan": tuned,
        "algorithmic_gb": abytes / 1e9, "achieved_gbs": round(abytes / (ms_batch * 1e-3) / 1e9, 1),
        "hbm_frac": round(abytes / (ms_batch * 1e-3) / 8e12, 4),
        "max_abs_dr_vs_fp64_oracle_sample": max(errs),
    }
    print(json.dumps(line), flush=True)


def bench_c5(args, torch, np, synth, B, dev):
    """Learned q/k choice on 8192 x 8192 FP32 matrices with mixed spectra:
    pbpqlp_factor_auto against the plain method with q = 3 and the true
    epsilon-rank k*, both judged by tau = 1.05 r_opt(k* + p)."""
    from paper_2103_07245_amd import train_qk as T
    plan = args.plan or "native"
    count = args.count if args.count != 1024 else 12
    size = 8192
    model = B.Model.load(args.model)
    p = 8
    rows = []
    t_all = time.time()
    for i in range(count + 1):                   # matrix 0 is a warm-up
        spec = synth.qk_spec(i, 777, (size, size), (size, size), 512)
        A = T.make_matrix(spec, dev).float().contiguous()
        ks = T.k_star(spec.sigma)
        tau = T.Q_SLACK * T.r_opt(spec.sigma, ks + p)
        fplain = B.Factorizer(size, size, ks, p, 3, torch.float32, plan, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, res, info = B.factor_auto(model, A, p, spec.seed_omega, B.PROBE_K, tau, plan=plan)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fplain(A, spec.seed_omega)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r_plain = fplain.info().resid_rel_est
        if i > 0:
            rows.append({"family": spec.family, "k_star": ks, "tau": tau, "q_pred": res["q_pred"],
                         "k_pred": res["k_pred"], "q_used": res["q_used"], "k_used": res["k_used"],
                         "fell_back": res["fell_back"], "passes": res["passes"],
                         "r_learned": res["resid_final"], "r_plain": r_plain,
                         "ms_learned": (t1 - t0) * 1e3, "ms_plain": (t2 - t1) * 1e3})
            log(f"matrix {i}: {spec.family:4s} k*={ks:2d} q_hat={res['q_pred']} k_hat={res['k_pred']:2d} "
                f"passes {res['passes']:2d} fell_back={res['fell_back']} "
                f"r {res['resid_final']:.3e} / plain {r_plain:.3e} (tau {tau:.3e}) "
                f"ms {rows[-1]['ms_learned']:.2f} / {rows[-1]['ms_plain']:.2f}")
        del A, fplain
    ml = float(np.mean([r["ms_learned"] for r in rows]))
    mp = float(np.mean([r["ms_plain"] for r in rows]))
    ok_l = float(np.mean([r["r_learned"] <= r["tau"] for r in rows]))
    ok_p = float(np.mean([r["r_plain"] <= r["tau"] for r in rows]))
    line = {
        "metric": "learned q/k: ms per factorization of 8192x8192 FP32, learned vs plain q=3",
        "value": round(ml, 3), "unit": "ms/factorization", "n_gpus": 1, "steps": len(rows),
        "warmup": 1, "ms_per_step": round(ml, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if plan == "native" else "bf16", "data": "synthetic",
        "config": {"workload": f"{len(rows)} FP32 {size}x{size} matrices, spectra step/poly/exp, "
                               "planted rank <= 512, p=8, probe l=64", "plan": plan},
        "plain_q3_ms": round(mp, 3), "speedup_vs_plain_q3": round(mp / ml, 3),
        "passes_learned_mean": float(np.mean([r["passes"] for r in rows])), "passes_plain": 8,
        "success_learned": ok_l, "success_plain_q3": ok_p,
        "fallback_rate": float(np.mean([r["fell_back"] for r in rows])),
        "k_hat_abs_log_err": float(np.mean([abs(math.log(r["k_pred"] / r["k_star"])) for r in rows])),
        "q_hat_hist": np.bincount([r["q_pred"] for r in rows], minlength=5).tolist(),
        "wall_s": round(time.time() - t_all, 1),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
