#!/usr/bin/env python3
"""Throughput of the anisotropic 3PCF hot path on one MI355X.

A step is one pass of the whole hot path over the synthetic catalogue:
g3pcf_forward (cell list, pair kernel, FP64 conversion, zeta on MFMA) followed
by g3pcf_backward (recomputed a_lm, adjoint coefficients, adjoint pair kernel)
for a random c ~ N(0, 1).  ``value`` = accepted ordered pairs of the catalogue
divided by the step time, with the inputs resident in HBM.  The pair kernel's
duration is measured with HIP events that the library records on its own
stream around every launch.

Default workload: N = 2^20 uniform galaxies, periodic L = 1000 Mpc/h, float32
positions, w ~ U(0.5, 1.5), R_max = 200 Mpc/h, 10 shells, l_max = 10, line of
sight = z.  Besides the timed FP32 step the default run reports, as extra keys
of the same line: the plain FP64 form (the paper's precision) timed with the
same warm-up / median protocol, the BF16x3 zeta stage (time and error), the
zeta stage's matrix-core rate, the clustered and adjoint catalogues, and the
FP64 CPU oracle on all host cores and on one.

``python bench.py --summarise-rocprof ...`` turns rocprofv3 CSV output into
the per-launch counter record kept under profiles/ (see summarise_rocprof).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks (dense)
    "fp32_vector_tflops": 157.3,
    "fp64_vector_tflops": 78.6,
    "fp32_mfma_tflops": 157.3,
    "fp64_mfma_tflops": 78.6,
    "bf16_mfma_tflops": 2500.0,
    "hbm_gbs": 8000.0,
}
# Algorithmic flops per accepted pair of the pair kernel (an FMA counts 2).
# Cartesian basis: 286 monomials x (1 mul + 1 add) = 572, the paper's count.
# Spin basis, SpinChunk::add: the Chebyshev polynomials T_2..T_10 of u_z
# (2 u_z: one add, then 9 FMAs: 19); m = 0: one add and 10 FMAs (21); the
# chain w (x - i y)^m: 2 multiplies, then 9 steps of 2 multiplies and 2 FMAs
# (2 + 54 = 56); m >= 1: per m two adds and 2 (10 - m) FMAs, i.e. 20 adds +
# 90 FMAs (200).  19 + 21 + 56 + 200 = 296.
FLOPS_PER_PAIR = {"cartesian": 572, "spin": 296}
# Algorithmic flops per pair of the FP32 adjoint pair kernel (either basis):
# the polynomial in (x - i y)^m T_n(z): T_n by recurrence (1 + 9 x 2 = 19),
# m = 0 (10 FMAs, 20), the chain (9 x 6 = 54), m >= 1 (90 FMAs, 180), the Re
# parts (20 FMAs, 40), times the primary's weight (1) = 314.
ADJ_FLOPS_PER_PAIR_FP32 = 314
# Real Gram width per m at l_max = 10, 10 shells: 110 for m = 0, 2 (11 - m) 10
# for m >= 1; sum of squares 166,100.  The zeta stage's algorithmic work is the
# full square Gram, 2 x 166,100 flops per primary.
ZETA_FLOPS_PER_PRIMARY = 2 * 166100

WORKLOADS = {
    "c1": "config1",
    "c2": "config2",
    "c3": "config3",
    "c5": "config5",
}
PROFILE = os.path.join(ROOT, "profiles", "pair_kernel_uniform_n1048576_traffic.json")
PAIR_KERNEL_SOURCES = ["paper_1709_00086_amd/csrc/pairs.hip",
                       "paper_1709_00086_amd/csrc/monomials.h",
                       "paper_1709_00086_amd/csrc/internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha256(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def measured_profile(basis, precision, workload):
    """The committed rocprofv3 counter record of the pair kernel (HBM bytes
    from FETCH_SIZE / WRITE_SIZE, FP32 VALU instructions from the SQ
    counters, per launch), or None if the kernel sources changed since then
    or the profile does not cover this configuration."""
    if not (os.path.exists(PROFILE) and basis == "spin" and precision != "fp64"
            and workload == "c2"):
        return None
    rec = json.load(open(PROFILE))
    if sources_sha256(rec["source_files"]) != rec["source_sha256"]:
        return None
    return rec


# ---------------------------------------------------------------- rocprofv3 summaries
def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _find(dirs, suffix):
    out = []
    for d in dirs:
        out += glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    return sorted(out)


def summarise_rocprof(args):
    """Per-launch averages of rocprofv3 counters for one kernel.

    --counters DIR...: directories of `rocprofv3 --pmc ... --output-format csv`
    runs (each *counter_collection.csv row is one counter of one dispatch);
    --kernel-stats DIR: a `--kernel-trace --stats` run (its *kernel_stats.csv).
    FETCH_SIZE / WRITE_SIZE are scaled by what the same counters read for the
    plain device copy of --copy-mib MiB in the same runs (kernel names
    containing "copyBuffer").  Writes the JSON record to --out and prints it."""
    import re
    pat = re.compile(args.kernel_regex)
    per = {}            # counter -> list of per-dispatch values of the kernel
    copy = {}           # counter -> list of per-dispatch values of the copy
    for path in _find(args.counters, "counter_collection.csv"):
        rows = _csv_rows(path)
        acc = {}
        for r in rows:
            name = r.get("Kernel_Name", "")
            key = (r.get("Dispatch_Id"), r.get("Counter_Name"))
            acc.setdefault(key, [name, 0.0])
            acc[key][1] += float(r.get("Counter_Value", 0.0))
        for (disp, counter), (name, val) in acc.items():
            if pat.search(name):
                per.setdefault(counter, []).append(val)
            elif "copyBuffer" in name:
                copy.setdefault(counter, []).append(val)
    sources = args.sources or PAIR_KERNEL_SOURCES
    rec = {"kernel": args.label or args.kernel_regex,
           "source_sha256": sources_sha256(sources),
           "source_files": sources,
           "counters_per_launch": {k: statistics.fmean(v) for k, v in sorted(per.items())},
           "launches_counted": {k: len(v) for k, v in sorted(per.items())},
           "commands": args.commands or []}
    if args.copy_mib and "FETCH_SIZE" in copy and "WRITE_SIZE" in copy:
        # the calibration copy is the largest copy dispatch of each run (the
        # runs also copy a few bytes back to the host)
        kib = args.copy_mib * 1024.0
        cf, cw = max(copy["FETCH_SIZE"]), max(copy["WRITE_SIZE"])
        fs, wsc = kib / cf, kib / cw
        rec.update({"copy_reference_mib": args.copy_mib, "copy_fetch_kib_raw": cf,
                    "copy_write_kib_raw": cw, "fetch_scale": fs, "write_scale": wsc})
        if "FETCH_SIZE" in per and "WRITE_SIZE" in per:
            f = statistics.fmean(per["FETCH_SIZE"])
            w = statistics.fmean(per["WRITE_SIZE"])
            rec.update({"fetch_kib_per_launch_raw": f, "write_kib_per_launch_raw": w,
                        "traffic_bytes_per_launch": (f * fs + w * wsc) * 1024.0})
    c = rec["counters_per_launch"]
    fl = 0.0
    for k, mult in (("SQ_INSTS_VALU_FMA_F32", 2), ("SQ_INSTS_VALU_MUL_F32", 1),
                    ("SQ_INSTS_VALU_ADD_F32", 1), ("SQ_INSTS_VALU_TRANS_F32", 1)):
        if k in c:
            fl += 64.0 * mult * c[k]
    if fl:
        rec["valu_f32_flops_per_launch"] = fl
    # matrix-core work: each MOPS count is 512 flops
    mf = {k: 512.0 * v for k, v in c.items() if k.startswith("SQ_INSTS_VALU_MFMA_MOPS_")}
    if mf:
        rec["mfma_flops_per_launch"] = mf
    for path in _find(args.kernel_stats, "kernel_stats.csv"):
        for r in _csv_rows(path):
            if pat.search(r.get("Name", "")):
                rec["trace_avg_ms"] = float(r["AverageNs"]) * 1e-6
                rec["trace_calls"] = int(r["Calls"])
    if "trace_avg_ms" not in rec:  # a --kernel-trace run without --stats
        durs = [float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
                for path in _find(args.kernel_stats, "kernel_trace.csv")
                for r in _csv_rows(path) if pat.search(r.get("Kernel_Name", ""))]
        if durs:
            rec["trace_avg_ms"] = statistics.fmean(durs) * 1e-6
            rec["trace_calls"] = len(durs)
    if mf and "trace_avg_ms" in rec:
        peaks = {"F32": PEAK["fp32_mfma_tflops"], "F64": PEAK["fp64_mfma_tflops"],
                 "BF16": PEAK["bf16_mfma_tflops"]}
        rec["mfma_tflops"] = {k: v / (rec["trace_avg_ms"] * 1e-3) / 1e12 for k, v in mf.items()}
        rec["mfma_frac_of_peak"] = {
            k: v / peaks[k.rsplit("_", 1)[1]] for k, v in rec["mfma_tflops"].items()
            if k.rsplit("_", 1)[1] in peaks and v > 0}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
    print(json.dumps(rec, indent=1))


# ---------------------------------------------------------------- precision report
def _errors(z, ref, floor=1e-6):
    """Per m and per (l, l'): the normwise error max|dz| / max|ref| and the
    largest per-entry relative error over entries with |ref| >= floor max|ref|."""
    L1 = z.shape[0]
    scale = np.abs(ref).max()
    d = np.abs(z - ref)
    big = np.abs(ref) >= floor * scale
    rel = np.where(big, d / np.where(big, np.abs(ref), 1.0), 0.0)
    per_m = [(float(d[m].max() / scale), float(rel[m].max())) for m in range(L1)]
    per_ll = [[float(rel[:, l, lp].max()) for lp in range(L1)] for l in range(L1)]
    return {"norm": float(d.max() / scale), "per_entry": float(rel.max()), "per_m": per_m,
            "per_ll": per_ll}


def precision_report():
    """Errors of the zeta stage on its own (the same FP64 pair stage feeding
    FP64, FP32 and BF16x3 Gram products) and of the FP32 pair path, against
    the FP64 oracle: config1 (one block of 4096 primaries) and the config2
    catalogue with 65,536 seeded primaries (16 blocks, so the FP64 sum across
    blocks is exercised).  Prints JSON and markdown tables."""
    import torch
    import oracle
    from paper_1709_00086_amd import api, catalogues as C
    dev = torch.device("cuda:0")
    report = {}
    for label, cat, mask_np in (
            ("config1", C.config1(), None),
            ("config2_16_blocks", C.config2(), C.primary_mask(1 << 20, 65536, seed=9))):
        t = time.perf_counter()
        ref = oracle.zeta(cat, primary_mask=mask_np)
        log(f"{label}: oracle {time.perf_counter() - t:.1f} s")
        pos = torch.from_numpy(cat.pos).to(dev)
        w = torch.from_numpy(cat.w).to(dev)
        m = torch.from_numpy(mask_np).to(dev) if mask_np is not None else None

        def run(prec, zp=None):
            cfg = api.Config(box=cat.box, rmax=cat.rmax, nbins=cat.nbins, lmax=cat.lmax,
                             los=cat.los, observer=cat.observer, periodic=cat.periodic,
                             box_lo=cat.box_lo, precision=prec, basis="spin", zeta_precision=zp)
            return api.zeta(pos, w, cfg, primary_mask=m).cpu().numpy()
        rows = {}
        z64 = run("fp64", "fp64")
        rows["FP64 pairs, FP64 zeta stage"] = _errors(z64, ref)
        for zp in ("fp32", "bf16x3"):
            rows[f"FP64 pairs, {zp.upper()} zeta stage"] = _errors(run("fp64", zp), ref)
        for zp in ("fp32", "bf16x3"):
            rows[f"FP32 pairs, {zp.upper()} zeta stage"] = _errors(run("fp32", zp), ref)
        report[label] = rows
    print(json.dumps(report))
    for label, rows in report.items():
        print(f"\n### {label}: normwise error max|dz|/max|z| and largest per-entry relative "
              f"error (entries with |z| >= 1e-6 max|z|)\n")
        print("| path | all | " + " | ".join(f"m={m}" for m in range(11)) + " |")
        print("|---|---|" + "---|" * 11)
        for name, e in rows.items():
            cells = " | ".join(f"{a:.1e} / {b:.1e}" for a, b in e["per_m"])
            print(f"| {name} | {e['norm']:.1e} / {e['per_entry']:.1e} | {cells} |")
        for name in ("FP32 pairs, FP32 zeta stage", "FP32 pairs, BF16X3 zeta stage"):
            e = rows[name]
            print(f"\n{label}, {name}: largest per-entry relative error per (l, l') "
                  f"(rows l, columns l')\n")
            print("| l \\ l' | " + " | ".join(str(l) for l in range(11)) + " |")
            print("|---|" + "---|" * 11)
            for l in range(11):
                print(f"| {l} | " + " | ".join(f"{v:.0e}" for v in e["per_ll"][l]) + " |")


# ---------------------------------------------------------------- probes
PROBE_SRC = os.path.join(ROOT, "bench_probes.hip")
PROBE_BIN = os.path.join(ROOT, "paper_1709_00086_amd", "_build", "bench_probes")


def probes(args):
    """Build (on any machine with hipcc) or run (on the GPU) bench_probes.hip."""
    import subprocess
    if args.build_probes:
        os.makedirs(os.path.dirname(PROBE_BIN), exist_ok=True)
        subprocess.check_call(["hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang",
                               "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-Wno-unused-command-line-argument", "-I", ROOT, PROBE_SRC,
                               "-o", PROBE_BIN])
        log(f"built {PROBE_BIN}")
    if args.probes:
        if not os.path.exists(PROBE_BIN):
            raise SystemExit(f"{PROBE_BIN} is missing: python bench.py --build-probes")
        sys.exit(subprocess.call([PROBE_BIN, args.probes]))


# ---------------------------------------------------------------- timing helpers
def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def median_ms(fn, reps, torch):
    """Median wall time of fn() over reps calls, each bracketed by syncs."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    return statistics.median(ts)


def stage_table(recs, nsteps):
    out = {}
    for name, ms in recs:
        out[name] = out.get(name, 0.0) + ms
    return {k: v / nsteps for k, v in out.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3", "fp64"],
                    help="fp32: FP32 pairs, FP32 MFMA zeta stage; bf16x3 (default): FP32 "
                         "pairs, BF16x3-split MFMA zeta stage; fp64: FP64 throughout")
    ap.add_argument("--basis", default="spin", choices=["cartesian", "spin"])
    ap.add_argument("--forward-only", action="store_true",
                    help="time the forward pass only (not the contract's step)")
    ap.add_argument("--distinct", action="store_true",
                    help="leave out the degenerate j = k triangles (forward only, so it "
                         "implies --forward-only)")
    ap.add_argument("--regions", type=int, default=0, metavar="K",
                    help="partial zeta of K^3 spatial cubes of primaries (jack-knife regions; "
                         "forward only)")
    ap.add_argument("--batch", type=int, default=0, metavar="K",
                    help="K mock catalogues of n/K galaxies each in the workload's box, in one "
                         "batched forward call (forward only; no CPU baseline or FP64 compare)")
    ap.add_argument("--keep-alm", action="store_true",
                    help="the forward keeps the a_lm in a store (n * nbins * (lmax+1)^2 "
                         "doubles) and the backward reads them instead of recomputing them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the extra legs (BF16x3 zeta stage, zeta-stage error sweep, "
                         "clustered and adjoint catalogues)")
    ap.add_argument("--leg-steps", type=int, default=3,
                    help="timed repetitions (median) of every extra leg")
    ap.add_argument("--sample", type=int, default=8192,
                    help="primaries in the seeded sample used for errors and the CPU baseline")
    ap.add_argument("--sample-1t", type=int, default=512,
                    help="primaries of the one-thread CPU baseline sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--precision-report", action="store_true",
                    help="per-(m, l, l') errors of the FP32 and BF16x3 zeta stages and of the "
                         "FP32 path against the FP64 oracle (config1 and a 16-block 2^20 "
                         "sample); prints a markdown report")
    ap.add_argument("--build-probes", action="store_true",
                    help="compile bench_probes.hip (issue-rate and counter-calibration probes)")
    ap.add_argument("--probes", default=None, metavar="MODE",
                    help="run the built probes: fma, accum, count, mfma or all (GPU)")
    ap.add_argument("--summarise-rocprof", action="store_true",
                    help="summarise rocprofv3 CSV output instead of running (no GPU)")
    ap.add_argument("--counters", nargs="*", default=[])
    ap.add_argument("--kernel-stats", nargs="*", default=[])
    ap.add_argument("--kernel-regex", default=r"k_pairs<float, 1, false, false, false>")
    ap.add_argument("--label", default=None)
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--commands", nargs="*", default=None)
    ap.add_argument("--sources", nargs="*", default=None,
                    help="source files whose hash the record keeps (default: the pair "
                         "kernel's)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.summarise_rocprof:
        summarise_rocprof(args)
        return
    if args.precision_report:
        precision_report()
        return
    if args.build_probes or args.probes:
        probes(args)
        return
    if args.distinct or args.regions or args.batch:
        args.forward_only = True
    if args.batch:
        args.no_cpu_baseline = True
        args.no_fp64_compare = True
    default_run = not (args.forward_only or args.keep_alm or args.batch or args.regions
                       or args.distinct) and args.precision != "fp64"

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); the multi-GPU path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1709_00086_amd import _lib, api, catalogues as C

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written once")
        del src, dst
    t = time.time()
    cat = getattr(C, WORKLOADS[args.workload])()
    log(f"workload {cat.name}: n={cat.n} generated in {time.time() - t:.1f}s")
    pos = torch.from_numpy(cat.pos).to(dev)
    w = torch.from_numpy(cat.w).to(dev)

    def config(c, precision, basis=args.basis, zeta_precision=None):
        return api.Config(box=c.box, rmax=c.rmax, nbins=c.nbins, lmax=c.lmax, los=c.los,
                          observer=c.observer, periodic=c.periodic, box_lo=c.box_lo,
                          precision=precision, basis=basis, distinct=args.distinct,
                          zeta_precision=zeta_precision)

    cfg = config(cat, args.precision)
    c = torch.from_numpy(C.loss_weights(cat.lmax, cat.nbins, seed=55)).to(dev)
    ws = api.Workspace()
    zeta_out = torch.empty(api.zeta_shape(cat.lmax, cat.nbins), dtype=torch.float64, device=dev)

    offs = None
    if args.batch:
        # K seeded mock catalogues of the workload's box and dtype in place of it
        k = args.batch
        mp, mw, offs = C.mock_batch([cat.n // k] * k, cat.box[0], seed=97, dtype=cat.pos.dtype)
        pos = torch.from_numpy(mp).to(dev)
        w = torch.from_numpy(mw).to(dev)
        zeta_batch_out = torch.empty((k,) + api.zeta_shape(cat.lmax, cat.nbins),
                                     dtype=torch.float64, device=dev)
        _, pairs = api.zeta_batch(pos, w, cfg, offs, out=zeta_batch_out, workspace=ws,
                                  return_pairs=True)
    else:
        # accepted pairs (counted by the kernel; outside the timed region)
        _, pairs = api.zeta(pos, w, cfg, out=zeta_out, workspace=ws, return_pairs=True)
    log(f"accepted ordered pairs: {pairs} ({pairs / cat.n:.1f} per primary)")

    region = None
    if args.regions:
        k = args.regions
        p64 = np.asarray(cat.pos, dtype=np.float64)
        cube = np.clip(np.floor((p64 - np.asarray(cat.box_lo)) / np.asarray(cat.box) * k),
                       0, k - 1).astype(np.int64)
        region = torch.from_numpy(((cube[:, 0] * k + cube[:, 1]) * k + cube[:, 2])
                                  .astype(np.int32)).to(dev)
        zeta_regions_out = torch.empty((k ** 3,) + api.zeta_shape(cat.lmax, cat.nbins),
                                       dtype=torch.float64, device=dev)

    # the backward recomputes the a_lm on the pair kernel; --keep-alm keeps
    # them in a store instead (one row per primary, allocated once like the
    # workspace, rewritten by every forward)
    store = None
    if not args.forward_only and args.keep_alm:
        store = api.alm_store(pos, w, cfg)
        log(f"a_lm store: {store.numel() / 1e9:.2f} GB")

    def step(trace=None, cfg_=cfg):
        if offs is not None:
            api.zeta_batch(pos, w, cfg_, offs, out=zeta_batch_out, workspace=ws, trace=trace)
        elif region is not None:
            api.zeta_regions(pos, w, cfg_, region, args.regions ** 3, out=zeta_regions_out,
                             workspace=ws, trace=trace)
        else:
            api.zeta(pos, w, cfg_, out=zeta_out, workspace=ws, trace=trace, alm=store)
        if not args.forward_only:
            api.zeta_backward(pos, w, cfg_, c, workspace=ws, trace=trace, alm=store)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    trace = _lib.Trace(capacity=max(4096, 2048 * args.steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(trace)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    recs = trace.read()
    stage_ms = stage_table(recs, args.steps)
    pair_launches = [ms for name, ms in recs if name == "pairs"]
    # forward pair kernel passes in one step (a backward without the store
    # recomputes the a_lm on it)
    per_step_pair_passes = 2 if (not args.forward_only and store is None) else 1
    avg_launch_ms = sum(pair_launches) / max(1, len(pair_launches))
    launches_per_pass = len(pair_launches) / (args.steps * per_step_pair_passes)
    pairs_per_launch = pairs / launches_per_pass
    fpp = FLOPS_PER_PAIR[args.basis]
    achieved_tflops = pairs_per_launch * fpp / (avg_launch_ms * 1e-3) / 1e12
    peak = PEAK["fp64_vector_tflops"] if args.precision == "fp64" else PEAK["fp32_vector_tflops"]
    pair_kernel_pairs_per_s = pairs_per_launch / (avg_launch_ms * 1e-3)
    # the profile covers full pair-blocks of the workload itself
    prof = measured_profile(args.basis, args.precision,
                            None if (args.batch or args.regions) else args.workload)
    value = pairs / (ms_per_step * 1e-3)
    log(f"step {ms_per_step:.1f} ms; stages (ms/step) {json.dumps(stage_ms)}")
    log(f"pair kernel: {len(pair_launches)} launches, avg {avg_launch_ms:.2f} ms, "
        f"{pair_kernel_pairs_per_s:.3e} pairs/s, {achieved_tflops:.1f} TFLOP/s")

    out = {
        "metric": "pairs/s at lmax=10, % of FP32 VALU peak; split-MFMA vs FP64 speedup at "
                  "stated error",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": cat.name,
            "n": cat.n,
            "rmax": cat.rmax,
            "nbins": cat.nbins,
            "lmax": cat.lmax,
            "los": cat.los,
            "periodic": cat.periodic,
            "precision": args.precision,
            "basis": args.basis,
            "step": "forward" if args.forward_only else "forward+backward",
            "backward_alm": None if args.forward_only else ("recomputed" if store is None
                                                            else "kept from the forward"),
            "distinct": bool(args.distinct),
            "regions": args.regions ** 3 if args.regions else 0,
            "batch": (f"{args.batch} mock catalogues of {cat.n // args.batch} galaxies "
                      f"(uniform, seed 97) in the workload's box") if args.batch else None,
            "accepted_pairs": pairs,
        },
        "stage_ms_per_step": stage_ms,
        "pair_kernel": {
            "launches_per_pass": launches_per_pass,
            "avg_launch_ms": avg_launch_ms,
            "pairs_per_s": pair_kernel_pairs_per_s,
            "flops_per_pair": fpp,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / peak,
            "traffic": prof.get("traffic_bytes_per_launch") if prof else None,
        },
    }
    if prof and "valu_f32_flops_per_launch" in prof:
        # FP32 VALU flops the counters saw per launch (every instruction the
        # kernel issues, not only the accumulation), over the live launch time
        counted = prof["valu_f32_flops_per_launch"] / (avg_launch_ms * 1e-3) / 1e12
        out["pair_kernel"]["counted_valu_tflops"] = counted
        out["pair_kernel"]["counted_frac_of_fp32_peak"] = counted / PEAK["fp32_vector_tflops"]
        cpl = prof["counters_per_launch"]
        if "SQ_INSTS_VALU" in cpl:
            out["pair_kernel"]["valu_insts_per_pair"] = cpl["SQ_INSTS_VALU"] / pairs_per_launch
    adj_launches = [ms for name, ms in recs if name == "pair_adjoint"]
    if adj_launches:
        # the adjoint pair kernel visits the same pairs once per step
        adj_avg = sum(adj_launches) / len(adj_launches)
        adj_pps = pairs / (len(adj_launches) / args.steps) / (adj_avg * 1e-3)
        out["adjoint_kernel"] = {"avg_launch_ms": adj_avg, "pairs_per_s": adj_pps}
        if args.precision != "fp64":
            afpp = ADJ_FLOPS_PER_PAIR_FP32
            out["adjoint_kernel"]["flops_per_pair"] = afpp
            out["adjoint_kernel"]["tflops"] = adj_pps * afpp / 1e12
            out["adjoint_kernel"]["frac_of_fp32_peak"] = adj_pps * afpp / 1e12 / PEAK[
                "fp32_vector_tflops"]
    zeta_launch_ms = stage_ms.get("zeta")
    if zeta_launch_ms and not (args.batch or args.regions):
        # matrix-core rate of the zeta stage (Gram products and their FP64 sum),
        # counted as the full square Gram
        zfl = ZETA_FLOPS_PER_PRIMARY * cat.n / (zeta_launch_ms * 1e-3) / 1e12
        zp = cfg.zeta_prec()
        # BF16x3 does six bfloat16 products per FP32-equivalent product
        key, work = {_lib.PREC_FP32: ("fp32_mfma_tflops", 1), _lib.PREC_FP64: ("fp64_mfma_tflops", 1),
                     _lib.PREC_BF16X3: ("bf16_mfma_tflops", 6)}[zp]
        out["zeta_stage"] = {"ms_per_pass": zeta_launch_ms, "tflops_full_square": zfl,
                             "mfma_tflops": zfl * work,
                             "frac_of_mfma_peak": zfl * work / PEAK[key], "peak": key}

    # the same seeded primary sample for the errors, the FP64 comparison and the
    # CPU baseline
    mask_np = C.primary_mask(cat.n, min(args.sample, cat.n), seed=7)
    mask = torch.from_numpy(mask_np).to(dev)
    ref = None
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.default_threads()
        t = time.perf_counter()
        ref, ref_pairs = oracle.zeta(cat, primary_mask=mask_np, nthreads=threads,
                                     return_pairs=True, distinct=args.distinct)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": ref_pairs / dt,
            "unit": "pairs/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"{int(mask_np.sum())} primaries (seeded mask, seed 7) of the same "
                      f"catalogue against all {cat.n} secondaries; {ref_pairs} pairs in "
                      f"{dt:.1f} s",
            "cpu_model": cpu_model(),
        }
        log(f"oracle: {ref_pairs} pairs in {dt:.1f} s on {threads} threads")
        if args.sample_1t > 0:
            m1 = C.primary_mask(cat.n, min(args.sample_1t, cat.n), seed=8)
            t = time.perf_counter()
            _, p1 = oracle.zeta(cat, primary_mask=m1, nthreads=1, return_pairs=True,
                                distinct=args.distinct)
            dt1 = time.perf_counter() - t
            out["cpu_baseline"]["one_thread"] = {
                "value": p1 / dt1, "unit": "pairs/s", "cores": 1,
                "sample": f"{int(m1.sum())} primaries (seeded mask, seed 8); {p1} pairs in "
                          f"{dt1:.1f} s"}
            log(f"oracle, one thread: {p1} pairs in {dt1:.1f} s")
        zs = api.zeta(pos, w, cfg, primary_mask=mask, workspace=ws).cpu().numpy()
        out["err_vs_oracle_sample"] = float(np.abs(zs - ref).max() / np.abs(ref).max())

    if not args.no_fp64_compare and args.precision != "fp64":
        # the plain FP64 form (the paper's precision) on the same input, timed
        # with the same protocol: warm-up, then the median of --leg-steps runs
        cfg64 = config(cat, "fp64")
        reps = max(1, args.leg_steps)
        fwd = lambda cf: api.zeta(pos, w, cf, out=zeta_out, workspace=ws)  # noqa: E731
        fwd(cfg64)
        fp64_fwd_ms = median_ms(lambda: fwd(cfg64), reps, torch)
        fwd(cfg)
        fwd_ms = median_ms(lambda: fwd(cfg), reps, torch)
        cmp_ = {"forward_ms": fwd_ms, "fp64_forward_ms": fp64_fwd_ms,
                "forward_speedup": fp64_fwd_ms / fwd_ms,
                "forward_pairs_per_s": pairs / (fwd_ms * 1e-3), "reps": reps}
        if not args.forward_only and store is None:
            step(cfg_=cfg64)
            tr64 = _lib.Trace(capacity=4096)
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                step(tr64, cfg_=cfg64)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t) * 1e3)
            r64 = tr64.read()
            st64 = stage_table(r64, reps)
            l64 = [ms for name, ms in r64 if name == "pairs"]
            avg64 = sum(l64) / max(1, len(l64))
            ppl64 = pairs / (len(l64) / (2 * reps))
            tf64 = ppl64 * fpp / (avg64 * 1e-3) / 1e12
            step_ms64 = statistics.median(ts)
            cmp_.update({
                "fp64_ms_per_step": step_ms64,
                "fp64_pairs_per_s": pairs / (step_ms64 * 1e-3),
                "step_speedup": step_ms64 / ms_per_step,
                "fp64_stage_ms_per_step": st64,
                "fp64_pair_kernel": {"avg_launch_ms": avg64,
                                     "pairs_per_s": ppl64 / (avg64 * 1e-3),
                                     "tflops": tf64,
                                     "frac_of_fp64_peak": tf64 / PEAK["fp64_vector_tflops"]},
            })
            log(f"FP64 step {step_ms64:.1f} ms (FP32 {ms_per_step:.1f} ms); FP64 pair kernel "
                f"{avg64:.2f} ms per launch, {tf64:.1f} TFLOP/s")
        if ref is not None:
            z64 = api.zeta(pos, w, cfg64, primary_mask=mask, workspace=ws).cpu().numpy()
            cmp_["fp64_err_vs_oracle_sample"] = float(np.abs(z64 - ref).max() /
                                                      np.abs(ref).max())
            cmp_["err_vs_oracle_sample"] = out.get("err_vs_oracle_sample")
        out["fp64_form"] = cmp_
        log(f"forward {fwd_ms:.1f} ms vs plain FP64 {fp64_fwd_ms:.1f} ms")

    if default_run and not args.no_legs:
        reps = max(1, args.leg_steps)
        legs = {}
        # the other FP32-path zeta stage: FP32 MFMA, or BF16x3 (each FP32
        # operand split into three bfloat16 terms, FP32 accumulation, FP64 sum
        # across blocks)
        alt = "fp32" if args.precision == "bf16x3" else "bf16x3"
        cfgb = config(cat, alt)
        api.zeta(pos, w, cfgb, out=zeta_out, workspace=ws)
        trb = _lib.Trace(capacity=1024)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            api.zeta(pos, w, cfgb, out=zeta_out, workspace=ws, trace=trb)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        stb = stage_table(trb.read(), reps)
        bleg = {"precision": alt, "forward_ms": statistics.median(ts),
                "zeta_stage_ms": stb.get("zeta")}
        if stb.get("zeta"):
            bleg["zeta_tflops_fp32_equivalent"] = (ZETA_FLOPS_PER_PRIMARY * cat.n /
                                                   (stb["zeta"] * 1e-3) / 1e12)
        if ref is not None:
            zb = api.zeta(pos, w, cfgb, primary_mask=mask, workspace=ws).cpu().numpy()
            bleg["err_vs_oracle_sample"] = float(np.abs(zb - ref).max() / np.abs(ref).max())
        # the zeta stage alone: the same FP64 pair stage (FP64 a_lm) into
        # FP64, FP32 and BF16x3 Gram products on the sample
        zsw = {}
        base = None
        for zp in ("fp64", "fp32", "bf16x3"):
            zz = api.zeta(pos, w, config(cat, "fp64", zeta_precision=zp), primary_mask=mask,
                          workspace=ws).cpu().numpy()
            if base is None:
                base = zz
            else:
                zsw[zp] = float(np.abs(zz - base).max() / np.abs(base).max())
        bleg["zeta_stage_err_vs_fp64_zeta_stage"] = zsw
        legs["zeta_" + alt] = bleg
        log(f"{alt} zeta stage: forward {bleg['forward_ms']:.1f} ms; zeta stage errors {zsw}")
        # the clustered observer-LOS catalogue and the adjoint catalogue, same step
        for key in ("c3", "c5"):
            t = time.time()
            oc = getattr(C, WORKLOADS[key])()
            gen = time.time() - t
            opos = torch.from_numpy(oc.pos).to(dev)
            ow = torch.from_numpy(oc.w).to(dev)
            ocfg = config(oc, args.precision)
            oc_c = torch.from_numpy(C.loss_weights(oc.lmax, oc.nbins, seed=55)).to(dev)
            _, opairs = api.zeta(opos, ow, ocfg, out=None, workspace=ws, return_pairs=True)

            def ostep(cf=ocfg):
                api.zeta(opos, ow, cf, workspace=ws)
                api.zeta_backward(opos, ow, cf, oc_c, workspace=ws)
            ostep()
            oms = median_ms(ostep, reps, torch)
            legs[oc.name] = {"ms_per_step": oms, "pairs_per_s": opairs / (oms * 1e-3),
                             "accepted_pairs": opairs, "step": "forward+backward",
                             "precision": args.precision, "basis": args.basis}
            log(f"{oc.name}: {oms:.1f} ms per step, {opairs / (oms * 1e-3):.3e} pairs/s "
                f"(generated in {gen:.1f} s)")
            del opos, ow
        out["legs"] = legs

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
