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
sight = z.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "fp32_vector_tflops": 157.3,
    "fp64_vector_tflops": 78.6,
    "hbm_gbs": 8000.0,
}
# Algorithmic flops per accepted pair of the pair kernel.  Cartesian basis:
# 286 monomials x (1 mul + 1 add) = 572, the paper's count.  Spin basis:
# 11 adds/FMAs for m = 0 (21 flops), 110 FMAs for m >= 1 (220), the complex
# chain (x - i y)^m (2 + 9 x 6 = 56) and z^n (9) = 306.
FLOPS_PER_PAIR = {"cartesian": 572, "spin": 306}
# Algorithmic flops per pair of the FP32 adjoint pair kernel (either basis):
# the polynomial in (x - i y)^m T_n(z): T_n by recurrence (1 + 9 x 2 = 19),
# m = 0 (10 FMAs, 20), the chain (9 x 6 = 54), m >= 1 (90 FMAs, 180), the Re
# parts (20 FMAs, 40), times the primary's weight (1) = 314.
ADJ_FLOPS_PER_PAIR_FP32 = 314

WORKLOADS = {
    "c1": "config1",
    "c2": "config2",
    "c3": "config3",
    "c5": "config5",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_profile(basis, precision, workload):
    """The committed rocprofv3 counter record of the pair kernel (HBM bytes
    from FETCH_SIZE / WRITE_SIZE, FP32 VALU instructions from the SQ
    counters, per launch), or None if the kernel sources changed since then
    or the profile does not cover this configuration."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pair_kernel_uniform_n1048576_traffic.json")
    if not (os.path.exists(path) and basis == "spin" and precision != "fp64"
            and workload == "c2"):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp64"])
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
    ap.add_argument("--sample", type=int, default=8192,
                    help="primaries in the seeded sample used for errors and the CPU baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.distinct or args.regions or args.batch:
        args.forward_only = True
    if args.batch:
        args.no_cpu_baseline = True
        args.no_fp64_compare = True

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
    cfg = api.Config(box=cat.box, rmax=cat.rmax, nbins=cat.nbins, lmax=cat.lmax, los=cat.los,
                     observer=cat.observer, periodic=cat.periodic, box_lo=cat.box_lo,
                     precision=args.precision, basis=args.basis, distinct=args.distinct)
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

    def step(trace=None):
        if offs is not None:
            api.zeta_batch(pos, w, cfg, offs, out=zeta_batch_out, workspace=ws, trace=trace)
        elif region is not None:
            api.zeta_regions(pos, w, cfg, region, args.regions ** 3, out=zeta_regions_out,
                             workspace=ws, trace=trace)
        else:
            api.zeta(pos, w, cfg, out=zeta_out, workspace=ws, trace=trace, alm=store)
        if not args.forward_only:
            api.zeta_backward(pos, w, cfg, c, workspace=ws, trace=trace, alm=store)

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
    stage_ms = {}
    for name, ms in recs:
        stage_ms[name] = stage_ms.get(name, 0.0) + ms
    stage_ms = {k: v / args.steps for k, v in stage_ms.items()}
    pair_launches = [ms for name, ms in recs if name == "pairs"]
    # forward pair kernel passes in one step (a backward without the store
    # recomputes the a_lm on it)
    per_step_pair_passes = 2 if (not args.forward_only and store is None) else 1
    pair_ms_total = sum(pair_launches) / args.steps
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
            "paper_equivalent_frac_of_fp32_peak": pair_kernel_pairs_per_s * 572 / 157.3e12,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / peak,
            "traffic": prof["traffic_bytes_per_launch"] if prof else None,
        },
    }
    if prof and "valu_flops_per_launch" in prof:
        # FP32 VALU flops the counters saw per launch (every instruction the
        # kernel issues, not only the accumulation), over the live launch time
        counted = prof["valu_flops_per_launch"] / (avg_launch_ms * 1e-3) / 1e12
        out["pair_kernel"]["counted_valu_tflops"] = counted
        out["pair_kernel"]["counted_frac_of_fp32_peak"] = counted / PEAK["fp32_vector_tflops"]
    adj_launches = [ms for name, ms in recs if name == "pair_adjoint"]
    if adj_launches:
        # the adjoint pair kernel visits the same pairs once per step
        adj_avg = sum(adj_launches) / len(adj_launches)
        adj_pps = pairs / (len(adj_launches) / args.steps) / (adj_avg * 1e-3)
        out["adjoint_kernel"] = {"avg_launch_ms": adj_avg, "pairs_per_s": adj_pps}
        afpp = ADJ_FLOPS_PER_PAIR_FP32 if args.precision != "fp64" else None
        if afpp:
            out["adjoint_kernel"]["flops_per_pair"] = afpp
            out["adjoint_kernel"]["tflops"] = adj_pps * afpp / 1e12
            out["adjoint_kernel"]["frac_of_fp32_peak"] = adj_pps * afpp / 1e12 / PEAK[
                "fp32_vector_tflops"]

    # the same seeded primary sample for the errors, the FP64 speedup and the CPU baseline
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
        }
        log(f"oracle: {ref_pairs} pairs in {dt:.1f} s on {threads} threads")
        zs = api.zeta(pos, w, cfg, primary_mask=mask, workspace=ws).cpu().numpy()
        out["err_vs_oracle_sample"] = float(np.abs(zs - ref).max() / np.abs(ref).max())

    if not args.no_fp64_compare and args.precision != "fp64":
        cfg64 = api.Config(box=cat.box, rmax=cat.rmax, nbins=cat.nbins, lmax=cat.lmax,
                           los=cat.los, observer=cat.observer, periodic=cat.periodic,
                           box_lo=cat.box_lo, precision="fp64", basis=args.basis,
                           distinct=args.distinct)
        api.zeta(pos, w, cfg64, out=zeta_out, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        api.zeta(pos, w, cfg64, out=zeta_out, workspace=ws)
        torch.cuda.synchronize()
        fp64_ms = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        api.zeta(pos, w, cfg, out=zeta_out, workspace=ws)
        torch.cuda.synchronize()
        fwd_ms = (time.perf_counter() - t) * 1e3
        cmp_ = {"forward_ms": fwd_ms, "fp64_forward_ms": fp64_ms, "speedup": fp64_ms / fwd_ms,
                "forward_pairs_per_s": pairs / (fwd_ms * 1e-3)}
        if ref is not None:
            z64 = api.zeta(pos, w, cfg64, primary_mask=mask, workspace=ws).cpu().numpy()
            cmp_["fp64_err_vs_oracle_sample"] = float(np.abs(z64 - ref).max() /
                                                      np.abs(ref).max())
        out["speedup_vs_fp64"] = cmp_
        log(f"forward {fwd_ms:.1f} ms vs plain FP64 {fp64_ms:.1f} ms")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
