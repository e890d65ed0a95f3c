"""Throughput of k-point band solves + adjoint on one MI355X.

Workload (FCC M=5 headline): 16 seeded designs, FCC primitive cell, 32^3 voxels
(uniform[0,1] then periodic 3x3x3 box mean, seeds 400-415), plane-wave order
M=5 (N=1331: 3993 displacement / 7986 stress unknowns), 60 k-points on the
IBZ boundary G-X-W-K-G-L-U-W-L-K|U-X, lowest 12 bands, d omega / d rho_e for
bands 6 and 7 at every k, mixed precision (FP32 pencil factorisation and
preconditioner, FP64 residuals and Rayleigh-Ritz).  One step = all 16 designs
x 60 k-points.  Inputs are resident on the device (torch tensors) when the
timed region starts; outputs stay on the device.

Prints one JSON line (rank 0) with the metric, a roofline entry for the
dominant kernel class measured with HIP events on the library stream over the
timed region, the mixed-vs-FP64 accuracy gate and a CPU-oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--designs", type=int, default=16)
    ap.add_argument("--nk", type=int, default=60)
    ap.add_argument("--M", type=int, default=5)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--streams", type=int, default=12, help="designs solved concurrently (library option)")
    ap.add_argument("--coarse-tol", type=float, default=None, help="library option coarse_tol")
    ap.add_argument("--shift", type=float, default=None, help="library option shift")
    ap.add_argument("--opt", action="append", default=[], metavar="KEY=VALUE",
                    help="any other library option (phx_set_option), repeatable")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-gate", action="store_true", help="skip the mixed-vs-FP64 accuracy gate")
    ap.add_argument("--no-host", action="store_true", help="skip the host-copy (PCIe-inclusive) rate")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (sharding over GPUs is "
                                   "not built)"}), flush=True)
        sys.exit(2)

    # One hardware queue per design stream (HIP maps streams onto GPU_MAX_HW_QUEUES queues,
    # 4 by default; two streams on one queue run their kernels one after the other).  Read
    # when the HIP runtime starts, so set before torch touches the GPU.
    os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(4, args.streams)))

    import numpy as np
    import torch

    from paper_1603_06855_amd import phx, synth

    dev = torch.device("cuda:0")
    ctx = phx.Context(0)
    wl = synth.config4(all_m5=True, ndesign=args.designs)
    cells = [synth.Cell(c.lattice, c.a, c.nv, args.M, c.phase0, c.phase1, c.simp_p) for c in wl.cells]
    q = phx.kpath("FCC", args.nk) if args.nk >= 12 else phx.kpath("FCC", 12)[: args.nk]
    bands = (6, 7)
    nb = 12
    rho_dev = [torch.from_numpy(np.ascontiguousarray(d.reshape(-1))).to(dev) for d in wl.designs]
    torch.cuda.synchronize()

    ctx.set_option("streams", args.streams)
    if args.coarse_tol is not None:
        ctx.set_option("coarse_tol", args.coarse_tol)
    if args.shift is not None:
        ctx.set_option("shift", args.shift)
    # The headline designs are smooth (box-smoothed random fields): neighbouring k-points
    # share preconditioner factors more widely than the library default.
    opts = {"kshare": 8.0, "kshare_dist": 1.0}
    for kv in args.opt:
        key, val = kv.split("=", 1)
        opts[key] = float(val)
    for key, val in opts.items():
        ctx.set_option(key, val)

    def step():
        # every design of the step through one batched call (designs spread over
        # concurrent library streams)
        return ctx.sens_batch_dev(cells, rho_dev, q, nb, bands, args.precision)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Timed steps: only the launches of the single-kernel classes record events (their
    # kernel's start and end); the stage intervals of the breakdown come from one more,
    # untimed step afterwards (their events on every stage would slow the timed steps).
    ctx.set_option("profile_reset", 1)
    ctx.set_option("profile", 2)
    torch.cuda.synchronize()
    w0 = time.monotonic_ns()
    t0 = time.perf_counter()
    iters = 0
    sweeps = 0
    coarse_iters = 0
    iters_mean_k = 0
    for _ in range(args.steps):
        res = step()
        iters = max(iters, ctx.stat("iters"))
        sweeps = max(sweeps, ctx.stat("rr_sweeps"))
        coarse_iters = max(coarse_iters, ctx.stat("coarse_iters"))
        iters_mean_k = ctx.stat("iters_mean_k")
        factors = ctx.stat("factors")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    w1 = time.monotonic_ns()
    ctx.set_option("profile", 0)

    elapsed = t1 - t0
    units = args.designs * args.nk * args.steps
    value = units / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    classes = ["potrf_diag", "panel", "herk", "trsm_diag", "trsm_update", "solve_upd", "solve_diag", "sbinv",
               "assemble", "apply", "op_gemm", "gram", "small", "update", "residual", "adjoint"]
    prof = {c: {k: ctx.stat(f"prof.{c}.{k}") for k in ("ms", "flops", "bytes", "count")} for c in classes}
    # the untimed, fully profiled step of the per-stage breakdown
    ctx.set_option("profile_reset", 1)
    ctx.set_option("profile", 1)
    step()
    torch.cuda.synchronize()
    ctx.set_option("profile", 0)
    stage_ms = {c: round(ctx.stat(f"prof.{c}.ms"), 3) for c in classes}
    # Classes that are exactly one kernel, each launch timed by HIP events that the launch
    # itself records at the kernel's start and end (hipExtLaunchKernelGGL, on the library
    # stream the kernel runs on): the roofline entry is the one of them that took the most
    # time in the timed region; the others follow under "others".
    fp_chol = "float" if args.precision == "mixed" else "double"
    fpn = "fp32" if fp_chol == "float" else "fp64"
    nbk = 1 if min(21, nb + max(8, nb)) <= 16 else 2
    # the block-column steps of the preconditioner solves (both directions); in FP64 the
    # backward diagonal-block steps run the same kernel outside the class
    upd = (f"phx::zgemm_kernel<float, 1, 0, 128, 32, 0>" if fp_chol == "float"
           else f"phx::nrhs_kernel<double, 1, {nbk}, 1>")
    single = {"herk": (f"phx::zgemm_kernel<{fp_chol}, 0, 1, 64, 64, 1>", fpn, "mfma"),
              "op_gemm": ("phx::zgemm_kernel<double, 0, 0, 64, 64, 2>", "fp64", "mfma"),
              "solve_upd": (upd, fpn, "hbm")}
    # The library counts the work of the padded problem (Np = 64 ceil(N / 64) waves per
    # displacement component); the algorithmic work is that of the N-wave problem: the
    # Cholesky update scales as the cube of the size, the operator products as the square.
    N = (2 * args.M + 1) ** 3
    Np = 64 * ((N + 63) // 64)
    unpad = {"herk": (N / Np) ** 3, "op_gemm": (N / Np) ** 2}
    for c in unpad:
        prof[c]["flops"] *= unpad[c]

    def entry(c):
        p = prof[c]
        name, fp, bound = single[c]
        us = 1e3 * p["ms"] / max(p["count"], 1)
        if bound == "mfma":
            achieved = p["flops"] / max(p["ms"] * 1e-3, 1e-12) / 1e12
            e = {"bound": "mfma", "achieved": achieved, "peak": PEAK[fp] / 1e12, "unit": "TFLOP/s",
                 "frac": achieved / (PEAK[fp] / 1e12)}
        else:
            achieved = p["bytes"] / max(p["ms"] * 1e-3, 1e-12) / 1e9
            e = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
                 "frac": achieved / (PEAK["hbm"] / 1e9)}
        e.update({"traffic": measured_traffic(name), "kernel": name, "dtype": fp, "launches": int(p["count"]),
                  "avg_launch_us": us, "flops_per_launch": p["flops"] / max(p["count"], 1),
                  "alg_bytes_per_launch": p["bytes"] / max(p["count"], 1), "total_ms": p["ms"]})
        return e

    order = sorted(single, key=lambda c: -prof[c]["ms"])
    roof = entry(order[0])
    roof["others"] = [entry(c) for c in order[1:]]
    breakdown = stage_ms

    # Accuracy gate (untimed, after the timed steps): the last timed step's own mixed-precision
    # results for every design at a subset of its k-points against FP64 solves (tolerance
    # 1e-10) of the same designs at those k-points, one batched call.  Frequencies: relative
    # error, bands below 1e-3 of the largest frequency (the acoustic bands near Gamma)
    # excluded; sensitivities: norm-relative per (design, k, band), bands closer than 1e-4
    # (relative) to a neighbour excluded (their per-vector sensitivity is not unique).
    gate = None
    if not args.no_gate:
        sub_idx = np.arange(0, args.nk, max(1, args.nk // 8))
        ctx.set_option("tol_fp64", 1e-10)
        o64, d64 = ctx.sens_batch_dev(cells, rho_dev, q[sub_idx], nb, bands, "fp64")
        torch.cuda.synchronize()
        ctx.set_option("tol_fp64", 1e-8)
        om_err, sens_err, skipped = 0.0, 0.0, 0
        for d in range(args.designs):
            om32 = res[0][d].cpu().numpy()[sub_idx]
            dw32 = res[1][d].cpu().numpy()[sub_idx]
            om64, dw64 = o64[d].cpu().numpy(), d64[d].cpu().numpy()
            rel = np.where(om64 > 1e-3 * om64.max(), np.abs(om32 - om64) / np.maximum(om64, 1e-300), 0.0)
            om_err = max(om_err, float(rel.max()))
            for k in range(len(sub_idx)):
                w = om64[k]
                for j, b in enumerate(bands):
                    i = b - 1
                    gap = min(abs(w[i] - w[i - 1]), abs(w[i + 1] - w[i]) if i + 1 < nb else np.inf)
                    if w[i] <= 0 or gap < 1e-4 * w[i]:
                        skipped += 1
                        continue
                    e = np.abs(dw32[k, j] - dw64[k, j]).max() / max(np.abs(dw64[k, j]).max(), 1e-300)
                    sens_err = max(sens_err, float(e))
        gate = {"designs": args.designs, "k_points": int(len(sub_idx)), "source": "timed step",
                "max_rel_omega_err": om_err, "max_sens_err": sens_err, "sens_skipped_degenerate": skipped,
                "pass": bool(om_err <= 1e-6 and sens_err <= 1e-6)}

    # PCIe-inclusive rate (untimed for `value`): the same steps with every design's density
    # copied in from pinned host memory before the step and all frequencies and
    # sensitivities copied back to pinned host memory after it.
    host = None
    if not args.no_host and res[1] is not None:
        rho_h = [r.cpu().pin_memory() for r in rho_dev]
        om_h = [torch.empty(o.shape, dtype=o.dtype, pin_memory=True) for o in res[0]]
        dw_h = [torch.empty(d.shape, dtype=d.dtype, pin_memory=True) for d in res[1]]
        nbytes = sum(r.numel() for r in rho_h) * 8 + sum(o.numel() for o in om_h) * 8 + sum(d.numel() for d in dw_h) * 8
        torch.cuda.synchronize()
        th0 = time.perf_counter()
        for _ in range(args.steps):
            for r_d, r_h in zip(rho_dev, rho_h):
                r_d.copy_(r_h, non_blocking=True)
            oms, dws = step()
            for o_h, o in zip(om_h, oms):
                o_h.copy_(o, non_blocking=True)
            for d_h, d in zip(dw_h, dws):
                d_h.copy_(d, non_blocking=True)
            torch.cuda.synchronize()
        th = (time.perf_counter() - th0) / args.steps
        # the copies alone (same buffers, no solve), for their own cost
        tc0 = time.perf_counter()
        for r_d, r_h in zip(rho_dev, rho_h):
            r_d.copy_(r_h, non_blocking=True)
        for o_h, o in zip(om_h, oms):
            o_h.copy_(o, non_blocking=True)
        for d_h, d in zip(dw_h, dws):
            d_h.copy_(d, non_blocking=True)
        torch.cuda.synchronize()
        tc = time.perf_counter() - tc0
        host = {"value": args.designs * args.nk / th, "unit": "k-solves/s", "ms_per_step": 1e3 * th,
                "bytes_per_step": nbytes, "copies_alone_ms": 1e3 * tc, "copy_GB_per_s": nbytes / tc / 1e9}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.M)

    line = {
        "metric": "k-point band solves+adjoint/sec, FCC M=5; mixed vs FP64 at <=1e-6 rel omega err",
        "value": value,
        "unit": "k-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64" if args.precision == "mixed" else "fp64",
        "data": "synthetic",
        "config": {"workload": f"FCC 32^3, M={args.M} (3N={3 * (2 * args.M + 1) ** 3}), {args.designs} designs x "
                               f"{args.nk} k, 12 bands, adjoint bands 6/7, {args.precision}",
                   "designs": args.designs, "k_points": args.nk, "nbands": nb, "sens_bands": list(bands),
                   "M": args.M, "precision": args.precision, "parallelism": f"single GPU, {args.streams} design streams",
                   "eigensolver_iters_max": iters, "jacobi_sweeps_max": sweeps,
                   "coarse_start_iters_max": coarse_iters, "iters_to_converge_mean_over_k": iters_mean_k,
                   "preconditioner_factors_per_design": factors / args.designs,
                   "library_options": opts},
        "roofline": roof,
        "stage_ms_per_step": breakdown,
        "accuracy_gate": gate,
        "timed_window_monotonic_ns": [w0, w1],
        "cpu_baseline": cpu,
        "host_copies": host,
    }
    print(json.dumps(line), flush=True)


def kernel_source_sha(kernel: str):
    """SHA-256 of the text of the template definition of `kernel` ("phx::name<...>") in the
    HIP sources, or None."""
    import glob
    import hashlib
    base = kernel.split("<")[0].split("::")[-1]
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_1603_06855_amd", "csrc", "*.hip"))):
        src = open(path).read()
        i = src.find(f" void {base}(")
        if i < 0:
            continue
        start = src.rfind("template <", 0, i)
        end = src.index("\n}\n", i) + 3
        return hashlib.sha256(src[start:end].encode()).hexdigest()
    return None


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summaries (profiles/*_traffic.md, one per kernel), or None when there is none or the
    kernel's source text (its template's definition) changed since the counters were taken."""
    import glob
    sha = kernel_source_sha(kernel)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        fields = {}
        for line in open(path):
            key = line.split(":", 1)[0]
            if ":" in line and key in ("kernel", "traffic_bytes_per_launch", "kernel_source_sha256"):
                fields[key] = line.split(":", 1)[1].strip()
        if fields.get("kernel") == kernel and sha and fields.get("kernel_source_sha256") == sha:
            return float(fields["traffic_bytes_per_launch"])
    return None


def cpu_baseline(M: int):
    """The FP64 oracle on one design x two k-points (+ adjoint of bands 6 and 7), FCC 32^3."""
    from oracle import adjoint, geometry
    from paper_1603_06855_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    cell = synth.Cell("FCC", 1.0, 32, M)
    rho = synth.box_smoothed_uniform(32, 400)
    Q = geometry.kpath("FCC", 60)[[7, 23]]
    t = time.perf_counter()
    adjoint.sensitivities(cell, rho, Q, 12, (6, 7))
    dt = time.perf_counter() - t
    return {"value": len(Q) / dt, "unit": "k-solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"1 design x {len(Q)} k-points (FCC 32^3, M={M}, 12 bands, adjoint bands 6/7, "
                      f"per-design compliance factorisation included), {dt:.1f} s"}


if __name__ == "__main__":
    main()
