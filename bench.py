"""Throughput of k-point band solves + adjoint on one MI355X.

Workload (FCC M=5 headline): 16 seeded designs, FCC primitive cell, 32^3 voxels
(uniform[0,1] then periodic 3x3x3 box mean, seeds 400-415), plane-wave order
M=5 (N=1331: 3993 displacement / 7986 stress unknowns), 60 k-points on the
IBZ boundary G-X-W-K-G-L-U-W-L-K|U-X, lowest 12 bands, d omega / d rho_e for
bands 6 and 7 at every k, mixed precision (FP32 pencil factorisation and
preconditioner, FP64 residuals and Rayleigh-Ritz).  One step = all 16 designs
x 60 k-points.  Inputs are resident on the device (torch tensors) when the
timed region starts; outputs stay on the device.

Prints one JSON line (rank 0) with the metric; a roofline entry for the dominant
kernel class measured with HIP events on the library stream over the timed
region, beside the same kernel's rate on one stream; the factorisation stage's
rate per precision; the FP64 path on the same workload; the rate at the
library's default options; the mixed-vs-FP64 accuracy gate and a CPU-oracle
baseline.
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
CLASSES = ["potrf_diag", "panel", "herk", "trsm_diag", "trsm_update", "solve_upd", "solve_diag", "sbinv",
           "assemble", "apply", "op_gemm", "gram", "small", "update", "residual", "adjoint", "op_conv"]
FACTOR_CLASSES = ["potrf_diag", "panel", "herk", "sbinv"]


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
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 leg on the same workload")
    ap.add_argument("--no-defaults", action="store_true", help="skip the rate at the library's default options")
    ap.add_argument("--no-one-stream", action="store_true", help="skip the one-stream profiled steps")
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
    wl = synth.config4(all_m5=True, ndesign=args.designs)
    cells = [synth.Cell(c.lattice, c.a, c.nv, args.M, c.phase0, c.phase1, c.simp_p) for c in wl.cells]
    q = phx.kpath("FCC", args.nk) if args.nk >= 12 else phx.kpath("FCC", 12)[: args.nk]
    bands = (6, 7)
    nb = 12
    rho_dev = [torch.from_numpy(np.ascontiguousarray(d.reshape(-1))).to(dev) for d in wl.designs]
    torch.cuda.synchronize()
    N = (2 * args.M + 1) ** 3
    Np = 64 * ((N + 63) // 64)

    # The headline designs are smooth (box-smoothed random fields): the library's default
    # preconditioner (block Jacobi, the pencil factors only where it stalls) stays on block
    # Jacobi; should it switch, neighbouring k-points share pencil factors more widely than
    # the library default.  The coarse start runs at order M - 3 (order 2 at M = 5; the
    # library default is M - 2): on these designs its cheaper solve outweighs the half
    # iteration more that the order-5 solve then takes.
    opts = {"streams": float(args.streams), "kshare": 8.0, "kshare_dist": 1.0, "coarse_drop": 3.0}
    if args.coarse_tol is not None:
        opts["coarse_tol"] = args.coarse_tol
    if args.shift is not None:
        opts["shift"] = args.shift
    for kv in args.opt:
        key, val = kv.split("=", 1)
        opts[key] = float(val)

    def make_ctx(options):
        c = phx.Context(0)
        for key, val in options.items():
            c.set_option(key, val)
        return c

    def step(c, prec):
        # every design of the step through one batched call (designs spread over
        # concurrent library streams)
        return c.sens_batch_dev(cells, rho_dev, q, nb, bands, prec)

    def timed(c, prec, steps, warmup):
        """Warm-up steps, then `steps` timed steps with the single-kernel classes' own
        events on (profile mode 2).  Returns rate, ms per step, the last result, the
        solver statistics of the last step, the class counters and the window."""
        for _ in range(warmup):
            step(c, prec)
        torch.cuda.synchronize()
        c.set_option("profile_reset", 1)
        c.set_option("profile", 2)
        torch.cuda.synchronize()
        w0 = time.monotonic_ns()
        t0 = time.perf_counter()
        st = {}
        for _ in range(steps):
            r = step(c, prec)
            for key, agg in (("iters", max), ("rr_sweeps", max), ("coarse_iters", max)):
                st[key] = agg(st.get(key, 0), c.stat(key))
            st["iters_mean_k"] = c.stat("iters_mean_k")
            st["factors"] = c.stat("factors")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        w1 = time.monotonic_ns()
        c.set_option("profile", 0)
        prof = {k: {f: c.stat(f"prof.{k}.{f}") for f in ("ms", "flops", "bytes", "count")} for k in CLASSES}
        for k in prof:  # per step
            for f in prof[k]:
                prof[k][f] /= steps
        return {"value": args.designs * args.nk * steps / el, "ms_per_step": 1e3 * el / steps, "res": r,
                "stats": st, "prof": prof, "window": [w0, w1]}

    def profiled(c, prec):
        """One untimed step with every stage timed (profile mode 1): per-class summed stage
        milliseconds, the class counters and the step's wall time."""
        c.set_option("profile_reset", 1)
        c.set_option("profile", 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(c, prec)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        c.set_option("profile", 0)
        prof = {k: {f: c.stat(f"prof.{k}.{f}") for f in ("ms", "flops", "bytes", "count")} for k in CLASSES}
        return prof, 1e3 * wall

    def kernel_names(prec):
        fp_chol = "float" if prec == "mixed" else "double"
        fpn = "fp32" if fp_chol == "float" else "fp64"
        nbk = 1 if min(21, nb + max(8, nb)) <= 16 else 2
        # the block-column steps of the preconditioner solves (both directions); in FP64 the
        # backward diagonal-block steps run the same kernel outside the class
        upd = ("phx::zgemm_kernel<float, 1, 0, 128, 32, 0>" if fp_chol == "float"
               else f"phx::nrhs_kernel<double, 1, {nbk}, 1>")
        names = {"herk": (f"phx::zgemm_kernel<{fp_chol}, 0, 1, 64, 64, 1>", fpn, "mfma"),
                 "op_gemm": ("phx::opgemm_kernel<8>", "fp64", "mfma"),
                 "solve_upd": (upd, fpn, "hbm")}
        if args.M <= 5:  # Omega_s X as a convolution: FP64 vector arithmetic through LDS
            names["op_conv"] = (f"phx::omega_conv_kernel<{args.M}>", "fp64", "alu")
        return names

    # The library counts the work of the padded problem (Np = 64 ceil(N / 64) waves per
    # displacement component); the algorithmic work is that of the N-wave problem: the
    # Cholesky update scales as the cube of the size, the operator products as the square.
    unpad = {"herk": (N / Np) ** 3, "op_gemm": (N / Np) ** 2}

    def entry(prof, c, single):
        """Roofline entry of single-kernel class c from per-step class counters."""
        p = dict(prof[c])
        p["flops"] = p["flops"] * unpad.get(c, 1.0)
        name, fp, bound = single[c]
        us = 1e3 * p["ms"] / max(p["count"], 1)
        if bound in ("mfma", "alu"):  # FP64: matrix and vector peaks are the same on MI355X
            achieved = p["flops"] / max(p["ms"] * 1e-3, 1e-12) / 1e12
            e = {"bound": bound, "achieved": achieved, "peak": PEAK[fp] / 1e12, "unit": "TFLOP/s",
                 "frac": achieved / (PEAK[fp] / 1e12)}
        else:
            achieved = p["bytes"] / max(p["ms"] * 1e-3, 1e-12) / 1e9
            e = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
                 "frac": achieved / (PEAK["hbm"] / 1e9)}
        e.update({"traffic": measured_traffic(name), "kernel": name, "dtype": fp, "launches": int(p["count"]),
                  "avg_launch_us": us, "flops_per_launch": p["flops"] / max(p["count"], 1),
                  "alg_bytes_per_launch": p["bytes"] / max(p["count"], 1), "total_ms": p["ms"]})
        return e

    def factorisation(prof, factors_per_step, prec):
        """The pencil factorisations of one step on one stream (the four classes of the
        factorisation: 64-wide diagonal blocks, panels, trailing updates, super-block
        inverses): algorithmic flops (3N)^3 / 3 complex multiply-adds = 8 (3N)^3 / 6 per
        order-M factor, plus the same for the factors of the coarse start at its own order
        (one per order-M factor), over the summed stage time."""
        Mc = max(1, args.M - int(opts.get("coarse_drop", 2)))  # the coarse start's order
        Nc = (2 * Mc + 1) ** 3
        flops = factors_per_step * 8.0 * ((3.0 * N) ** 3 + ((3.0 * Nc) ** 3 if args.M >= 4 else 0.0)) / 6.0
        ms = sum(prof[c]["ms"] for c in FACTOR_CLASSES)
        fp = "fp32" if prec == "mixed" else "fp64"
        tf = flops / max(ms * 1e-3, 1e-12) / 1e12
        return {"precision": prec, "dtype": fp, "tflops": tf, "peak": PEAK[fp] / 1e12, "frac": tf / (PEAK[fp] / 1e12),
                "ms_per_step": ms, "factors_per_step": factors_per_step,
                "stage_ms": {c: round(prof[c]["ms"], 3) for c in FACTOR_CLASSES},
                "note": "pencil route (precond 0), one stream (no other design's kernels beside it); stage "
                        "intervals summed"}

    # ---------------------------------------------------------------- headline: mixed, tuned options
    ctx = make_ctx(opts)
    head = timed(ctx, args.precision, args.steps, args.warmup)
    value, ms_per_step, res = head["value"], head["ms_per_step"], head["res"]
    single = kernel_names(args.precision)
    # the roofline kernel: the operator products, the class that holds the most of the chip
    # (summed event times under 12 streams also count the time a launch waits for room on
    # the chip, which ranks the convolution, whose workgroups need 78 KB of LDS, too high);
    # the other event-timed classes follow
    present = [c for c in single if head["prof"][c]["count"] > 0]
    first = "op_gemm" if "op_gemm" in present else max(single, key=lambda c: head["prof"][c]["ms"])
    order = [first] + sorted((c for c in present if c != first), key=lambda c: -head["prof"][c]["ms"])
    roof = entry(head["prof"], order[0], single)
    roof["others"] = [entry(head["prof"], c, single) for c in order[1:]]
    for e in roof["others"]:
        if e["kernel"].startswith("phx::omega_conv_kernel") and args.M >= 4:
            mc = max(1, args.M - int(opts.get("coarse_drop", 2)))
            e["note"] = f"with the coarse start's launches at order {mc} (the same kernel for that order)"
    # the dominant kernel's summed launch time per step over the step's wall time: how many
    # of its launches run at once on average (its per-launch rate is that of a kernel
    # sharing the chip with the other designs' kernels)
    roof["launch_time_over_wall"] = roof["total_ms"] / ms_per_step
    # the untimed, fully profiled step of the per-stage breakdown
    prof_all, wall_all = profiled(ctx, args.precision)
    stage_ms = {c: round(prof_all[c]["ms"], 3) for c in CLASSES}
    stage_sum = sum(prof_all[c]["ms"] for c in CLASSES)

    # ---------------------------------------------------------------- one stream: kernel alone, factorisation rate
    one_stream = {}
    fact = {}
    if not args.no_one_stream:
        # the dominant kernel with one design stream (the headline's options)
        c1 = make_ctx(dict(opts, streams=1.0))
        step(c1, args.precision)  # workspaces
        torch.cuda.synchronize()
        p1, w1ms = profiled(c1, args.precision)
        e1 = entry(p1, order[0], single)
        one_stream = {"kernel": e1["kernel"], "achieved": e1["achieved"], "unit": e1["unit"], "frac": e1["frac"],
                      "avg_launch_us": e1["avg_launch_us"], "launches": e1["launches"], "step_ms": w1ms,
                      "note": "the same kernel class in one profiled step with one design stream"}
        for c, e in zip(order[1:], roof["others"]):
            if p1[c]["count"] > 0:
                eo = entry(p1, c, single)
                e["one_stream"] = {"achieved": eo["achieved"], "frac": eo["frac"], "avg_launch_us": eo["avg_launch_us"],
                                   "launches": eo["launches"]}
        c1.close()
        # the pencil factorisation stage (precond 0: every k-point group factors K(k) + sigma Omega)
        cp = make_ctx(dict(opts, streams=1.0, precond=0.0))
        precs = [args.precision] + ([] if args.no_fp64 or args.precision == "fp64" else ["fp64"])
        for prec in precs:
            step(cp, prec)  # workspaces for this precision
            torch.cuda.synchronize()
            pp, _ = profiled(cp, prec)
            fact[prec] = factorisation(pp, cp.stat("factors"), prec)
        cp.close()
    roof["one_stream"] = one_stream or None

    # ---------------------------------------------------------------- the pencil route (precond 0), same workload
    pencil = None
    if not args.no_defaults:
        cpen = make_ctx(dict(opts, precond=0.0))
        pres = timed(cpen, args.precision, args.steps, 1)
        ppen = pres["prof"]
        pencil = {"value": pres["value"], "unit": "k-solves/s", "ms_per_step": pres["ms_per_step"],
                  "factors_per_design": pres["stats"]["factors"] / args.designs,
                  "iters_to_converge_mean_over_k": pres["stats"]["iters_mean_k"],
                  "solve_upd": entry(ppen, "solve_upd", single),
                  "note": "the headline's options with precond 0: K(k) + sigma Omega assembled and Cholesky-"
                          "factored per group of k-points, triangular solves as the preconditioner"}
        cpen.close()

    # ---------------------------------------------------------------- the FP64 path on the same workload
    fp64 = None
    if not args.no_fp64 and args.precision != "fp64":
        f = timed(ctx, "fp64", 1, 1)
        pf, wf = profiled(ctx, "fp64")
        fp64 = {"value": f["value"], "unit": "k-solves/s", "ms_per_step": f["ms_per_step"],
                "mixed_over_fp64": value / f["value"], "stats": f["stats"],
                "stage_ms_per_step": {c: round(pf[c]["ms"], 3) for c in CLASSES},
                "library_options": opts, "steps": 1, "warmup": 1}

    # ---------------------------------------------------------------- the library's default options
    defaults = None
    if not args.no_defaults:
        cd = phx.Context(0)
        dres = timed(cd, args.precision, args.steps, 1)
        defaults = {"value": dres["value"], "unit": "k-solves/s", "ms_per_step": dres["ms_per_step"],
                    "factors_per_design": dres["stats"]["factors"] / args.designs,
                    "iters_to_converge_mean_over_k": dres["stats"]["iters_mean_k"],
                    "note": "every library option at its default (streams 4, precond 2, kshare 2 within 0.15)"}
        cd.close()

    # Accuracy gate (untimed, after the timed steps): the last timed step's own mixed-precision
    # results for every design at a subset of its k-points against FP64 solves (tolerance
    # 1e-10) of the same designs at those k-points, one batched call.  Frequencies: relative
    # error, bands below 1e-3 of the largest frequency (the acoustic bands near Gamma)
    # excluded.  Sensitivities, norm-relative: bands 6 and 7 are compared by clusters of
    # nearly equal frequency (relative gap below 1e-4 in the FP64 result), each by the sum of
    # its members' derivatives (inside a nearly degenerate pair the per-vector derivative
    # depends on the basis the solver picked; the sum does not).  A cluster inside {6, 7} is
    # compared on the timed step's own output; one that reaches band 5 or 8 (or beyond) on a
    # second, untimed mixed-precision call at the same k-points that computes bands 3..10.
    gate = None
    if not args.no_gate:
        sub_idx = np.arange(0, args.nk, max(1, args.nk // 8))
        ext = tuple(range(3, 11))
        ctx.set_option("tol_fp64", 1e-10)
        o64, d64 = ctx.sens_batch_dev(cells, rho_dev, q[sub_idx], nb, ext, "fp64")
        torch.cuda.synchronize()
        ctx.set_option("tol_fp64", 1e-8)
        o32x, d32x = ctx.sens_batch_dev(cells, rho_dev, q[sub_idx], nb, ext, "mixed")
        torch.cuda.synchronize()
        om_err, sens_err, n_timed, n_ext, n_left = 0.0, 0.0, 0, 0, 0
        om_band = np.zeros(nb)           # max over designs and k of |dw|/w, per band
        sens_band = {}                   # band -> max sensitivity error of its cluster
        for d in range(args.designs):
            om32 = res[0][d].cpu().numpy()[sub_idx]
            dw32 = res[1][d].cpu().numpy()[sub_idx]
            om64, dw64 = o64[d].cpu().numpy(), d64[d].cpu().numpy()
            dw32x = d32x[d].cpu().numpy()
            rel = np.where(om64 > 1e-3 * om64.max(), np.abs(om32 - om64) / np.maximum(om64, 1e-300), 0.0)
            om_err = max(om_err, float(rel.max()))
            om_band = np.maximum(om_band, rel.max(axis=0))
            for k in range(len(sub_idx)):
                w = om64[k]
                done = set()
                for b in bands:
                    i = b - 1
                    if i in done:
                        continue
                    lo, hi = i, i
                    while lo > 0 and w[lo] - w[lo - 1] < 1e-4 * w[lo]:
                        lo -= 1
                    while hi + 1 < nb and w[hi + 1] - w[hi] < 1e-4 * w[hi + 1]:
                        hi += 1
                    cl = list(range(lo, hi + 1))
                    done.update(cl)
                    if w[i] <= 0:
                        continue
                    ref = dw64[k, [ext.index(c + 1) for c in cl]].sum(axis=0) if all(c + 1 in ext for c in cl) \
                        else None
                    if ref is None or hi == nb - 1:
                        n_left += 1  # cannot be formed from the bands computed
                        continue
                    if all(c + 1 in bands for c in cl):
                        got = dw32[k, [bands.index(c + 1) for c in cl]].sum(axis=0)
                        n_timed += 1
                    else:
                        got = dw32x[k, [ext.index(c + 1) for c in cl]].sum(axis=0)
                        n_ext += 1
                    e = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
                    sens_err = max(sens_err, float(e))
                    for c in cl:
                        sens_band[c + 1] = max(sens_band.get(c + 1, 0.0), float(e))
        gate = {"designs": args.designs, "k_points": int(len(sub_idx)), "source": "timed step",
                "max_rel_omega_err": om_err, "max_sens_err": sens_err,
                "rel_omega_err_per_band": [float(f"{e:.2e}") for e in om_band],
                "sens_err_per_band": {str(b): float(f"{e:.2e}") for b, e in sorted(sens_band.items())},
                "sens_clusters_from_timed_step": n_timed, "sens_clusters_from_bands_3_to_10": n_ext,
                "sens_clusters_not_compared": n_left,
                "pass": bool(om_err <= 1e-6 and sens_err <= 1e-6 and n_left == 0)}

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
            oms, dws = step(ctx, args.precision)
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

    st = head["stats"]
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
        "config": {"workload": f"FCC 32^3, M={args.M} (3N={3 * N}), {args.designs} designs x "
                               f"{args.nk} k, 12 bands, adjoint bands 6/7, {args.precision}",
                   "designs": args.designs, "k_points": args.nk, "nbands": nb, "sens_bands": list(bands),
                   "M": args.M, "precision": args.precision, "parallelism": f"single GPU, {args.streams} design streams",
                   "eigensolver_iters_max": st["iters"], "jacobi_sweeps_max": st["rr_sweeps"],
                   "coarse_start_iters_max": st["coarse_iters"], "iters_to_converge_mean_over_k": st["iters_mean_k"],
                   "preconditioner_factors_per_design": st["factors"] / args.designs,
                   "library_options": opts},
        "roofline": roof,
        "factorisation": fact or None,
        "fp64_path": fp64,
        "pencil_route": pencil,
        "library_defaults": defaults,
        "stage_ms_per_step": stage_ms,
        "stage_sum_over_wall": stage_sum / wall_all,
        "accuracy_gate": gate,
        "timed_window_monotonic_ns": head["window"],
        "cpu_baseline": cpu,
        "host_copies": host,
    }
    print(json.dumps(line), flush=True)


def kernel_source_sha(kernel: str):
    """SHA-256 of the text of the definition of `kernel` ("phx::name" or "phx::name<...>":
    the whole template) in the HIP sources, or None."""
    import glob
    import hashlib
    base = kernel.split("<")[0].split("::")[-1]
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_1603_06855_amd", "csrc", "*.hip"))):
        src = open(path).read()
        i = src.find(f" void {base}(")
        if i < 0:
            continue
        # the template line of a template kernel, else the line after the previous definition
        start = max(src.rfind("template <", 0, i), src.rfind("\n}\n", 0, i) + 3)
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
