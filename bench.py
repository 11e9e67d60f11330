"""Benchmark of the constant-time bilateral filter on one MI355X.

One step = one plain FP32 forward pass of the whole filter (plan, pointwise
transforms, horizontal and vertical moving sums, recombination, ratio) over a
4096x4096 synthetic "rect" image (64 random rectangles + N(0, 20^2) noise),
box radius 20, sigma_r = 30, T = 255, N = 30 (16 folded orders).  Inputs are
resident in HBM before timing starts; steps are timed with HIP events on the
stream the library launches on.  The same run also times, at their own
workloads, the training forward + adjoint, the 16-bit precision forms (BF16,
FP16, Q15 stack; with and without Kahan-compensated sums), the 8192^2 r=32
workload, the 16 x 1024^2 differentiation workload and the batched
persistent/graph launch, and the FP64 CPU oracle on a bounded sample of the
headline workload (reported as cpu_baseline).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6       # MI355X published FP64 vector peak
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E
# Algorithmic FP32 work of the method per (pixel, folded order): rotation of
# (cos, sin) 6, f-weighted channels 2, four channels x two directions x two
# running-sum updates 16, recombination of P and Q 10.
FLOP_PER_PX_ORDER = 34
BYTES_PER_PX = 8              # FP32 in + FP32 out; the stack never reaches HBM
# HBM bytes and VALU wave-instructions per launch of the headline kernel, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE (scaled by a 256 MiB copy) and
# SQ_INSTS_VALU (profiles/strip_kernel_fwd_rect4096_r20_s30.md).  Valid for this
# kernel build only: set to None when the kernel changes.
HEADLINE_KERNEL = "strip_kernel<float,256,16,4,PolForward<float,0>,0,false,3,20>"
HEADLINE_HBM_BYTES = 282.7e6
HEADLINE_VALU_INSTS = 194.15e6
# SQ_LDS_IDX_ACTIVE per launch (cycles summed over the CUs in which the LDS
# serves this kernel's accesses), from the same profile
HEADLINE_LDS_ACTIVE = 144.648e6
# VALU issue: one wave64 instruction per SIMD every 4 cycles (16 lanes, no
# packed FP32), 4 SIMDs per CU, 256 CUs at 2.4 GHz
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
METRIC = "Mpixel/s + %HBM roofline, 4096\u00b2 r=20 \u03c3r=30; fwd+bwd and BF16 vs plain FP32"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_calls(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        fn()
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return float(np.mean(ms)), float(np.median(ms)), wall


def cpu_baseline(img, radius, sigma, N, T, gpu_out=None, budget_s=20.0):
    """Times the FP64 oracle on a seeded sample of pixels; with the GPU output of the
    same workload, also returns its errors against the oracle on that sample."""
    import oracle
    H, W = img.shape
    rng = np.random.default_rng(123)
    n0 = 2000
    idx = rng.integers(0, H * W, n0)
    t0 = time.perf_counter()
    oracle.bilateral_at(img, idx, radius, sigma, N)
    t_cal = time.perf_counter() - t0
    n = int(min(H * W, max(n0, n0 * budget_s / max(t_cal, 1e-6))))
    idx = rng.integers(0, H * W, n)
    t0 = time.perf_counter()
    ref = oracle.bilateral_at(img, idx, radius, sigma, N)
    dt = time.perf_counter() - t0
    base = {"value": n / dt / 1e6, "unit": "Mpixel/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} seeded random pixels of the {H}x{W} r={radius} image, direct FP64 window sums "
                      f"({(2 * radius + 1) ** 2} kernel evaluations per pixel), {dt:.1f} s"}
    if gpu_out is None:
        return base, None
    err = np.abs(gpu_out.ravel()[idx].astype(np.float64) - ref)
    parity = {"vs": "oracle", "pixels": n, "max_abs": float(err.max()), "rms": float(np.sqrt(np.mean(err ** 2))),
              "p99.99": float(np.quantile(err, 0.9999)), "tolerance": 1e-4 * T}
    return base, parity


class OracleErrors:
    """Errors of GPU outputs against the FP64 oracle, evaluated in the CPU-baseline leg.

    sample() picks, while the GPU output still exists, n seeded random pixels plus, when
    worst_vs (another output of the same workload, e.g. the plain FP32 one) is given, the
    `worst` pixels where the output departs most from it, and keeps the output's values
    there; evaluate() later runs the oracle at those pixels (ref_at(idx): the oracle
    at flat pixel indices) and writes the errors into the result dictionaries."""

    def __init__(self):
        self.pending = []

    def sample(self, into, out, ref_at, tol, n=100_000, seed=321, worst_vs=None, worst=2000):
        import torch
        flat = out.detach().double().ravel()
        idx = np.random.default_rng(seed).integers(0, flat.numel(), n)
        if worst_vs is not None:
            d = (out.double() - worst_vs.double()).abs().ravel()
            top = torch.topk(d, min(worst, d.numel())).indices.cpu().numpy()
            idx = np.concatenate([idx, top])
        idx = np.unique(idx)
        vals = flat[torch.from_numpy(idx).to(flat.device)].cpu().numpy()
        self.pending.append((into, vals, idx, ref_at, tol))

    def evaluate(self):
        for into, vals, idx, ref_at, tol in self.pending:
            err = np.abs(vals - ref_at(idx))
            m = float(err.max())
            e = {"vs": "oracle", "pixels": int(idx.size), "max_abs": m, "rms": float(np.sqrt(np.mean(err ** 2))),
                 "p99.99": float(np.quantile(err, 0.9999)), "tolerance": tol, "within": bool(m <= tol)}
            if "error" in into and isinstance(into["error"], list):
                into["error"].append(e)
            else:
                into["error"] = e
        self.pending = []


def _oracle():
    import oracle
    return oracle


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def copy_bandwidth(dev, mib=1024, reps=10):
    """Device-to-device copy rate (read + write bytes per second) of a plain torch copy."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * 4 * n / (ms * 1e-3) / 1e9


def child_processes():
    """Processes this one has started that still exist (the benchmark starts none; the
    oracle's OpenMP workers are threads)."""
    try:
        import psutil
        return [f"{c.pid}:{c.name()}" for c in psutil.Process().children(recursive=True)]
    except Exception as e:  # noqa: BLE001
        return [f"unknown ({type(e).__name__})"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 200 warm-up calls (about 90 ms of the headline) let the GPU's clocks settle
    # before the timed calls; with 20 the first timed calls still ran slower
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--kernel-only", nargs="?", const="headline", default=None,
                    choices=["headline", "spatial", "poly", "poly_trunc", "nlm2", "fp64", "fwd_bwd", "bf16",
                             "batched", "alg1", "denoise16"],
                    help="profiling mode: run the headline forward (or the spatial-kernel, polynomial-"
                         "kernel, patch, FP64, training forward + adjoint, 16-bit or Algorithm 1 form at the same "
                         "size, "
                         "or the 256-image batch) --steps times after --warmup, and a device copy of "
                         "--copy-mib MiB; print nothing but a summary line")
    ap.add_argument("--copy-mib", type=int, default=256)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is "
              "described in DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1107_4617_amd import (autotune_batched, batched_shape, bilateral, bilateral_backward,
                                     bilateral_batched, bilateral_train, nlm2, order_for, plan_info,
                                     poly_order_for, poly_plan_info, spatial_filter, spatial_sigma_for,
                                     tune_cache_clear)
    from paper_1107_4617_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    H = W = 4096
    radius, sigma, T, N = 20, 30.0, 255.0, 30
    K, _ = plan_info(N, 0.0)
    log("generating rect4096 image")
    img_np = wl.rect_image(H, W, seed=2)
    img = torch.from_numpy(img_np).to(dev)
    out = torch.empty_like(img)

    fwd = lambda: bilateral(img, radius, sigma, T, N=N, out=out)  # noqa: E731
    # the separable q_2 spatial kernel over the same window (Algorithm 2 with M = 9)
    sig_s = spatial_sigma_for(radius, 2)
    fwd_sp = lambda: bilateral(img, radius, sigma, T, N=N, out=out, spatial_sigma=sig_s, spatial_N=2)  # noqa: E731
    # the polynomial range kernel (Section 3's p_N, eq. (5) scaling) at the same sigma_r:
    # N_p = ceil(T^2 / (2 sigma_r^2)) = 37, all 75 Chebyshev coefficients or those above 1e-7
    fwd_poly = lambda: bilateral(img, radius, sigma, T, out=out, range_kernel="poly")  # noqa: E731
    fwd_poly_t = lambda: bilateral(img, radius, sigma, T, out=out, range_kernel="poly", weight_eps=1e-7)  # noqa: E731
    # two-pixel-patch non-local means (Section 5, p = 2): patches {x, x + (0, 1)}, sigma 60 per
    # patch pixel (N_0 = 8 each: 9 x 5 terms)
    fwd_nlm = lambda: nlm2(img, radius, 60.0, 60.0, (0, 1), T, out=out)  # noqa: E731
    if args.kernel_only:
        if args.kernel_only == "spatial":
            fwd = fwd_sp
        elif args.kernel_only == "nlm2":
            fwd = fwd_nlm
        elif args.kernel_only == "poly":
            fwd = fwd_poly
        elif args.kernel_only == "poly_trunc":
            fwd = fwd_poly_t
        elif args.kernel_only == "fp64":
            img64 = img.double()
            out64 = torch.empty_like(img64)
            fwd = lambda: bilateral(img64, radius, sigma, T, N=N, precision="fp64", out=out64)  # noqa: E731
        elif args.kernel_only == "fwd_bwd":
            g = torch.randn(img.shape, generator=torch.Generator().manual_seed(5)).to(dev)

            def fwd():
                o, sv = bilateral_train(img, radius, sigma, T, N)
                bilateral_backward(img, g, radius, sigma, T, N, out=o, saved=sv)
        elif args.kernel_only == "denoise16":
            # the 16 x 1024^2 differentiation workload as one stacked launch pair
            pairs = [wl.denoise_pair(i) for i in range(16)]
            x16 = torch.from_numpy(np.stack([p[0] for p in pairs])).to(dev)
            t16 = torch.from_numpy(np.stack([p[1] for p in pairs])).to(dev)

            def fwd():
                o, sv = bilateral_train(x16, 10, 25.0, T, 43)
                bilateral_backward(x16, (2.0 / x16.numel()) * (o - t16), 10, 25.0, T, 43, out=o, saved=sv)
        elif args.kernel_only == "alg1":
            # Algorithm 1: the q_2 Gaussian-like spatial filter alone, over the same window
            fwd = lambda: spatial_filter(img, radius, sig_s, 2, out=out)  # noqa: E731
        elif args.kernel_only == "bf16":
            fwd = lambda: bilateral(img, radius, sigma, T, N=N, precision="bf16", weight_eps=1e-7,  # noqa: E731
                                    out=out)
        elif args.kernel_only == "batched":
            specs = wl.batch_specs(256, seed=4)
            imgs = [torch.from_numpy(wl.gradient_image(h, w, s)).to(dev) for (h, w, r, sg, s) in specs]
            outs = [torch.empty_like(x) for x in imgs]
            radii, sigs = [s[2] for s in specs], [s[3] for s in specs]
            fwd = lambda: bilateral_batched(imgs, radii, sigs, T, outs=outs)  # noqa: E731
        # a plain device copy of known size: reference for the HBM byte counters
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        for _ in range(args.warmup):
            fwd()
        torch.cuda.synchronize()
        for _ in range(args.steps):
            fwd()
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": True, "steps": args.steps, "copy_bytes": 4 * n}), flush=True)
        return
    log("timing FP32 forward")
    mean_ms, med_ms, wall = time_calls(fwd, args.steps, args.warmup, stream)
    torch.cuda.synchronize()
    out_head = out.cpu().numpy()   # the headline output, for the oracle comparison
    px = H * W
    value = px / (mean_ms * 1e-3) / 1e6
    flops = FLOP_PER_PX_ORDER * K * px
    achieved = flops / (mean_ms * 1e-3) / 1e12
    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mean_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rect4096_r20_s30", "H": H, "W": W, "radius": radius, "sigma_r": sigma, "T": T,
                   "N": N, "folded_orders": K},
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": (round(HEADLINE_HBM_BYTES / (mean_ms * 1e-3) / 1e9, 1)
                        if HEADLINE_HBM_BYTES is not None else None),
            "traffic_unit": "GB/s",
            "traffic_bytes_per_launch": HEADLINE_HBM_BYTES,
            "kernel": HEADLINE_KERNEL,
            "flop_per_launch": flops,
            "algorithmic_bytes_per_launch": BYTES_PER_PX * px,
            "hbm_frac": round(BYTES_PER_PX * px / (mean_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        },
        "median_ms": round(med_ms, 4),
    }
    log("timing a 1 GiB device copy")
    copy_gbs = copy_bandwidth(dev)
    rl = rec["roofline"]
    rl["copy_GB/s"] = round(copy_gbs, 1)
    rl["hbm_frac_vs_copy"] = round(BYTES_PER_PX * px / (mean_ms * 1e-3) / 1e9 / copy_gbs, 4)
    if HEADLINE_VALU_INSTS is not None:
        # share of the launch during which the SIMDs issue VALU instructions
        rl["valu_busy"] = round(HEADLINE_VALU_INSTS / VALU_ISSUE_PER_S / (mean_ms * 1e-3), 4)
        rl["valu_lane_instructions_per_pixel_order"] = round(HEADLINE_VALU_INSTS * 64 / (px * K), 2)
    else:
        rl["valu_busy"] = None
    # share of the launch during which the CUs' LDS is busy with the kernel's accesses
    # (timing probes with LDS traffic removed show the launch time following it)
    rl["lds_busy"] = (round(HEADLINE_LDS_ACTIVE / (256 * 2.4e9) / (mean_ms * 1e-3), 4)
                      if HEADLINE_LDS_ACTIVE is not None else None)
    # Errors of each variant below against the FP64 oracle, evaluated in the CPU-baseline leg:
    # 100,000 seeded random pixels plus the 2,000 where the variant departs most from the
    # plain FP32 output.
    oe = OracleErrors()
    at_head = lambda idx: _oracle().bilateral_at(img_np, idx, radius, sigma, N)  # noqa: E731

    if not args.no_extra:
        variants = {}
        # precision forms at the headline workload: the cos/sin stack quantised to
        # 16 bits, Kahan-compensated vertical sums, weights below 1e-7 dropped
        kb, eps = plan_info(N, 1e-7)
        outq = torch.empty_like(img)
        for prec in ("bf16", "fp16", "i16"):
            for kahan in (True, False):
                log(f"timing {prec} precision form, kahan={kahan}")
                ms_q, _, _ = time_calls(lambda: bilateral(img, radius, sigma, T, N=N, precision=prec,
                                                          weight_eps=1e-7, kahan=kahan, out=outq),
                                        args.steps, args.warmup, stream)
                name = f"{prec}{'_kahan' if kahan else ''}_trunc1e-7"
                variants[name] = {"Mpixel/s": round(px / ms_q / 1e3, 2), "ms": round(ms_q, 4),
                                  "folded_orders": kb, "dropped_weight": eps,
                                  "max_abs_vs_fp32": float((outq - out).abs().max())}
                oe.sample(variants[name], outq, at_head, 2e-3 * T, worst_vs=out)
        # plain FP32 with the same truncation: the precision forms' order count in FP32
        log("timing fp32 with weights below 1e-7 dropped")
        ms_t, _, _ = time_calls(lambda: bilateral(img, radius, sigma, T, N=N, weight_eps=1e-7, out=outq),
                                args.steps, args.warmup, stream)
        variants["fp32_trunc1e-7"] = {"Mpixel/s": round(px / ms_t / 1e3, 2), "ms": round(ms_t, 4),
                                      "folded_orders": kb, "dropped_weight": eps,
                                      "max_abs_vs_fp32": float((outq - out).abs().max())}
        oe.sample(variants["fp32_trunc1e-7"], outq, at_head, 1e-4 * T, worst_vs=out)
        del outq
        # FP64 throughout (transforms, sums, recombination) at the headline workload
        log("timing fp64 form")
        img64 = img.double()
        out64 = torch.empty_like(img64)
        ms_d, _, _ = time_calls(lambda: bilateral(img64, radius, sigma, T, N=N, precision="fp64", out=out64),
                                max(5, args.steps // 5), max(2, args.warmup // 5), stream)
        variants["fp64_rect4096_r20_s30"] = {"Mpixel/s": round(px / ms_d / 1e3, 2), "ms": round(ms_d, 4),
                                             "fp64_TFLOP/s": round(px * K * FLOP_PER_PX_ORDER / (ms_d * 1e-3) / 1e12, 2),
                                             "fp64_frac": round(px * K * FLOP_PER_PX_ORDER / (ms_d * 1e-3) / 1e12
                                                                / PEAK_FP64_TFLOPS, 4),
                                             "max_abs_vs_fp32": float((out64.float() - out).abs().max())}
        oe.sample(variants["fp64_rect4096_r20_s30"], out64, at_head, 1e-9 * T, worst_vs=out)
        del img64, out64
        # Algorithm 2 with the separable q_2 spatial kernel (M = 9) and Algorithm 1 at the
        # headline size and window
        log("timing spatial kernels")
        outv = torch.empty_like(img)
        ms_sp, _, _ = time_calls(lambda: bilateral(img, radius, sigma, T, N=N, out=outv, spatial_sigma=sig_s,
                                                   spatial_N=2), args.steps, args.warmup, stream)
        v = variants["spatial_q2_M9_rect4096_r20_s30"] = {
            "Mpixel/s": round(px / ms_sp / 1e3, 2), "ms": round(ms_sp, 4), "spatial_sigma": sig_s, "spatial_N": 2,
            "vs_box": round(mean_ms / ms_sp, 3)}
        oe.sample(v, outv, lambda idx: _oracle().bilateral_sp_at(img_np, idx, radius, sigma, N, sig_s, 2), 1e-4 * T)
        ms_a1, _, _ = time_calls(lambda: spatial_filter(img, radius, sig_s, 2, out=outv), args.steps, args.warmup,
                                 stream)
        v = variants["algorithm1_q2_rect4096_r20"] = {"Mpixel/s": round(px / ms_a1 / 1e3, 2), "ms": round(ms_a1, 4)}
        oe.sample(v, outv, lambda idx: _oracle().bilateral_sp_at(img_np, idx, radius, 1.0, 0, sig_s, 2), 1e-4 * T)
        log("timing two-pixel-patch non-local means")
        ms_nl, _, _ = time_calls(lambda: nlm2(img, radius, 60.0, 60.0, (0, 1), T, out=outv),
                                 max(5, args.steps // 5), max(2, args.warmup // 5), stream)
        n60 = order_for(60.0, T)
        v = variants["nlm2_patch_u01_s60_rect4096_r20"] = {"Mpixel/s": round(px / ms_nl / 1e3, 2),
                                                           "ms": round(ms_nl, 4), "terms": 45}
        oe.sample(v, outv, lambda idx: _oracle().nlm2_at(img_np, idx, radius, 60.0, n60, 60.0, n60, (0, 1)), 1e-4 * T)
        ms_b60, _, _ = time_calls(lambda: bilateral(img, radius, 60.0, T, out=outv), args.steps, args.warmup, stream)
        v["bilateral_s60_ms"] = round(ms_b60, 4)
        log("timing polynomial range kernel")
        n_p = poly_order_for(sigma, T)
        at_poly = lambda idx: _oracle().bilateral_poly_at(img_np, idx, radius, sigma, n_p)  # noqa: E731
        for name, eps_p in (("poly_pN37_rect4096_r20_s30", 0.0), ("poly_pN37_trunc1e-7_rect4096_r20_s30", 1e-7)):
            ms_pl, _, _ = time_calls(lambda: bilateral(img, radius, sigma, T, out=outv, range_kernel="poly",
                                                       weight_eps=eps_p), args.steps, args.warmup, stream)
            kp, bp = poly_plan_info(sigma, T, eps=eps_p)
            variants[name] = {"Mpixel/s": round(px / ms_pl / 1e3, 2), "ms": round(ms_pl, 4), "N": n_p,
                              "chebyshev_coefficients": kp, "dropped_bound": bp,
                              "vs_raised_cosine": round(mean_ms / ms_pl, 3)}
            oe.sample(variants[name], outv, at_poly, 1e-4 * T)
        # the paper's timed instance: 512x512, T = 5 (11x11 window), M x N = 3^2 x 5, i.e. the
        # spatial q_2 on [-5, 5] and the range q_4 on [-255, 255] (sigma_r = 255 / pi)
        small_np = wl.smooth_image(512, 512, seed=1)
        small = torch.from_numpy(small_np).to(dev)
        outs_ = torch.empty_like(small)
        ss5 = spatial_sigma_for(5, 2)
        ms_p, _, _ = time_calls(lambda: bilateral(small, 5, T / math.pi, T, N=4, out=outs_,
                                                  spatial_sigma=ss5, spatial_N=2),
                                args.steps, args.warmup, stream)
        v = variants["paper_instance_512_T5_M9_N5"] = {"ms": round(ms_p, 4),
                                                       "Mpixel/s": round(512 * 512 / ms_p / 1e3, 2),
                                                       "paper_matlab_s": 2.5}
        oe.sample(v, outs_, lambda idx: _oracle().bilateral_sp_at(small_np, idx, 5, T / math.pi, 4, ss5, 2),
                  1e-4 * T, n=512 * 512)
        del small, outs_, outv
        # training forward + adjoint at the headline workload
        g = torch.randn_like(img)

        def fb():
            o, s = bilateral_train(img, radius, sigma, T, N)
            bilateral_backward(img, g, radius, sigma, T, N, out=o, saved=s)

        log("timing forward+backward")
        ms_fb, _, _ = time_calls(fb, max(3, args.steps // 2), 1, stream)
        o_tr, _ = bilateral_train(img, radius, sigma, T, N)
        v = variants["fwd_bwd_fp32"] = {"Mpixel/s": round(px / ms_fb / 1e3, 2), "ms": round(ms_fb, 4),
                                        "error_note": "the training forward's output; the gradients are compared "
                                                      "with the oracle's in the GPU tests"}
        oe.sample(v, o_tr, at_head, 1e-4 * T)
        del g, o_tr
        # 8192^2, r=32, sigma_r=15, N=117: plain FP32 (59 orders) vs truncation at 1e-7 (28 orders)
        # in FP32 and in the 16-bit stacks
        log("timing 8192^2 r=32 workload")
        big_np = wl.rect_image(8192, 8192, seed=3)
        big = torch.from_numpy(big_np).to(dev)
        outb = torch.empty_like(big)
        out8 = torch.empty_like(big)
        at8 = lambda idx: _oracle().bilateral_at(big_np, idx, 32, 15.0, 117)  # noqa: E731
        px8 = 8192 * 8192
        ms_p, _, _ = time_calls(lambda: bilateral(big, 32, 15.0, T, N=117, out=out8), 3, 1, stream)
        v8 = {"fp32": {"Mpixel/s": round(px8 / ms_p / 1e3, 2), "ms": round(ms_p, 3),
                       "orders": plan_info(117, 0.0)[0]}}
        oe.sample(v8["fp32"], out8, at8, 1e-4 * T, n=20_000)
        for name, kw in (("fp32_trunc", {}), ("i16_trunc", {"precision": "i16"}),
                         ("i16_kahan_trunc", {"precision": "i16", "kahan": True}),
                         ("fp16_trunc", {"precision": "fp16"}), ("bf16_trunc", {"precision": "bf16"})):
            log(f"timing 8192^2 {name}")
            ms_v, _, _ = time_calls(lambda: bilateral(big, 32, 15.0, T, N=117, weight_eps=1e-7, out=outb, **kw),
                                    3, 1, stream)
            v8[name] = {"Mpixel/s": round(px8 / ms_v / 1e3, 2), "ms": round(ms_v, 3),
                        "orders": plan_info(117, 1e-7)[0]}
            # every truncated form is held to the precision form's 2e-3 T: at |B| = 65^2 the
            # dropped weight mass alone moves the output by up to 2 eps |B| T / Q (eps = 1.28e-7)
            oe.sample(v8[name], outb, at8, 2e-3 * T, n=20_000, worst_vs=out8)
        variants["rect8192_r32_s15"] = v8
        del big, outb, out8
        # differentiation workload: 16 x 1024^2, r=10, sigma_r=25, N=43
        log("timing 16x1024^2 fwd+bwd")
        pairs = [wl.denoise_pair(i) for i in range(16)]
        x16 = torch.from_numpy(np.stack([p[0] for p in pairs])).to(dev)
        t16 = torch.from_numpy(np.stack([p[1] for p in pairs])).to(dev)

        def fb16():
            # the 16 images as one stack: one training-forward launch and one adjoint
            # launch; loss = mean((u - target)^2) over the batch
            o, s = bilateral_train(x16, 10, 25.0, T, 43)
            gg = (2.0 / x16.numel()) * (o - t16)
            bilateral_backward(x16, gg, 10, 25.0, T, 43, out=o, saved=s)

        def fb16_each():
            for b in range(16):
                o, s = bilateral_train(x16[b], 10, 25.0, T, 43)
                gg = (2.0 / x16.numel()) * (o - t16[b])
                bilateral_backward(x16[b], gg, 10, 25.0, T, 43, out=o, saved=s)

        ms16, _, _ = time_calls(fb16, 5, 1, stream)
        ms16e, _, _ = time_calls(fb16_each, 3, 1, stream)
        o16, _ = bilateral_train(x16, 10, 25.0, T, 43)
        x0 = pairs[0][0]
        v = variants["denoise16x1024_fwd_bwd"] = {"Mpixel/s": round(16 * 1024 * 1024 / ms16 / 1e3, 2),
                                                  "ms": round(ms16, 3), "one_image_at_a_time_ms": round(ms16e, 3),
                                                  "error_note": "image 0's training-forward output"}
        oe.sample(v, o16[0], lambda idx: _oracle().bilateral_at(x0, idx, 10, 25.0, 43), 1e-4 * T, n=50_000)
        del x16, t16, pairs, o16
        # batched workload: 256 images, one persistent launch replayed from a HIP graph,
        # with the default launch shapes and with those the autotuner picks for the batch
        log("generating 256-image batch")
        specs = wl.batch_specs(256, seed=4)
        imgs_np = [wl.gradient_image(h, w, s) for (h, w, r, sg, s) in specs]
        imgs = [torch.from_numpy(x).to(dev) for x in imgs_np]
        outs = [torch.empty_like(x) for x in imgs]
        radii, sigs = [s[2] for s in specs], [s[3] for s in specs]
        tot_px = sum(h * w for (h, w, *_r) in specs)
        side = torch.cuda.Stream()
        log("timing batched graph (default launch shapes)")
        tune_cache_clear()
        with torch.cuda.stream(side):
            ms_b0, _, _ = time_calls(lambda: bilateral_batched(imgs, radii, sigs, T, outs=outs, graph_key=40),
                                     5, 1, side)
            log("autotuning the batched launch")
            t0 = time.perf_counter()
            blk, _ = autotune_batched(imgs, radii, sigs, T, outs=outs)
            tune_s = time.perf_counter() - t0
            log("timing batched graph (tuned launch shapes)")
            ms_bt, _, _ = time_calls(lambda: bilateral_batched(imgs, radii, sigs, T, outs=outs, graph_key=41),
                                     5, 1, side)
        side.synchronize()
        _, rows_t, chunk_t = batched_shape([tuple(x.shape) for x in imgs], radii, sigs, T)
        v = variants["batched256_graph"] = {
            "Mpixel/s": round(tot_px / ms_bt / 1e3, 2), "ms": round(ms_bt, 3), "pixels": tot_px,
            "default_shape_ms": round(ms_b0, 3), "tuned_block": blk, "tune_s": round(tune_s, 1),
            "tuned_rows_used": sorted(set(rows_t)), "tuned_chunks_used": sorted(set(chunk_t)), "error": [],
            "error_note": "images 0, 100 and 255"}
        for b in (0, 100, 255):
            _, _, r_, sg_, _ = specs[b]
            n_b = order_for(sg_, T)
            oe.sample(v, outs[b], lambda idx, f=imgs_np[b], r_=r_, sg_=sg_, n_b=n_b:
                      _oracle().bilateral_at(f, idx, r_, sg_, n_b), 1e-4 * T, n=20_000)
        tune_cache_clear()
        del imgs, outs
        rec["variants"] = variants

    if not args.no_cpu:
        log("timing CPU oracle sample")
        rec["cpu_baseline"], rec["parity"] = cpu_baseline(img_np, radius, sigma, N, T, gpu_out=out_head)
        rec["cpu_baseline"]["host"] = host_info()
        log("evaluating the variants' errors against the oracle")
        oe.evaluate()
    rec["child_processes_at_end"] = child_processes()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
