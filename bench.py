"""Benchmark: Fourier-accelerated Landau gauge fixing of a 32^4 SU(3) lattice on one MI355X.

A step is one iteration of Alg. 1 (transform of the divergence, momentum
scaling, inverse transform, g with reunitarisation, link update, theta/F
reduction) over the whole lattice. `value` is FP64 iterations per second with
the links resident in HBM. Also reported: the same with the FP32 transform,
time to theta <= 1e-15 from the generated configuration for both, per-kernel
durations measured with HIP events on the library's stream, the roofline of
the dominant kernel, and the CPU oracle on a bounded sample.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-iters N] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "iters/s & time-to-theta<=1e-15 at 32^4 SU(3), FP64 vs FP32-FFT; HBM GB/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Algorithmic HBM bytes per site per launch of each kernel, for FP64 and
# FP32 transform fields (c = bytes per complex transform element):
#   divergence: read 4 links (576) + write 4 packed fields (4c)
#   transform pass: read + write 4 fields (8c)
#   gauge, or the inverse (x, y) pass fused with it: read 4 fields (4c) + write g (144)
#   link update: read 4 links (576) + g(x) (144) + write 4 links (576);
#     neighbour g(x + mu) is counted once (its own site's read)
#   fused link update + divergence of the new links: the link update's bytes
#     + 4 fields written (neighbour links and g recomputed from cache)
#   reduction: negligible (one double-double pair per 256 sites)


def kernel_bytes_per_site(name: str, c: int) -> float:
    if name == "fft_xy_inv_gauge":  # inverse (x, y) pass fused with g: read 4 fields, write g
        return 4 * c + 144
    if name.startswith("delta"):
        return 576 + 4 * c
    if name.startswith("fft"):
        return 8 * c
    if name.startswith("gauge"):
        return 4 * c + 144
    if name == "link_update_delta":  # fused update + divergence: the update's bytes + 4 fields written
        return 576 + 144 + 576 + 4 * c
    if name.startswith("link_update"):
        return 576 + 144 + 576
    return 0.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-iters", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--dims", default="32,32,32,32")
    ap.add_argument("--eps", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the method's data-parallel kernel runs on one GPU's share); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1210_8018_amd.api import GaugeFixer
    from paper_1210_8018_amd.inputs import random_links

    dims = tuple(int(v) for v in args.dims.split(","))
    V = int(np.prod(dims))
    log(f"generating {dims} eps={args.eps} seed={args.seed}")
    t0 = time.time()
    U_host = random_links(dims, args.eps, args.seed)
    log(f"generated in {time.time() - t0:.1f}s")
    U0 = torch.from_numpy(U_host).to("cuda")
    torch.cuda.synchronize()

    res = {}
    for prec in (0, 1):
        tag = "fp64" if prec == 0 else "fp32_fft"
        # throughput: K iterations regardless of theta
        U = U0.clone()
        fx = GaugeFixer(U, fft_prec=prec)
        log(f"[{tag}] warmup {args.warmup}")
        fx.step(args.warmup)
        torch.cuda.synchronize()
        log(f"[{tag}] timed {args.steps} steps")
        t0 = time.perf_counter()
        fx.step(args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # per-kernel durations with HIP events on the library's stream
        log(f"[{tag}] event-timed {args.steps} steps")
        fx.set_timing(True)
        fx.reset_timing()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fx.step(args.steps)
        torch.cuda.synchronize()
        dt_ev = time.perf_counter() - t1
        kt = fx.kernel_times()
        sched = fx.fft_schedule
        fx.set_timing(False)
        fx.close()
        del fx, U
        # time to theta <= 1e-15 from the generated configuration
        U = U0.clone()
        fx = GaugeFixer(U, fft_prec=prec)
        torch.cuda.synchronize()
        log(f"[{tag}] fix_until 1e-15")
        t2 = time.perf_counter()
        it, F, th = fx.fix_until(1e-15, 100000)
        torch.cuda.synchronize()
        ttt = time.perf_counter() - t2
        fx.close()
        del fx, U
        res[tag] = dict(iters_per_s=args.steps / dt, ms_per_step=1e3 * dt / args.steps,
                        event_region_iters_per_s=args.steps / dt_ev, kernels=kt,
                        time_to_theta_s=ttt, iterations=it, F_final=F, theta_final=th, fft_schedule=sched)
        log(f"[{tag}] {args.steps / dt:.1f} it/s, fixed in {it} its / {ttt * 1e3:.2f} ms, F={F:.15f}")

    c = 16
    per_iter_bytes = 0.0
    kern = {}
    for name, (ms, n) in res["fp64"]["kernels"].items():
        b = kernel_bytes_per_site(name, c) * V
        if n:
            per_iter_bytes += b
            avg = ms / n
            kern[name] = {"avg_us": round(1e3 * avg, 2), "launches": n,
                          "alg_GBs": round(b / (avg * 1e-3) / 1e9, 1) if b else None}
    dom = max(res["fp64"]["kernels"].items(), key=lambda kv: kv[1][0])
    dom_name, (dom_ms, dom_n) = dom
    dom_avg_s = dom_ms / dom_n * 1e-3
    dom_bytes = kernel_bytes_per_site(dom_name, c) * V
    achieved = dom_bytes / dom_avg_s / 1e9
    traffic_file = os.path.join(ROOT, "profiles", "traffic_link_update_32x4.json")
    traffic = None
    if os.path.exists(traffic_file):
        try:
            t = json.load(open(traffic_file))
            if t.get("kernel") == dom_name and t.get("source_hash") == _source_hash():
                traffic = t.get("bytes_per_launch")
        except Exception:
            traffic = None

    cpu = None
    if not args.no_cpu:
        import oracle

        nthr = oracle.num_threads()
        log(f"cpu oracle: {args.cpu_iters} iterations at {dims} on {nthr} threads")
        t3 = time.perf_counter()
        oracle.fix(dims, U_host, alpha=0.08, eps=-1.0, max_iter=args.cpu_iters)
        dcpu = time.perf_counter() - t3
        cpu = {"value": args.cpu_iters / dcpu, "unit": "iters/s", "cores": nthr, "kind": "oracle",
               "sample": f"{args.cpu_iters} iterations of Alg. 1 on the same {'x'.join(map(str, dims))} "
                         f"configuration (FP64 C oracle, OpenMP), {dcpu:.1f} s"}

    f64 = res["fp64"]
    f32 = res["fp32_fft"]
    out = {
        "metric": METRIC,
        "value": round(f64["iters_per_s"], 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} SU(3) links, generator eps={args.eps} seed={args.seed}, "
                               f"alpha=0.08, FP64 (plain method)",
                   "dims": list(dims), "alpha": 0.08, "theta_eps": 1e-15},
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "avg_us": round(dom_avg_s * 1e6, 2), "alg_bytes_per_launch": dom_bytes},
        "cpu_baseline": cpu,
        "time_to_theta": {"fp64": {"seconds": round(f64["time_to_theta_s"], 5), "iterations": f64["iterations"],
                                   "F_final": f64["F_final"], "theta_final": f64["theta_final"]},
                          "fp32_fft": {"seconds": round(f32["time_to_theta_s"], 5), "iterations": f32["iterations"],
                                       "F_final": f32["F_final"], "theta_final": f32["theta_final"]}},
        "fp32_fft": {"iters_per_s": round(f32["iters_per_s"], 2), "ms_per_step": round(f32["ms_per_step"], 4),
                     "fft_schedule": f32["fft_schedule"]},
        "fft_schedule": f64["fft_schedule"],
        "hbm": {"alg_bytes_per_iter": per_iter_bytes,
                "effective_GBs": round(per_iter_bytes * f64["iters_per_s"] / 1e9, 1),
                "effective_frac": round(per_iter_bytes * f64["iters_per_s"] / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_fp64": kern,
        "event_region_iters_per_s": round(f64["event_region_iters_per_s"], 2),
    }
    print(json.dumps(out), flush=True)


def _source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in ("gf_kernels.hip", "gf_device.h", "gf_internal.h"):
        with open(os.path.join(ROOT, "paper_1210_8018_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
