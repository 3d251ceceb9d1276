"""Benchmark: Fourier-accelerated Landau gauge fixing of a 32^4 SU(3) lattice on one MI355X.

A step is one iteration of Alg. 1 (transform of the divergence, momentum
scaling, inverse transform, g with reunitarisation, link update, theta/F
reduction) over the whole lattice. `value` is FP64 iterations per second with
the links resident in HBM. Also reported: the same with the FP32 transform,
time to theta <= 1e-15 from the generated configuration for both, per-kernel
durations measured with HIP events on the library's stream, the roofline of
the dominant kernel, and the CPU oracle on a bounded sample.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-iters N] [--no-cpu]
python bench.py --workload batch|batch_small|large48|large64|diff|thermal   (other measured workloads)
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
#   transform pass: read + write 4 fields (8c); the (z, t) pass with the
#     scaling also reads K(p), one real of the transform precision (c/2)
#   gauge: read 4 fields (4c) + write g (144); the inverse (x, y) pass, which
#     ends the transform, writes the 4 filtered fields (4c) for the fused pass
#   link update: read 4 links (576) + g(x) (144) + write 4 links (576);
#     neighbour g(x + mu) is counted once (its own site's read)
#   fused link update + divergence of the new links, links in two-row
#     (12-real) form, g formed from the 4 filtered fields: read links (384) +
#     filtered fields (4c) + write links (384) + 4 fields (4c) (neighbour
#     links and g recomputed from cache)
#   reduction: negligible (one double-double pair per 256 sites)


def kernel_bytes_per_site(name: str, c: int) -> float:
    if name == "fft_xy_inv_gauge":  # inverse (x, y) pass: read and write 4 fields
        return 8 * c
    if name.startswith("delta"):
        return 576 + 4 * c
    if name == "fft_zt_scale":  # (z, t) forward, K(p) (one real of the transform precision), backward
        return 8 * c + c // 2
    if name.startswith("fft"):
        return 8 * c
    if name.startswith("gauge"):
        return 4 * c + 144
    if name == "link_update_delta":  # fused update + divergence, two-row links, g from the filtered fields
        return 384 + 4 * c + 384 + 4 * c
    if name.startswith("link_update"):
        return 576 + 144 + 576
    return 0.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=60)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--dims", default="32,32,32,32")
    ap.add_argument("--eps", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "batch", "batch_small", "large48", "large64", "diff", "thermal"])
    ap.add_argument("--beta", type=float, default=6.0)
    ap.add_argument("--sweeps", type=int, default=300)
    ap.add_argument("--oracle-iters", type=int, default=20,
                    help="large48/large64: iterations compared with the oracle")
    ap.add_argument("--fft-schedule", type=int, default=0,
                    help="transform schedule of the headline contexts (0: autotuned; see gf_params.fft_schedule)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the method's data-parallel kernel runs on one GPU's share); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1210_8018_amd.api import GaugeFixer
    from paper_1210_8018_amd.inputs import random_links

    if args.workload != "headline":
        {"batch": bench_batch, "batch_small": bench_batch, "large48": bench_large, "large64": bench_large,
         "diff": bench_diff, "thermal": bench_thermal}[args.workload](args)
        return

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
        fx = GaugeFixer(U, fft_prec=prec, fft_schedule=args.fft_schedule)
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
        fx = GaugeFixer(U, fft_prec=prec, fft_schedule=args.fft_schedule)
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

    # single-precision link storage (the paper's single-precision mode, 12-real
    # in binary32, FP64 arithmetic) with the FP32 transform; fix_until then
    # refines in FP64 storage from theta <= 1e-10 down to 1e-15
    U = U0.clone()
    fx = GaugeFixer(U, fft_prec=1, link_prec=1, fft_schedule=args.fft_schedule)
    fx.step(args.warmup)
    torch.cuda.synchronize()
    log(f"[sp_links] timed {args.steps} steps")
    t0 = time.perf_counter()
    fx.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fx.set_timing(True)
    fx.reset_timing()
    fx.step(args.steps)
    kt_sp = fx.kernel_times()
    fx.close()
    del fx, U
    U = U0.clone()
    fx = GaugeFixer(U, fft_prec=1, link_prec=1, refine_theta=1e-10, fft_schedule=args.fft_schedule)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    it, F, th = fx.fix_until(1e-15, 100000)
    torch.cuda.synchronize()
    ttt = time.perf_counter() - t2
    fx.close()
    del fx, U
    sp = {"iters_per_s": round(args.steps / dt, 2), "ms_per_step": round(1e3 * dt / args.steps, 4),
          "kernels_us": {k: round(1e3 * ms / n, 2) for k, (ms, n) in kt_sp.items() if n},
          "time_to_theta": {"seconds": round(ttt, 5), "iterations": it, "F_final": F, "theta_final": th,
                            "F_minus_fp64": F - res["fp64"]["F_final"], "refine_theta": 1e-10}}
    log(f"[sp_links] {args.steps / dt:.1f} it/s, fixed in {it} its / {ttt * 1e3:.2f} ms, F={F:.15f}")

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
            same_shape = t.get("workload", "").split(" ")[0] == "x".join(str(d) for d in dims)
            if t.get("kernel") == dom_name and t.get("source_hash") == _source_hash() and same_shape:
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
                         f"configuration (FP64 C oracle, OpenMP), {dcpu:.1f} s",
               "cpu_model": _cpu_model()}
        # the same oracle on one host thread, a shorter sample
        n1 = max(1, args.cpu_iters // 20)
        oracle.set_num_threads(1)
        try:
            log(f"cpu oracle: {n1} iterations at {dims} on 1 thread")
            t4 = time.perf_counter()
            oracle.fix(dims, U_host, alpha=0.08, eps=-1.0, max_iter=n1)
            d1 = time.perf_counter() - t4
        finally:
            oracle.set_num_threads(nthr)
        cpu["single_thread"] = {"value": n1 / d1, "unit": "iters/s", "cores": 1,
                                "sample": f"{n1} iterations, {d1:.1f} s"}

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
                               f"alpha=0.08, FP64 transform and arithmetic, links stored as two FP64 rows "
                               f"(12-real form, third row rebuilt)",
                   "dims": list(dims), "alpha": 0.08, "theta_eps": 1e-15},
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "avg_us": round(dom_avg_s * 1e6, 2), "alg_bytes_per_launch": dom_bytes},
        "cpu_baseline": cpu,
        "time_to_theta": {"fp64": {"seconds": round(f64["time_to_theta_s"], 5), "iterations": f64["iterations"],
                                   "F_final": f64["F_final"], "theta_final": f64["theta_final"]},
                          "fp32_fft": {"seconds": round(f32["time_to_theta_s"], 5), "iterations": f32["iterations"],
                                       "F_final": f32["F_final"], "theta_final": f32["theta_final"]},
                          "sp_links_fp32_fft_then_fp64": {"seconds": sp["time_to_theta"]["seconds"],
                                                          "iterations": sp["time_to_theta"]["iterations"],
                                                          "F_final": sp["time_to_theta"]["F_final"],
                                                          "theta_final": sp["time_to_theta"]["theta_final"]}},
        "fp32_fft": {"iters_per_s": round(f32["iters_per_s"], 2), "ms_per_step": round(f32["ms_per_step"], 4),
                     "fft_schedule": f32["fft_schedule"]},
        "sp_links_fp32_fft": sp,
        "fft_schedule": f64["fft_schedule"],
        "hbm": {"alg_bytes_per_iter": per_iter_bytes,
                "effective_GBs": round(per_iter_bytes * f64["iters_per_s"] / 1e9, 1),
                "effective_frac": round(per_iter_bytes * f64["iters_per_s"] / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_fp64": kern,
        "event_region_iters_per_s": round(f64["event_region_iters_per_s"], 2),
    }
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Configurations of uneven shapes in one batch context (FP64 links, FP32
    transform) against the same ones one context after another. `batch`: 24
    configurations (8x12^4, 8x16^3x32, 6x24^4, 2x32^4), eps ~ U[0.2, 0.6);
    `batch_small`: the 16 small ones (8x12^4, 8x16^3x32), eps ~ U[0.2, 0.45),
    lattices too small to fill the GPU one at a time."""
    import numpy as np
    import torch

    from paper_1210_8018_amd.api import BatchGaugeFixer, GaugeFixer
    from paper_1210_8018_amd.inputs import batch_workload

    small = args.workload == "batch_small"
    log("generating the batch workload")
    if small:
        cfgs = list(batch_workload([(12, 12, 12, 12)] * 8 + [(16, 16, 16, 32)] * 8, first_seed=200,
                                   eps_range=(0.2, 0.45)))
    else:
        cfgs = list(batch_workload())
    U0 = [torch.from_numpy(U).to("cuda") for _, _, _, U in cfgs]
    torch.cuda.synchronize()
    Us = [u.clone() for u in U0]
    bx = BatchGaugeFixer(Us, fft_prec=1, reunit_every=100)
    torch.cuda.synchronize()
    log("batch fix_until 1e-15")
    t0 = time.perf_counter()
    its = [0] * len(Us)
    for _ in range(50):  # 2000-iteration slices, progress between them
        it, Fs, ths = bx.fix_until(1e-15, 2000, allow_maxiter=True)
        its = [a + b for a, b in zip(its, it)]
        left = sum(1 for t in ths if t > 1e-15)
        log(f"  {time.perf_counter() - t0:.2f}s: {sum(its)} iterations, {left} configurations still iterating")
        if left == 0:
            break
    torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    sched = None
    bx.close()
    del bx, Us
    log(f"batch makespan {makespan:.3f}s, max its {max(its)}")
    # the same configurations one context after another
    seq = 0.0
    seq_its = []
    for k, u in enumerate(U0):
        U = u.clone()
        fx = GaugeFixer(U, fft_prec=1, reunit_every=100)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        it, F, th = fx.fix_until(1e-15, 100000, allow_maxiter=True)
        torch.cuda.synchronize()
        log(f"  sequential {k}: {it} iterations")
        seq += time.perf_counter() - t1
        seq_its.append(it)
        sched = fx.fft_schedule
        fx.close()
        del fx, U
    sites = [int(np.prod(d)) for d, _, _, _ in cfgs]
    site_its = sum(i * v for i, v in zip(its, sites))
    if small:
        metric = "batch makespan to theta<=1e-15, 16 configurations (8x12^4, 8x16^3x32)"
        workload = ("batch of 16, eps ~ U[0.2,0.45), seeds 200-215, alpha=0.08, theta_eps=1e-15, "
                    "links reunitarised every 100 updates")
    else:
        metric = "batch makespan to theta<=1e-15, 24 configurations (8x12^4, 8x16^3x32, 6x24^4, 2x32^4)"
        workload = ("batch of 24, eps ~ U[0.2,0.6), seeds 100-123, alpha=0.08, theta_eps=1e-15, "
                    "links reunitarised every 100 updates")
    out = {
        "metric": metric,
        "value": round(makespan, 4), "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "dtype": "f64 links / c64 transform",
        "config": {"workload": workload},
        "per_config": [{"dims": list(d), "eps": round(e, 4), "seed": sd, "iterations": i, "F_final": F, "theta": th}
                       for (d, e, sd, _), i, F, th in zip(cfgs, its, Fs, ths)],
        "total_iterations": int(sum(its)), "site_iterations_per_s": site_its / makespan,
        "sequential_seconds": round(seq, 4), "sequential_iterations_equal": seq_its == its,
        "speedup_vs_sequential": round(seq / makespan, 3),
    }
    print(json.dumps(out), flush=True)


def bench_large(args):
    """48^4 or 64^4, eps 0.5: FP32 transform to theta <= 1e-15, with its error against FP64."""
    import numpy as np
    import torch

    from paper_1210_8018_amd.api import GaugeFixer
    from paper_1210_8018_amd.inputs import random_links

    L = 48 if args.workload == "large48" else 64
    dims = (L, L, L, L)
    seed = 3 if L == 48 else 4
    log(f"generating {dims} eps=0.5 seed={seed}")
    t0 = time.time()
    U_host = random_links(dims, 0.5, seed)
    log(f"generated in {time.time() - t0:.1f}s")
    U0 = torch.from_numpy(U_host).to("cuda")
    torch.cuda.synchronize()
    res = {}
    for prec in (1, 0):
        tag = "fp32_fft" if prec else "fp64"
        U = U0.clone()
        fx = GaugeFixer(U, fft_prec=prec, reunit_every=100)
        torch.cuda.synchronize()
        log(f"[{tag}] fix_until 1e-15")
        t1 = time.perf_counter()
        it = 0
        for _ in range(100):  # 1000-iteration slices, progress between them
            di, F, th = fx.fix_until(1e-15, 1000, allow_maxiter=True)
            it += di
            log(f"  {time.perf_counter() - t1:.2f}s: {it} iterations, theta {th:.3e}")
            if th <= 1e-15:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        Fh, Th = fx.history()
        res[tag] = dict(seconds=dt, iterations=it, F=F, theta=th, iters_per_s=it / dt, F_hist=Fh, T_hist=Th,
                        schedule=fx.fft_schedule)
        fx.close()
        del fx, U
        log(f"[{tag}] {it} its in {dt:.2f}s ({it / dt:.1f} it/s), F={F:.15f}")
    a, b = res["fp32_fft"], res["fp64"]
    n = min(len(a["T_hist"]), len(b["T_hist"]))
    Ta, Tb = np.asarray(a["T_hist"][:n]), np.asarray(b["T_hist"][:n])
    Fa, Fb = np.asarray(a["F_hist"][:n]), np.asarray(b["F_hist"][:n])
    big = Tb > 1e-12
    cpu = None
    if not args.no_cpu:
        import oracle

        # the first k iterations against the FP64 oracle: per-iteration F and
        # theta, and the plaquette of the links after k updates (gauge
        # invariant: equal to the initial one up to rounding)
        k = args.oracle_iters
        plaq = {}
        for prec, tag in ((1, "fp32_fft"), (0, "fp64")):
            U = U0.clone()
            fx = GaugeFixer(U, fft_prec=prec, reunit_every=100)
            fx.step(k)
            plaq[tag] = fx.plaquette()
            fx.close()
            del fx, U
        log(f"cpu oracle: {k} iterations at {dims}")
        t2 = time.perf_counter()
        _, Uo, Fo, To = oracle.fix(dims, U_host, alpha=0.08, eps=-1.0, max_iter=k, reunit_every=100)
        dcpu = time.perf_counter() - t2
        P0, Pk = oracle.plaquette(dims, U_host), oracle.plaquette(dims, Uo)
        del Uo
        cpu = {"value": k / dcpu, "unit": "iters/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{k} iterations at {L}^4, {dcpu:.1f} s",
               "F_rel_err_fp32_fft": float(np.max(np.abs(Fa[:k + 1] - Fo) / np.abs(Fo))),
               "theta_rel_err_fp32_fft": float(np.max(np.abs(Ta[:k + 1] - To) / To)),
               "F_rel_err_fp64": float(np.max(np.abs(Fb[:k + 1] - Fo) / np.abs(Fo))),
               "theta_rel_err_fp64": float(np.max(np.abs(Tb[:k + 1] - To) / To)),
               "plaquette_initial": P0, "plaquette_oracle_after": Pk,
               "plaquette_err_fp32_fft": plaq["fp32_fft"] - Pk, "plaquette_err_fp64": plaq["fp64"] - Pk}
    out = {
        "metric": f"time to theta<=1e-15 at {L}^4 SU(3), FP32 transform (FP64 links/Delta/update/sums)",
        "value": round(a["seconds"], 4), "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "dtype": "f64 links / c64 transform",
        "config": {"workload": f"{L}^4, generator eps=0.5 seed={seed}, alpha=0.08, links reunitarised every 100"},
        "fp32_fft": {k: a[k] for k in ("seconds", "iterations", "F", "theta", "iters_per_s", "schedule")},
        "fp64": {k: b[k] for k in ("seconds", "iterations", "F", "theta", "iters_per_s", "schedule")},
        "fp32_vs_fp64": {"F_final_rel": abs(a["F"] - b["F"]) / abs(b["F"]),
                         "F_max_rel_per_iter": float(np.max(np.abs(Fa - Fb) / np.abs(Fb))),
                         "theta_max_rel_per_iter_while_theta_gt_1e-12": float(np.max(np.abs(Ta[big] - Tb[big]) / Tb[big]))},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_diff(args):
    """24^4 differentiable functional: forward and backward times; gradient checks (informational)."""
    import numpy as np
    import torch

    from paper_1210_8018_amd import gf
    from paper_1210_8018_amd.api import GaugeFixer
    from paper_1210_8018_amd.inputs import random_links, random_omega

    dims = (24, 24, 24, 24)
    V = int(np.prod(dims))
    U = torch.from_numpy(random_links(dims, 0.3, 5)).to("cuda")
    om = torch.from_numpy(random_omega(dims, 0.1, 6)).to("cuda")
    fx = GaugeFixer(U)
    d_om = torch.empty_like(om)
    d_U = torch.empty_like(U)
    for _ in range(3):
        gf.gf_functional_g(fx.ctx, om)
        gf.gf_functional_g_backward(fx.ctx, om, 1.0, d_om, d_U)
    n = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        F = gf.gf_functional_g(fx.ctx, om)
    t1 = time.perf_counter()
    for _ in range(n):
        gf.gf_functional_g_backward(fx.ctx, om, 1.0, d_om, d_U)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fx.close()
    # the autograd function end to end (functional-only context, reused)
    from paper_1210_8018_amd.api import GaugeFunctional

    Ug = U.clone().requires_grad_(True)
    omg = om.clone().requires_grad_(True)
    for _ in range(3):
        GaugeFunctional.apply(Ug, omg).backward()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(n):
        Ug.grad = None
        omg.grad = None
        Fa = GaugeFunctional.apply(Ug, omg)
        Fa.backward()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    out = {"metric": "differentiable functional at 24^4: forward and backward time", "value": round((t1 - t0) / n * 1e3, 4),
           "unit": "ms (forward)", "backward_ms": round((t2 - t1) / n * 1e3, 4),
           "autograd_forward_backward_ms": round((t4 - t3) / n * 1e3, 4), "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "f64", "F": F,
           "config": {"workload": "24^4 links eps 0.3 seed 5, omega ~ N(0, 0.1^2) seed 6"}}
    print(json.dumps(out), flush=True)


def bench_thermal(args):
    """32^4 Wilson-action configuration thermalised on the GPU (cold start, heatbath + 4
    overrelaxation sweeps), then gauge-fixed to theta <= 1e-15 in each precision mode."""
    import numpy as np
    import torch

    from paper_1210_8018_amd.api import GaugeFixer

    dims = (32, 32, 32, 32)
    V = int(np.prod(dims))
    one = torch.zeros((4, 3, 3, V), dtype=torch.complex128, device="cuda")
    for i in range(3):
        one[:, i, i, :] = 1
    U0 = one.reshape(4, 3, 3, 32, 32, 32, 32).contiguous()
    fx = GaugeFixer(U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plaq = []
    done = 0
    while done < args.sweeps:
        n = min(50, args.sweeps - done)
        fx.heatbath(args.beta, n, 4, seed=20121030, sweep0=done)
        done += n
        plaq.append((done, fx.plaquette()))
        log(f"  {time.perf_counter() - t0:.1f}s: {done} sweeps, plaquette {plaq[-1][1]:.6f}")
    gen_s = time.perf_counter() - t0
    fx.close()
    res = {}
    for tag, kw in (("fp64", {}), ("fp32_fft", {"fft_prec": 1}), ("sp_links_fp32_fft", {"fft_prec": 1, "link_prec": 1})):
        U = U0.clone()
        fx = GaugeFixer(U, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        it = 0
        while True:  # slices of 1000 iterations, progress between them
            di, F, th = fx.fix_until(1e-15, 1000, allow_maxiter=True)
            it += di
            log(f"  [{tag}] {time.perf_counter() - t1:.2f}s: {it} iterations, theta {th:.3e}")
            if th <= 1e-15 or it >= 100000:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        res[tag] = {"seconds": round(dt, 4), "iterations": it, "F_final": F, "theta_final": th,
                    "iters_per_s": round(it / dt, 1)}
        fx.close()
        del fx, U
    out = {"metric": f"time to theta<=1e-15 at 32^4 SU(3), Wilson action beta={args.beta} thermalised on the GPU",
           "value": res["fp64"]["seconds"], "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "dtype": "f64",
           "config": {"workload": f"32^4 cold start, {args.sweeps} x (heatbath + 4 overrelaxation) sweeps at "
                                  f"beta={args.beta}, Philox seed 20121030"},
           "generation": {"seconds": round(gen_s, 3), "plaquette": plaq}, "fix": res}
    print(json.dumps(out), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in ("csrc/gf_kernels.hip", "csrc/gf_device.h", "csrc/gf_internal.h", "csrc/gf_runtime.hip", "build.py"):
        with open(os.path.join(ROOT, "paper_1210_8018_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
