#!/usr/bin/env python3
"""Benchmark: whole-slice solves per second on the 512^2 slice.

With --workload uneven64 it times instead the batch of 64 uneven slices
(image 256/384/512 at 0.8 mm, 360/720/984 views, 512-888 bins): slices of
one image size run as one batch (one launch per kernel and iteration for
all of them), against the same 64 slices solved one at a time.

With --workload image512 it times the image-domain form (Algorithm 1 on the
attenuation image pair of the same 512^2 phantom, 50 iterations).

With --workload serve it replays Poisson arrival streams of single-slice
requests (image 256-768, 360-1152 views, 20-80 iterations) through the
continuous-batching server and reports latency percentiles and slices/s per
arrival rate.

Workload: 512x512 image at 0.8 mm, 720 views over 360 deg, 736 detector bins,
SID 1000 mm, SDD 1500 mm, dual-energy sinograms of an elliptical water body
with 40 bone / soft-tissue / lung inserts, Poisson noise 5e4 / 1e5, 50 outer
iterations of the sinogram-form Algorithm 1.  A step is one whole solve of one
slice (FBP start, 50 iterations, output maps) with the sinograms already in
HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu-baseline]
                    [--storage fp32|bf16|bf16_state]
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

N_ITER = 50
PEAK_FP32_TFLOPS = 157.3      # MI355X dense FP32 vector (published)
PEAK_HBM_GBS = 8000.0


def count_nonzeros(g) -> int:
    """Nonzeros of the system matrix: ray-pixel intersections, counted as
    (grid lines crossed inside the image) + 1 per ray that meets the image."""
    from paper_2308_01290_amd import phantoms as P
    src, dst = P.ray_endpoints(g)
    S = np.broadcast_to(src[:, None, :], dst.shape).reshape(-1, 2)
    d = dst.reshape(-1, 2) - S
    half = np.array([g.n_x, g.n_y]) * g.pixel_mm / 2
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = (-half[None, :] - S) / d
        tb = (half[None, :] - S) / d
    t0 = np.max(np.minimum(ta, tb), axis=1)
    t1 = np.min(np.maximum(ta, tb), axis=1)
    hit = t1 > t0
    total = 0
    for a, n in ((0, g.n_x), (1, g.n_y)):
        c0 = (S[:, a] + t0 * d[:, a] + half[a]) / g.pixel_mm
        c1 = (S[:, a] + t1 * d[:, a] + half[a]) / g.pixel_mm
        lo, hi = np.minimum(c0, c1), np.maximum(c0, c1)
        cross = np.clip(np.ceil(hi) - 1, 0, n) - np.clip(np.floor(lo) + 1, 0, n) + 1
        total += int(np.sum(np.where(hit, np.maximum(cross, 0), 0)))
    return total + int(hit.sum())


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel's source changed since the counters."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "backproject_traffic_512.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or "kernel_source" not in kv:
        return None
    src = os.path.join(ROOT, kv["kernel_source"])
    if not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("kernel_source_sha256"):
        return None
    return float(kv["traffic_bytes_per_launch"])


def timeline_summary(tl):
    """Medians over the timed outer iterations (dect_solver_timeline rows, us
    after the previous update): when the f-step reaches the gradient, its
    forward projection and update end (the period), when the t' PCG finishes
    its set-up and its solve, and how long before the next gradient the PCG's
    result is ready (its slack; the f-step chain sets the period while it is
    positive)."""
    import numpy as np
    if len(tl) < 3:
        return None
    med = lambda x: float(np.median(x))  # noqa: E731
    slack = tl[1:, 0] - (tl[:-1, 4] - tl[:-1, 2])
    return {"iterations": int(len(tl)), "period": med(tl[:, 2]), "gradient_reached": med(tl[:, 0]),
            "projection_done": med(tl[:, 1]), "pcg_setup_done": med(tl[:, 3]), "pcg_done": med(tl[:, 4]),
            "pcg_slack_before_next_gradient": med(slack)}


def small_workload_times(threads):
    """The 128^2 workload (180 views, 256 bins, 10 iterations): the whole
    oracle solve on all host cores, and the same solve on the GPU (a solver
    kept across solves, as in the timed 512^2 steps; median of five after one
    untimed)."""
    import torch
    from oracle import solve as S
    from oracle.physics import Physics
    from paper_2308_01290_amd import dect
    from paper_2308_01290_amd import phantoms as P
    phys = Physics()
    g, _, pL, pH = P.workload_small(phys.mu_pair)
    k = 10
    t0 = time.perf_counter()
    S.solve(pL.astype(np.float64), pH.astype(np.float64), g, phys, S.Params(n_iter=k), nthreads=threads)
    t_cpu = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    lo = torch.as_tensor(pL.astype(np.float32)[None], device=dev)
    hi = torch.as_tensor(pH.astype(np.float32)[None], device=dev)
    sol = dect.Solver(g, dect.default_params(n_iter=k))
    ts = []
    for r in range(6):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        sol.init(lo, hi)
        sol.iterate(k)
        sol.finish()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - s0)
    sol.close()
    t_gpu = float(np.median(ts[1:]))
    return {"workload": "128x128 at 1 mm, 180 views, 256 bins, 10 outer iterations",
            "oracle_s_per_slice": t_cpu, "oracle_cores": threads, "gpu_ms_per_slice": 1e3 * t_gpu}


def cpu_baseline(g, pL, pH, iters: int):
    """The FP64 oracle (as it stands) on the host cores: FBP start plus `iters`
    outer iterations, extrapolated to the 50-iteration solve.  A 1-core figure
    comes from one forward and one back-projection of one channel (the
    oracle's dominant work) timed on 1 core and on all cores."""
    from oracle import operators as O
    from oracle import solve as S
    from oracle.physics import Physics
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    phys = Physics()
    params = S.Params(n_iter=N_ITER).resolved(phys, g)
    a = pL.astype(np.float64)
    b = pH.astype(np.float64)
    t0 = time.perf_counter()
    st = S.init_state(a, b, g, phys, params, nthreads=threads)
    t1 = time.perf_counter()
    for _ in range(iters):
        st = S.iterate(st, a, b, g, phys, params, nthreads=threads)
    t2 = time.perf_counter()
    per_slice = (t1 - t0) + N_ITER * (t2 - t1) / iters

    def fp_bp(nthreads):
        s0 = time.perf_counter()
        O.project(g, st.f2, nthreads)
        O.backproject(g, a, nthreads)
        return time.perf_counter() - s0

    t_all = fp_bp(threads)
    t_one = fp_bp(1)
    per_slice_1 = per_slice * t_one / t_all
    return {"value": 1.0 / per_slice, "unit": "slices/s", "cores": threads, "kind": "oracle",
            "small_workload": small_workload_times(threads),
            "sample": f"FBP start + {iters} of {N_ITER} outer iterations on the same 512^2 slice "
                      f"({t2 - t0:.1f} s), extrapolated to {N_ITER} iterations "
                      f"({per_slice:.1f} s per slice)",
            "one_core": {"value": 1.0 / per_slice_1, "unit": "slices/s", "cores": 1,
                         "sample": f"one forward and one back-projection of one channel: "
                                   f"{t_one:.2f} s on 1 core, {t_all:.2f} s on {threads}; the "
                                   f"all-core solve time scaled by that ratio "
                                   f"({per_slice_1:.0f} s per slice)"}}


def _uneven_slice(i):
    from paper_2308_01290_amd import dect
    from paper_2308_01290_amd import phantoms as P
    params = dect.default_params()
    g, ph, pL, pH = P.slice_uneven(3000 + i, lambda Z, R: dect.attenuation(params, Z, R))
    return g, pL.astype(np.float32), pH.astype(np.float32)


def tune(args, sol, lo, hi, default_mode):
    """Autotune `sol` on its inputs when asked, or apply --set; returns
    (schedule, seconds)."""
    if args.set:
        sol.set_schedule(**dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in args.set))
    if (args.schedule or default_mode) != "autotune":
        return sol.schedule(), 0.0
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chosen, _ = sol.autotune(lo, hi, iters=4, reps=3)
    torch.cuda.synchronize()
    return chosen, time.perf_counter() - t0


def bench_uneven(args):
    """64 uneven slices of mixed image sizes, 50 iterations each: one handle
    for the whole batch (one uneven-batch solver per image size, iterated
    together) against one slice at a time; a step solves all 64 slices."""
    import multiprocessing as mp
    import torch
    from paper_2308_01290_amd import dect
    n_slices = 64
    workers = min(16, os.cpu_count() or 1)
    with mp.get_context("spawn").Pool(workers) as pool:
        data = pool.map(_uneven_slice, range(n_slices))
    params = dect.default_params(n_iter=N_ITER)
    dev = torch.device("cuda:0")
    geoms = [d[0] for d in data]
    groups = {}
    for i, g in enumerate(geoms):
        groups.setdefault(g.n_x, []).append(i)
    lo = dect.concat_sinograms([torch.as_tensor(d[1], device=dev) for d in data])
    hi = dect.concat_sinograms([torch.as_tensor(d[2], device=dev) for d in data])
    batch = dect.UnevenSolver(geoms, params)
    single = []
    for g, pL, pH in data:
        single.append((dect.Solver(g, params), torch.as_tensor(pL[None], device=dev),
                       torch.as_tensor(pH[None], device=dev)))
    t_tune = 0.0
    if (args.schedule or "autotune") == "autotune":
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.autotune(lo, hi, iters=4, reps=3)
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
    schedules = [batch.schedule(q) for q in range(batch.groups())]

    def run_batch():
        batch.init(lo, hi)
        batch.iterate(N_ITER)
        return batch.finish()

    def run_single():
        out = []
        for sol, a, b in single:
            sol.init(a, b)
            sol.iterate(N_ITER)
            out.append(sol.finish())
        return out

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res

    t_b, (Zb, Rb) = timed(run_batch, args.steps, args.warmup)
    t_s, res_s = timed(run_single, max(1, args.steps // 2), 1)
    # the batch must give each slice's own result
    same = True
    for i, (z, r) in enumerate(zip(dect.split_images(Zb, geoms), dect.split_images(Rb, geoms))):
        same = same and bool(torch.equal(z, res_s[i][0][0])) and bool(torch.equal(r, res_s[i][1][0]))
    out = {
        "metric": "uneven batch slices/s (64 slices, 256-512^2, 360-984 views, 50 iters)",
        "value": n_slices / t_b, "unit": "slices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_b, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 uneven slices: n in {256, 384, 512} at 0.8 mm, views in "
                               "{360, 720, 984}, bins 512-888, scaled body phantom with 40 inserts, "
                               "Poisson 5e4/1e5, 50 outer iterations",
                   "groups": {str(n): len(idx) for n, idx in sorted(groups.items())}},
        "one_slice_at_a_time": {"value": n_slices / t_s, "unit": "slices/s", "ms_per_step": 1e3 * t_s},
        "speedup": t_s / t_b,
        "results_identical_to_one_at_a_time": same,
        "schedule": {"mode": args.schedule or "autotune", "per_group": schedules,
                     "autotune_s": t_tune},
    }
    print(json.dumps(out), flush=True)


def _serve_slice(args):
    """One pool slice for the serving stream (image n, views and bins drawn
    from the seed)."""
    n, seed = args
    from paper_2308_01290_amd import dect
    from paper_2308_01290_amd import phantoms as P
    params = dect.default_params()
    g, ph, pL, pH = P.slice_served(n, seed, lambda Z, R: dect.attenuation(params, Z, R))
    return g, pL.astype(np.float32), pH.astype(np.float32)


def serve_streams(rates, n_requests, seed=20230801, budget_bytes=200e9):
    """Poisson streams of single-slice requests (image 256-768, 360-1152 views,
    20-80 iterations) through the continuous-batching server, one stream per
    rate; per rate: latency p50/p99 (arrival to maps ready) and slices/s.  Two
    requests per rate are re-solved alone and compared bit for bit."""
    import multiprocessing as mp
    import torch
    from paper_2308_01290_amd import dect
    from paper_2308_01290_amd import phantoms as P
    from paper_2308_01290_amd.serve import EngineSpec, Request, Server
    per_size = 4
    jobs = [(n, 5000 + 10 * n + i) for n in P.SERVE_SIZES for i in range(per_size)]
    with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
        data = pool.map(_serve_slice, jobs)
    dev = torch.device("cuda:0")
    pool_dev = [(g, torch.as_tensor(pL, device=dev), torch.as_tensor(pH, device=dev))
                for g, pL, pH in data]
    params = dect.default_params()
    specs = [EngineSpec(n, 0.8, 16, 1152, 1024) for n in P.SERVE_SIZES]
    rng = np.random.Generator(np.random.PCG64(seed))
    results = []
    checked = 0
    identical = True
    for rate in rates:
        server = Server(specs, params, hbm_budget_bytes=budget_bytes)
        t = 0.0
        reqs = []
        for i in range(n_requests):
            t += rng.exponential(1.0 / rate)
            g, lo, hi = pool_dev[int(rng.integers(len(pool_dev)))]
            reqs.append(Request(g, lo, hi, int(rng.integers(20, 81)), arrival=t, tag=i))
        t0 = time.perf_counter()
        server.run(reqs)
        wall = time.perf_counter() - t0
        lat = np.array([r.latency for r in reqs])
        results.append({"rate_req_s": rate, "requests": len(reqs),
                        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                        "mean_ms": 1e3 * float(lat.mean()),
                        "slices_per_s": len(reqs) / wall,
                        "hbm_peak_gb": server.hbm_peak / 1e9,
                        "engines_created": server.engines_created})
        # a served request equals the same slice solved alone
        for r in reqs[:2]:
            Z1, R1 = dect.solve(r.sino_lo[None], r.sino_hi[None], r.geom, dect.default_params(n_iter=r.n_iter))
            identical = identical and bool(torch.equal(Z1[0], r.Z)) and bool(torch.equal(R1[0], r.rho))
            checked += 1
        server.close()
        del server
    return results, {"checked": checked, "identical": identical}


SERVE_WORKLOAD = ("Poisson arrivals of single-slice requests: image 256/384/512/768 at 0.8 mm, "
                  "views 360-1152, bins 512-1024, iterations 20-80; engines of 16 slots per image "
                  "size created on demand under a 200 GB HBM budget")


def bench_serve(args):
    """Poisson streams of single-slice requests through the continuous-batching
    server; per rate: latency p50/p99 (arrival to maps ready) and slices/s."""
    results, same = serve_streams([float(r) for r in args.rates.split(",")], args.requests)
    mid = results[len(results) // 2]
    out = {
        "metric": "served p99 latency (single-slice requests, 256-768^2, 360-1152 views, 20-80 iters)",
        "value": mid["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": len(results), "warmup": 0,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": SERVE_WORKLOAD, "value_at_rate_req_s": mid["rate_req_s"]},
        "per_rate": results,
        "served_equals_alone": same,
    }
    print(json.dumps(out), flush=True)


def bench_image(args):
    """The image-domain form on the 512^2 phantom's attenuation image pair: a
    step is one whole solve (closed-form start, 50 iterations, output maps)
    with the images already in HBM."""
    import torch
    from paper_2308_01290_amd import dect
    from paper_2308_01290_amd import phantoms as P
    params = dect.default_params(n_iter=N_ITER)
    g, ph, L, H = P.workload_image512(lambda Z, R: dect.attenuation(params, Z, R))
    dev = torch.device("cuda:0")
    lo = torch.as_tensor(L[None].astype(np.float32), device=dev)
    hi = torch.as_tensor(H[None].astype(np.float32), device=dev)
    sol = dect.ImageSolver(g.n_x, g.n_y, params)
    schedule, t_tune = tune(args, sol, lo, hi, "default")
    Z = torch.empty((1, g.n_y, g.n_x), device=dev)
    R = torch.empty_like(Z)

    def step():
        sol.init(lo, hi)
        sol.iterate(N_ITER)
        dect._check(dect.lib().dect_solver_finish(sol._h, dect._ptr(Z), dect._ptr(R)), "finish")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sol.enable_timing(True)
    sol.timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fs_ms, fs_n, _, _ = sol.timing()
    sol.enable_timing(False)
    elapsed = t1 - t0
    value = args.steps / elapsed
    npix = g.n_x * g.n_y
    fs_avg_s = fs_ms / max(fs_n, 1) / 1e3
    # algorithmic HBM bytes of one f-step (the joint 2x2 solve of both bases):
    # per pixel read f (8 B), mu_L, mu_H, rho_e, t' (16 B) and write f (8 B)
    fs_bytes = 32 * npix
    achieved = fs_bytes / fs_avg_s / 1e9
    out = {
        "metric": "512^2 image-domain solves/s (50 iters)",
        "value": value,
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x512 attenuation image pair at 0.8 mm (water body + 40 inserts, "
                               "15/10 HU white noise), image-domain Algorithm 1, 50 outer iterations",
                   "image": [g.n_y, g.n_x], "iterations": N_ITER, "slices_per_solve": 1},
        "f_step_ms": 1e3 * fs_avg_s,
        "roofline": {"kernel": "f-step (k_fft_rows_fwd + k_fft_cols + k_fft_rows_inv, both bases)",
                     "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None},
        "schedule": {"mode": args.schedule or "default", "chosen": schedule, "autotune_s": t_tune},
    }
    if not args.no_cpu_baseline:
        from oracle import image as I
        from oracle.physics import Physics
        from oracle.solve import Params
        phys = Physics()
        p = I.resolved(Params(n_iter=N_ITER), phys)
        a, b = L.astype(np.float32).astype(np.float64), H.astype(np.float32).astype(np.float64)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        c0 = time.perf_counter()
        st = I.init_from_mu(a, b, phys, p)
        c1 = time.perf_counter()
        for _ in range(args.cpu_iters):
            st = I.iterate(st, a, b, phys, p)
        c2 = time.perf_counter()
        per = (c1 - c0) + N_ITER * (c2 - c1) / args.cpu_iters
        out["cpu_baseline"] = {"value": 1.0 / per, "unit": "slices/s", "cores": threads, "kind": "oracle",
                               "sample": f"closed-form start + {args.cpu_iters} of {N_ITER} outer "
                                         f"iterations on the same image pair ({c2 - c0:.1f} s), "
                                         f"extrapolated ({per:.1f} s per slice)"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--workload", choices=["slice512", "uneven64", "serve", "image512"],
                    default="slice512")
    ap.add_argument("--storage", choices=["fp32", "bf16", "bf16_state"], default="fp32",
                    help="slice512: storage of the projector operands (bf16) and also of the "
                         "state images (bf16_state)")
    ap.add_argument("--schedule", choices=["default", "autotune"], default=None,
                    help="launch schedule of the timed solvers: the library default, or the one "
                         "the library's autotuner picks on the workload before the warmup "
                         "(default: autotune for uneven64, default otherwise)")
    ap.add_argument("--set", nargs="*", default=[], metavar="KEY=VALUE",
                    help="slice512 / image512: schedule fields (dect_schedule) set before timing")
    ap.add_argument("--rates", default="20,50,100,200", help="serve: arrival rates (req/s)")
    ap.add_argument("--requests", type=int, default=96, help="serve: requests per rate")
    ap.add_argument("--served-requests", type=int, default=48,
                    help="slice512: requests of the served leg at 20 req/s (0: none)")
    ap.add_argument("--batch", type=int, default=1,
                    help="slice512: solve this many copies of the slice per launch (one solver, "
                         "batch slices; value counts every slice)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first copy a device buffer of this many MiB once: the reference "
                         "kernel of known traffic for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "slices are independent solves, so more GPUs would each take whole slices",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2308_01290_amd import dect
    from paper_2308_01290_amd import phantoms as P
    if args.workload == "uneven64":
        bench_uneven(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "image512":
        bench_image(args)
        return

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    storage = {"fp32": dect.DECT_STORAGE_FP32, "bf16": dect.DECT_STORAGE_BF16,
               "bf16_state": dect.DECT_STORAGE_BF16_STATE}[args.storage]
    params = dect.default_params(n_iter=N_ITER, storage=storage)
    g, ph, pL, pH = P.workload_slice512(lambda Z, R: dect.attenuation(params, Z, R))
    pL = pL.astype(np.float32)
    pH = pH.astype(np.float32)
    dev = torch.device("cuda:0")
    nb = args.batch
    if nb < 1:
        raise SystemExit("--batch must be at least 1")
    lo = torch.as_tensor(np.repeat(pL[None], nb, 0), device=dev)
    hi = torch.as_tensor(np.repeat(pH[None], nb, 0), device=dev)
    sol = dect.Solver(g, params, batch=nb)
    schedule, t_tune = tune(args, sol, lo, hi, "default")
    Z = torch.empty((nb, g.n_y, g.n_x), device=dev)
    R = torch.empty_like(Z)

    def step():
        sol.init(lo, hi)
        sol.iterate(N_ITER)
        dect._check(dect.lib().dect_solver_finish(sol._h, dect._ptr(Z), dect._ptr(R)), "finish")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed solves time their back-projections (the roofline's kernel)
    sol.enable_timing(True, bp_only=True)
    sol.timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bp_ms, bp_n, _, _ = sol.timing()
    # the forward projections' in-solve time and the iteration timeline from
    # three more solves, outside the timed region (their events add host work
    # to every iteration)
    sol.enable_timing(True, timeline=True)
    for _ in range(3):
        step()
    _, _, fp_ms, fp_n = sol.timing()
    tl = sol.timeline()
    sol.enable_timing(False)

    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = nb * args.steps / elapsed
    nnz = count_nonzeros(g)
    # every copy of the slice must come out bit-identical to the first
    batch_identical = bool(all(torch.equal(Z[i], Z[0]) and torch.equal(R[i], R[0])
                               for i in range(1, nb)))
    bp_avg_s = bp_ms / max(bp_n, 1) / 1e3
    fp_avg_s = fp_ms / max(fp_n, 1) / 1e3
    # the same back-projection of both channels alone on the GPU (the stand-alone
    # operator: pairing the two sinograms, then the kernel), for comparison with
    # the in-solve duration, where it shares the GPU with the concurrent PCG
    sino2 = torch.stack([lo[0], hi[0]])
    for _ in range(3):
        dect.backproject(g, sino2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dect.backproject(g, sino2)
    e1.record()
    torch.cuda.synchronize()
    bp_alone_s = e0.elapsed_time(e1) / 10 / 1e3
    # the forward projection of the image pair alone (plain mode: the same
    # traversal and reads as the solver's line-search projection)
    img2 = torch.stack([Z[0], R[0]])
    for _ in range(3):
        dect.project(g, img2)
    e0.record()
    for _ in range(10):
        dect.project(g, img2)
    e1.record()
    torch.cuda.synchronize()
    fp_alone_s = e0.elapsed_time(e1) / 10 / 1e3
    # algorithmic work of one back-projection launch: both channels of the
    # sparse transpose product, one multiply-add per nonzero and channel, for
    # each slice of the batch
    bp_flops = 2 * 2 * nnz * nb
    achieved = bp_flops / bp_avg_s / 1e12
    nray = g.n_views * g.n_det
    npix = g.n_x * g.n_y
    bp_bytes = nray * 8 + npix * 8
    fp_bytes = npix * 8 + nray * 8
    out = {
        "metric": "512^2 slices/s (720 views, 50 iters)",
        "value": value,
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x512 slice at 0.8 mm, 720 views, 736 bins, SID 1000 / SDD 1500 mm, "
                               "water body + 40 inserts, Poisson 5e4/1e5, 50 outer iterations"
                               + (f", {nb} copies per launch" if nb > 1 else ""),
                   "image": [g.n_y, g.n_x], "views": g.n_views, "bins": g.n_det,
                   "iterations": N_ITER, "slices_per_solve": nb, "storage": args.storage},
        "rays_per_s": 4.0 * nray * N_ITER * value,
        "projector": {
            "system_matrix_nonzeros": nnz,
            # in-solve durations per launch (a launch covers the whole batch);
            # the alone figures are for one slice
            "backproject_ms": 1e3 * bp_avg_s,
            "backproject_alone_ms": 1e3 * bp_alone_s,
            "backproject_alone_tflops": 2 * 2 * nnz / bp_alone_s / 1e12,
            "project_ms": 1e3 * fp_avg_s,
            "project_alone_ms": 1e3 * fp_alone_s,
            "backproject_visits_per_s": 2 * nnz * nb / bp_avg_s,
            "project_visits_per_s": 2 * nnz * nb / fp_avg_s,
            # effective touch bandwidth: every (pixel, ray) visit of both images
            # counted as one 4-byte access; not HBM traffic (the images and
            # sinograms are reread from L2 and the Infinity Cache)
            "backproject_effective_touch_gbs": 2 * nnz * nb * 4 / bp_avg_s / 1e9,
            "project_effective_touch_gbs": 2 * nnz * nb * 4 / fp_avg_s / 1e9,
            "backproject_algorithmic_hbm_gbs": bp_bytes * nb / bp_avg_s / 1e9,
            "project_algorithmic_hbm_gbs": fp_bytes * nb / fp_avg_s / 1e9,
        },
        "roofline": {"kernel": "k_backproject_sym8", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic("k_backproject_sym8") if storage == 0 and nb == 1 else None},
        "schedule": {"mode": args.schedule or "default", "chosen": schedule, "autotune_s": t_tune},
        "iteration_timeline_us": timeline_summary(tl),
    }
    if nb > 1:
        out["batch_slices_identical"] = batch_identical
    if args.served_requests > 0:
        # the metric's served part: a short Poisson stream at 20 req/s
        results, same = serve_streams([20.0], args.served_requests)
        out["served"] = dict(results[0], workload=SERVE_WORKLOAD, served_equals_alone=same)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, pL, pH, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
