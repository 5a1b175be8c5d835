"""Benchmark of the short-range TreePM tree force on one MI355X.

One step = the whole hot path on one box already resident in HBM: build (keys, radix sort,
gather, octree, moments, groups), walk (interaction lists) and the FP32 force.  The workload
is the 256^3 clustered box (2000 NFW halos plus a uniform half, mesh 256^3, r_cut = 3/256,
eps = 1/(20*256), theta = 0.5).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload nfw256] [--n-crit C]
                  [--no-cpu-baseline] [--no-fp64]
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles/s + interactions/s at θ=0.5, FP32 vs FP64 path; ensemble p50/p99"
K_PP = 38  # flops per pair interaction (FMA = 2, add/mul/rsqrt/sqrt = 1, selects = 0)
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes of one particle-mesh call: per mesh point, clearing and filling the
# fixed-point mass mesh (8 + 8), five FFT passes (16 + 16 + 16 + 16 + 12), the differences
# (4 read + 16 written) and one read of the force mesh (16); per particle, the key-ordered
# record read by the max-mass pass, the assignment and the interpolation (3 x 32), its index
# (4) and three FP32 outputs (12).
PM_BYTES_PER_POINT = 8 + 8 + 16 + 16 + 16 + 16 + 12 + 4 + 16 + 16
PM_BYTES_PER_PARTICLE = 3 * 32 + 4 + 12
FP64_VECTOR_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_f32_traffic.json")
FORCE_SRC = os.path.join(ROOT, "paper_0910_0121_amd", "csrc", "k_force.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="nfw256")
    ap.add_argument("--theta", type=float, default=None, help="override the workload's theta")
    ap.add_argument("--n-crit", type=int, default=0,
                    help="group size limit; 0 = autotune over --n-crit-candidates")
    ap.add_argument("--n-crit-candidates", default="128,192,256",
                    help="the n_crit values the autotuner tries (each is parity-tested at full "
                         "size on the 256^3 box)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="oracle sample: every k-th group (0 = choose for ~15 s of work)")
    ap.add_argument("--no-theta-r", action="store_true",
                    help="skip the distance-dependent opening angle leg")
    ap.add_argument("--theta0", type=float, default=0.3,
                    help="theta_0 of the distance-dependent opening angle leg")
    ap.add_argument("--theta-max", type=float, default=0.5,
                    help="cap of the distance-dependent opening angle leg")
    ap.add_argument("--no-quadrupole", action="store_true",
                    help="skip the quadrupole-cells leg")
    ap.add_argument("--no-time-step", action="store_true",
                    help="skip the full TreePM time-step leg")
    ap.add_argument("--no-pm", action="store_true",
                    help="skip the particle-mesh long-range leg")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the force-accuracy leg on the 128^3 box")
    ap.add_argument("--no-scale", action="store_true",
                    help="skip the 512^3 clustered box at theta 0.5 and 0.4")
    ap.add_argument("--scale-n-crit", type=int, default=192)
    ap.add_argument("--serving-boxes", type=int, default=64)
    ap.add_argument("--serving-requests-per-box", type=int, default=10)
    ap.add_argument("--serving-inflight", type=int, default=8)
    ap.add_argument("--serving-batching", action="store_true",
                    help="serve with shared walk and force launches across boxes")
    ap.add_argument("--serving-budget-frac", type=float, default=0.25)
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def measured_traffic(n_crit, workload):
    """HBM bytes per force call from the committed rocprofv3 counter runs (one per n_crit
    measured), if one was taken on the current force-kernel source, the same workload and the
    same n_crit; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        with open(FORCE_SRC, "rb") as f:
            sha = hashlib.sha1(f.read()).hexdigest()
        for run in [t] + t.get("other_runs", []):
            if (run.get("source_sha1") == sha and run.get("n_crit") == n_crit
                    and run.get("workload", "").startswith(workload)):
                return run
        return None
    except (OSError, ValueError):
        return None


def run_steps(tp, torch, ctx, dev, acc, k):
    times, st = [], None
    for _ in range(k):
        tp.treepm_build(ctx, *dev)
        tp.treepm_walk(ctx)
        tp.treepm_force_short(ctx, *acc)
        st = tp.treepm_get_stats(ctx)
        times.append(list(st.t_ms))
    return times, st


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, arrays, n_crit, stride_arg):
    """The oracle's tree build (one thread) and its walk + FP64 list force on a stratified
    sample of groups (every k-th group in key order), once on all the host's threads (up to
    16) and once on one thread, each sample sized for about 15 s of work; the full-box time is
    extrapolated from the sampled groups' share."""
    import oracle
    x, y, z, m = arrays
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    T = oracle.Tree(x, y, z, m, spec.L, spec.r_cut, spec.eps, spec.theta, spec.n_leaf, n_crit)
    t_build = time.perf_counter() - t0
    G = T.n_groups

    def sized(nthreads, budget_s):
        # pilot on a sparse sample, then a stride for about budget_s of work
        pilot = max(1, G // (nthreads * 16))
        t1 = time.perf_counter()
        T.walk_force_sample(pilot, 0, nthreads)
        per_group = (time.perf_counter() - t1) / max(1, len(range(0, G, pilot)))
        return max(1, G // max(1, int(budget_s / max(per_group, 1e-9))))

    out = {}
    for label, nth in (("all", threads), ("one", 1)):
        stride = stride_arg if (stride_arg > 0 and label == "all") else sized(nth, 15.0)
        t2 = time.perf_counter()
        _, _, _, inter, parts = T.walk_force_sample(stride, 0, nth)
        t_sample = time.perf_counter() - t2
        n_sampled = len(range(0, G, stride))
        out[label] = (stride, n_sampled, parts, inter, t_sample,
                      t_build + t_sample * (G / n_sampled))
    T.close()
    stride, n_s, parts, inter, t_s, t_full = out["all"]
    stride1, n_s1, parts1, inter1, t_s1, t_full1 = out["one"]
    # per core: the one-thread walk + force rate with the (one-thread) build included
    return {
        "value": spec.n / t_full,
        "unit": "particles/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"oracle tree build on all {spec.n} particles ({t_build:.1f} s, 1 thread) + "
                   f"walk and FP64 list force for every {stride}th group in key order "
                   f"({n_s} of {G} groups, {parts} particles, {inter} interactions, "
                   f"{t_s:.1f} s on {threads} threads), extrapolated by group count"),
        "interactions_per_s": inter / t_s,
        "one_core": {
            "particles_per_s": spec.n / t_full1,
            "interactions_per_s": inter1 / t_s1,
            "sample": (f"the same build + every {stride1}th group ({n_s1} groups, {parts1} "
                       f"particles, {inter1} interactions, {t_s1:.1f} s on 1 thread), "
                       f"extrapolated by group count"),
            "paper_per_core_particles_per_s": 5.0e4,
        },
    }


def serving_bench(tp, n_boxes, per_box, inflight, budget_frac=0.25, batching=False):
    """The ensemble serving workload: n_boxes independent clustered boxes with N log-uniform
    in [32^3, 256^3] (seed 999; box i uses seed 1000 + i and max(1, round(N/1e4)) halos),
    mesh = N^(1/3), r_cut = 3/mesh, eps = mesh/20, theta = 0.5, FP32.  First the closed-loop
    capacity (2 * inflight requests kept outstanding, over the whole request sequence); then
    the same n_boxes * per_box requests in
    seeded order arriving as a Poisson process at 0.8 x that capacity, then again at 0.5 x,
    with the HBM budget set to 25% of the ensemble's total resident footprint.  Reports p50/p99
    latency (completion minus submission), its queued and service parts, the median service
    stages, the mean number of boxes per shared launch and aggregate particles/s for both
    rates."""
    import concurrent.futures as cf
    import threading

    import numpy as np

    import boxgen

    ns, halos = boxgen.serving_sizes(n_boxes, 999)
    log(f"[serving] generating {n_boxes} boxes, {int(ns.sum())} particles ...")
    t0 = time.time()

    def gen(i):
        return boxgen.nfw_box(int(ns[i]), int(halos[i]), 1000 + i)

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        boxes = list(ex.map(gen, range(n_boxes)))
    log(f"[serving] generated in {time.time() - t0:.1f} s")
    params = []
    for i in range(n_boxes):
        mesh_n = round(float(ns[i]) ** (1.0 / 3.0))
        mesh = 1.0 / mesh_n
        params.append(tp.treepm_params(1.0, mesh, 3.0 * mesh, mesh / 20.0, 0.5, 10, 256,
                                       tp.TREEPM_FP32))
    footprint = int(sum(int(n) * 320 + (64 << 20) for n in ns))
    budget = max(int(footprint * budget_frac), int(ns.max()) * 320 + (64 << 20))
    ens = tp.treepm_ens_create(0, budget, inflight)
    tp.treepm_ens_set_batching(ens, batching)
    rng = boxgen.SplitMix64(998)
    order = np.argsort(rng.next_u64(n_boxes * per_box), kind="stable") % n_boxes

    def drain(pending, done, out_lat):
        for t in list(pending):
            rc, st = tp.treepm_ensemble_poll(ens, t)
            if rc == tp.TREEPM_OK:
                out_lat.append((st.latency_ms, st.queue_ms, st.stage_ms[0], st.stage_ms[1],
                                st.stage_ms[2], st.batch_boxes))
                done.append(pending.pop(t))

    try:
        # closed loop: keep 2 * inflight requests outstanding, over the whole request sequence
        # (a prefix can draw an easier mix of box sizes and evictions than the open loops get)
        n_closed = len(order)
        pending, done, lat = {}, [], []
        t0 = time.perf_counter()
        k = 0
        shown = 0
        while len(done) < n_closed:
            while k < n_closed and len(pending) < 2 * inflight:
                i = int(order[k]); k += 1
                pending[tp.treepm_ensemble_submit(ens, i, params[i], *boxes[i])] = i
            drain(pending, done, lat)
            if len(done) >= shown + 160:
                shown = len(done) // 160 * 160
                log(f"[serving] closed loop: {len(done)} of {n_closed} done")
            time.sleep(0.0005)
        t_closed = time.perf_counter() - t0
        cap = n_closed / t_closed
        log(f"[serving] closed loop: {n_closed} requests in {t_closed:.1f} s ({cap:.1f} req/s)")
        def open_loop(frac):
            """Poisson arrivals at frac x capacity: (latencies, requests done, makespan)."""
            lam = frac * cap
            gaps = -np.log(1.0 - rng.uniform(len(order))) / lam
            arrivals = np.cumsum(gaps)
            pending, done, lat = {}, [], []
            lock = threading.Lock()
            t_start = time.perf_counter()

            def submitter():
                for j, i in enumerate(order):
                    wait = arrivals[j] - (time.perf_counter() - t_start)
                    if wait > 0:
                        time.sleep(wait)
                    t = tp.treepm_ensemble_submit(ens, int(i), params[int(i)],
                                                  *boxes[int(i)])
                    with lock:
                        pending[t] = int(i)

            th = threading.Thread(target=submitter)
            th.start()
            shown = 0
            while th.is_alive() or pending:
                with lock:
                    drain(pending, done, lat)
                if len(done) >= shown + 160:
                    shown = len(done) // 160 * 160
                    log(f"[serving] open loop at {frac} x: {len(done)} of {len(order)} done")
                time.sleep(0.0005)
            th.join()
            return lam, np.array(lat).reshape(-1, 6), done, time.perf_counter() - t_start

        lam, lat, done, makespan = open_loop(0.8)
        log(f"[serving] open loop at 0.8 x capacity: {len(done)} requests in {makespan:.1f} s")
        info = tp.treepm_ens_info(ens)
        lam5, lat5, done5, makespan5 = open_loop(0.5)
        log(f"[serving] open loop at 0.5 x capacity: {len(done5)} requests in {makespan5:.1f} s")
    finally:
        tp.treepm_ens_destroy(ens)
    def stages(l):
        # median of each part of the service time: context, input copy and build; wait for a
        # batch; the batch's walk, force and result copy
        return {k: float(np.percentile(l[:, 2 + j], 50))
                for j, k in enumerate(("build", "wait_for_batch", "batch"))}

    parts = float(sum(int(ns[i]) for i in done))
    parts5 = float(sum(int(ns[i]) for i in done5))
    return {
        "boxes": n_boxes,
        "requests": len(done),
        "particles": int(ns.sum()),
        "n_range": [int(ns.min()), int(ns.max())],
        "hbm_budget_gib": budget / 2 ** 30,
        "footprint_gib": footprint / 2 ** 30,
        "max_inflight": inflight,
        "shared_launches": bool(batching),
        "closed_loop_requests_per_s": cap,
        "arrival_rate_per_s": lam,
        "latency_ms_p50": float(np.percentile(lat[:, 0], 50)),
        "latency_ms_p99": float(np.percentile(lat[:, 0], 99)),
        "latency_ms_max": float(lat[:, 0].max()),
        "queue_ms_p50": float(np.percentile(lat[:, 1], 50)),
        "queue_ms_p99": float(np.percentile(lat[:, 1], 99)),
        "service_ms_p50": float(np.percentile(lat[:, 0] - lat[:, 1], 50)),
        "service_ms_p99": float(np.percentile(lat[:, 0] - lat[:, 1], 99)),
        "particles_per_s": parts / makespan,
        "stage_ms_p50": stages(lat),
        "batch_boxes_mean": float(lat[:, 5].mean()),
        "resident_boxes_at_end": info["resident_boxes"],
        "at_half_capacity": {
            "arrival_rate_per_s": lam5,
            "requests": len(done5),
            "latency_ms_p50": float(np.percentile(lat5[:, 0], 50)),
            "latency_ms_p99": float(np.percentile(lat5[:, 0], 99)),
            "queue_ms_p50": float(np.percentile(lat5[:, 1], 50)),
            "queue_ms_p99": float(np.percentile(lat5[:, 1], 99)),
            "service_ms_p50": float(np.percentile(lat5[:, 0] - lat5[:, 1], 50)),
            "service_ms_p99": float(np.percentile(lat5[:, 0] - lat5[:, 1], 99)),
            "particles_per_s": parts5 / makespan5,
            "stage_ms_p50": stages(lat5),
            "batch_boxes_mean": float(lat5[:, 5].mean()),
        },
    }


def accuracy_bench(tp, torch, np, n_crit):
    """Force accuracy on the 128^3 clustered box, all computed by the library: the reference is
    the FP64 path at theta = 0, whose lists hold every particle within r_cut of each group (the
    exact short-range sum).  For each setting: interactions and the RMS, median and 99th
    percentile over particles of |a - a_exact| / |a_exact|.  The FP32 path at theta = 0 gives
    the kernel's own rounding against FP64 on the same lists."""
    import boxgen
    spec = boxgen.CONFIGS["nfw128"]
    arrays = spec.generate()
    dev = [torch.from_numpy(a).cuda() for a in arrays]
    log("[bench] accuracy leg (nfw128)")

    def run(prec, theta, opening=0, theta_max=0.0, quad=0):
        p = tp.make_params(spec.L, spec.mesh, spec.r_cut, spec.eps, theta, spec.n_leaf, n_crit,
                           prec, opening=opening, theta_max=theta_max, quadrupole=quad)
        ctx = tp.treepm_create(p, 0)
        try:
            tp.treepm_build(ctx, *dev)
            st = tp.treepm_walk(ctx)
            acc = [torch.empty(spec.n, dtype=torch.float64, device="cuda") for _ in range(3)]
            tp.treepm_force_short(ctx, *acc)
            torch.cuda.synchronize()
            return torch.stack(acc), int(st.interactions)
        finally:
            tp.treepm_destroy(ctx)

    ref, inter0 = run(tp.TREEPM_FP64, 0.0)
    nr = torch.linalg.norm(ref, dim=0)
    nz = nr > 0

    def err(a):
        rel = (torch.linalg.norm(a - ref, dim=0)[nz] / nr[nz]).cpu().numpy()
        return {"rms": float(np.sqrt(np.mean(rel * rel))), "p50": float(np.median(rel)),
                "p99": float(np.quantile(rel, 0.99))}

    out = {"workload": f"{spec.name}, n_crit={n_crit}", "exact_interactions": inter0}
    a, i = run(tp.TREEPM_FP32, 0.0)
    out["fp32_kernel_theta_0"] = dict(err(a), interactions=i)
    for name, kw in (("monopole_theta_0.5", dict(theta=0.5)),
                     ("monopole_theta_0.4", dict(theta=0.4)),
                     ("quadrupole_theta_0.5", dict(theta=0.5, quad=1)),
                     ("quadrupole_theta_0.7", dict(theta=0.7, quad=1)),
                     ("theta_r_0.3_cap_0.5", dict(theta=0.3, opening=1, theta_max=0.5))):
        a, i = run(tp.TREEPM_FP32, **kw)
        out[name] = dict(err(a), interactions=i)
    del dev
    torch.cuda.empty_cache()
    return out


def scale_bench(tp, torch, np, n_crit, steps=4, warmup=2):
    """The scale workload: the 512^3 clustered box (10,000 halos holding 70 % of the particles,
    mesh 512^3, r_cut = 3/512, eps = 1/(20*512)), FP32 path, n_crit fixed (parity-tested at
    this size), at theta = 0.5 (Table 2's setting) and theta = 0.4.  Step = build + walk +
    force on the resident box, as in the main leg."""
    import boxgen
    spec = boxgen.CONFIGS["nfw512"]
    log(f"[bench] scale leg: generating {spec.name} (N={spec.n}) ...")
    t0 = time.time()
    arrays = spec.generate()
    log(f"[bench] generated in {time.time() - t0:.1f} s")
    dev = [torch.from_numpy(a).cuda() for a in arrays]
    del arrays
    acc = [torch.empty(spec.n, dtype=torch.float32, device="cuda") for _ in range(3)]
    out = {"workload": (f"{spec.name}: N={spec.n} clustered box ({spec.n_halos} NFW halos, "
                        f"{int(spec.f_halo * 100)}% in halos), mesh {spec.mesh_n}^3, "
                        f"r_cut=3/{spec.mesh_n}, eps=1/(20*{spec.mesh_n}), n_leaf={spec.n_leaf}, "
                        f"n_crit={n_crit}, FP32; step = build + walk + force"),
           "n": spec.n, "n_crit": n_crit}
    for theta in (0.5, 0.4):
        p = tp.treepm_params(spec.L, spec.mesh, spec.r_cut, spec.eps, theta, spec.n_leaf,
                             n_crit, tp.TREEPM_FP32)
        ctx = tp.treepm_create(p, 0)
        tp.treepm_set_timing(ctx, True)
        log(f"[bench] scale leg: theta = {theta}")
        run_steps(tp, torch, ctx, dev, acc, warmup)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        times, st = run_steps(tp, torch, ctx, dev, acc, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        tp.treepm_destroy(ctx)
        ph = np.array(times)
        tf = float(np.mean(ph[:, 2])) * 1e-3
        inter = int(st.interactions)
        pps = spec.n * steps / el
        out[f"theta_{theta}"] = {
            "ms_per_step": el / steps * 1e3,
            "particles_per_s": pps,
            "interactions": inter,
            "interactions_per_particle": inter / spec.n,
            "interactions_per_s": inter / tf,
            "evaluated_pairs": int(st.evaluated),
            "phase_ms": {"build": float(np.mean(ph[:, 0])), "walk": float(np.mean(ph[:, 1])),
                         "force_f32": float(np.mean(ph[:, 2]))},
            "groups": int(st.n_groups),
            "force_roofline_frac": K_PP * inter / tf / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
            "paper_core_equivalents": pps / 5.0e4,
        }
    del dev, acc
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (the tree force of one box on one "
              f"MI355X); --gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import boxgen
    import paper_0910_0121_amd as tp

    if args.copy_calibration:
        # a plain copy of known size: reads and writes 2^30 bytes per dispatch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "dispatches": 3}), flush=True)
        return
    if args.serving_only:
        print(json.dumps(serving_bench(tp, args.serving_boxes, args.serving_requests_per_box,
                                       args.serving_inflight, args.serving_budget_frac,
                                       args.serving_batching)),
              flush=True)
        return
    spec = boxgen.CONFIGS[args.workload]
    if args.theta is not None:
        import dataclasses
        spec = dataclasses.replace(spec, theta=args.theta)
    n_crit = args.n_crit
    log(f"[bench] generating {spec.name} (N={spec.n}) ...")
    t0 = time.time()
    arrays = spec.generate()
    log(f"[bench] generated in {time.time() - t0:.1f} s")
    dev = [torch.from_numpy(a).cuda() for a in arrays]
    acc = [torch.empty(spec.n, dtype=torch.float32, device="cuda") for _ in range(3)]

    autotune = None
    if n_crit <= 0:
        cands = [int(v) for v in args.n_crit_candidates.split(",")]
        p0 = tp.treepm_params(spec.L, spec.mesh, spec.r_cut, spec.eps, spec.theta,
                              spec.n_leaf, cands[0], tp.TREEPM_FP32)
        ctx = tp.treepm_create(p0, 0)
        t0 = time.time()
        n_crit, best_ms = tp.treepm_autotune(ctx, *dev, cands)
        tp.treepm_destroy(ctx)
        autotune = {"candidates": cands, "chosen": n_crit, "step_ms": best_ms,
                    "seconds": time.time() - t0}
        log(f"[bench] autotuned n_crit = {n_crit} ({best_ms:.2f} ms)")

    p32 = tp.treepm_params(spec.L, spec.mesh, spec.r_cut, spec.eps, spec.theta, spec.n_leaf,
                           n_crit, tp.TREEPM_FP32)
    ctx = tp.treepm_create(p32, 0)
    tp.treepm_set_timing(ctx, True)
    log(f"[bench] warmup {args.warmup} steps")
    run_steps(tp, torch, ctx, dev, acc, args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, st = run_steps(tp, torch, ctx, dev, acc, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tp.treepm_destroy(ctx)
    ms_per_step = elapsed / args.steps * 1e3
    ph = np.array(times)  # per step: build, walk, force, sum (device event times, ms)
    t_force = float(np.mean(ph[:, 2])) * 1e-3
    inter = int(st.interactions)
    evaluated = int(st.evaluated)
    # Achieved FLOP/s in the survey's unit: K_pp flops per list interaction (sum over groups of
    # n_g L_g, the paper's N_int x N), over the force call's device time.  The kernel skips
    # the pairs whose source lies at least r_cut from the group's box (they add exactly zero);
    # the same rate counted on the pairs it evaluated is reported beside it.
    achieved = K_PP * inter / t_force / 1e12
    achieved_eval = K_PP * evaluated / t_force / 1e12
    traffic = measured_traffic(n_crit, spec.name)
    result = {
        "metric": METRIC,
        "value": spec.n * args.steps / elapsed,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{spec.name}: N={spec.n} clustered box ({spec.n_halos} NFW halos, "
                         f"c=10, dN/dM~M^-1.9, {int(spec.f_halo * 100)}% in halos), unit "
                         f"periodic box, mesh {spec.mesh_n}^3, r_cut=3/{spec.mesh_n}, "
                         f"eps=1/(20*{spec.mesh_n}), theta={spec.theta}, n_leaf={spec.n_leaf}, "
                         f"n_crit={n_crit}; step = build + walk + FP32 force"),
            "n": spec.n, "theta": spec.theta, "n_crit": n_crit, "n_leaf": spec.n_leaf,
            "r_cut": spec.r_cut, "eps": spec.eps,
        },
        "autotune": autotune,
        "interactions_per_s": inter / t_force,
        "interactions": inter,
        "interactions_per_particle": inter / spec.n,
        "evaluated_pairs": evaluated,
        "evaluated_pairs_per_s": evaluated / t_force,
        "zero_pairs_skipped_frac": 1.0 - evaluated / inter,
        "phase_ms": {"build": float(np.mean(ph[:, 0])), "walk": float(np.mean(ph[:, 1])),
                     "force_f32": float(np.mean(ph[:, 2]))},
        "tree": {"nodes": int(st.n_nodes), "groups": int(st.n_groups),
                 "cell_entries": int(st.n_cell_entries), "particle_entries": int(st.n_part_entries),
                 "max_level": int(st.max_level), "max_group": int(st.max_group)},
        "roofline": {
            "kernel": "k_force_f32",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": (traffic["fetch_bytes"] + traffic["write_bytes"]) if traffic else None,
            "flops_per_interaction": K_PP,
            "flops_counted_on": "list interactions (sum over groups of n_g L_g)",
            "achieved_on_evaluated_pairs": achieved_eval,
            "frac_on_evaluated_pairs": achieved_eval / FP32_VECTOR_PEAK_TFLOPS,
        },
    }
    if not args.no_fp64:
        p64 = tp.treepm_params(spec.L, spec.mesh, spec.r_cut, spec.eps, spec.theta, spec.n_leaf,
                               n_crit, tp.TREEPM_FP64)
        ctx = tp.treepm_create(p64, 0)
        tp.treepm_set_timing(ctx, True)
        log("[bench] FP64 path")
        run_steps(tp, torch, ctx, dev, acc, 1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        k64 = max(1, min(3, args.steps))
        times64, st64 = run_steps(tp, torch, ctx, dev, acc, k64)
        torch.cuda.synchronize()
        e64 = time.perf_counter() - t1
        tp.treepm_destroy(ctx)
        f64 = float(np.mean(np.array(times64)[:, 2])) * 1e-3
        ev64 = int(st64.evaluated)
        result["fp64_path"] = {
            "particles_per_s": spec.n * k64 / e64,
            "interactions_per_s": inter / f64,
            "force_ms": f64 * 1e3,
            "evaluated_pairs": ev64,
            "achieved_tflops": K_PP * inter / f64 / 1e12,
            "frac_fp64_peak": K_PP * inter / f64 / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "achieved_tflops_on_evaluated_pairs": K_PP * ev64 / f64 / 1e12,
            "force_speedup_fp32_over_fp64": f64 / t_force,
        }
    if not args.no_theta_r:
        # The same box and step under the distance-dependent angle of eq. (12).
        pr = tp.make_params(spec.L, spec.mesh, spec.r_cut, spec.eps, args.theta0, spec.n_leaf,
                            n_crit, tp.TREEPM_FP32, opening=tp.TREEPM_OPEN_DISTANCE,
                            theta_max=args.theta_max)
        ctx = tp.treepm_create(pr, 0)
        tp.treepm_set_timing(ctx, True)
        log(f"[bench] theta(r) leg: theta_0={args.theta0}, cap={args.theta_max}")
        run_steps(tp, torch, ctx, dev, acc, 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kr = max(1, min(5, args.steps))
        timesr, str_ = run_steps(tp, torch, ctx, dev, acc, kr)
        torch.cuda.synchronize()
        er = time.perf_counter() - t1
        tp.treepm_destroy(ctx)
        phr = np.array(timesr)
        fr = float(np.mean(phr[:, 2])) * 1e-3
        result["theta_r"] = {
            "theta0": args.theta0, "theta_max": args.theta_max,
            "ms_per_step": er / kr * 1e3,
            "particles_per_s": spec.n * kr / er,
            "interactions": int(str_.interactions),
            "interactions_per_s": int(str_.interactions) / fr,
            "cell_entries": int(str_.n_cell_entries),
            "phase_ms": {"build": float(np.mean(phr[:, 0])), "walk": float(np.mean(phr[:, 1])),
                         "force_f32": float(np.mean(phr[:, 2]))},
        }
    if not args.no_quadrupole:
        # The same box and step with the cells' second-order terms (Section 4.1).
        pq = tp.make_params(spec.L, spec.mesh, spec.r_cut, spec.eps, spec.theta, spec.n_leaf,
                            n_crit, tp.TREEPM_FP32, quadrupole=1)
        ctx = tp.treepm_create(pq, 0)
        tp.treepm_set_timing(ctx, True)
        log("[bench] quadrupole leg")
        run_steps(tp, torch, ctx, dev, acc, 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kq = max(1, min(5, args.steps))
        timesq, stq = run_steps(tp, torch, ctx, dev, acc, kq)
        torch.cuda.synchronize()
        eq = time.perf_counter() - t1
        tp.treepm_destroy(ctx)
        phq = np.array(timesq)
        result["quadrupole"] = {
            "ms_per_step": eq / kq * 1e3,
            "particles_per_s": spec.n * kq / eq,
            "interactions": int(stq.interactions),
            "phase_ms": {"build": float(np.mean(phq[:, 0])), "walk": float(np.mean(phq[:, 1])),
                         "force_f32_with_quadrupole": float(np.mean(phq[:, 2]))},
        }
    if not args.no_pm:
        # The long-range half of the split on the same box and its own mesh (N_PM^3 = N).
        pp = tp.make_params(spec.L, spec.mesh, spec.r_cut, spec.eps, spec.theta, spec.n_leaf,
                            n_crit, tp.TREEPM_FP32)
        ctx = tp.treepm_create(pp, 0)
        log(f"[bench] particle-mesh leg: N_PM = {spec.mesh_n}")
        tp.treepm_build(ctx, *dev)
        for _ in range(2):
            tp.treepm_force_long(ctx, *acc)
        torch.cuda.synchronize()
        kp = max(1, min(10, args.steps))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pm_total = 0.0
        for _ in range(kp):
            # each timed call follows a fresh (untimed) build, as in a time step: one mesh
            # force per build
            tp.treepm_build(ctx, *dev)
            e0.record()
            tp.treepm_force_long(ctx, *acc)
            e1.record()
            torch.cuda.synchronize()
            pm_total += e0.elapsed_time(e1)
        tp.treepm_destroy(ctx)
        pm_ms = pm_total / kp
        pm_bytes = PM_BYTES_PER_POINT * spec.mesh_n ** 3 + PM_BYTES_PER_PARTICLE * spec.n
        result["pm"] = {
            "n_pm": spec.mesh_n,
            "ms": pm_ms,
            "particles_per_s": spec.n / (pm_ms * 1e-3),
            "short_plus_long_ms_per_step": ms_per_step + pm_ms,
            "roofline": {"bound": "hbm", "achieved": pm_bytes / (pm_ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": pm_bytes / (pm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes": pm_bytes},
        }
    if not args.no_time_step:
        # Whole TreePM time steps on copies of the box: short- and long-range forces into one
        # FP32 array, the shared step of eq. (7) and a kick and drift (Section 2.2, 2.4).
        ps_ = tp.make_params(spec.L, spec.mesh, spec.r_cut, spec.eps, spec.theta, spec.n_leaf,
                             n_crit, tp.TREEPM_FP32)
        ctx = tp.treepm_create(ps_, 0)
        pos = [t.clone() for t in dev[:3]]
        vel = [torch.zeros(spec.n, dtype=torch.float64, device="cuda") for _ in range(3)]
        log("[bench] time-step leg")

        def one_step(first):
            tp.treepm_build(ctx, *pos, dev[3])
            tp.treepm_walk(ctx)
            tp.treepm_force_short(ctx, *acc)
            tp.treepm_force_long(ctx, *acc, accumulate=True)
            dt = tp.treepm_timestep(ctx, *vel, *acc, spec.eps, 1.0)
            tp.treepm_kick_drift(ctx, *pos, *vel, *acc, 0.5 * dt if first else dt, dt)
            return dt

        for k in range(2):
            one_step(k == 0)
        torch.cuda.synchronize()
        ks = max(1, min(5, args.steps))
        t1 = time.perf_counter()
        dts = [one_step(False) for _ in range(ks)]
        torch.cuda.synchronize()
        es = time.perf_counter() - t1
        tp.treepm_destroy(ctx)
        del pos, vel
        result["time_step"] = {
            "ms_per_step": es / ks * 1e3,
            "particles_per_s": spec.n * ks / es,
            "dt_last": dts[-1],
            "content": "build + walk + FP32 short-range + PM long-range + eq. (7) step + "
                       "kick-drift",
        }
    if not args.no_accuracy:
        result["accuracy"] = accuracy_bench(tp, torch, np, n_crit)
    if not args.no_scale:
        result["scale"] = scale_bench(tp, torch, np, args.scale_n_crit)
    if not args.no_serving:
        log("[bench] ensemble serving")
        result["ensemble"] = serving_bench(tp, args.serving_boxes, args.serving_requests_per_box,
                                           args.serving_inflight, args.serving_budget_frac,
                                           args.serving_batching)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (bounded sample)")
        result["cpu_baseline"] = cpu_baseline(spec, arrays, n_crit, args.cpu_stride)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
