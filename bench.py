#!/usr/bin/env python3
"""Throughput of the full SPH step (tree + density + force) on one MI355X.

A "step" is one kick-drift-kick step of the whole hot path over one instance:
leapfrog predict, Morton keys, radix sort, gather, keep mask + reduction,
Karras tree, bottom-up boxes, two-stage neighbour cache, h/rho Newton
iteration with Omega, force + du/dt, corrector and the CFL reduction.  The
default workload is the Sedov-like blast on a jittered 256^3 lattice in FP32
(seeded synthetic input standing in for the paper's Sedov restart files).

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s/GPU (tree+density+force), %HBM peak; batched/served vs plain, p99"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per particle of one launch of each stage, FP32: every
# array the stage must touch crosses HBM once, neighbour data re-read through
# LDS / L2 is not counted, 81 cache entries of 4 B, two Newton passes over the
# cache per density launch, 8 radix passes.  Split as (integer bytes,
# floating-point bytes); the floating part doubles in FP64.
STAGE_BYTES = {
    "predict_morton": (12, 100),        # x, v, a, u, du/dt in; x, v^{n+1/2}, v*, u's out; key, iota
    "radix_sort": (192, 0),
    "gather": (4, 126),
    "mask_reduce_compact": (45, 0),
    "karras": (3, 0),
    "boxes": (0, 23),
    "group_leaf_cache": (25, 0),
    "particle_cache": (324, 46),        # 81 indices out; positions, h in
    "density": (648, 62),               # the cache read twice (two Newton passes); x, h in; h, rho, Omega out
    "force": (324, 56),                 # the cache; own fields in; a, du/dt out
    "correct": (0, 64),
}


def stage_bytes_pp(stage, T):
    ib, fb = STAGE_BYTES[stage]
    return ib + fb * T // 4

# HBM traffic of the dominant kernel per launch, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) scaled by what the same counters read for a plain
# 1 GiB device copy (FETCH x2.0000, WRITE x1.0000), with the sha256 of the
# kernel's sources at the time: the figure is reported only while they match.
TRAFFIC = {
    ("particle_cache", "sedov256"): {
        "bytes_per_launch": 5.4318e9,     # FETCH + WRITE of k_group_cache<float, 1>
        "sources_sha256": "112eeb6a4b11c376453a6b27877a8e82b7a2d3978a430d2e95c14c8f9453691d"},
    ("force", "sedov256"): {
        "bytes_per_launch": 7.0283e9,     # FETCH + WRITE of k_force<float, 1536, 0, 2>
        "sources_sha256": "f466f47c110d2f1247b9383f85758a36738f149c5a29d41c6b65209ef0f4ad03"},
}
KERNEL_SOURCES = {"particle_cache": ("neigh.hip", "common.hpp", "kernels.hpp"),
                  "force": ("sph.hip", "common.hpp", "kernels.hpp")}

# Vector instructions the dominant kernel issues per launch (rocprofv3 --pmc
# SQ_INSTS_VALU, wave instructions summed over the chip), with the sha256 of
# its sources at the time, set against the nominal rate of one wave64 VALU
# instruction per compute unit per clock at 2.4 GHz (a 64-lane FP32 operation
# occupies a 16-lane SIMD for four clocks, four SIMDs per CU).  A secondary
# figure beside the HBM roofline; the clock under load is not measured here.
VALU_INSTS = {
    ("particle_cache", "sedov256"): {
        "valu_insts_per_launch": 1.3700e9,   # k_group_cache<float, 1>
        "sources_sha256": "112eeb6a4b11c376453a6b27877a8e82b7a2d3978a430d2e95c14c8f9453691d"},
    ("force", "sedov256"): {
        "valu_insts_per_launch": 2.0369e9,   # k_force<float, 1536, 0, 2>
        "sources_sha256": "f466f47c110d2f1247b9383f85758a36738f149c5a29d41c6b65209ef0f4ad03"},
}
CU_COUNT, CLOCK_HZ = 256, 2.4e9


def valu_issue_for(stage, workload, avg_ms):
    t = VALU_INSTS.get((stage, workload))
    if not t or t["sources_sha256"] != sources_sha(stage):
        return None
    n = t["valu_insts_per_launch"]
    return {"valu_insts_per_launch": n,
            "frac_of_nominal_issue": round(n / (CU_COUNT * CLOCK_HZ * avg_ms * 1e-3), 4)}


def sources_sha(stage):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(stage, ()):
        with open(os.path.join(ROOT, "paper_2503_09713_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(stage, workload):
    t = TRAFFIC.get((stage, workload))
    if not t or t["sources_sha256"] != sources_sha(stage):
        return None
    return t["bytes_per_launch"]


WORKLOADS = {
    # name: (generator, lattice side, seed, dtype)
    "sedov256": ("sedov", 256, 3, "f32"),
    "uniform128": ("lattice", 128, 2, "f32"),
    "tiny16": ("lattice", 16, 1, "f64"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_input(name):
    import numpy as np
    import gen
    fam, n1, seed, dt = WORKLOADS[name]
    T = np.float32 if dt == "f32" else np.float64
    if fam == "sedov":
        return gen.sedov(n1, seed, dtype=T)
    return gen.lattice(n1, seed, dtype=T)


def cpu_baseline(ps_host, p, args):
    """The CPU oracle (FP64; its neighbour, density and force loops use OpenMP)
    on a bounded sample of the same workload.  Tree half at full size: Morton
    keys, stable sort, keep mask + reduction, radix tree and tight boxes of
    all N particles.  Particle half on S random targets against all N:
    neighbour sets, density (h root) and force, timed at two sample sizes and
    extrapolated linearly (slope per particle + the O(N) search-grid builds).
    The full step is the sum."""
    import numpy as np
    import oracle
    oracle.lib()
    n = p.n
    rng = np.random.default_rng(0)
    x, y, z = (ps_host[k].astype(np.float64) for k in ("x", "y", "z"))
    vx, vy, vz, u, h = (ps_host[k].astype(np.float64) for k in ("vx", "vy", "vz", "u", "h"))

    def tree():
        t0 = time.perf_counter()
        keys = oracle.morton(x, y, z, p.lo, p.hi)
        eps, mu = oracle.sort(keys)
        _, ids, ml = oracle.leaves(mu, args.n_red)
        t = oracle.radix_tree(ml)
        oracle.tight_boxes(ids, t, x[eps], y[eps], z[eps], h[eps])
        return time.perf_counter() - t0

    def run(S):
        t = np.sort(rng.choice(n, size=S, replace=False))
        t0 = time.perf_counter()
        oracle.neighbours(ps_host["x"], ps_host["y"], ps_host["z"], ps_host["h"], p.lo, p.hi,
                          p.periodic, 2.2, targets=t)
        hh, rho, om, _ = oracle.density(x, y, z, h, p.lo, p.hi, p.periodic, p.mass, targets=t)
        hfull = h.copy()
        hfull[t] = hh
        rfull = p.mass * (1.2 / hfull) ** 3
        ofull = np.ones(n)
        ofull[t] = om
        oracle.force(x, y, z, vx, vy, vz, u, hfull, rfull, ofull, p.lo, p.hi, p.periodic, p.mass,
                     targets=t)
        return time.perf_counter() - t0

    def rate(s1, s2, t_tree):
        log(f"[cpu] oracle sample {s1} ({oracle.threads()} threads) ...")
        t1 = run(s1)
        log(f"[cpu] oracle sample {s2} ({oracle.threads()} threads) ...")
        t2 = run(s2)
        slope = max((t2 - t1) / (s2 - s1), 1e-12)
        overhead = max(t1 - slope * s1, 0.0)
        return n / (t_tree + slope * n + overhead), t1, t2

    cores = oracle.threads()
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    log(f"[cpu] oracle tree half on all {n} particles ...")
    t_tree = tree()
    s1, s2 = args.cpu_sample // 8, args.cpu_sample
    v, t1, t2 = rate(s1, s2, t_tree)
    # one thread: a sample an eighth the size (the same extrapolation; the
    # tree half is single-threaded already)
    oracle.set_threads(1)
    v1, u1, u2 = rate(s1 // 8, s2 // 8, t_tree)
    oracle.set_threads(cores)
    return {"value": v, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "value_one_thread": v1, "cpu_model": cpu_model, "host_cpus": os.cpu_count(),
            "tree_half_s": t_tree,
            "sample": (f"tree half (keys, sort, reduction, radix tree, boxes) of all {n} "
                       f"particles of the {args.workload} state in {t_tree:.1f}s; neighbours, "
                       f"density (h root) and force of {s2} and {s1} random particles against "
                       f"all {n} ({t1:.1f}s, {t2:.1f}s; one thread: {s2 // 8} and {s1 // 8}, "
                       f"{u1:.1f}s, {u2:.1f}s), extrapolated to all particles; FP64")}


def run_lattice(args, shsph, torch, name="uniform128", steps=20, warmup=3):
    """The jittered-lattice workload (128^3, FP32, CFL steps) with the same
    kernels and defaults: particle-steps/s beside the Sedov line."""
    p = make_input(name)
    log(f"[{name}] {p.n} particles")
    ps = shsph.ParticleSet.from_particles(p)
    ctx = shsph.Context(0, n_red=args.n_red)
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    for _ in range(warmup):
        ctx.step(ps, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(ps, 0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    log(f"[{name}] {1e3 * el / steps:.2f} ms/step")
    return {"workload": name, "particles": p.n, "steps": steps, "warmup": warmup,
            "ms_per_step": 1e3 * el / steps, "value": p.n * steps / el,
            "unit": "particle-steps/s"}


def run_f64(args, shsph, torch, steps=10, warmup=3):
    """The Sedov 256^3 workload in FP64 (the paper's arithmetic), CFL steps."""
    import numpy as np
    import gen
    p = gen.sedov(256, gen.SEEDS["sedov"], dtype=np.float64)
    log(f"[f64] sedov256 FP64, {p.n} particles")
    ps = shsph.ParticleSet.from_particles(p)
    ctx = shsph.Context(0, n_red=args.n_red, eps_h=1e-12)
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    for _ in range(warmup):
        ctx.step(ps, 0.0)
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(ps, 0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stages = ctx.stage_times()
    ctx.close()
    log(f"[f64] {1e3 * el / steps:.2f} ms/step")
    return {"workload": "sedov256", "dtype": "f64", "particles": p.n, "steps": steps,
            "warmup": warmup, "ms_per_step": 1e3 * el / steps, "value": p.n * steps / el,
            "unit": "particle-steps/s",
            "stages_ms_per_step": {k: round(v[0] / steps, 4) for k, v in stages.items()}}


def run_tree_build_key_bits(args, shsph, torch, reps=5):
    """Tree build from the input's random order (full radix sort) with 63-bit
    and 30-bit Morton codes (Sect. 5.2.1 reports about 30% faster builds with
    32-bit codes): the tree stages (keys, sort, gather, mask/reduction,
    Karras, boxes) of shsph_build_tree, Sedov 256^3 FP32."""
    import numpy as np
    import gen
    p = gen.sedov(256, gen.SEEDS["sedov"], dtype=np.float32)
    ps = shsph.ParticleSet.from_particles(p)
    tree = ("predict_morton", "radix_sort", "gather", "mask_reduce_compact", "karras", "boxes")
    res = {"workload": "sedov256", "particles": p.n, "repetitions": reps}
    for bits in (63, 30):
        ctx = shsph.Context(0, n_red=args.n_red, key_bits=bits)
        ctx.build_tree(ps)
        torch.cuda.synchronize()
        ctx.set_profiling(True)
        for _ in range(reps):
            ctx.build_tree(ps)
        torch.cuda.synchronize()
        st = ctx.stage_times()
        ctx.close()
        ms = sum(st[k][0] for k in tree) / reps
        res[f"key_bits_{bits}"] = {"tree_ms": round(ms, 4),
                                   "stages_ms": {k: round(st[k][0] / reps, 4) for k in tree},
                                   "objects_per_s": p.n / (ms * 1e-3)}
        log(f"[tree] {bits}-bit codes: {ms:.3f} ms per tree build")
    res["speedup_30_vs_63"] = res["key_bits_63"]["tree_ms"] / res["key_bits_30"]["tree_ms"]
    return res


def run_m6(args, shsph, torch, steps=10, warmup=3):
    """The M6 kernel with h_fact = 1.0 (the paper's physics tests, about 113
    neighbours) on the jittered 128^3 lattice, FP32, CFL steps."""
    import numpy as np
    import gen
    p = gen.lattice(128, gen.SEEDS["uniform"], dtype=np.float32, hfact=1.0)
    ps = shsph.ParticleSet.from_particles(p)
    ctx = shsph.Context(0, n_red=args.n_red, kernel="M6", hfact=1.0)
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    for _ in range(warmup):
        ctx.step(ps, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(ps, 0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = ctx.get_info()
    ctx.close()
    log(f"[m6] {1e3 * el / steps:.2f} ms/step")
    return {"workload": "uniform128", "kernel": "M6", "hfact": 1.0, "particles": p.n,
            "cache_entries_per_particle": info["n_neigh"] / p.n, "steps": steps,
            "ms_per_step": 1e3 * el / steps, "value": p.n * steps / el, "unit": "particle-steps/s"}


def run_batched(args, shsph, torch):
    """64 uneven instances (half jittered lattices, half Plummer spheres,
    N_i log-uniform in [2^12, 2^20]): K CFL steps as one batched pass per step,
    against the same kernels run one instance per pass (plain launches)."""
    import gen
    log("[batched] generating 64 instances")
    insts = gen.batch(seed=gen.SEEDS["batch"], n_inst=64)
    ntot = sum(p.n for p in insts)
    sets = [shsph.ParticleSet.from_particles(p) for p in insts]
    K, W = args.batch_steps, args.batch_warmup
    res = {"workload": "batched64", "instances": len(insts), "particles": ntot,
           "n_min": min(p.n for p in insts), "n_max": max(p.n for p in insts), "steps": K}
    ctx = shsph.Context(0, n_red=args.n_red)
    hs = [ctx.instance_create(s) for s in sets]
    tune = ctx.autotune(hs)
    log(f"[batched] autotuned: n_red {tune['n_red']}, stage-2 walk {tune['stage2_mode']}, "
        f"force split {tune['force_split']}, fused density+force {tune['fused_density_force']}")
    res["autotuned"] = tune
    for _ in range(W):
        ctx.step_batch(hs)
    torch.cuda.synchronize()
    g0 = ctx.get_info()
    t0 = time.perf_counter()
    for _ in range(K):
        ctx.step_batch(hs)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    g1 = ctx.get_info()
    res["captured_passes"] = g1["graph_passes"] - g0["graph_passes"]
    res["captured_aborts"] = g1["graph_aborts"] - g0["graph_aborts"]
    # stage breakdown: two more steps launch by launch with stage events
    SP = 2
    ctx.set_profiling(True)
    for _ in range(SP):
        ctx.step_batch(hs)
    torch.cuda.synchronize()
    stages = ctx.stage_times()
    ctx.set_profiling(False)
    ctx.close()
    log(f"[batched] batched {1e3 * tb / K:.2f} ms/step ({res['captured_passes']} of {K} passes "
        f"from the captured graph, {res['captured_aborts']} switched off)")
    # plain: the same kernels, one instance per pass, launch by launch
    ctx = shsph.Context(0, n_red=tune["n_red"], stage2_mode=tune["stage2_mode"],
                        force_split=tune["force_split"],
                        fused_density_force=tune["fused_density_force"], graph_batch=0)
    hs = [ctx.instance_create(s) for s in sets]
    for _ in range(W):
        for h in hs:
            ctx.step_batch([h])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        for h in hs:
            ctx.step_batch([h])
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    ctx.close()
    log(f"[batched] plain {1e3 * tp / K:.2f} ms/step")
    res.update({"value": ntot * K / tb, "unit": "particle-steps/s", "ms_per_step": 1e3 * tb / K,
                "plain_value": ntot * K / tp, "plain_ms_per_step": 1e3 * tp / K,
                "speedup_vs_plain": tp / tb,
                "stages_ms_per_step": {k: round(v[0] / SP, 4) for k, v in stages.items()}})
    return res


def serve_templates(seed):
    """Seeded instance templates for the serving trace: per family, 16 sizes
    evenly spaced in log N over [2^12, 2^22] (bin centres); a job takes the
    template of its family nearest to its drawn size."""
    import numpy as np
    import gen
    out = {"lattice": [], "plummer": []}
    sizes = np.floor(2.0 ** (12 + 10 * (np.arange(16) + 0.5) / 16)).astype(int)
    for fam in out:
        for k, n in enumerate(sizes):
            if fam == "lattice":
                n1 = max(16, int(round(n ** (1.0 / 3.0))))
                p = gen.lattice(n1, seed * 100 + k)
            else:
                p = gen.plummer(int(n), seed * 100 + 50 + k)
            out[fam].append(p)
    return out


def run_served(args, shsph, torch, tune=None):
    """Poisson arrivals of STEP (1-10 CFL steps) and EVAL jobs, each bringing
    its own instance, served under a 200 GB budget with continuous batching and,
    on the same trace, one job at a time: each policy's saturation capacity
    (a burst), then a sweep of offered rates below and above the one-at-a-time
    capacity with p50 / p99 latency and throughput."""
    import numpy as np
    import gen
    kw = dict(n_red=args.n_red) if not tune else dict(n_red=tune["n_red"],
                                                      stage2_mode=tune["stage2_mode"],
                                                      force_split=tune["force_split"],
                        fused_density_force=tune["fused_density_force"])
    log("[served] generating templates")
    tpl = serve_templates(gen.SEEDS["serve"])
    sets = {f: [shsph.ParticleSet.from_particles(p) for p in ps] for f, ps in tpl.items()}
    # instances come from running simulations: settle each template's h once
    pre = shsph.Context(0, **kw)
    for f in sets:
        for ps in sets[f]:
            h = pre.instance_create(ps)
            pre.eval_batch([h])
            pre.instance_read(h, ps)
            pre.instance_destroy(h)
    pre.close()
    logn = {f: np.log([p.n for p in ps]) for f, ps in tpl.items()}
    base = gen.serve_trace(1.0, args.serve_jobs, seed=gen.SEEDS["serve"])
    jobs = []
    for j in base:
        k = int(np.argmin(np.abs(logn[j["family"]] - np.log(j["n"]))))
        jobs.append(dict(j, tpl=k, n=tpl[j["family"]][k].n))

    def submit(ctx, j):
        kind = shsph.JOB_EVAL if j["kind"] == "eval" else shsph.JOB_STEP
        return ctx.submit(init=sets[j["family"]][j["tpl"]], kind=kind, nsteps=j["nsteps"],
                          release=True)

    def serve(policy, jobs_run, rate, label):
        """Serve `jobs_run` with one policy; rate None = every job at once
        (a burst: the policy's saturation capacity), else Poisson arrivals at
        `rate` jobs/s on the trace's own arrival times."""
        # the one-at-a-time baseline is plain per-job launches (no captured
        # passes); continuous batching records repeating pass shapes
        plain = policy == shsph.SERVE_ONE_AT_A_TIME
        ctx = shsph.Context(0, **kw, graph_batch=0 if plain else 1)
        ctx.serve_start(200e9, max_batch=256, policy=policy,
                        max_batch_particles=args.serve_pass_particles)
        log(f"[served] {label}: {len(jobs_run)} jobs" + ("" if rate is None else f" at {rate:.1f}/s"))
        tk = []
        t0 = time.perf_counter()
        t_first = jobs_run[0]["t"]
        for i, j in enumerate(jobs_run):
            if i and i % 250 == 0:
                st = ctx.serve_stats()
                log(f"[served] {label}: {i} submitted, {st['jobs_done']} done, {st['passes']} passes")
            if rate is not None:
                due = t0 + (j["t"] - t_first) / rate
                while True:
                    d = due - time.perf_counter()
                    if d <= 0:
                        break
                    time.sleep(d if d > 2e-3 else 0)
            tk.append(submit(ctx, j))
        t_end = time.perf_counter() + args.serve_timeout
        while not ctx.serve_wait(5.0):
            st = ctx.serve_stats()
            log(f"[served] {label}: draining, {st['jobs_done']} of {len(jobs_run)} done")
            if time.perf_counter() > t_end:
                raise RuntimeError(f"serving run ({label}) did not finish in {args.serve_timeout} s")
        st = [ctx.poll(t) for t in tk]
        stats = ctx.serve_stats()
        ctx.serve_stop()
        ctx.close()
        errs = {}
        for x in st:
            if x["state"] != "done":
                errs[str(x["error"])] = errs.get(str(x["error"]), 0) + 1
        if errs:
            log(f"[served] {label}: failed jobs by error code {errs}")
        lat = np.array([x["t_done"] - x["t_submit"] for x in st])
        span = max(x["t_done"] for x in st) - min(x["t_submit"] for x in st)
        steps = sum(j["n"] * (j["nsteps"] if j["kind"] == "step" else 1) for j in jobs_run)
        r = {"p50_ms": 1e3 * float(np.percentile(lat, 50)),
             "p99_ms": 1e3 * float(np.percentile(lat, 99)),
             "mean_ms": 1e3 * float(lat.mean()),
             "jobs_done": int(sum(x["state"] == "done" for x in st)),
             "throughput_particle_steps_per_s": steps / span,
             "throughput_jobs_per_s": len(jobs_run) / span, "makespan_s": span,
             "failed_by_error": errs, "passes": stats["passes"],
             "peak_jobs_per_pass": stats["peak_jobs"], "peak_GB": stats["peak_bytes"] / 1e9}
        log(f"[served] {label}: {r['throughput_jobs_per_s']:.1f} jobs/s, "
            f"p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms")
        return r

    policies = (("continuous", shsph.SERVE_CONTINUOUS), ("one_at_a_time", shsph.SERVE_ONE_AT_A_TIME))
    # saturation capacity of each policy: the same burst of the trace's first jobs
    nb = min(args.serve_burst, len(jobs))
    cap = {name: serve(pol, jobs[:nb], None, f"{name} capacity (burst)") for name, pol in policies}
    c1 = cap["one_at_a_time"]["throughput_jobs_per_s"]
    res = {"workload": "served", "jobs_per_rate": args.serve_jobs, "budget_GB": 200,
           "pass_particles_max": args.serve_pass_particles, "templates": 32,
           "eval_fraction": float(np.mean([j["kind"] == "eval" for j in jobs])),
           "capacity_burst_jobs": nb, "capacity": cap,
           "capacity_vs_one_at_a_time": (cap["continuous"]["throughput_particle_steps_per_s"] /
                                         cap["one_at_a_time"]["throughput_particle_steps_per_s"]),
           "rates": []}
    # offered loads relative to the one-at-a-time capacity, below and above it
    for f in args.serve_loads:
        rate = f * c1
        row = {"offered_load_of_one_at_a_time_capacity": f, "rate_jobs_per_s": rate}
        for name, pol in policies:
            row[name] = serve(pol, jobs[:args.serve_jobs], rate, f"{name} at {f:g}x")
        row["throughput_vs_one_at_a_time"] = (row["continuous"]["throughput_particle_steps_per_s"] /
                                              row["one_at_a_time"]["throughput_particle_steps_per_s"])
        row["p99_vs_one_at_a_time"] = row["continuous"]["p99_ms"] / row["one_at_a_time"]["p99_ms"]
        res["rates"].append(row)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sedov256", choices=sorted(WORKLOADS))
    ap.add_argument("--n-red", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=160000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance batch run")
    ap.add_argument("--no-lattice", action="store_true", help="skip the 128^3 lattice run")
    ap.add_argument("--no-served", action="store_true", help="skip the serving run")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the FP64 line, the 30-bit tree build and the M6 line")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--serve-jobs", type=int, default=600, help="jobs per offered rate")
    ap.add_argument("--serve-burst", type=int, default=300,
                    help="jobs submitted at once to measure each policy's capacity")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 1.0, 2.0, 4.0],
                    help="offered loads as multiples of the one-at-a-time capacity")
    ap.add_argument("--serve-pass-particles", type=int, default=1 << 25,
                    help="particles in one serving pass (bounds working memory and pass time)")
    ap.add_argument("--serve-timeout", type=float, default=300.0,
                    help="give up a serving run that has not drained after this many seconds")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against known bytes) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the sharded design is described, "
              "not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.calibrate_copy > 0:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb, "launches": 5}), flush=True)
        return
    import paper_2503_09713_amd as shsph

    log(f"[bench] generating {args.workload}")
    p = make_input(args.workload)
    T = p.x.dtype.itemsize
    log(f"[bench] {p.n} particles, uploading")
    ps = shsph.ParticleSet.from_particles(p)
    ctx = shsph.Context(0, n_red=args.n_red)
    torch.cuda.synchronize()
    log("[bench] initial tree, density, force")
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    for i in range(args.warmup):
        ctx.step(ps, 0.0)
        log(f"[bench] warmup step {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.step(ps, 0.0)
        if (i + 1) % 10 == 0:
            log(f"[bench] step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = ctx.stage_times()
    work = ctx.work()
    ctx.set_profiling(False)
    info = ctx.get_info()
    ms_per_step = 1e3 * elapsed / args.steps
    value = p.n * args.steps / elapsed

    # dominant stage (largest time per step) and its roofline.  The bound is
    # HBM bandwidth: achieved = the stage's algorithmic bytes per particle
    # (STAGE_BYTES) times the particles one launch processes, over the live
    # average launch time (HIP events on the library's stream)
    cand = {k: v for k, v in stages.items() if k in STAGE_BYTES and v[1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    avg_ms = cand[dom][0] / cand[dom][1]
    bpp = stage_bytes_pp(dom, T)
    by = bpp * p.n
    hbm = by / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(hbm / HBM_PEAK_GBS, 4),
            "traffic": traffic_for(dom, args.workload),
            "avg_launch_ms": round(avg_ms, 4), "bytes_per_particle": bpp,
            "particles_per_launch": p.n, "bytes_per_launch": int(by),
            "launches_per_step": round(cand[dom][1] / args.steps, 3),
            "valu_issue": valu_issue_for(dom, args.workload, avg_ms)}
    # whole step: one launch of every stage per step at its algorithmic bytes
    step_bytes = sum(stage_bytes_pp(k, T) for k in STAGE_BYTES) * p.n

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if T == 4 else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "particles": p.n, "kernel": "M4", "hfact": 1.2,
                   "n_red": args.n_red, "dt": "cfl", "periodic": p.periodic,
                   "neighbours_per_particle": info["n_neigh"] / p.n,
                   "leaves": info["n_leaf"],
                   "cache_capacity_entries": info["cache_capacity"]},
        "roofline": roof,
        "step_hbm": {"algorithmic_bytes_per_step": int(step_bytes),
                     "GBs": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                     "frac_of_8TBs": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "work_per_step": {k: v / args.steps for k, v in work.items()},
        # density passes over the cache per step (Newton evaluations, cache
        # rebuild re-runs included) and the largest per-particle iteration count
        "newton": {"passes_per_step": round(work["density_pair_evals"] / args.steps / max(info["n_neigh"], 1), 3),
                   "max_iterations_last_step": info["max_iter_seen"]},
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
    }
    host = ps.host("x", "y", "z", "vx", "vy", "vz", "u", "h") if not args.no_cpu_baseline else None
    ctx.close()
    del ps
    torch.cuda.empty_cache()
    if not args.no_lattice:
        out["uniform128"] = run_lattice(args, shsph, torch)
        torch.cuda.empty_cache()
    if not args.no_extra:
        out["fp64"] = run_f64(args, shsph, torch)
        torch.cuda.empty_cache()
        out["tree_build"] = run_tree_build_key_bits(args, shsph, torch)
        torch.cuda.empty_cache()
        out["m6"] = run_m6(args, shsph, torch)
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = run_batched(args, shsph, torch)
        torch.cuda.empty_cache()
    if not args.no_served:
        out["served"] = run_served(args, shsph, torch, out.get("batched", {}).get("autotuned"))
    if host is not None:
        out["cpu_baseline"] = cpu_baseline(host, p, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
