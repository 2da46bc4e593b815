"""Pooled instances, batched passes and the serving loop on the GPU.

A batched pass must give every instance exactly what it gets alone (the
kernels never mix instances, and h iterations that settled are not re-run
when another instance forces a cache rebuild), so batch-vs-alone and
serving-mix-vs-alone comparisons are bit-exact.  Batched results are also
checked against the CPU oracle at the same tolerances as the plain path."""
import sys

import numpy as np
import pytest

import gen
import oracle
import parity_util

pytestmark = pytest.mark.gpu

shsph = pytest.importorskip("paper_2503_09713_amd")

STATE = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az", "dudt", "rho", "omega", "pid")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _random_state(p, seed, vscale=0.1, uvar=0.3):
    rng = np.random.default_rng(seed)
    T = p.x.dtype
    p.vx = (rng.standard_normal(p.n) * vscale).astype(T)
    p.vy = (rng.standard_normal(p.n) * vscale).astype(T)
    p.vz = (rng.standard_normal(p.n) * vscale).astype(T)
    p.u = (p.u * (1 + uvar * rng.uniform(-1, 1, p.n))).astype(T)
    return p


def _mix():
    """Uneven FP32 instances: periodic lattices, isolated Plummer spheres, a
    Sedov blast, one smaller than a group of 256."""
    return [
        _random_state(gen.lattice(8, 31, dtype=np.float32), 1),
        _random_state(gen.plummer(3000, 32, dtype=np.float32), 2, vscale=0.3),
        gen.sedov(10, 33, dtype=np.float32),
        _random_state(gen.lattice(6, 34, dtype=np.float32), 3, vscale=0.05),
        _random_state(gen.lattice(12, 35, dtype=np.float32), 4),
        _random_state(gen.plummer(1500, 36, dtype=np.float32), 5, vscale=0.1),
    ]


def _read(ctx, h, p):
    out = shsph.ParticleSet.from_particles(p)
    ctx.instance_read(h, out)
    return out.host(*STATE)


def _same(a, b, what):
    for k in STATE:
        assert a[k].dtype == b[k].dtype
        assert np.array_equal(a[k], b[k], equal_nan=True), f"{what}: field {k} differs"


def _box(p):
    if p.periodic:
        return p.lo, p.hi
    return ((float(p.x.min()), float(p.y.min()), float(p.z.min())),
            (float(p.x.max()), float(p.y.max()), float(p.z.max())))


def test_batch_step_equals_alone(torch_cuda):
    _say("[batch] 6 uneven instances: 3 CFL steps batched vs each alone (bit-exact)")
    ps = _mix()
    ctx = shsph.Context(0)
    hs = [ctx.instance_create(shsph.ParticleSet.from_particles(p)) for p in ps]
    used_b = []
    for s in range(3):
        order = hs if s != 1 else hs[::-1]          # the order within a pass is irrelevant
        u = ctx.step_batch(order)
        used_b.append(dict(zip(order, u)))
    got = [_read(ctx, h, p) for h, p in zip(hs, ps)]
    usage = ctx.pool_usage()
    assert usage["instances"] == len(ps) and usage["particles"] == sum(p.n for p in ps)
    ctx.close()
    alone = shsph.Context(0)
    pad = alone.instance_create(shsph.ParticleSet.from_particles(ps[2]))   # shifts the pool offsets
    for k, p in enumerate(ps):
        h = alone.instance_create(shsph.ParticleSet.from_particles(p))
        for s in range(3):
            u = alone.step_batch([h])
            assert u[0] == used_b[s][hs[k]], (k, s)
        _same(got[k], _read(alone, h, p), f"instance {k}")
        alone.instance_destroy(h)
    alone.instance_destroy(pad)
    alone.close()


def test_eval_batch_vs_oracle(torch_cuda):
    _say("[batch] eval pass of 3 instances vs oracle density / force / CFL")
    ps = [_random_state(gen.lattice(16, gen.SEEDS["tiny"], dtype=np.float32), 3),
          _random_state(gen.plummer(3000, 4, dtype=np.float32), 4, vscale=0.3),
          gen.sedov(12, 3, dtype=np.float32)]
    ctx = shsph.Context(0)
    hs = [ctx.instance_create(shsph.ParticleSet.from_particles(p)) for p in ps]
    ctx.eval_batch(hs)
    for p, h in zip(ps, hs):
        g = _read(ctx, h, p)
        j = g["pid"].astype(np.int64)          # pooled state is in Morton order
        lo, hi = _box(p)
        # positions, velocities and u are unchanged by an evaluation
        for k in ("x", "y", "z", "vx", "vy", "vz", "u"):
            assert np.array_equal(g[k], getattr(p, k)[j]), k
        hr, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, lo, hi, p.periodic, p.mass)
        ok = fl[j] == 0
        assert np.abs(g["h"][ok] / hr[j][ok] - 1).max() <= 1e-5
        hg = g["h"].astype(np.float64)
        rho_g = p.mass * (1.2 / hg) ** 3
        ref = oracle.force(p.x[j], p.y[j], p.z[j], p.vx[j], p.vy[j], p.vz[j], p.u[j], hg, rho_g,
                           g["omega"].astype(np.float64), lo, hi, p.periodic, p.mass)
        sa = np.maximum(ref["scale_a"], 1e-300)
        su = np.maximum(ref["scale_u"], 1e-300)
        ea = np.max(np.sqrt((g["ax"] - ref["ax"]) ** 2 + (g["ay"] - ref["ay"]) ** 2 +
                            (g["az"] - ref["az"]) ** 2) / sa)
        eu = np.max(np.abs(g["dudt"] - ref["dudt"]) / su)
        assert ea <= 1e-4 and eu <= 1e-4, (ea, eu)
        dt_ref = oracle.cfl(hg, ref["vsig"], ref["ax"], ref["ay"], ref["az"])
        assert abs(ctx.instance_info(h)["dt_cfl"] / dt_ref - 1) < 1e-4
    ctx.close()


def test_step_batch_vs_oracle(torch_cuda):
    _say("[batch] one fixed-dt step of 2 instances vs oracle step")
    ps = [_random_state(gen.lattice(12, 21, dtype=np.float32), 5, vscale=0.05, uvar=0.2),
          _random_state(gen.lattice(10, 22, dtype=np.float32), 6, vscale=0.05, uvar=0.2)]
    ps[1].vy = (ps[1].vy - 4.0).astype(np.float32)      # a drift across the periodic faces
    ctx = shsph.Context(0)
    hs = [ctx.instance_create(shsph.ParticleSet.from_particles(p)) for p in ps]
    ctx.eval_batch(hs)
    s0 = [_read(ctx, h, p) for h, p in zip(hs, ps)]
    dt = 0.5 * min(ctx.instance_info(h)["dt_cfl"] for h in hs)
    used = ctx.step_batch(hs, dt)
    assert used == [dt, dt]
    for p, h, a in zip(ps, hs, s0):
        st = {k: a[k] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az", "dudt")}
        ref = oracle.step(st, p.lo, p.hi, True, p.mass, dt)
        b = _read(ctx, h, p)
        parity_util.check_step_vs_oracle(a, b, ref, ctx.instance_info(h), p, dt, np.float32)
    ctx.close()


def _alone(p, kind, nsteps):
    c = shsph.Context(0)
    h = c.instance_create(shsph.ParticleSet.from_particles(p))
    if kind == shsph.JOB_EVAL:
        c.eval_batch([h])
    else:
        for _ in range(nsteps):
            c.step_batch([h])
    r = _read(c, h, p)
    c.close()
    return r


def test_serve_mix_equals_alone(torch_cuda):
    _say("[serve] 8 jobs (STEP 1-3 steps, EVAL) served together vs each alone (bit-exact)")
    ps = _mix() + [_random_state(gen.lattice(9, 37, dtype=np.float32), 7),
                   _random_state(gen.plummer(2200, 38, dtype=np.float32), 8, vscale=0.2)]
    jobs = [(shsph.JOB_STEP, 3), (shsph.JOB_EVAL, 1), (shsph.JOB_STEP, 1), (shsph.JOB_STEP, 2),
            (shsph.JOB_EVAL, 1), (shsph.JOB_STEP, 3), (shsph.JOB_STEP, 2), (shsph.JOB_STEP, 1)]
    ctx = shsph.Context(0)
    ctx.serve_start(budget_bytes=8e9, max_batch=16)
    sets = [shsph.ParticleSet.from_particles(p) for p in ps]
    # half the jobs first; the rest arrive once the loop has run a pass, so
    # they are admitted between passes while the first ones are running
    tk = [ctx.submit(init=s, kind=k, nsteps=n) for s, (k, n) in zip(sets[:4], jobs[:4])]
    import time
    t_end = time.time() + 60.0
    while ctx.serve_stats()["passes"] < 1 and time.time() < t_end:
        time.sleep(1e-4)
    passes_before = ctx.serve_stats()["passes"]
    assert passes_before >= 1
    tk += [ctx.submit(init=s, kind=k, nsteps=n) for s, (k, n) in zip(sets[4:], jobs[4:])]
    ctx.serve_drain(120.0)
    st = [ctx.poll(t) for t in tk]
    stats = ctx.serve_stats()
    got = [_read(ctx, s["handle"], p) for s, p in zip(st, ps)]
    overlap = sum(1 for a in st[4:] for b in st[:4] if a["t_start"] < b["t_done"])
    _say(f"[serve] late jobs admitted while an early one ran: {overlap} pairs")
    ctx.serve_stop()
    ctx.close()
    assert stats["jobs_done"] == len(jobs) and stats["jobs_failed"] == 0
    assert stats["peak_jobs"] > 1, "jobs were not batched"
    for s, (k, n) in zip(st, jobs):
        assert s["state"] == "done" and s["error"] == 0
        assert s["steps_done"] == (0 if k == shsph.JOB_EVAL else n)
        assert s["t_submit"] <= s["t_start"] <= s["t_done"]
    for k, (p, (kind, n)) in enumerate(zip(ps, jobs)):
        _same(got[k], _alone(p, kind, n), f"job {k}")


def test_serve_budget_policy_and_errors(torch_cuda):
    _say("[serve] budget admission, one-at-a-time policy, error codes")
    ps = [gen.lattice(8, 41 + k, dtype=np.float32) for k in range(4)]
    ctx = shsph.Context(0)
    with pytest.raises(shsph.ShsphError) as e:            # not serving yet
        ctx.submit(init=shsph.ParticleSet.from_particles(ps[0]))
    assert e.value.code == shsph.SHSPH_ESTATE
    st_b, wk_b = ctx.footprint(ps[0].n)
    # room for one job at a time (its instance + work), released at the end
    ctx.serve_start(budget_bytes=1.5 * (st_b + wk_b), max_batch=8)
    sets = [shsph.ParticleSet.from_particles(p) for p in ps]
    tk = [ctx.submit(init=s, nsteps=2, release=True) for s in sets]
    big = shsph.ParticleSet.from_particles(gen.lattice(16, 1, dtype=np.float32))
    with pytest.raises(shsph.ShsphError) as e:            # can never fit
        ctx.submit(init=big)
    assert e.value.code == shsph.SHSPH_ENOMEM
    with pytest.raises(shsph.ShsphError) as e:            # unknown instance
        ctx.submit(handle=12345)
    assert e.value.code == shsph.SHSPH_EINVAL
    ctx.serve_drain(120.0)
    st = [ctx.poll(t) for t in tk]
    stats = ctx.serve_stats()
    assert all(s["state"] == "done" and s["handle"] == 0 for s in st)
    assert stats["peak_jobs"] == 1 and stats["peak_bytes"] <= 1.5 * (st_b + wk_b)
    for a, b in zip(st, st[1:]):
        assert b["t_start"] >= a["t_done"]                 # admitted only after the previous left
    assert ctx.pool_usage()["instances"] == 0
    ctx.serve_stop()
    # one-at-a-time policy with a large budget: still a single job per pass
    ctx.serve_start(budget_bytes=8e9, max_batch=8, policy=shsph.SERVE_ONE_AT_A_TIME)
    tk = [ctx.submit(init=s, nsteps=1, release=True) for s in sets]
    ctx.serve_drain(120.0)
    assert ctx.serve_stats()["peak_jobs"] == 1
    assert all(ctx.poll(t)["state"] == "done" for t in tk)
    ctx.serve_stop()
    ctx.close()


def test_batch_flags_instance_that_does_not_converge(torch_cuda):
    _say("[batch] no cache rebuilds allowed; one instance starts with h at half its root")
    good = _random_state(gen.lattice(8, 31, dtype=np.float32), 1)
    bad = gen.plummer(3000, 34, dtype=np.float32)
    bad.h = (bad.h * 0.5).astype(np.float32)       # must grow past chi h_cache
    ctx = shsph.Context(0, max_restarts=0)
    hg = ctx.instance_create(shsph.ParticleSet.from_particles(good))
    hb = ctx.instance_create(shsph.ParticleSet.from_particles(bad))
    with pytest.raises(shsph.ShsphError) as e:
        ctx.eval_batch([hg, hb])
    assert e.value.code == shsph.SHSPH_ENOCONV
    assert ctx.instance_info(hb)["n_noconv"] > 0
    assert ctx.instance_info(hg)["n_noconv"] == 0
    got = _read(ctx, hg, good)
    ctx.close()
    alone = shsph.Context(0, max_restarts=0)
    h = alone.instance_create(shsph.ParticleSet.from_particles(good))
    alone.eval_batch([h])
    _same(got, _read(alone, h, good), "converged instance next to a failing one")
    alone.close()


def test_leaf_size_and_walk_do_not_change_results(torch_cuda):
    _say("[batch] leaf size and stage-2 walk: bit-exact; autotuner")
    ps = _mix()
    got = []
    for kw in (dict(n_red=2, stage2_mode=1), dict(n_red=4, stage2_mode=2),
               dict(n_red=3, stage2_mode=0)):
        ctx = shsph.Context(0, **kw)
        hs = [ctx.instance_create(shsph.ParticleSet.from_particles(p)) for p in ps]
        ctx.step_batch(hs)
        ctx.step_batch(hs)
        got.append([_read(ctx, h, p) for h, p in zip(hs, ps)])
        ctx.close()
    for k in range(len(ps)):
        _same(got[0][k], got[1][k], f"instance {k}")
        _same(got[0][k], got[2][k], f"instance {k}")
    ctx = shsph.Context(0)
    hs = [ctx.instance_create(shsph.ParticleSet.from_particles(p)) for p in ps]
    t = ctx.autotune(hs)
    assert t["n_red"] in (2, 3, 4) and t["stage2_mode"] in (0, 1, 2) and t["pass_ms"] > 0
    assert t["force_split"] in (1, 2)
    ctx.step_batch(hs)
    ctx.close()


def test_instance_errors(torch_cuda):
    _say("[batch] instance error codes")
    ctx = shsph.Context(0)
    p32 = gen.lattice(8, 1, dtype=np.float32)
    h = ctx.instance_create(shsph.ParticleSet.from_particles(p32))
    with pytest.raises(shsph.ShsphError) as e:            # pool holds FP32 instances
        ctx.instance_create(shsph.ParticleSet.from_particles(gen.lattice(8, 1, dtype=np.float64)))
    assert e.value.code == shsph.SHSPH_EINVAL
    with pytest.raises(shsph.ShsphError) as e:
        ctx.step_batch([h, h])
    assert e.value.code == shsph.SHSPH_EINVAL
    with pytest.raises(shsph.ShsphError) as e:
        ctx.instance_read(h, shsph.ParticleSet.from_particles(gen.lattice(9, 1, dtype=np.float32)))
    assert e.value.code == shsph.SHSPH_EINVAL
    with pytest.raises(shsph.ShsphError) as e:
        ctx.eval_batch([h + 100])
    assert e.value.code == shsph.SHSPH_EINVAL
    ctx.instance_destroy(h)
    with pytest.raises(shsph.ShsphError) as e:
        ctx.instance_destroy(h)
    assert e.value.code == shsph.SHSPH_EINVAL
    # an empty pool may switch dtype
    h64 = ctx.instance_create(shsph.ParticleSet.from_particles(gen.lattice(8, 1, dtype=np.float64)))
    ctx.eval_batch([h64])
    assert ctx.instance_info(h64)["dt_cfl"] > 0
    ctx.close()
