"""The persistent fused density + force launch (fused_density_force = 1)
against the separate kernels with one thread per particle in the force
(force_split = 1): the same code per group, so every output is bit-identical,
for the plain step (CFL steps from a random state, FP32 and FP64), a step
whose h leaves chi h_cache (the fused launch skips its force and the separate
passes take over after the cache rebuild), and a batched pass of uneven
instances.  The fused step is also checked against the oracle's step."""
import sys

import numpy as np
import pytest

import gen
import oracle
import parity_util

pytestmark = pytest.mark.gpu

shsph = pytest.importorskip("paper_2503_09713_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _state(p, seed, vscale=0.1, uvar=0.3):
    rng = np.random.default_rng(seed)
    T = p.x.dtype
    for k in ("vx", "vy", "vz"):
        setattr(p, k, (rng.standard_normal(p.n) * vscale).astype(T))
    p.u = (p.u * (1 + uvar * rng.uniform(-1, 1, p.n))).astype(T)
    return p


def _run(p, steps, **kw):
    ctx = shsph.Context(0, **kw)
    ps = shsph.ParticleSet.from_particles(p)
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    infos = []
    for _ in range(steps):
        ctx.step(ps, 0.0)
        infos.append(ctx.get_info())
    out = ps.host()
    ctx.close()
    return out, infos


@pytest.mark.parametrize("T", [np.float32, np.float64])
def test_fused_step_equals_separate(torch_cuda, T):
    _say(f"[fused] plain CFL steps, {np.dtype(T).name}")
    p = _state(gen.lattice(24, 91, dtype=T), 4)
    eps = 1e-6 if T == np.float32 else 1e-12
    a, ia = _run(p, 3, eps_h=eps, force_split=1, fused_density_force=0)
    b, ib = _run(p, 3, eps_h=eps, force_split=1, fused_density_force=1)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    for x, y in zip(ia, ib):
        assert x["dt_cfl"] == y["dt_cfl"] and x["restarts"] == y["restarts"]


def test_fused_step_with_cache_rebuild(torch_cuda):
    """Smoothing lengths a quarter too small: the first h iteration leaves
    chi h_cache, so the fused launch stops after the density and the step
    finishes through the rebuild and the separate force."""
    _say("[fused] step whose h leaves chi h_cache")
    p = _state(gen.lattice(20, 92, dtype=np.float32), 5)
    out = []
    for fused in (0, 1):
        ctx = shsph.Context(0, force_split=1, fused_density_force=fused)
        ps = shsph.ParticleSet.from_particles(p)
        ctx.build_tree(ps)
        ctx.density(ps)
        ctx.force(ps)
        dt = ctx.get_info()["dt_cfl"]
        h = ps.t["h"]
        h.mul_(0.75)                       # h far below its root: it must grow past chi h
        ctx.step(ps, 0.5 * dt)
        info = ctx.get_info()
        assert info["restarts"] >= 1
        out.append(ps.host())
        ctx.close()
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def test_fused_step_vs_oracle(torch_cuda):
    _say("[fused] step against the oracle")
    T = np.float32
    p = _state(gen.lattice(12, 93, dtype=T), 6, vscale=0.05, uvar=0.2)
    ctx = shsph.Context(0, eps_h=1e-6, force_split=1, fused_density_force=1)
    ps = shsph.ParticleSet.from_particles(p)
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    s0 = ps.host()
    dt = 0.5 * ctx.get_info()["dt_cfl"]
    st = {k: s0[k] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az", "dudt")}
    ref = oracle.step(st, p.lo, p.hi, True, p.mass, dt)
    used = ctx.step(ps, dt, want_dt=True)
    assert used == dt
    s1 = ps.host()
    parity_util.check_step_vs_oracle(s0, s1, ref, ctx.get_info(), p, dt, T)
    ctx.close()


def test_fused_batch_equals_separate(torch_cuda):
    _say("[fused] batched pass of uneven instances")
    insts = [_state(gen.lattice(12, 94, dtype=np.float32), 7),
             _state(gen.plummer(3000, 95, dtype=np.float32), 8, vscale=0.3),
             _state(gen.lattice(17, 96, dtype=np.float32), 9)]
    res = []
    for fused in (0, 1):
        ctx = shsph.Context(0, force_split=1, fused_density_force=fused)
        hs = [ctx.instance_create(shsph.ParticleSet.from_particles(p)) for p in insts]
        for _ in range(2):
            ctx.step_batch(hs)
        got = []
        for h, p in zip(hs, insts):
            o = shsph.ParticleSet.from_particles(p)
            ctx.instance_read(h, o)
            got.append(o.host())
        res.append(got)
        ctx.close()
    for k in range(len(insts)):
        for f in res[0][k]:
            assert np.array_equal(res[0][k][f], res[1][k][f]), (k, f)
