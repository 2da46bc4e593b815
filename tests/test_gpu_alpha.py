"""The shock-detection switch (App. G, Shock detection) on the GPU against the
oracle: per-particle alpha read by the force, and evolved by the step from
v*, grad v* and grad a^n (implicit update of Eq. evolalphaanalytic)."""
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


def _converging(p, seed):
    """Random velocities plus a converging flow towards the box centre, so
    that the detector fires in the middle and alpha decays elsewhere."""
    rng = np.random.default_rng(seed)
    T = p.x.dtype
    for k, c in (("vx", p.x), ("vy", p.y), ("vz", p.z)):
        r = c.astype(np.float64) - 0.5
        setattr(p, k, (-0.8 * r * np.exp(-(r / 0.25) ** 2) + 0.03 * rng.standard_normal(p.n)).astype(T))
    p.u = (p.u * (1 + 0.2 * rng.uniform(-1, 1, p.n))).astype(T)
    return p


@pytest.mark.parametrize("T", [np.float32, np.float64])
def test_force_with_per_particle_alpha(torch_cuda, T):
    _say(f"[alpha] force with per-particle alpha, {np.dtype(T).name}")
    p = _converging(gen.lattice(14, 91, dtype=T), 1)
    alpha = np.random.default_rng(2).uniform(0.0, 1.0, p.n).astype(T)
    ctx = shsph.Context(0, eps_h=1e-6 if T == np.float32 else 1e-12)
    ps = shsph.ParticleSet.from_particles(p, alpha=alpha)
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    g = {k: v.astype(np.float64) for k, v in ps.host("h", "omega", "ax", "ay", "az", "dudt").items()}
    rho_g = p.mass * (1.2 / g["h"]) ** 3
    ref = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, g["h"], rho_g, g["omega"], p.lo, p.hi,
                       True, p.mass, alpha_arr=alpha)
    ea, eu = parity_util.force_err(g, ref)
    tol = 1e-4 if T == np.float32 else 1e-9
    assert ea.max() <= tol and eu.max() <= tol, (ea.max(), eu.max())
    # and it differs from the constant-alpha force by far more than the bar
    ref1 = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, g["h"], rho_g, g["omega"], p.lo,
                        p.hi, True, p.mass)
    assert parity_util.force_err(g, ref1)[1].max() > 100 * tol
    ctx.close()


@pytest.mark.parametrize("T", [np.float32, np.float64])
def test_step_with_alpha_switch_vs_oracle(torch_cuda, T):
    _say(f"[alpha] two steps with the switch, {np.dtype(T).name}")
    p = _converging(gen.lattice(14, 92, dtype=T), 3)
    alpha0 = np.random.default_rng(4).uniform(0.0, 1.0, p.n).astype(T)
    eps_h = 1e-6 if T == np.float32 else 1e-12
    ctx = shsph.Context(0, eps_h=eps_h, alpha_switch=1)
    ps = shsph.ParticleSet.from_particles(p, alpha=alpha0)
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    s0 = ps.host()
    dt = 0.5 * ctx.get_info()["dt_cfl"]
    fired = 0
    for it in range(2):
        st = {k: s0[k] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az",
                                 "dudt", "alpha")}
        ref = oracle.step(st, p.lo, p.hi, True, p.mass, dt, alpha_switch=True)
        ctx.step(ps, dt)
        s1 = ps.host()
        j = parity_util.map_to_start(s0["pid"], s1["pid"])
        # alpha^{n+1}: a smooth function of the step's sums (FP32: 1e-4 absolute)
        err = np.abs(s1["alpha"].astype(np.float64) - ref["alpha"][j])
        assert err.max() <= (1e-4 if T == np.float32 else 1e-9), err.max()
        parity_util.check_step_vs_oracle(s0, s1, ref, ctx.get_info(), p, dt, T)
        fired += int((ref["alpha"] > st["alpha"].astype(np.float64) + 1e-3).sum())
        s0 = s1
    assert fired > 0, "the detector never raised alpha"
    ctx.close()
