"""Pins of the oracle's physics half (M4 kernel, h/rho root, Omega, force,
du/dt, leapfrog) against closed forms, conservation laws and symmetry."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import gen
import oracle


# ------------------------------------------------------------- kernel ----
def test_m4_normalisation():
    # 3-D normalisation: int W dV = 4 pi C_norm int_0^2 f(q) q^2 dq = 1, C_norm = 1/pi
    val, _ = integrate.quad(lambda q: oracle.m4_f(q) * q * q, 0.0, 2.0, points=[1.0])
    assert abs(4.0 * math.pi * val / math.pi - 1.0) < 1e-12


def test_m4_shape_and_continuity():
    assert oracle.m4_f(0.0) == 1.0 and oracle.m4_f(2.0) == 0.0 and oracle.m4_f(2.5) == 0.0
    for q0 in (1.0, 2.0):
        e = 1e-9
        assert abs(oracle.m4_f(q0 - e) - oracle.m4_f(q0 + e)) < 1e-8
        assert abs(oracle.m4_df(q0 - e) - oracle.m4_df(q0 + e)) < 1e-8
    # f' is the derivative of f
    for q in np.linspace(0.05, 1.95, 39):
        fd = (oracle.m4_f(q + 1e-6) - oracle.m4_f(q - 1e-6)) / 2e-6
        assert abs(fd - oracle.m4_df(q)) < 1e-7


# -------------------------------------------- lattice closed form (h) ----
def _lattice_sum(eta, fn):
    R = int(np.ceil(2 * eta)) + 1
    r = np.arange(-R, R + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    q = np.sqrt(X ** 2 + Y ** 2 + Z ** 2).ravel() / eta
    return sum(fn(float(v)) for v in q if v < 2.0)


def _lattice_fixed_point():
    """Unjittered cubic lattice, h = eta*dx, m = rho0 dx^3: rho_sum/rho0 =
    S(eta)/(pi eta^3) with S = sum over integer offsets of f(|n|/eta); the
    fixed point of rho_sum = m (hfact/h)^3 is S(eta) = pi hfact^3."""
    g = lambda eta: _lattice_sum(eta, oracle.m4_f) - math.pi * 1.2 ** 3
    eta = optimize.brentq(g, 1.0, 1.5, xtol=1e-15)
    return eta


def test_lattice_fixed_point_closed_form():
    eta = _lattice_fixed_point()
    p = gen.lattice(16, 1, dtype=np.float64, jitter=0.0)
    h, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    dx = 1.0 / 16
    assert fl.max() == 0
    assert np.allclose(h / dx, eta, rtol=1e-12, atol=0)
    assert np.allclose(rho, (1.2 / eta) ** 3, rtol=1e-12, atol=0)
    # Omega = 1 + h/(3 rho) sum m dW/dh, with dW/dh = -(3f + q f')/(pi h^4)
    s = _lattice_sum(eta, lambda q: -(3 * oracle.m4_f(q) + q * oracle.m4_df(q)))
    om_ref = 1.0 + s / (3.0 * math.pi * 1.2 ** 3)
    assert np.allclose(om, om_ref, rtol=1e-12, atol=0)
    # the values quoted for this lattice
    assert abs(eta - 1.199670052480077) < 1e-12
    assert abs(om_ref - 0.980895317192107) < 1e-12


def test_h_rho_relation_holds_on_jittered_lattice():
    p = gen.lattice(12, 3, dtype=np.float64)
    h, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    assert fl.max() == 0
    s, _ = oracle.density_sum(p.x, p.y, p.z, h, p.lo, p.hi, True, p.mass)
    assert np.abs(s - rho).max() / rho.max() < 1e-12
    assert abs(rho.mean() - 1.0) < 2e-2


def test_density_plummer_converges():
    p = gen.plummer(2000, 7, dtype=np.float64)
    h, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, False, p.mass)
    assert fl.max() == 0
    s, _ = oracle.density_sum(p.x, p.y, p.z, h, p.lo, p.hi, False, p.mass)
    assert np.abs(s / rho - 1).max() < 1e-11


# -------------------------------------------------------------- force ----
def _state(p, rng, vscale=0.1, uvar=0.3):
    v = [p.vx + vscale * rng.standard_normal(p.n) for _ in range(3)]
    u = p.u * (1.0 + uvar * rng.uniform(-1, 1, p.n))
    h, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, p.periodic, p.mass)
    return v, u, h, rho, om


@pytest.mark.parametrize("family", ["lattice", "plummer"])
def test_momentum_and_energy_conservation(family):
    rng = np.random.default_rng(2)
    p = gen.lattice(10, 5, dtype=np.float64) if family == "lattice" else gen.plummer(1500, 5, dtype=np.float64)
    v, u, h, rho, om = _state(p, rng)
    f = oracle.force(p.x, p.y, p.z, *v, u, h, rho, om, p.lo, p.hi, p.periodic, p.mass)
    m = p.mass
    S = (m * f["scale_a"]).sum()
    for c in ("ax", "ay", "az"):
        assert abs(m * f[c].sum()) < 1e-13 * S
    # d/dt sum m (v^2/2 + u) = sum m (v.a + du/dt) = 0: pins the minus sign of
    # dv/dt and q inside the du/dt sum
    e = m * (v[0] * f["ax"] + v[1] * f["ay"] + v[2] * f["az"] + f["dudt"])
    scale = m * (np.abs(v[0] * f["ax"]) + np.abs(v[1] * f["ay"]) + np.abs(v[2] * f["az"]) + f["scale_u"])
    assert abs(e.sum()) < 1e-12 * scale.sum()
    if family == "plummer":   # central pair forces conserve angular momentum
        L = np.cross(np.stack([p.x, p.y, p.z], 1), np.stack([f["ax"], f["ay"], f["az"]], 1)) * m
        assert np.abs(L.sum(0)).max() < 1e-12 * S


def test_conductivity_conserves_energy_alone():
    # v = 0: only the conductivity term moves u, and it moves it pairwise
    rng = np.random.default_rng(4)
    p = gen.lattice(10, 6, dtype=np.float64)
    u = 1.0 + rng.uniform(0, 1, p.n)
    h, rho, om, _ = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    f = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, u, h, rho, om, p.lo, p.hi, True, p.mass)
    assert abs((p.mass * f["dudt"]).sum()) < 1e-12 * (p.mass * f["scale_u"]).sum()
    # heat flows from hot to cold: the hottest particle cools
    assert f["dudt"][np.argmax(u)] < 0
    f0 = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, u, h, rho, om, p.lo, p.hi, True,
                      p.mass, beta_u=0.0)
    assert np.abs(f0["dudt"]).max() == 0.0


def test_lattice_symmetry_zero_force():
    p = gen.lattice(12, 1, dtype=np.float64, jitter=0.0)
    h, rho, om, _ = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    f = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, h, rho, om, p.lo, p.hi, True, p.mass)
    for c in ("ax", "ay", "az"):
        assert np.abs(f[c]).max() < 1e-12 * f["scale_a"].max()
    assert np.abs(f["dudt"]).max() == 0.0


def test_compression_heats_and_galilean_invariance():
    p = gen.lattice(10, 8, dtype=np.float64)
    h, rho, om, _ = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    # converging flow towards the box centre, away from the periodic seam
    c = 0.05
    vx, vy, vz = -c * (p.x - 0.5), -c * (p.y - 0.5), -c * (p.z - 0.5)
    f = oracle.force(p.x, p.y, p.z, vx, vy, vz, p.u, h, rho, om, p.lo, p.hi, True, p.mass)
    r = np.sqrt((p.x - .5) ** 2 + (p.y - .5) ** 2 + (p.z - .5) ** 2)
    inner = r < 0.3
    assert (f["dudt"][inner] > 0).all()
    g = oracle.force(p.x, p.y, p.z, vx + 0.7, vy - 0.2, vz + 0.1, p.u, h, rho, om, p.lo,
                     p.hi, True, p.mass)
    for k in ("ax", "ay", "az"):
        assert np.abs(g[k] - f[k]).max() < 1e-12 * f["scale_a"].max()
    assert np.abs(g["dudt"] - f["dudt"]).max() < 1e-12 * f["scale_u"].max()


def test_sedov_pushes_outwards():
    p = gen.sedov(16, 3, dtype=np.float64)
    h, rho, om, _ = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    f = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, h, rho, om, p.lo, p.hi, True, p.mass)
    d = np.stack([p.x - .5, p.y - .5, p.z - .5], 1)
    a = np.stack([f["ax"], f["ay"], f["az"]], 1)
    hot = p.u > 1.0
    assert hot.sum() == 56
    assert ((d * a).sum(1)[hot] > 0).all()


def test_force_brute_force_small():
    # direct double loop over all pairs, written from the equations, on 64
    # particles: the oracle's cell search must not miss any pair
    rng = np.random.default_rng(12)
    p = gen.plummer(64, 12, dtype=np.float64)
    v, u, h, rho, om = _state(p, rng, vscale=0.3)
    f = oracle.force(p.x, p.y, p.z, *v, u, h, rho, om, p.lo, p.hi, False, p.mass)
    g, a = 5.0 / 3.0, np.zeros((p.n, 3))
    P = (g - 1) * rho * u
    cs = np.sqrt(g * P / rho)
    X = np.stack([p.x, p.y, p.z], 1)
    V = np.stack(v, 1)
    for i in range(p.n):
        for j in range(p.n):
            d = X[i] - X[j]
            r = np.linalg.norm(d)
            if i == j or r >= 2 * max(h[i], h[j]):
                continue
            rh = d / r
            w = (V[i] - V[j]) @ rh
            qa = -0.5 * rho[i] * (cs[i] + 2 * abs(w)) * w if w < 0 else 0
            qb = -0.5 * rho[j] * (cs[j] + 2 * abs(w)) * w if w < 0 else 0
            Fa = oracle.m4_df(r / h[i]) / (math.pi * h[i] ** 4)
            Fb = oracle.m4_df(r / h[j]) / (math.pi * h[j] ** 4)
            a[i] -= p.mass * ((P[i] + qa) / (rho[i] ** 2 * om[i]) * Fa
                              + (P[j] + qb) / (rho[j] ** 2 * om[j]) * Fb) * rh
    ref = np.stack([f["ax"], f["ay"], f["az"]], 1)
    assert np.abs(ref - a).max() < 1e-12 * np.abs(a).max()


def test_cfl_closed_form_at_rest():
    # unjittered lattice at rest, uniform u: a = 0 and the signal speed is the
    # sound speed, so dt = C_cour h / c_s with c_s = sqrt(gamma (gamma-1) u)
    p = gen.lattice(10, 1, dtype=np.float64, jitter=0.0)
    p.u = np.full(p.n, 2.5)
    h, rho, om, _ = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    f = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, h, rho, om, p.lo, p.hi, True, p.mass)
    g = 5.0 / 3.0
    cs = math.sqrt(g * (g - 1) * 2.5)
    assert np.allclose(f["vsig"], cs, rtol=1e-14)
    dt = oracle.cfl(h, f["vsig"], f["ax"], f["ay"], f["az"])
    assert abs(dt - 0.3 * h.min() / cs) < 1e-12 * dt


# ---------------------------------------------------------------- step ----
def test_kdk_step_conserves_momentum_and_is_reversible():
    rng = np.random.default_rng(9)
    p = gen.lattice(10, 9, dtype=np.float64)
    v, u, h, rho, om = _state(p, rng, vscale=0.05, uvar=0.2)
    f = oracle.force(p.x, p.y, p.z, *v, u, h, rho, om, p.lo, p.hi, True, p.mass)
    st = dict(x=p.x, y=p.y, z=p.z, vx=v[0], vy=v[1], vz=v[2], u=u, h=h,
              ax=f["ax"], ay=f["ay"], az=f["az"], dudt=f["dudt"])
    dt = 0.2 * oracle.cfl(h, f["vsig"], f["ax"], f["ay"], f["az"])
    p0 = np.array([v[0].sum(), v[1].sum(), v[2].sum()]) * p.mass
    e0 = (0.5 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) + u).sum() * p.mass
    s = st
    for _ in range(3):
        s = oracle.step(s, p.lo, p.hi, True, p.mass, dt)
        assert ((s["x"] >= 0) & (s["x"] < 1)).all()
    p1 = np.array([s["vx"].sum(), s["vy"].sum(), s["vz"].sum()]) * p.mass
    e1 = (0.5 * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2) + s["u"]).sum() * p.mass
    assert np.abs(p1 - p0).max() < 1e-14
    assert abs(e1 - e0) / e0 < 1e-5
    # corrector size relative to the rms velocity stays small (App. H.1)
    assert s["diag"][0] / math.sqrt(s["diag"][2] / p.n) < 1e-2
