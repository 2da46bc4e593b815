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
    # corrector size relative to the rms velocity stays small (App. G.1)
    assert s["diag"][0] / math.sqrt(s["diag"][2] / p.n) < 1e-2


# ------------------------------------------ exact identities at the root --
# At a self-consistent h (sum_b m W_ab(h_a) = rho_a = m (hfact/h_a)^3) the
# definition of Omega (Eq. sphomega with dh/drho = -h/(3 rho)) reduces to
#     Omega_a = -(1/(3 rho_a)) sum_b m q f'(q) / (pi h_a^3),   q = r_ab/h_a,
# because sum_b m W_ab = rho_a cancels the 1.  Two closed forms follow that
# hold for every particle whose h is the root, on any particle set:
#   * uniform compression v = -c r (+ any constant): the pressure part of
#     du_a/dt (Eq. sphuint) is exactly 3 c P_a / rho_a = -(P/rho) div v;
#   * on a cubic lattice, a linear pressure P = P0 + g x: dv_a/dt is exactly
#     -g/rho x (cubic symmetry makes sum r_x^2 F / r = sum r F / 3).
# A dropped factor (m, rho^2, Omega), a wrong kernel argument (h_b for h_a)
# or a transposed term breaks them.

def _interior(p, h, margin):
    """Particles whose 2h-neighbourhood stays clear of the periodic seam."""
    ok = np.ones(p.n, bool)
    for c in (p.x, p.y, p.z):
        ok &= np.abs(c - 0.5) + margin * h < 0.5
    return ok


@pytest.mark.parametrize("family", ["lattice", "plummer"])
def test_uniform_compression_heats_at_exactly_3cP_over_rho(family):
    if family == "lattice":
        p = gen.lattice(12, 14, dtype=np.float64)
    else:
        p = gen.plummer(2500, 14, dtype=np.float64)
    h, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, p.periodic, p.mass)
    assert fl.max() == 0
    c, g = 0.3, 5.0 / 3.0
    u = 1.0 + 0.5 * np.sin(7 * p.x) * np.cos(5 * p.y)     # any u: the identity is per particle
    vx, vy, vz = -c * (p.x - 0.5) + 0.2, -c * (p.y - 0.5) - 0.1, -c * (p.z - 0.5)
    f = oracle.force(p.x, p.y, p.z, vx, vy, vz, u, h, rho, om, p.lo, p.hi, p.periodic,
                     p.mass, gamma=g, alpha=0.0, beta=0.0, beta_u=0.0)
    sel = _interior(p, h, 2.5) if p.periodic else np.ones(p.n, bool)
    assert sel.sum() > 50
    want = 3.0 * c * (g - 1.0) * u
    assert np.abs(f["dudt"][sel] / want[sel] - 1).max() < 1e-9


def test_linear_pressure_gives_exact_acceleration_on_cubic_lattice():
    p = gen.lattice(16, 1, dtype=np.float64, jitter=0.0)
    h, rho, om, _ = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    g, k = 5.0 / 3.0, 0.5
    u = 1.0 + k * (p.x - 0.5)                  # P = (gamma-1) rho u, grad P = (gamma-1) rho k x
    f = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, u, h, rho, om, p.lo, p.hi, True,
                     p.mass, gamma=g)
    sel = _interior(p, h, 2.5)
    assert sel.sum() > 100
    ax = -(g - 1.0) * k                        # -grad P / rho
    assert np.abs(f["ax"][sel] / ax - 1).max() < 1e-9
    for c in ("ay", "az"):
        assert np.abs(f[c][sel]).max() < 1e-9 * abs(ax)


# ------------------------------------------- two-particle hand values ----
# Particles a at the origin and b at (1.5, 0, 0) with prescribed h, rho,
# Omega, u and v (force() takes them as inputs), m = 1:
#   r_ab = r_a - r_b = (-1.5, 0, 0), rhat_ab = -x;  h_a = 1, h_b = 1.5, so
#   q_a = 1.5, q_b = 1 and, for the M4 spline, f'(1.5) = -3/16, f'(1) = -3/4:
#   F_a = f'(q_a)/(pi h_a^4) = -3/(16 pi),  F_b = -(3/4)/(pi 1.5^4) = -4/(27 pi).
#   rho_a = 2, rho_b = 1, Omega_a = 0.8, Omega_b = 1.25.
#   v_a = (0.5,0,0), v_b = (-0.5,0,0): v_ab = (1,0,0), w = v_ab . rhat = -1.
_PAIR = dict(x=[0.0, 1.5], y=[0.0, 0.0], z=[0.0, 0.0], vx=[0.5, -0.5], vy=[0.0, 0.0],
             vz=[0.0, 0.0], h=[1.0, 1.5], rho=[2.0, 1.0], omega=[0.8, 1.25])


def _pair_force(u, **kw):
    a = {k: np.array(v, np.float64) for k, v in _PAIR.items()}
    return oracle.force(a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                        np.array(u, np.float64), a["h"], a["rho"], a["omega"],
                        (0, 0, 0), (1, 1, 1), False, 1.0, **kw)


def test_pair_viscosity_by_hand():
    # gamma = 2: P = rho u, c_s = sqrt(2u).  u = (2, 0.5): P = (4, 0.5), c = (2, 1).
    # alpha = 1, beta = 2: vsig_a = 2 + 2 = 4, vsig_b = 1 + 2 = 3;
    # q^a = -rho_a vsig_a w / 2 = 4, q^b = 1.5.
    # (P_a+q^a)/(rho_a^2 Om_a) = 8/3.2 = 5/2;  (P_b+q^b)/(rho_b^2 Om_b) = 2/1.25 = 8/5.
    # dv_a/dt = -m [5/2 F_a + 8/5 F_b] rhat = [5/2 (-3/16) + 8/5 (-4/27)]/pi x
    #         = -(15/32 + 32/135)/pi x = -3049/(4320 pi) x
    # du_a/dt = m 5/2 w F_a = 15/(32 pi)          (beta_u = 0)
    f = _pair_force([2.0, 0.5], gamma=2.0, alpha=1.0, beta=2.0, beta_u=0.0)
    assert abs(f["ax"][0] - (-3049.0 / (4320.0 * math.pi))) < 1e-15
    assert abs(f["ay"][0]) == 0.0 and abs(f["az"][0]) == 0.0
    assert abs(f["dudt"][0] - 15.0 / (32.0 * math.pi)) < 1e-15
    assert f["vsig"][0] == 4.0               # the largest alpha c_a + beta |w|
    # particle b feels the opposite momentum flux (equal masses)
    assert abs(f["ax"][1] + f["ax"][0]) < 1e-15


def test_pair_conductivity_by_hand():
    # gamma = 5/3, u = (21/4, 3/2): P = (2/3) rho u = (7, 1);
    # vsig_u = sqrt(|P_a - P_b| / ((rho_a + rho_b)/2)) = sqrt(6 / 1.5) = 2.
    # Lambda_a = m beta_u vsig_u (u_a - u_b) (F_a/(Om_a rho_a) + F_b/(Om_b rho_b))/2
    #          = 2 (15/4) (-15/128 - 16/135)/(2 pi) = -(15/4)(4073/17280)/pi
    # Pressure part with no viscosity (alpha = beta = 0):
    #   m (P_a/(rho_a^2 Om_a)) w F_a = (7/3.2)(-1)(-3/16)/pi = 105/(256 pi)
    f = _pair_force([5.25, 1.5], gamma=5.0 / 3.0, alpha=0.0, beta=0.0, beta_u=1.0)
    lam = -(15.0 / 4.0) * (4073.0 / 17280.0) / math.pi
    assert abs(f["dudt"][0] - (105.0 / (256.0 * math.pi) + lam)) < 1e-14
    g = _pair_force([5.25, 1.5], gamma=5.0 / 3.0, alpha=0.0, beta=0.0, beta_u=0.0)
    assert abs((f["dudt"][0] - g["dudt"][0]) - lam) < 1e-14
    # pairwise: b gains what a loses (equal masses)
    assert abs((f["dudt"][1] - g["dudt"][1]) + lam) < 1e-14
    # the conductivity grows as |du|^(3/2): doubling both u doubles u_a - u_b
    # and P_a - P_b, which scales Lambda by 2 sqrt 2
    f2 = _pair_force([10.5, 3.0], gamma=5.0 / 3.0, alpha=0.0, beta=0.0, beta_u=1.0)
    g2 = _pair_force([10.5, 3.0], gamma=5.0 / 3.0, alpha=0.0, beta=0.0, beta_u=0.0)
    assert abs((f2["dudt"][0] - g2["dudt"][0]) / lam - 2.0 * math.sqrt(2.0)) < 1e-13


def test_cfl_force_branch_by_hand():
    # particle 0: C_cour h / vsig = 0.3 * 0.01 / 1e-6 = 3000, but
    # C_force sqrt(h/|a|) = 0.25 sqrt(0.01/5) = 0.25 sqrt(0.002) = 0.011180339887498949;
    # particle 1: C_cour h/vsig = 0.3 * 1/10 = 0.03, a = 0.
    h = np.array([0.01, 1.0])
    vsig = np.array([1e-6, 10.0])
    ax, ay, az = np.array([3.0, 0.0]), np.array([4.0, 0.0]), np.zeros(2)
    dt = oracle.cfl(h, vsig, ax, ay, az)
    assert abs(dt - 0.011180339887498949) < 1e-17
    # Courant branch when the force term is the larger: vsig_0 = 1 gives
    # 0.3 * 0.01 = 0.003 against 0.25 sqrt(0.01 / 5e-6) = 11.18
    dt2 = oracle.cfl(h, np.array([1.0, 10.0]), ax * 1e-6, ay * 1e-6, az)
    assert abs(dt2 - 0.003) < 1e-18


def test_kdk_step_is_velocity_verlet_and_diagnostics():
    """One fixed-dt step against the textbook velocity-Verlet forms (App. G.1):
    r^{n+1} = r^n + dt v^n + dt^2 a^n / 2 (wrapped into the box),
    v^{n+1} = v^n + dt (a^n + a^{n+1}) / 2, same for u with du/dt; and the
    corrector diagnostics (Eq. deltavi) from the returned derivatives:
    dv = dt (a^{n+1} - a^n) / 2, max |dv|, sum |dv|^2, sum |v^{n+1}|^2."""
    rng = np.random.default_rng(19)
    p = gen.lattice(8, 19, dtype=np.float64)
    v, u, h, rho, om = _state(p, rng, vscale=0.2, uvar=0.3)
    f = oracle.force(p.x, p.y, p.z, *v, u, h, rho, om, p.lo, p.hi, True, p.mass)
    # a^n deliberately not the derivative of the state, so that a^{n+1} - a^n is large
    an = [f[c] + 0.3 * rng.standard_normal(p.n) for c in ("ax", "ay", "az")]
    dun = f["dudt"] + 0.1 * rng.standard_normal(p.n)
    st = dict(x=p.x, y=p.y, z=p.z, vx=v[0], vy=v[1], vz=v[2], u=u, h=h,
              ax=an[0], ay=an[1], az=an[2], dudt=dun)
    dt = 0.2 * oracle.cfl(h, f["vsig"], f["ax"], f["ay"], f["az"])
    s = oracle.step(st, p.lo, p.hi, True, p.mass, dt)
    for c, vc, ac in zip(("x", "y", "z"), v, an):
        want = np.mod(st[c] + dt * vc + 0.5 * dt * dt * ac, 1.0)
        d = np.abs(s[c] - want)
        assert np.minimum(d, 1 - d).max() < 1e-15 and (s[c] >= 0).all() and (s[c] < 1).all()
    dv = []
    for c, vc, ac, nc in zip(("vx", "vy", "vz"), v, an, ("ax", "ay", "az")):
        assert np.abs(s[c] - (vc + 0.5 * dt * (ac + s[nc]))).max() < 1e-14
        dv.append(0.5 * dt * (s[nc] - ac))
    assert np.abs(s["u"] - (u + 0.5 * dt * (dun + s["dudt"]))).max() < 1e-14
    dvn = np.sqrt(dv[0] ** 2 + dv[1] ** 2 + dv[2] ** 2)
    assert dvn.max() > 1e-3 * np.abs(v[0]).max()
    assert abs(s["diag"][0] - dvn.max()) < 1e-15
    assert abs(s["diag"][1] / (dvn ** 2).sum() - 1) < 1e-13
    assert abs(s["diag"][2] / (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2).sum() - 1) < 1e-13
    # the CFL dt of the new state
    g = oracle.force(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["u"], s["h"],
                     s["rho"], s["omega"], p.lo, p.hi, True, p.mass)
    assert s["diag"][3] > 0
