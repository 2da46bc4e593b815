"""Pins of the oracle's extensions: the kernel family of Sect. 2.1.1 (M4, M5,
M6 B-splines, Wendland C2, C4, C6), the corrector re-run and CFL multiplier
(App. G.1, App. G CFL multiplier), and the shock-detection switch (App. G,
Shock detection).  Each pin is a closed form, an integral, a value the paper
prints, or an exact identity, chosen so that a plausible slip fails it."""
import math

import numpy as np
import pytest
from scipy import integrate

import gen
import oracle

KERNELS = ["M4", "M5", "M6", "C2", "C4", "C6"]
BREAKS = {"M4": [1.0], "M5": [0.5, 1.5], "M6": [1.0, 2.0], "C2": [], "C4": [], "C6": []}
# h_fact used with each kernel in these tests (M6: the paper's 1.0)
HFACT = {"M4": 1.2, "M5": 1.2, "M6": 1.0, "C2": 1.2, "C4": 1.3, "C6": 1.5}


# ------------------------------------------------------------- kernels ----
@pytest.mark.parametrize("k", KERNELS)
def test_kernel_normalisation(k):
    # int W dV = 4 pi C_norm int_0^R f(q) q^2 dq = 1 in three dimensions
    R, C = oracle.kernel_support(k), oracle.kernel_norm(k)
    val, _ = integrate.quad(lambda q: oracle.kernel_f(k, q) * q * q, 0.0, R,
                            points=BREAKS[k] or None, epsabs=1e-14, epsrel=1e-13)
    assert abs(4.0 * math.pi * C * val - 1.0) < 1e-11


@pytest.mark.parametrize("k", KERNELS)
def test_kernel_shape(k):
    R = oracle.kernel_support(k)
    assert oracle.kernel_f(k, R) == 0.0 and oracle.kernel_f(k, R + 0.3) == 0.0
    assert abs(oracle.kernel_df(k, 0.0)) < 1e-12            # smooth at the origin
    e = 1e-8
    for q0 in BREAKS[k] + [R]:                               # f, f' continuous
        assert abs(oracle.kernel_f(k, q0 - e) - oracle.kernel_f(k, q0 + e)) < 1e-6
        assert abs(oracle.kernel_df(k, q0 - e) - oracle.kernel_df(k, q0 + e)) < 1e-6
    for q in np.linspace(0.03, R - 0.03, 57):                # f' is the derivative of f
        fd = (oracle.kernel_f(k, q + 1e-6) - oracle.kernel_f(k, q - 1e-6)) / 2e-6
        assert abs(fd - oracle.kernel_df(k, q)) < 1e-6 * max(1.0, oracle.kernel_f(k, 0.0))
        assert oracle.kernel_df(k, q) < 0                    # bell-shaped: decreasing


@pytest.mark.parametrize("k,hfact,paper", [("M6", 1.0, 113.0), ("M4", 1.2, 60.0)])
def test_mean_neighbour_count_paper_values(k, hfact, paper):
    """Sect. 4.1: M6 with h_fact = 1.0 has on average 113 neighbours; Sect. 2:
    M4 with h_fact = 1.2 about 60.  With rho = m (h_fact/h)^3 the mean count
    within R h is (4 pi / 3)(R h_fact)^3 (113.1 and 57.9)."""
    p = gen.lattice(20, 31, dtype=np.float64, jitter=0.3, hfact=hfact)
    h, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass, hfact=hfact,
                                    kernel=k)
    assert fl.max() == 0
    R = oracle.kernel_support(k)
    off, _ = oracle.neighbours(p.x, p.y, p.z, h, p.lo, p.hi, True, R)
    # neighbours of a within R max(h_a, h_b): count those within R h_a
    lst = oracle.neighbours(p.x, p.y, p.z, h, p.lo, p.hi, True, R)[1]
    cnt = np.zeros(p.n)
    o = off.astype(np.int64)
    for a in range(p.n):
        b = lst[o[a]:o[a + 1]]
        d = np.stack([p.x[b] - p.x[a], p.y[b] - p.y[a], p.z[b] - p.z[a]], 1)
        d -= np.round(d)
        cnt[a] = (np.sqrt((d ** 2).sum(1)) < R * h[a]).sum()
    want = 4.0 * math.pi / 3.0 * (R * hfact) ** 3
    assert abs(cnt.mean() / want - 1) < 0.05
    assert abs(cnt.mean() / paper - 1) < 0.06


def _interior(p, h, margin):
    ok = np.ones(p.n, bool)
    for c in (p.x, p.y, p.z):
        ok &= np.abs(c - 0.5) + margin * h < 0.5
    return ok


@pytest.mark.parametrize("k", KERNELS)
def test_identities_at_the_root_for_every_kernel(k):
    """The exact identities of the M4 pins hold for every kernel at its
    self-consistent h: uniform compression heats at 3cP/rho (jittered
    lattice), a linear pressure accelerates at -grad P/rho (cubic lattice)."""
    hf, R, g = HFACT[k], oracle.kernel_support(k), 5.0 / 3.0
    p = gen.lattice(14, 41, dtype=np.float64, hfact=hf)
    h, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass, hfact=hf,
                                    kernel=k)
    assert fl.max() == 0
    c = 0.3
    u = 1.0 + 0.5 * np.sin(7 * p.x) * np.cos(5 * p.y)
    f = oracle.force(p.x, p.y, p.z, -c * (p.x - .5), -c * (p.y - .5), -c * (p.z - .5), u, h,
                     rho, om, p.lo, p.hi, True, p.mass, gamma=g, alpha=0.0, beta=0.0,
                     beta_u=0.0, kernel=k)
    sel = _interior(p, h, 1.2 * R)
    assert sel.sum() > 20
    assert np.abs(f["dudt"][sel] / (3 * c * (g - 1) * u[sel]) - 1).max() < 1e-9
    q = gen.lattice(16, 1, dtype=np.float64, jitter=0.0, hfact=hf)
    h, rho, om, _ = oracle.density(q.x, q.y, q.z, q.h, q.lo, q.hi, True, q.mass, hfact=hf,
                                   kernel=k)
    f = oracle.force(q.x, q.y, q.z, q.vx, q.vy, q.vz, 1.0 + 0.5 * (q.x - 0.5), h, rho, om, q.lo,
                     q.hi, True, q.mass, gamma=g, kernel=k)
    sel = _interior(q, h, 1.2 * R)
    assert np.abs(f["ax"][sel] / (-(g - 1) * 0.5) - 1).max() < 1e-9


# ------------------------------------------------ gradients, alpha switch --
_A = np.array([[0.3, -0.7, 0.2], [0.5, -0.1, 0.9], [-0.4, 0.6, 0.25]])
_B = np.array([[0.2, 0.4, -0.3], [-0.6, 0.1, 0.5], [0.7, -0.2, -0.45]])


def _cubic(k):
    hf = HFACT[k]
    q = gen.lattice(16, 1, dtype=np.float64, jitter=0.0, hfact=hf)
    h, rho, om, _ = oracle.density(q.x, q.y, q.z, q.h, q.lo, q.hi, True, q.mass, hfact=hf,
                                   kernel=k)
    r = np.stack([q.x - 0.5, q.y - 0.5, q.z - 0.5], 1)
    return q, h, rho, om, r, _interior(q, h, 1.2 * oracle.kernel_support(k))


@pytest.mark.parametrize("k", ["M4", "M6"])
def test_gradient_of_linear_field_is_exact_on_cubic_lattice(k):
    """v = A r: the SPH estimate -1/(rho Omega) sum m v_ab (x) rhat F equals A
    on the unjittered lattice at the root (cubic symmetry and the Omega
    identity), with A not symmetric so that a transposed index fails."""
    q, h, rho, om, r, sel = _cubic(k)
    v = r @ _A.T
    G = oracle.gradient(q.x, q.y, q.z, v[:, 0], v[:, 1], v[:, 2], h, rho, om, q.lo, q.hi, True,
                        q.mass, kernel=k)
    assert sel.sum() > 50
    assert np.abs(G[sel] - _A).max() < 1e-9


def test_alpha_switch_hand_cases():
    """Cubic lattice at the root, so grad v and grad a are exact (test above):
    * v = A r, a = B r: d(div v)/dt = tr B - tr(A A);
    * isotropic compression v = -w r with a = b r, b chosen so that
      A_shock = -d(div v)/dt = c_s^2/(10 h^2) (curl 0, so xi = 1): then
      alpha_loc = alpha_max / 2, and alpha^{n+1} = max((alpha^n + x/2)/(1+x), 1/2)
      with x = dt sigma c_s / h;
    * a rigid rotation (div v = 0): xi = 0, alpha_loc = alpha_min, alpha decays
      as alpha^n / (1 + x);
    * an expansion whose divergence is steady (a = w^2 r): no trigger."""
    q, h, rho, om, r, sel = _cubic("M4")
    g, u0, dt, sig = 5.0 / 3.0, 0.9, 0.002, 0.1
    u = np.full(q.n, u0)
    cs = math.sqrt(g * (g - 1) * u0)
    hh = h[sel][0]
    assert np.allclose(h[sel], hh, rtol=1e-12)
    x = dt * sig * cs / hh

    def run(v, a, alpha_n):
        return oracle.alpha_switch(q.x, q.y, q.z, v[:, 0], v[:, 1], v[:, 2], a[:, 0], a[:, 1],
                                   a[:, 2], u, h, rho, om, alpha_n, q.lo, q.hi, True, q.mass, dt,
                                   gamma=g, sigma_decay=sig, alpha_max=1.0, alpha_min=0.0)

    o = run(r @ _A.T, r @ _B.T, np.zeros(q.n))
    assert np.abs(o["ddivv_dt"][sel] - (np.trace(_B) - np.trace(_A @ _A))).max() < 1e-9
    assert np.abs(o["divv"][sel] - np.trace(_A)).max() < 1e-9
    w = 0.4
    b = w * w - cs * cs / (30.0 * hh * hh)         # 3b - 3w^2 = -c^2/(10 h^2)
    for a_n in (0.0, 1.0):
        o = run(-w * r, b * r, np.full(q.n, a_n))
        assert np.abs(o["alpha_loc"][sel] - 0.5).max() < 1e-9
        want = max((a_n + 0.5 * x) / (1 + x), 0.5)
        assert np.abs(o["alpha"][sel] - want).max() < 1e-9
    rot = np.array([[0.0, -0.8, 0.0], [0.8, 0.0, 0.0], [0.0, 0.0, 0.0]])
    o = run(r @ rot.T, -3.0 * r, np.full(q.n, 0.7))  # strongly decelerating, but no divergence
    assert np.abs(o["alpha_loc"][sel]).max() < 1e-20
    assert np.abs(o["alpha"][sel] - 0.7 / (1 + x)).max() < 1e-12
    o = run(w * r, w * w * r, np.full(q.n, 0.3))
    assert np.abs(o["alpha_loc"][sel]).max() < 1e-9


def test_alpha_decay_follows_the_ode():
    """With alpha_loc fixed, the implicit step approximates
    alpha(t) = alpha_loc + (alpha^n - alpha_loc) exp(-t/tau) to O((dt/tau)^2)
    (Eq. evolalphaanalytic)."""
    q, h, rho, om, r, sel = _cubic("M4")
    g, u0, sig = 5.0 / 3.0, 1.0, 0.1
    u = np.full(q.n, u0)
    cs = math.sqrt(g * (g - 1) * u0)
    hh = h[sel][0]
    for dt in (1e-3, 3e-3, 1e-2):
        o = oracle.alpha_switch(q.x, q.y, q.z, *(np.zeros(q.n),) * 6, u, h, rho, om,
                                np.full(q.n, 1.0), q.lo, q.hi, True, q.mass, dt, gamma=g,
                                sigma_decay=sig)
        x = dt * sig * cs / hh
        exact = math.exp(-x)
        assert np.abs(o["alpha"][sel] - exact).max() <= 0.5 * x * x + 1e-12


# ---------------------------------------------- corrector re-run, CFL --
def test_cfl_multiplier_closed_form():
    """lambda^{n+1} = (1 + s lambda^n)/(1 + s): 1 is the fixed point and
    1 - lambda shrinks by s/(1+s) per step; a re-run halves lambda."""
    s = 0.75
    assert oracle.cfl_multiplier(1.0, False, s) == 1.0
    assert oracle.cfl_multiplier(0.8, True, s) == 0.4
    lam = 0.25
    for k in range(1, 12):
        lam = oracle.cfl_multiplier(lam, False, s)
        assert abs((1 - lam) - 0.75 * (s / (1 + s)) ** k) < 1e-15


def test_corrector_reruns_reach_the_trapezoidal_fixed_point():
    """Each re-run evaluates the force with v* <- v^{n+1}; repeated, v^{n+1}
    converges to the solution of v = v^{n+1/2} + dt/2 a(r^{n+1}, v, u)
    (u likewise), which the final state must satisfy."""
    rng = np.random.default_rng(5)
    p = gen.lattice(9, 61, dtype=np.float64)
    v = [0.3 * rng.standard_normal(p.n) for _ in range(3)]
    u = 1.0 + 0.3 * rng.uniform(-1, 1, p.n)
    h, rho, om, _ = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass)
    f = oracle.force(p.x, p.y, p.z, *v, u, h, rho, om, p.lo, p.hi, True, p.mass)
    dt = 0.5 * oracle.cfl(h, f["vsig"], f["ax"], f["ay"], f["az"])
    st = dict(x=p.x, y=p.y, z=p.z, vx=v[0], vy=v[1], vz=v[2], u=u, h=h, ax=f["ax"],
              ay=f["ay"], az=f["az"], dudt=f["dudt"])
    s0 = oracle.step(st, p.lo, p.hi, True, p.mass, dt)
    assert s0["diag"][4] == 0
    s = oracle.step(st, p.lo, p.hi, True, p.mass, dt, eps_v=1e-13, max_rerun=40)
    assert s["diag"][4] > 2
    # the fixed point: the force at the final state reproduces the final v, u
    g = oracle.force(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["u"], s["h"],
                     s["rho"], s["omega"], p.lo, p.hi, True, p.mass)
    for c, a in (("vx", "ax"), ("vy", "ay"), ("vz", "az")):
        vh = st[c] + 0.5 * dt * st[a]
        assert np.abs(s[c] - (vh + 0.5 * dt * g[a])).max() < 1e-10 * np.abs(vh).max()
    uh = u + 0.5 * dt * f["dudt"]
    assert np.abs(s["u"] - (uh + 0.5 * dt * g["dudt"])).max() < 1e-10
    # a loose tolerance stops at once; the first evaluation is the plain step
    s1 = oracle.step(st, p.lo, p.hi, True, p.mass, dt, eps_v=10.0, max_rerun=40)
    assert s1["diag"][4] == 0 and np.array_equal(s1["vx"], s0["vx"])
    # one re-run: the force of the plain step's v^{n+1} gives the next iterate
    s2 = oracle.step(st, p.lo, p.hi, True, p.mass, dt, eps_v=1e-13, max_rerun=1)
    g0 = oracle.force(s0["x"], s0["y"], s0["z"], s0["vx"], s0["vy"], s0["vz"], s0["u"], s0["h"],
                      s0["rho"], s0["omega"], p.lo, p.hi, True, p.mass)
    vh = st["vx"] + 0.5 * dt * st["ax"]
    assert np.abs(s2["vx"] - (vh + 0.5 * dt * g0["ax"])).max() < 1e-13 * np.abs(vh).max() + 1e-15
    assert s2["diag"][0] == pytest.approx(np.sqrt(((s2["vx"] - s0["vx"]) ** 2 + (s2["vy"] - s0["vy"]) ** 2
                                                   + (s2["vz"] - s0["vz"]) ** 2).max()), rel=1e-12)
