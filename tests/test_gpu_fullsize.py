"""GPU against the oracle at the benchmark's full size: the Sedov blast on a
jittered 256^3 lattice in FP32 (16,777,216 particles), built with the default
parameters that bench.py times (n_red 3, per-lane stage-2 walk).  The oracle
cannot take the whole state in seconds, so the checks are outputs it computes
one particle at a time (Morton keys, neighbour sets, h / rho / Omega,
acceleration and du/dt of sampled particles) and properties that hold at any
size (sort permutation, key order, stability of ties, CFL dt bound)."""
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

shsph = pytest.importorskip("paper_2503_09713_amd")

N1, SEED = 256, gen.SEEDS["sedov"]     # the benchmark's sedov256 workload


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _sample(p, k_rand=48, k_centre=8, k_corner=8):
    """Random particles, the blast centre and a corner of the periodic box."""
    rng = np.random.default_rng(11)
    s = list(rng.choice(p.n, size=k_rand, replace=False))
    x, y, z = (p.x.astype(np.float64), p.y.astype(np.float64), p.z.astype(np.float64))
    rc = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    s += list(np.argpartition(rc, k_centre)[:k_centre])
    r0 = np.minimum(x, 1 - x) ** 2 + np.minimum(y, 1 - y) ** 2 + np.minimum(z, 1 - z) ** 2
    s += list(np.argpartition(r0, k_corner)[:k_corner])
    return np.unique(np.array(s, np.int64))


def test_sedov256_full_size(torch_cuda):
    _say("[full] sedov 256^3 f32: generating")
    p = gen.sedov(N1, SEED, dtype=np.float32)
    assert p.n == N1 ** 3 and p.periodic
    s = _sample(p)
    ctx = shsph.Context(0)
    ps = shsph.ParticleSet.from_particles(p)
    _say("[full] build tree + caches")
    ctx.build_tree(ps)
    ex = ctx.export_tree(fields=["keys", "eps", "mu", "neigh_off", "neigh_list"])
    keys, eps, mu = ex["keys"], ex["eps"].astype(np.int64), ex["mu"]

    _say("[full] keys of a sample, sort permutation, order, stability")
    ks = np.random.default_rng(12).choice(p.n, size=8192, replace=False)
    assert np.array_equal(keys[ks], oracle.morton(p.x[ks], p.y[ks], p.z[ks], p.lo, p.hi))
    assert np.array_equal(np.bincount(eps, minlength=p.n), np.ones(p.n, np.int64))
    assert np.array_equal(mu, keys[eps])
    assert (mu[1:] >= mu[:-1]).all()
    assert ((mu[1:] > mu[:-1]) | (eps[1:] > eps[:-1])).all()

    _say("[full] neighbour sets of the sample (key order)")
    inv = np.empty(p.n, np.int64)
    inv[eps] = np.arange(p.n)
    t = inv[s]
    xs, ys, zs, hs = p.x[eps], p.y[eps], p.z[eps], p.h[eps]
    off, lst = oracle.neighbours(xs, ys, zs, hs, p.lo, p.hi, True, 2.2, targets=t)
    go, gl = ex["neigh_off"], ex["neigh_list"]
    for r, i in enumerate(t):
        assert np.array_equal(gl[go[i]:go[i + 1]], lst[off[r]:off[r + 1]]), f"particle {s[r]}"
    del ex, gl, xs, ys, zs, hs

    _say("[full] density of the sample")
    ctx.density(ps)
    g = {k: v.astype(np.float64) for k, v in ps.host("h", "rho", "omega").items()}
    h, rho, om, fl = oracle.density(p.x, p.y, p.z, p.h, p.lo, p.hi, True, p.mass, targets=s)
    assert fl.max() == 0
    assert np.abs(g["h"][s] / h - 1).max() <= 1e-5
    assert np.abs(g["rho"][s] / rho - 1).max() <= 1e-5
    assert np.abs(g["omega"][s] / om - 1).max() <= 1e-4

    _say("[full] force of the sample, CFL bound")
    ctx.force(ps)
    g.update({k: v.astype(np.float64) for k, v in ps.host("ax", "ay", "az", "dudt").items()})
    rho_g = p.mass * (1.2 / g["h"]) ** 3
    ref = oracle.force(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, g["h"], rho_g, g["omega"],
                       p.lo, p.hi, True, p.mass, targets=s)
    sa = np.maximum(ref["scale_a"], 1e-300)
    su = np.maximum(ref["scale_u"], 1e-300)
    ea = np.sqrt((g["ax"][s] - ref["ax"]) ** 2 + (g["ay"][s] - ref["ay"]) ** 2 +
                 (g["az"][s] - ref["az"]) ** 2) / sa
    eu = np.abs(g["dudt"][s] - ref["dudt"]) / su
    assert ea.max() <= 1e-4 and eu.max() <= 1e-4, (ea.max(), eu.max())
    # the CFL dt is a minimum over all particles: at most the sample's minimum
    dt_s = oracle.cfl(g["h"][s], ref["vsig"], ref["ax"], ref["ay"], ref["az"])
    assert ctx.get_info()["dt_cfl"] <= dt_s * (1 + 1e-4)

    _say("[full] one CFL step: ids stay a permutation, order and cache rebuilt")
    ctx.step(ps, 0.0)
    pid = ps.host("pid")["pid"].astype(np.int64)
    assert np.array_equal(np.sort(pid), np.arange(p.n))
    ex2 = ctx.export_tree(fields=["mu"])
    assert (ex2["mu"][1:] >= ex2["mu"][:-1]).all()
    ctx.close()
