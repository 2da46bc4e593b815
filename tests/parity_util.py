"""Comparisons shared by the GPU parity tests: one kick-drift-kick step of the
GPU (App. G.1) against the oracle's step or against the textbook
velocity-Verlet forms, raw positions included (no minimum-image fold)."""
import numpy as np

import oracle

F32_ULP = 2.0 ** -23


def box_for_oracle(p):
    """The oracle's box: the periodic box, or the data extent (isolated)."""
    if p.periodic:
        return p.lo, p.hi
    return ((float(p.x.min()), float(p.y.min()), float(p.z.min())),
            (float(p.x.max()), float(p.y.max()), float(p.z.max())))


def _oracle_tree(p, n_red, key_bits=63):
    lo, hi = box_for_oracle(p)
    keys = oracle.morton(p.x, p.y, p.z, lo, hi, bits=key_bits // 3)
    eps, mu = oracle.sort(keys)
    xi, ids, ml = oracle.leaves(mu, n_red)
    t = oracle.radix_tree(ml)
    return keys, eps, mu, xi, ids, ml, t


def check_tree(ctx, p, n_red, chi=1.1, r_kern=2.0, key_bits=63):
    """Every table of the GPU's last build against the oracle, bit for bit;
    the cache radius is r_kern chi max(h_a, h_b)."""
    T = p.x.dtype
    ex = ctx.export_tree(dtype=T)
    keys, eps, mu, xi, ids, ml, t = _oracle_tree(p, n_red, key_bits)
    assert np.array_equal(ex["keys"], keys), "Morton keys"
    assert np.array_equal(ex["eps"], eps), "sort permutation"
    assert np.array_equal(ex["mu"], mu)
    assert np.array_equal(ex["xi"], xi), "keep mask"
    assert np.array_equal(ex["id"], ids)
    assert np.array_equal(ex["mu_leaf"], ml)
    for k in ("lchild", "rchild", "lflag", "rflag", "endrange"):
        assert np.array_equal(ex[k], t[k]), k
    assert np.array_equal(ex["parent"], t["parent"]), "parent"
    xs, ys, zs, hs = p.x[eps], p.y[eps], p.z[eps], p.h[eps]
    bmin, bmax, hmax = oracle.tight_boxes(ids, t, xs, ys, zs, hs)
    assert np.array_equal(ex["bmin"].astype(np.float64), bmin), "tight box min"
    assert np.array_equal(ex["bmax"].astype(np.float64), bmax), "tight box max"
    assert np.array_equal(ex["hmax"].astype(np.float64), hmax), "h_max"
    # prefix boxes in the 63-bit layout (30-bit codes moved up by 33 bits)
    box, plen = oracle.prefix_boxes(ml << np.uint64(63 - key_bits), t)
    assert np.array_equal(ex["pbox"], box) and np.array_equal(ex["plen"], plen), "prefix boxes"
    lo, hi = box_for_oracle(p)
    off, lst = oracle.neighbours(xs, ys, zs, hs, lo, hi, p.periodic, r_kern * chi)
    assert np.array_equal(ex["neigh_off"], off), "neighbour counts"
    assert np.array_equal(ex["neigh_list"], lst), "neighbour sets / order"
    # stage-1 lists (per group of 256 key-order slots) are ascending and
    # cover the leaf of every neighbour of every particle of the group
    go, gl = ex["group_off"], ex["group_leaves"]
    leaf_of = np.searchsorted(ids, np.arange(p.n), side="right") - 1
    for a in range(0, p.n, max(1, p.n // 300)):
        g = a // 256
        seg = gl[go[g]:go[g + 1]]
        assert (np.diff(seg.astype(np.int64)) > 0).all()
        assert set(leaf_of[lst[off[a]:off[a + 1]]]) <= set(seg.tolist())
    return ex


def map_to_start(pid_start, pid_after):
    """Index into the start-of-step arrays for every particle of the output
    (the step returns the particles in the new key order, ids carried)."""
    pos = np.empty(pid_start.shape[0], np.int64)
    pos[pid_start.astype(np.int64)] = np.arange(pid_start.shape[0])
    return pos[pid_after.astype(np.int64)]


def check_positions(got, want, lo, hi, tol):
    """Raw comparison after the periodic wrap: every coordinate in [lo, hi),
    and within `tol` of the reference.  Only a particle whose reference lies
    within `tol` of a face may come out on the other side of the box (the
    FP32 and FP64 wraps can then differ); at most a few do."""
    amb_total = 0
    for d, (g, w) in enumerate(zip(got, want)):
        L = hi[d] - lo[d]
        assert (g >= lo[d]).all() and (g < hi[d]).all(), "position outside the box"
        err = np.abs(g.astype(np.float64) - w)
        bad = err > tol
        if bad.any():
            near = np.minimum(w - lo[d], hi[d] - w) <= tol
            assert (near[bad]).all(), f"axis {d}: max raw error {err.max()} away from the faces"
            assert (np.abs(err[bad] - L) <= tol).all(), f"axis {d}: wrapped by other than L"
            amb_total += int(bad.sum())
    assert amb_total <= max(4, got[0].shape[0] // 100000)
    return amb_total


def force_err(g, ref):
    sa = np.maximum(ref["scale_a"], 1e-300)
    su = np.maximum(ref["scale_u"], 1e-300)
    ea = np.sqrt((g["ax"] - ref["ax"]) ** 2 + (g["ay"] - ref["ay"]) ** 2 +
                 (g["az"] - ref["az"]) ** 2) / sa
    eu = np.abs(g["dudt"] - ref["dudt"]) / su
    return ea, eu


def check_corrector_forms(s0, s1, j, dt, T, lo, hi, periodic, info=None):
    """The GPU's step output against the velocity-Verlet forms of its own
    derivatives:
        r^{n+1} = r^n + dt v^n + dt^2 a^n / 2 (wrapped),
        v^{n+1} = v^n + dt (a^n + a^{n+1}) / 2,   u likewise with du/dt,
    and its corrector reductions (Eq. deltavi) from dv = dt (a^{n+1} - a^n)/2.
    Tolerances are rounding bounds of the storage type: each FP32 operation of
    the predictor / corrector adds at most half an ulp of its result."""
    f = lambda k, s: s[k].astype(np.float64)
    eps = F32_ULP if T == np.float32 else 2.0 ** -52
    vmag = np.sqrt(sum(f(k, s0)[j] ** 2 for k in ("vx", "vy", "vz")))
    amag = np.sqrt(sum(f(k, s0)[j] ** 2 for k in ("ax", "ay", "az")) +
                   sum(f(k, s1) ** 2 for k in ("ax", "ay", "az")))
    # positions: a few roundings of x, dt v and dt^2 a
    want = []
    for c, vc, ac in (("x", "vx", "ax"), ("y", "vy", "ay"), ("z", "vz", "az")):
        w = f(c, s0)[j] + dt * f(vc, s0)[j] + 0.5 * dt * dt * f(ac, s0)[j]
        if periodic:
            d = ("x", "y", "z").index(c)
            w = lo[d] + np.mod(w - lo[d], hi[d] - lo[d])
        want.append(w)
    tolx = 8 * eps * max(1.0, max(abs(v) for v in hi)) + 4 * eps * dt * vmag.max()
    amb = check_positions([s1["x"], s1["y"], s1["z"]], want, lo, hi, tolx) if periodic else 0
    if not periodic:
        for g, w in zip((s1["x"], s1["y"], s1["z"]), want):
            assert np.abs(g - w).max() <= tolx
    # velocities and u
    tolv = 6 * eps * (vmag + dt * amag) + 1e-30
    dv = []
    for vc, ac in (("vx", "ax"), ("vy", "ay"), ("vz", "az")):
        w = f(vc, s0)[j] + 0.5 * dt * (f(ac, s0)[j] + f(ac, s1))
        assert (np.abs(f(vc, s1) - w) <= tolv).all(), vc
        dv.append(0.5 * dt * (f(ac, s1) - f(ac, s0)[j]))
    umag = np.abs(f("u", s0)[j]) + dt * (np.abs(f("dudt", s0)[j]) + np.abs(f("dudt", s1)))
    wu = f("u", s0)[j] + 0.5 * dt * (f("dudt", s0)[j] + f("dudt", s1))
    assert (np.abs(f("u", s1) - wu) <= 6 * eps * umag + 1e-30).all(), "u"
    if info is not None:
        dvn = np.sqrt(dv[0] ** 2 + dv[1] ** 2 + dv[2] ** 2)
        e = 6 * eps * (vmag + dt * amag)           # per-particle bound on the GPU's dv
        assert abs(info["dv_max"] - dvn.max()) <= e.max() + 1e-30
        assert abs(info["dv2_sum"] - (dvn ** 2).sum()) <= (2 * dvn * e + e * e).sum() + 1e-30
        v2 = sum(f(k, s1) ** 2 for k in ("vx", "vy", "vz"))
        assert abs(info["v2_sum"] / max(v2.sum(), 1e-300) - 1) <= 1e-6
    return amb


def check_step_vs_oracle(s0, s1, ref, info, p, dt, T, **params):
    """A GPU step (s0 -> s1, FP32 or FP64) against oracle.step on the same
    start state (ref): raw positions, h, a, du/dt (scaled), v, u, and the
    corrector reductions max|dv|, sum|dv|^2, sum|v|^2 against the oracle's."""
    j = map_to_start(s0["pid"], s1["pid"])
    f32 = T == np.float32
    tolx = 2e-6 if f32 else 1e-12
    check_positions([s1["x"], s1["y"], s1["z"]], [ref["x"][j], ref["y"][j], ref["z"][j]],
                    p.lo, p.hi, tolx)
    hr = np.abs(s1["h"] / ref["h"][j] - 1).max()
    assert hr <= (1e-5 if f32 else 1e-10), hr
    fp = {k: params[k] for k in ("kernel", "gamma", "alpha", "beta", "beta_u") if k in params}
    if "alpha" in ref:
        fp["alpha_arr"] = ref["alpha"]
    fr = oracle.force(ref["x"], ref["y"], ref["z"], ref["vx"], ref["vy"], ref["vz"], ref["u"],
                      ref["h"], ref["rho"], ref["omega"], p.lo, p.hi, p.periodic, p.mass, **fp)
    g = {k: s1[k].astype(np.float64) for k in ("ax", "ay", "az", "dudt")}
    r = {k: ref[k][j] for k in ("ax", "ay", "az", "dudt")}
    r["scale_a"], r["scale_u"] = fr["scale_a"][j], fr["scale_u"][j]
    ea, eu = force_err(g, r)
    tol = 2e-4 if f32 else 1e-9
    assert ea.max() <= tol and eu.max() <= tol, (ea.max(), eu.max())
    # v^{n+1} and u^{n+1}: FP32 rounding of v plus dt/2 times the derivative error
    eps = F32_ULP if f32 else 2.0 ** -52
    vmax = max(np.abs(ref[k]).max() for k in ("vx", "vy", "vz"))
    for k in ("vx", "vy", "vz"):
        err = np.abs(s1[k] - ref[k][j])
        assert (err <= 8 * eps * vmax + dt * tol * r["scale_a"]).all(), k
    err = np.abs(s1["u"] - ref["u"][j])
    assert (err <= 8 * eps * np.abs(ref["u"][j]) + dt * tol * r["scale_u"]).all(), "u"
    # corrector reductions: dv = dt (a^{n+1} - a^n)/2 differs by at most
    # dt/2 times the derivative error (plus rounding of v) per particle
    e = 0.5 * dt * tol * r["scale_a"] + 8 * eps * vmax
    assert abs(info["dv_max"] - ref["diag"][0]) <= e.max()
    dvn = np.sqrt(ref["diag"][1] / max(p.n, 1))
    assert abs(info["dv2_sum"] - ref["diag"][1]) <= 2 * np.sqrt(ref["diag"][1] * (e ** 2).sum()) + (e ** 2).sum()
    assert abs(info["v2_sum"] / ref["diag"][2] - 1) <= 1e-5
    assert ref["diag"][0] > 0 and dvn > 0
    return j
