"""Pins of the oracle's tree half (Morton, sort, reduction, radix tree, boxes,
neighbour sets) against what the paper prints and what mathematics fixes."""
import json
import os

import numpy as np
import pytest

import gen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------- Morton ----
def test_interleave_x_is_msb_of_each_triple():
    # App. B.1: m = X0 Y0 Z0 X1 Y1 Z1 ..., X0 the most significant bit of X.
    assert oracle.interleave(1 << 20, 0, 0) == 1 << 62
    assert oracle.interleave(0, 1 << 20, 0) == 1 << 61
    assert oracle.interleave(0, 0, 1 << 20) == 1 << 60
    assert oracle.interleave(1, 0, 0) == 1 << 2
    assert oracle.interleave(0, 0, 1) == 1
    full = (1 << 21) - 1
    assert oracle.interleave(full, full, full) == (1 << 63) - 1


def test_interleave_roundtrip_random():
    rng = np.random.default_rng(11)
    for _ in range(500):
        X, Y, Z = (int(v) for v in rng.integers(0, 1 << 21, size=3))
        assert oracle.deinterleave(oracle.interleave(X, Y, Z)) == (X, Y, Z)


def test_morton_quantisation_unit_box():
    # [0,1) sampled on 2^21 cells; 1 itself is excluded (clamped to the last cell)
    x = np.array([0.0, 0.5, 1.0 - 2.0 ** -22, 1.0, -1e-9, 0.25 + 2.0 ** -21])
    k = oracle.morton(x, x, x, (0, 0, 0), (1, 1, 1))
    X = [oracle.deinterleave(int(v))[0] for v in k]
    assert X == [0, 1 << 20, (1 << 21) - 1, (1 << 21) - 1, 0, (1 << 19) + 1]


def test_morton_order_matches_octree_halving():
    # first key bit = x >= 1/2, second = y >= 1/2, third = z >= 1/2 (Fig. octree_morton)
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 1, size=(200, 3))
    k = oracle.morton(p[:, 0], p[:, 1], p[:, 2], (0, 0, 0), (1, 1, 1))
    top = (k >> np.uint64(60)).astype(int)
    want = 4 * (p[:, 0] >= 0.5) + 2 * (p[:, 1] >= 0.5) + (p[:, 2] >= 0.5)
    assert np.array_equal(top, want)


# ------------------------------------------------- sort + mask (Fig.) ----
def _codes3(strs):
    return np.array([int(s, 2) << 61 for s in strs], np.uint64)


def test_fig_mortonlistbuild_exact():
    g = _load("fig_mortonlistbuild.json")
    m = _codes3(g["codes"])
    eps, mu = oracle.sort(m)
    assert np.array_equal(mu, _codes3(g["sorted"]))
    assert np.array_equal(mu, m[eps])            # mu_i = m_{eps_i}
    # stability: equal codes keep their original order
    for i in range(len(mu) - 1):
        if mu[i] == mu[i + 1]:
            assert eps[i] < eps[i + 1]
    xi, ids, ml = oracle.leaves(mu, 0)
    assert xi.tolist() == g["xi"]
    assert ids.tolist() == g["id"]                # last slot = input length
    assert np.array_equal(ml, _codes3(g["mu_leaf"]))


def _tree_from_codes(codes):
    """Independent plain-Python radix tree: nested (left, right) tuples of
    leaf indices, splitting each range at its first differing bit."""
    def build(f, l):
        if f == l:
            return f
        a, b = int(codes[f]), int(codes[l])
        p = 64 - (a ^ b).bit_length()
        bit = 1 << (63 - p)
        g = f
        while g + 1 <= l and not (int(codes[g + 1]) & bit):
            g += 1
        return (build(f, g), build(g + 1, l))
    return build(0, len(codes) - 1)


def _sibling_reduction(mu, n_red):
    """The reduction as the paper states it in words (App. C.2): in the tree
    of the currently kept codes, a code that is the second leaf of an
    internal node whose two children are both leaves is removed."""
    n = len(mu)
    keep = [True] + [mu[i] != mu[i - 1] for i in range(1, n)]
    for _ in range(n_red):
        kept = [i for i in range(n) if keep[i]]
        if len(kept) < 2:
            break
        t = _tree_from_codes([mu[i] for i in kept])
        removed = set()

        def walk(node):
            if isinstance(node, tuple):
                l, r = node
                if not isinstance(l, tuple) and not isinstance(r, tuple):
                    removed.add(kept[r])
                walk(l)
                walk(r)
        walk(t)
        for i in removed:
            keep[i] = False
    return np.array(keep, np.uint8)


def test_reduction_on_fig_example():
    g = _load("fig_mortonlistbuild.json")
    mu = _codes3(g["sorted"])
    for n_red in range(4):
        xi, ids, ml = oracle.leaves(mu, n_red)
        assert np.array_equal(xi, _sibling_reduction(list(mu), n_red)), n_red
    # pass 1: leaves {000,000,001}, {010,011,011}, {100}
    xi, ids, _ = oracle.leaves(mu, 1)
    assert ids.tolist() == [0, 3, 6, 7]


@pytest.mark.parametrize("seed", range(6))
def test_reduction_matches_sibling_definition_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    bits = int(rng.integers(3, 12))
    codes = rng.integers(0, 1 << bits, size=n).astype(np.uint64) << np.uint64(63 - bits)
    _, mu = oracle.sort(codes)
    for n_red in range(5):
        xi, _, _ = oracle.leaves(mu, n_red)
        assert np.array_equal(xi, _sibling_reduction(list(mu), n_red)), (seed, n_red)
        # no two adjacent kept codes are removed by the same pass
        assert xi[0] == 1


def test_reduction_halves_leaves_on_power_of_two_lattice():
    # 16^3 unjittered lattice: each pass merges all sibling leaf pairs
    p = gen.lattice(16, 1, dtype=np.float64, jitter=0.0)
    k = oracle.morton(p.x, p.y, p.z, p.lo, p.hi)
    _, mu = oracle.sort(k)
    for n_red in range(5):
        _, ids, _ = oracle.leaves(mu, n_red)
        assert len(ids) - 1 == 4096 >> n_red


# ------------------------------------------------------ Karras (Table) ----
def test_karras_table_exact():
    g = _load("karras_table.json")
    codes = np.array([int(c, 16) for c in g["codes"]], np.uint64)
    t = oracle.radix_tree(codes)
    for key in ("lchild", "rchild", "lflag", "rflag", "endrange"):
        assert t[key].tolist() == g[key], key


def _check_tree_invariants(mu_leaf, t):
    nl = len(mu_leaf)
    ni = nl - 1
    seen_leaf = np.zeros(nl, int)
    seen_int = np.zeros(max(ni, 1), int)

    def rng_of(i):
        a, b = i, int(t["endrange"][i])
        return min(a, b), max(a, b)

    stack = [(0, False)] if ni > 0 else []
    while stack:
        i, _ = stack.pop()
        seen_int[i] += 1
        f, l = rng_of(i)
        lc, rc = int(t["lchild"][i]), int(t["rchild"][i])
        # children partition the parent's range at the split lc | rc = lc + 1
        assert rc == lc + 1 and f <= lc < l
        d_parent = oracle.delta(int(mu_leaf[f]), int(mu_leaf[l]))
        for c, flag, (cf, cl) in ((lc, t["lflag"][i], (f, lc)), (rc, t["rflag"][i], (rc, l))):
            if flag:
                assert cf == cl == c
                seen_leaf[c] += 1
                assert int(t["parent"][ni + c]) == i
            else:
                assert rng_of(c) == (cf, cl)
                assert oracle.delta(int(mu_leaf[cf]), int(mu_leaf[cl])) > d_parent
                assert int(t["parent"][c]) == i
                stack.append((c, False))
        # the split is at the first differing bit
        bit = np.uint64(1) << np.uint64(63 - d_parent)
        assert all((mu_leaf[j] & bit) == 0 for j in range(f, lc + 1))
        assert all((mu_leaf[j] & bit) != 0 for j in range(lc + 1, l + 1))
    assert (seen_leaf == 1).all()
    if ni:
        assert (seen_int[:ni] == 1).all()


@pytest.mark.parametrize("seed", range(5))
def test_radix_tree_invariants_random(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 600))
    keys = np.unique(rng.integers(0, 1 << 63, size=n, dtype=np.uint64))
    t = oracle.radix_tree(keys)
    _check_tree_invariants(keys, t)
    # same structure as the independent nested-tuple construction
    ref = _tree_from_codes(list(keys))

    def to_tuple(node, is_leaf):
        if is_leaf:
            return node
        return (to_tuple(int(t["lchild"][node]), bool(t["lflag"][node])),
                to_tuple(int(t["rchild"][node]), bool(t["rflag"][node])))
    assert to_tuple(0, len(keys) == 1) == ref


def test_single_leaf_tree():
    t = oracle.radix_tree(np.array([12345], np.uint64))
    assert len(t["lchild"]) == 0 and len(t["parent"]) == 1


# -------------------------------------------------------------- boxes ----
def _tree_for(p, n_red):
    k = oracle.morton(p.x, p.y, p.z, p.lo, p.hi)
    eps, mu = oracle.sort(k)
    xi, ids, ml = oracle.leaves(mu, n_red)
    t = oracle.radix_tree(ml)
    return eps, mu, ids, ml, t


@pytest.mark.parametrize("n_red", [0, 2, 3])
def test_tight_boxes_inside_prefix_boxes(n_red):
    p = gen.plummer(3000, 9, dtype=np.float64)
    eps, mu, ids, ml, t = _tree_for(p, n_red)
    xs, ys, zs, hs = p.x[eps], p.y[eps], p.z[eps], p.h[eps]
    bmin, bmax, hmax = oracle.tight_boxes(ids, t, xs, ys, zs, hs)
    box, plen = oracle.prefix_boxes(ml, t)
    lo = np.array(p.lo)
    s = (1 << 21) / (np.array(p.hi) - lo)
    # real image of the integer box [X0, X1+1) / s + lo contains the tight box
    assert (bmin >= lo + box[:, :3] / s - 1e-12).all()
    assert (bmax <= lo + (box[:, 3:].astype(np.float64) + 1) / s + 1e-12).all()
    # child boxes nest in their parents, h_max is monotone up the tree
    ni = len(ml) - 1
    for i in range(ni):
        for c, fl in ((t["lchild"][i], t["lflag"][i]), (t["rchild"][i], t["rflag"][i])):
            v = ni + c if fl else c
            assert (bmin[v] >= bmin[i]).all() and (bmax[v] <= bmax[i]).all()
            assert hmax[v] <= hmax[i]
            assert (box[v, :3] >= box[i, :3]).all() and (box[v, 3:] <= box[i, 3:]).all()
    # every particle lies in its leaf's tight box
    for k in range(len(ml)):
        sl = slice(ids[k], ids[k + 1])
        assert xs[sl].min() == bmin[ni + k, 0] and xs[sl].max() == bmax[ni + k, 0]


def test_aabb_extension_permutation_theorem():
    # Eq. AABB_theo: (A (+) h) n B != 0  <=>  A n (B (+) h) != 0
    rng = np.random.default_rng(5)
    for _ in range(4000):
        a = np.sort(rng.uniform(0, 1, (3, 2)), axis=1)
        b = np.sort(rng.uniform(0, 1, (3, 2)), axis=1)
        h = rng.uniform(0, 0.3)
        lhs = all(max(a[d, 0] - h, b[d, 0]) <= min(a[d, 1] + h, b[d, 1]) for d in range(3))
        rhs = all(max(a[d, 0], b[d, 0] - h) <= min(a[d, 1], b[d, 1] + h) for d in range(3))
        assert lhs == rhs


# --------------------------------------------------------- neighbours ----
def _lattice_shell_counts(eta, radius_factor):
    """Number of integer offsets n with |n| < radius_factor * eta (App. B,
    cubic lattice, unit spacing): the neighbour count of every particle."""
    R = int(np.ceil(radius_factor * eta)) + 1
    r = np.arange(-R, R + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    d2 = X ** 2 + Y ** 2 + Z ** 2
    return int((d2 < (radius_factor * eta) ** 2).sum())


@pytest.mark.parametrize("T", [np.float32, np.float64])
def test_neighbour_counts_jittered_lattice(T):
    p = gen.lattice(16, 1, dtype=T)
    n81 = _lattice_shell_counts(1.2, 2.2)
    n57 = _lattice_shell_counts(1.2, 2.0)
    assert (n81, n57) == (81, 57)
    off, _ = oracle.neighbours(p.x, p.y, p.z, p.h, p.lo, p.hi, True, 2.2)
    assert (np.diff(off.astype(np.int64)) == n81).all()
    off, _ = oracle.neighbours(p.x, p.y, p.z, p.h, p.lo, p.hi, True, 2.0)
    assert (np.diff(off.astype(np.int64)) == n57).all()


@pytest.mark.parametrize("family", ["lattice", "plummer"])
def test_neighbours_grid_equals_brute_force(family):
    if family == "lattice":
        p = gen.lattice(12, 7, dtype=np.float32)
        p.h = (p.h * np.random.default_rng(1).uniform(0.7, 1.3, p.n)).astype(np.float32)
    else:
        p = gen.plummer(3000, 4, dtype=np.float32)
    a = oracle.neighbours(p.x, p.y, p.z, p.h, p.lo, p.hi, p.periodic, 2.2)
    b = oracle.neighbours(p.x, p.y, p.z, p.h, p.lo, p.hi, p.periodic, 2.2, brute=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    off, lst = a
    for i in range(0, p.n, 97):       # ascending, self included, symmetric
        seg = lst[off[i]:off[i + 1]]
        assert (np.diff(seg.astype(np.int64)) > 0).all() and i in seg
        for j in seg[:5]:
            assert i in lst[off[j]:off[j + 1]]
    # a target subset gives exactly those rows
    t = np.array([p.n - 1, 0, 5, 5, 1234 % p.n])
    to, tl = oracle.neighbours(p.x, p.y, p.z, p.h, p.lo, p.hi, p.periodic, 2.2, targets=t)
    for r, i in enumerate(t):
        assert np.array_equal(tl[to[r]:to[r + 1]], lst[off[i]:off[i + 1]])


def test_neighbours_float_decision_in_float():
    # two particles exactly at a distance that is < rc in float but not in
    # double must be taken by the float decision (the storage precision)
    x = np.array([0.1, 0.1 + 0.05], np.float32)
    y = np.zeros(2, np.float32) + 0.5
    z = np.zeros(2, np.float32) + 0.5
    h = np.full(2, np.float32(0.05) / np.float32(2.2), np.float32)
    off, lst = oracle.neighbours(x, y, z, h, (0, 0, 0), (1, 1, 1), True, 2.2)
    dx = np.float32(x[1] - x[0])
    rc = np.float32(2.2) * h[0]
    want = 2 if dx * dx < rc * rc else 1
    assert int(off[1] - off[0]) == want


# Pairs (float32 positions, common h) on which r^2 formed with fused
# multiply-adds and r^2 formed as (dx*dx + dy*dy) + dz*dz fall on opposite
# sides of the squared cache radius.  Found by a seeded search; the decision
# the criterion of App. E asks for is the real-valued one.
_STRADDLE_F32 = [
    # h, particle b (particle a sits at (0.25, 0.375, 0.3125))
    (0.012568564154207706, (0.2501320242881775, 0.34750130772590637, 0.30960628390312195)),
    (0.013240364380180836, (0.25197258591651917, 0.39744433760643005, 0.33096206188201904)),
]


def _round_f32(v):
    """Round an exact rational to the nearest float32 (ties to even)."""
    from fractions import Fraction
    if v == 0:
        return Fraction(0)
    s, a = (-1 if v < 0 else 1), abs(v)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    sc = Fraction(2) ** (e - 23)
    m = a / sc
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return s * fl * sc


@pytest.mark.parametrize("case", range(len(_STRADDLE_F32)))
def test_neighbour_r2_rounding_takes_the_exact_side(case):
    """The storage-type r^2 is formed with fused multiply-adds (each partial
    sum rounded once).  On these pairs the unfused sum rounds to the other
    side of rc^2; the oracle must take the side of the exact real-valued
    comparison of the (exactly representable) differences with rc^2."""
    from fractions import Fraction as Fr
    h, pb = _STRADDLE_F32[case]
    pa = (0.25, 0.375, 0.3125)
    x = np.array([pa[0], pb[0]], np.float32)
    y = np.array([pa[1], pb[1]], np.float32)
    z = np.array([pa[2], pb[2]], np.float32)
    hh = np.full(2, h, np.float32)
    d = [Fr(float(c[1])) - Fr(float(c[0])) for c in (x, y, z)]
    for k, c in enumerate((x, y, z)):   # the float differences are exact
        assert Fr(float(np.float32(c[1] - c[0]))) == d[k]
    rc = _round_f32(_round_f32(Fr(11, 5)) * Fr(float(hh[0])))
    rc2 = _round_f32(rc * rc)
    exact = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 < rc2
    unfused = _round_f32(_round_f32(_round_f32(d[0] ** 2) + _round_f32(d[1] ** 2))
                         + _round_f32(d[2] ** 2)) < rc2
    assert exact != unfused            # the case does separate the two forms
    off, lst = oracle.neighbours(x, y, z, hh, (0, 0, 0), (1, 1, 1), False, 2.2)
    assert int(off[1] - off[0]) == (2 if exact else 1)
    assert int(off[2] - off[1]) == (2 if exact else 1)


def test_leaf_prefix_boxes_are_the_leaf_blocks():
    """16^3 lattice, three reduction passes: every leaf is one 2x2x2 block of
    lattice cells (each pass merges sibling leaves), so its prefix box
    (parent's prefix length + 1) is exactly that block: 2^18 grid cells per
    side, aligned to 2^18.  A leaf given its parent's length would be twice
    as long on one axis.  The root's box is the whole grid."""
    p = gen.lattice(16, 1, dtype=np.float64)
    k = oracle.morton(p.x, p.y, p.z, p.lo, p.hi)
    eps, mu = oracle.sort(k)
    _, ids, ml = oracle.leaves(mu, 3)
    assert len(ml) == 512
    t = oracle.radix_tree(ml)
    box, plen = oracle.prefix_boxes(ml, t)
    ni = len(ml) - 1
    side = 1 << 18
    leaf = box[ni:].astype(np.int64)
    assert (leaf[:, 3:] - leaf[:, :3] == side - 1).all()
    assert (leaf[:, :3] % side == 0).all()
    # the block holds exactly the leaf's particles
    g = (np.stack([p.x, p.y, p.z], 1)[eps] * (1 << 21)).astype(np.int64)
    for j in range(0, 512, 37):
        sl = slice(ids[j], ids[j + 1])
        assert ids[j + 1] - ids[j] == 8
        assert (g[sl] >= leaf[j, :3]).all() and (g[sl] <= leaf[j, 3:]).all()
    assert box[0].tolist() == [0, 0, 0, (1 << 21) - 1, (1 << 21) - 1, (1 << 21) - 1]
    assert plen[0] == 1            # only the unused top bit is common to all codes


# ----------------------------------------------------- 30-bit Morton codes --
def test_morton30_interleave_hand_values():
    # 10 bits per axis, X the most significant of each triple (App. B.1), the
    # 30-bit code in the low bits
    assert oracle.interleave_bits(1 << 9, 0, 0, 10) == 1 << 29
    assert oracle.interleave_bits(0, 1 << 9, 0, 10) == 1 << 28
    assert oracle.interleave_bits(0, 0, 1 << 9, 10) == 1 << 27
    assert oracle.interleave_bits(0, 0, 1, 10) == 1
    assert oracle.interleave_bits(1023, 1023, 1023, 10) == (1 << 30) - 1


def test_morton30_is_the_top_of_morton63():
    """Quantising to 2^10 cells is quantising to 2^21 and dropping 11 bits
    (scaling by powers of two is exact in FP64), so the 30-bit code is the
    63-bit code shifted right by 33: the two definitions pin each other."""
    rng = np.random.default_rng(23)
    p = rng.uniform(0, 1, size=(5000, 3))
    p[:7] = [[0, 0, 0], [1 - 2 ** -40, 0.5, 0.25], [1.0, 1.0, 1.0], [-0.1, 2.0, 0.5],
             [2 ** -11, 2 ** -10, 2 ** -22], [0.5 - 2 ** -30, 0.5, 0.5], [0.75, 0.125, 0.999]]
    k63 = oracle.morton(p[:, 0], p[:, 1], p[:, 2], (0, 0, 0), (1, 1, 1))
    k30 = oracle.morton(p[:, 0], p[:, 1], p[:, 2], (0, 0, 0), (1, 1, 1), bits=10)
    assert np.array_equal(k30, k63 >> np.uint64(33))
    assert int(k30.max()) < (1 << 30)
