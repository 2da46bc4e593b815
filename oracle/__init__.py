"""CPU FP64 oracle of the SPH hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2503_09713_amd``) and neither imports the other.

The arithmetic lives in ``oracle.c`` (plain C, built by gcc with
``-O2 -fopenmp -ffp-contract=off``); this module only marshals numpy arrays.
Every function cites the passage of the paper it restates; see oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
f32p = np.ctypeslib.ndpointer(np.float32, flags="C")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C")


KERNELS = {"M4": 0, "M5": 1, "M6": 2, "C2": 3, "C4": 4, "C6": 5}


class OrcParams(C.Structure):
    """Parameters of the oracle's step (mirrors orc_params in oracle.c)."""
    _fields_ = [("hfact", C.c_double), ("gamma", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("beta_u", C.c_double), ("c_cour", C.c_double),
                ("c_force", C.c_double), ("kernel", C.c_int), ("eps_v", C.c_double),
                ("max_rerun", C.c_int), ("alpha_switch", C.c_int), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("sigma_decay", C.c_double)]


def _kid(kernel) -> int:
    return KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def make_params(hfact=1.2, gamma=5.0 / 3.0, alpha=1.0, beta=2.0, beta_u=1.0, c_cour=0.3,
                c_force=0.25, kernel="M4", eps_v=0.0, max_rerun=0, alpha_switch=False,
                alpha_min=0.0, alpha_max=1.0, sigma_decay=0.1) -> OrcParams:
    return OrcParams(hfact, gamma, alpha, beta, beta_u, c_cour, c_force, _kid(kernel),
                     eps_v, max_rerun, int(bool(alpha_switch)), alpha_min, alpha_max,
                     sigma_decay)


def build() -> str:
    """Compile oracle.c into liboracle.so (gcc, no GPU code)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    L = C.CDLL(_LIB)
    i64, f64, i32 = C.c_int64, C.c_double, C.c_int
    vp = C.c_void_p
    L.orc_version.restype = i32
    L.orc_threads.restype = i32
    L.orc_set_threads.argtypes = [i32]
    L.orc_interleave.restype = C.c_uint64
    L.orc_interleave.argtypes = [C.c_uint32] * 3
    L.orc_deinterleave.argtypes = [C.c_uint64, vp, vp, vp]
    L.orc_morton.argtypes = [i64, f64p, f64p, f64p, f64p, f64p, u64p]
    L.orc_morton_bits.argtypes = [i64, f64p, f64p, f64p, f64p, f64p, i32, u64p]
    L.orc_interleave_bits.restype = C.c_uint64
    L.orc_interleave_bits.argtypes = [C.c_uint32] * 3 + [i32]
    L.orc_delta.restype = i32
    L.orc_delta.argtypes = [C.c_uint64, C.c_uint64]
    L.orc_sort.argtypes = [i64, u64p, u32p, u64p]
    L.orc_leaves.restype = i64
    L.orc_leaves.argtypes = [i64, u64p, i32, u8p, u32p, u64p]
    L.orc_radix_tree.argtypes = [i64, u64p, u32p, u32p, u8p, u8p, u32p, u32p]
    L.orc_prefix_boxes.argtypes = [i64, u64p, u32p, u32p, u32p, i32p]
    L.orc_tight_boxes.argtypes = [i64, u32p, u32p, f64p, f64p, f64p, f64p, f64p, f64p, f64p]
    for suf, fp in (("f32", f32p), ("f64", f64p)):
        fn = getattr(L, "orc_neigh_" + suf)
        fn.restype = i64
        fn.argtypes = [i64, fp, fp, fp, fp, f64p, f64p, i32, f64, i32, i64, vp, u64p, u32p, i64]
    L.orc_m4_f.restype = f64
    L.orc_m4_f.argtypes = [f64]
    L.orc_m4_df.restype = f64
    L.orc_m4_df.argtypes = [f64]
    L.orc_kernel_count.restype = i32
    for fn in ("orc_kernel_support", "orc_kernel_norm"):
        getattr(L, fn).restype = f64
        getattr(L, fn).argtypes = [i32]
    for fn in ("orc_kernel_f", "orc_kernel_df"):
        getattr(L, fn).restype = f64
        getattr(L, fn).argtypes = [i32, f64]
    L.orc_density.argtypes = [i64, f64p, f64p, f64p, f64p, f64p, f64p, i32, f64, f64, i32,
                              i64, vp, f64p, f64p, f64p, i32p]
    L.orc_density_sum.argtypes = [i64, f64p, f64p, f64p, f64p, f64p, f64p, i32, f64, i32,
                                  i64, vp, f64p, f64p]
    L.orc_force.argtypes = [i64] + [f64p] * 10 + [f64p, f64p, i32, f64, f64, f64, vp, f64, f64,
                                                   i32, i64, vp] + [f64p] * 7
    L.orc_gradient.argtypes = [i64] + [f64p] * 9 + [f64p, f64p, i32, f64, i32, i64, vp, f64p]
    L.orc_alpha_switch.argtypes = [i64] + [f64p] * 14 + [f64p, f64p, i32, f64,
                                                          C.POINTER(OrcParams), f64, f64p, vp, vp, vp]
    L.orc_cfl_multiplier.restype = f64
    L.orc_cfl_multiplier.argtypes = [f64, i32, f64]
    L.orc_cfl.restype = f64
    L.orc_cfl.argtypes = [i64, f64p, f64p, f64p, f64p, f64p, f64, f64]
    L.orc_step.argtypes = [i64] + [f64p] * 14 + [vp, f64p, f64p, i32, f64,
                                                  C.POINTER(OrcParams), f64, f64p]
    _lib = L
    return L


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _box(lo, hi):
    return _d(lo).reshape(3), _d(hi).reshape(3)


def _targets(targets):
    if targets is None:
        return None, None
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    return t, t.ctypes.data_as(C.c_void_p)


# ----------------------------------------------------------------- tree --
def interleave(X, Y, Z) -> int:
    """Morton interleave X0 Y0 Z0 X1 ... of 21-bit integers (App. B.1)."""
    return int(lib().orc_interleave(int(X), int(Y), int(Z)))


def deinterleave(key: int):
    a, b, c = C.c_uint32(), C.c_uint32(), C.c_uint32()
    lib().orc_deinterleave(C.c_uint64(int(key)), C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def delta(a: int, b: int) -> int:
    """Longest common prefix length clz(a ^ b) (Eq. delta_ab)."""
    return int(lib().orc_delta(C.c_uint64(int(a)), C.c_uint64(int(b))))


def morton(x, y, z, lo, hi, bits=21) -> np.ndarray:
    """Morton keys, `bits` per axis (21: 63-bit codes, 10: 30-bit codes),
    quantised in FP64 (App. B.1, Sect. 5.2.1)."""
    x, y, z = _d(x), _d(y), _d(z)
    lo, hi = _box(lo, hi)
    key = np.empty(x.shape[0], np.uint64)
    if bits == 21:
        lib().orc_morton(x.shape[0], x, y, z, lo, hi, key)
    else:
        lib().orc_morton_bits(x.shape[0], x, y, z, lo, hi, int(bits), key)
    return key


def interleave_bits(X, Y, Z, bits) -> int:
    return int(lib().orc_interleave_bits(int(X), int(Y), int(Z), int(bits)))


def sort(key):
    """Stable sort by key: returns (eps, mu) with mu[i] = key[eps[i]]."""
    key = np.ascontiguousarray(key, dtype=np.uint64)
    n = key.shape[0]
    eps = np.empty(n, np.uint32)
    mu = np.empty(n, np.uint64)
    lib().orc_sort(n, key, eps, mu)
    return eps, mu


def leaves(mu, n_red: int):
    """Keep mask after dedupe + n_red reduction passes, and its compaction
    (App. C, Alg. 1 and Fig. mortonlistbuild).  Returns (xi, id, mu_leaf)."""
    mu = np.ascontiguousarray(mu, dtype=np.uint64)
    n = mu.shape[0]
    xi = np.zeros(max(n, 1), np.uint8)
    ids = np.zeros(n + 1, np.uint32)
    ml = np.zeros(max(n, 1), np.uint64)
    nl = lib().orc_leaves(n, mu, int(n_red), xi, ids, ml)
    return xi[:n], ids[: nl + 1].copy(), ml[:nl].copy()


def radix_tree(mu_leaf):
    """Karras tables of the binary radix tree over distinct sorted codes
    (App. B.7 and its Table).  parent[] covers internal nodes then leaves."""
    ml = np.ascontiguousarray(mu_leaf, dtype=np.uint64)
    nl = ml.shape[0]
    ni = max(nl - 1, 0)
    t = dict(lchild=np.zeros(max(ni, 1), np.uint32), rchild=np.zeros(max(ni, 1), np.uint32),
             lflag=np.zeros(max(ni, 1), np.uint8), rflag=np.zeros(max(ni, 1), np.uint8),
             endrange=np.zeros(max(ni, 1), np.uint32),
             parent=np.zeros(max(2 * nl - 1, 1), np.uint32))
    lib().orc_radix_tree(nl, ml, t["lchild"], t["rchild"], t["lflag"], t["rflag"],
                         t["endrange"], t["parent"])
    for k in ("lchild", "rchild", "lflag", "rflag", "endrange"):
        t[k] = t[k][:ni]
    t["parent"] = t["parent"][: max(2 * nl - 1, 0)]
    return t


def prefix_boxes(mu_leaf, tree):
    """Integer prefix-class box of every node (App. B.6): (box[nn,6], len[nn])."""
    ml = np.ascontiguousarray(mu_leaf, dtype=np.uint64)
    nl = ml.shape[0]
    nn = 2 * nl - 1
    box = np.zeros((nn, 6), np.uint32)
    plen = np.zeros(nn, np.int32)
    er = tree["endrange"] if nl > 1 else np.zeros(1, np.uint32)
    par = tree["parent"] if nn > 0 else np.zeros(1, np.uint32)
    lib().orc_prefix_boxes(nl, ml, np.ascontiguousarray(er, np.uint32),
                           np.ascontiguousarray(par, np.uint32), box.reshape(-1), plen)
    return box, plen


def tight_boxes(ids, tree, xs, ys, zs, hs):
    """Tight AABB and h_max of every node by brute force (sorted-order fields)."""
    nl = ids.shape[0] - 1
    nn = 2 * nl - 1
    bmin = np.zeros((nn, 3))
    bmax = np.zeros((nn, 3))
    hmax = np.zeros(nn)
    er = tree["endrange"] if nl > 1 else np.zeros(1, np.uint32)
    lib().orc_tight_boxes(nl, np.ascontiguousarray(ids, np.uint32),
                          np.ascontiguousarray(er, np.uint32), _d(xs), _d(ys), _d(zs),
                          _d(hs), bmin.reshape(-1), bmax.reshape(-1), hmax)
    return bmin, bmax, hmax


def neighbours(x, y, z, h, lo, hi, periodic: bool, r_kern_chi: float, brute=False,
               targets=None):
    """Neighbour sets decided in the storage precision of x (App. E):
    returns (offsets[nt+1] uint64, list uint32), ascending, self included,
    for the targets (default: every particle)."""
    x = np.ascontiguousarray(x)
    T = x.dtype
    if T not in (np.float32, np.float64):
        raise TypeError(T)
    suf = "f32" if T == np.float32 else "f64"
    arrs = [np.ascontiguousarray(a, dtype=T) for a in (x, y, z, h)]
    lo, hi = _box(lo, hi)
    n = x.shape[0]
    t, tp = _targets(targets)
    nt = n if t is None else t.shape[0]
    off = np.zeros(nt + 1, np.uint64)
    cap = max(nt * 64, 1)
    fn = getattr(lib(), "orc_neigh_" + suf)
    while True:
        lst = np.zeros(cap, np.uint32)
        tot = fn(n, *arrs, lo, hi, int(bool(periodic)), float(r_kern_chi), int(brute), nt, tp,
                 off, lst, cap)
        if tot >= 0:
            return off, lst[:tot].copy()
        cap = -tot


# ---------------------------------------------------------------- physics --
def m4_f(q: float) -> float:
    return float(lib().orc_m4_f(float(q)))


def m4_df(q: float) -> float:
    return float(lib().orc_m4_df(float(q)))


def kernel_f(kernel, q: float) -> float:
    """f(q) of the named kernel (Sect. 2.1.1: M4, M5, M6, C2, C4, C6)."""
    return float(lib().orc_kernel_f(_kid(kernel), float(q)))


def kernel_df(kernel, q: float) -> float:
    return float(lib().orc_kernel_df(_kid(kernel), float(q)))


def kernel_support(kernel) -> float:
    """Support radius R in units of h."""
    return float(lib().orc_kernel_support(_kid(kernel)))


def kernel_norm(kernel) -> float:
    """3-D normalisation C_norm."""
    return float(lib().orc_kernel_norm(_kid(kernel)))


def density(x, y, z, h0, lo, hi, periodic, mass, hfact=1.2, targets=None, kernel="M4"):
    """Self-consistent h, rho = m (hfact/h)^3 and Omega (App. F, Eq. sphomega).
    Returns (h, rho, omega, flags) for the targets (default: all)."""
    x, y, z, h0 = _d(x), _d(y), _d(z), _d(h0)
    lo, hi = _box(lo, hi)
    t, tp = _targets(targets)
    nt = x.shape[0] if t is None else t.shape[0]
    h = np.zeros(nt); rho = np.zeros(nt); om = np.zeros(nt)
    fl = np.zeros(nt, np.int32)
    lib().orc_density(x.shape[0], x, y, z, h0, lo, hi, int(bool(periodic)), float(mass),
                      float(hfact), _kid(kernel), nt, tp, h, rho, om, fl)
    return h, rho, om, fl


def density_sum(x, y, z, h, lo, hi, periodic, mass, targets=None, kernel="M4"):
    """Plain SPH sum rho_a = sum_b m W_ab(h_a) (Eq. SPHmass) and sum m dW/dh."""
    x, y, z, h = _d(x), _d(y), _d(z), _d(h)
    lo, hi = _box(lo, hi)
    t, tp = _targets(targets)
    nt = x.shape[0] if t is None else t.shape[0]
    s = np.zeros(nt); ds = np.zeros(nt)
    lib().orc_density_sum(x.shape[0], x, y, z, h, lo, hi, int(bool(periodic)),
                          float(mass), _kid(kernel), nt, tp, s, ds)
    return s, ds


def force(x, y, z, vx, vy, vz, u, h, rho, omega, lo, hi, periodic, mass,
          gamma=5.0 / 3.0, alpha=1.0, beta=2.0, beta_u=1.0, targets=None, kernel="M4",
          alpha_arr=None):
    """dv/dt, du/dt (Eqs. sphvel, sphuint with AV and conductivity), the
    signal speed for the timestep and the per-particle error scales.
    alpha_arr: per-particle viscosity alpha (default: the constant alpha)."""
    arrs = [_d(a) for a in (x, y, z, vx, vy, vz, u, h, rho, omega)]
    lo, hi = _box(lo, hi)
    t, tp = _targets(targets)
    n = arrs[0].shape[0]
    nt = n if t is None else t.shape[0]
    out = [np.zeros(nt) for _ in range(7)]
    al = None if alpha_arr is None else _d(alpha_arr)
    lib().orc_force(n, *arrs, lo, hi, int(bool(periodic)), float(mass), float(gamma),
                    float(alpha), None if al is None else al.ctypes.data_as(C.c_void_p),
                    float(beta), float(beta_u), _kid(kernel), nt, tp, *out)
    keys = ("ax", "ay", "az", "dudt", "vsig", "scale_a", "scale_u")
    return dict(zip(keys, out))


def gradient(x, y, z, fx, fy, fz, h, rho, omega, lo, hi, periodic, mass, kernel="M4",
             targets=None):
    """SPH gradient of a vector field, (nt, 3, 3) with [i][j] = d_j f_i."""
    arrs = [_d(a) for a in (x, y, z, fx, fy, fz, h, rho, omega)]
    lo, hi = _box(lo, hi)
    t, tp = _targets(targets)
    n = arrs[0].shape[0]
    nt = n if t is None else t.shape[0]
    out = np.zeros(9 * nt)
    lib().orc_gradient(n, *arrs, lo, hi, int(bool(periodic)), float(mass), _kid(kernel),
                       nt, tp, out)
    return out.reshape(nt, 3, 3)


def alpha_switch(x, y, z, vx, vy, vz, ax, ay, az, u, h, rho, omega, alpha_n, lo, hi,
                 periodic, mass, dt, **params):
    """Shock detector and implicit alpha update (App. G, Shock detection):
    returns dict(alpha, alpha_loc, divv, ddivv_dt)."""
    arrs = [_d(a) for a in (x, y, z, vx, vy, vz, ax, ay, az, u, h, rho, omega, alpha_n)]
    lo, hi = _box(lo, hi)
    n = arrs[0].shape[0]
    P = make_params(**params)
    out = [np.zeros(n) for _ in range(4)]
    lib().orc_alpha_switch(n, *arrs, lo, hi, int(bool(periodic)), float(mass), C.byref(P),
                           float(dt), out[0], out[1].ctypes.data_as(C.c_void_p),
                           out[2].ctypes.data_as(C.c_void_p), out[3].ctypes.data_as(C.c_void_p))
    return dict(alpha=out[0], alpha_loc=out[1], divv=out[2], ddivv_dt=out[3])


def cfl_multiplier(lam: float, rerun: bool, lambda_stiff: float) -> float:
    """Next CFL multiplier (App. G, CFL multiplier)."""
    return float(lib().orc_cfl_multiplier(float(lam), int(bool(rerun)), float(lambda_stiff)))


def cfl(h, vsig, ax, ay, az, c_cour=0.3, c_force=0.25) -> float:
    h = _d(h)
    return float(lib().orc_cfl(h.shape[0], h, _d(vsig), _d(ax), _d(ay), _d(az),
                               float(c_cour), float(c_force)))


def step(state: dict, lo, hi, periodic, mass, dt, **params):
    """One fixed-dt KDK step (App. G.1).  ``state`` holds x,y,z,vx,vy,vz,u,h,
    ax,ay,az,dudt (and alpha with alpha_switch=True); FP64 copies are made.
    params: see make_params (hfact, kernel, eps_v / max_rerun for corrector
    re-runs, the alpha switch ...).  Returns the new state dict with rho,
    omega and diag = (max|dv|, sum|dv|^2, sum|v|^2, cfl dt, re-runs)."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az", "dudt")
    s = {k: _d(state[k]).copy() for k in keys}
    n = s["x"].shape[0]
    s["rho"] = np.zeros(n); s["omega"] = np.zeros(n)
    P = make_params(**params)
    al = None
    if P.alpha_switch:
        al = _d(state["alpha"]).copy() if "alpha" in state else np.full(n, P.alpha)
        s["alpha"] = al
    diag = np.zeros(5)
    lo, hi = _box(lo, hi)
    lib().orc_step(n, *[s[k] for k in keys], s["rho"], s["omega"],
                   None if al is None else al.ctypes.data_as(C.c_void_p), lo, hi,
                   int(bool(periodic)), float(mass), C.byref(P), float(dt), diag)
    s["diag"] = diag
    return s


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))
