"""shsph_step_noalloc (all device working memory in the library's static
per-device scratch array) against shsph_step on the same inputs: bit for bit,
over two calls in a row, the second with a smaller input, with the scratch
array used by another context in between, and CFL steps that take the dt of
the context's own previous allocation-free step; an FP64 step near the
particle limit; the size limit itself."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

shsph = pytest.importorskip("paper_2503_09713_amd")

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az", "dudt", "rho",
          "omega", "pid")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _state(n1, seed, T):
    """A jittered lattice with random v and u, its h, rho, Omega and
    derivatives from one plain build + density + force."""
    p = gen.lattice(n1, seed, dtype=T)
    rng = np.random.default_rng(seed)
    for k in ("vx", "vy", "vz"):
        setattr(p, k, (rng.standard_normal(p.n) * 0.1).astype(T))
    p.u = (p.u * (1 + 0.3 * rng.uniform(-1, 1, p.n))).astype(T)
    ctx = shsph.Context(0, eps_h=1e-6 if T == np.float32 else 1e-12)
    ps = shsph.ParticleSet.from_particles(p)
    ctx.build_tree(ps)
    ctx.density(ps)
    ctx.force(ps)
    dt = ctx.get_info()["dt_cfl"]
    s = ps.host()
    ctx.close()
    return p, s, dt


def _set(p, s):
    return shsph.ParticleSet(s, p.mass, p.lo, p.hi, p.periodic)


def _same(a, b, tag):
    ha, hb = a.host(*FIELDS), b.host(*FIELDS)
    for k in FIELDS:
        assert np.array_equal(ha[k], hb[k]), f"{tag}: {k} differs"


def test_noalloc_step_equals_step(torch_cuda):
    T = np.float32
    _say("[noalloc] 40^3 FP32 state")
    p1, s1, dt1 = _state(40, 31, T)
    eps = 1e-6
    ref = shsph.Context(0, eps_h=eps)          # shsph_step
    nal = shsph.Context(0, eps_h=eps)          # shsph_step_noalloc
    other = shsph.Context(0, eps_h=eps)        # another user of the scratch array
    a, b = _set(p1, s1), _set(p1, s1)

    _say("[noalloc] call 1: fixed dt, 64000 particles")
    u_ref = ref.step(a, dt1, want_dt=True)
    u_nal = nal.step_noalloc(b, dt1, want_dt=True)
    assert u_ref == u_nal == dt1
    _same(a, b, "call 1")

    _say("[noalloc] another context's allocation-free step on a smaller input")
    p0, s0, dt0 = _state(20, 33, T)
    c0 = _set(p0, s0)
    other.step_noalloc(c0, dt0)

    _say("[noalloc] call 2: CFL dt of the context's own previous step")
    u_ref = ref.step(a, 0.0, want_dt=True)
    u_nal = nal.step_noalloc(b, 0.0, want_dt=True)
    assert u_ref == u_nal and u_ref > 0
    _same(a, b, "call 2")

    _say("[noalloc] call 3: a smaller input (24^3, FP64)")
    T2 = np.float64
    p2, s2, dt2 = _state(24, 32, T2)
    ref2 = shsph.Context(0, eps_h=1e-12)
    nal.set_params(eps_h=1e-12)
    a2, b2 = _set(p2, s2), _set(p2, s2)
    u_ref = ref2.step(a2, dt2, want_dt=True)
    u_nal = nal.step_noalloc(b2, dt2, want_dt=True)
    assert u_ref == u_nal == dt2
    _same(a2, b2, "call 3")

    _say("[noalloc] call 4: CFL dt after the smaller input")
    u_ref = ref2.step(a2, 0.0, want_dt=True)
    u_nal = nal.step_noalloc(b2, 0.0, want_dt=True)
    assert u_ref == u_nal and u_ref > 0
    _same(a2, b2, "call 4")
    for c in (ref, ref2, nal, other):
        c.close()


def test_noalloc_at_size_limit(torch_cuda):
    """FP64 near the particle limit (50^3 = 125000 <= 131072): the working
    memory of the largest admitted FP64 step, lattice-like neighbour counts,
    fits the static array, and the step still equals shsph_step."""
    T = np.float64
    _say("[noalloc] 50^3 FP64 state (near the particle limit)")
    p, s, dt = _state(50, 36, T)
    ref = shsph.Context(0, eps_h=1e-12)
    nal = shsph.Context(0, eps_h=1e-12)
    a, b = _set(p, s), _set(p, s)
    for k, d in enumerate((dt, 0.0)):
        _say(f"[noalloc] 50^3 FP64 call {k + 1}, dt {d}")
        u_ref = ref.step(a, d, want_dt=True)
        u_nal = nal.step_noalloc(b, d, want_dt=True)
        assert u_ref == u_nal and u_ref > 0
        _same(a, b, f"50^3 call {k + 1}")
    ref.close()
    nal.close()


def test_noalloc_limits(torch_cuda):
    _say("[noalloc] size limit and state errors")
    ctx = shsph.Context(0)
    big = gen.lattice(51, 34, dtype=np.float32)       # 132651 > 131072 particles
    with pytest.raises(shsph.ShsphError) as e:
        ctx.step_noalloc(shsph.ParticleSet.from_particles(big), 1e-4)
    assert e.value.code == shsph.SHSPH_ECAPACITY
    small = gen.lattice(16, 35, dtype=np.float32)
    with pytest.raises(shsph.ShsphError) as e:             # no earlier step: no CFL dt
        ctx.step_noalloc(shsph.ParticleSet.from_particles(small), 0.0)
    assert e.value.code == shsph.SHSPH_ESTATE
    ctx.close()
