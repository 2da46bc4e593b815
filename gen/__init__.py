"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This module only draws particle sets; it contains none of the SPH method's
arithmetic (no kernel, no density, no tree).  Every draw is FP64 from numpy's
PCG64 and is rounded to the storage type at the end.

Recipes (they stand in for the paper's Sedov restart files and lattice setups,
Sect. 4 and 5, which are not available):

* ``lattice``  cell-centred cubic lattice (i+1/2)*dx in the periodic unit box,
  each coordinate jittered by U(-j, j)*dx, rho0 = 1 (m = 1/N), u = 1, v = 0,
  h = 1.2*dx.  The particle order is a seeded random permutation so that the
  first sort is not the identity.
* ``sedov``    the lattice plus an energy injection: the particles within
  r < 2*h0 of the box centre share E = 1 equally (u = 1e-6 elsewhere).
* ``plummer``  Plummer sphere, scale radius a = 0.1, total mass 1, truncated at
  r = 1, isotropic directions, v = 0, u = 1, isolated boundaries,
  h = 1.2*(m/rho_P(r))**(1/3) from the analytic profile.
* ``batch``    64 instances, N_i = floor(2**U(12, 20)), alternating lattice /
  Plummer (lattices use the largest cube n1**3 <= N_i).
* ``serve_trace`` Poisson arrivals, 1-10 steps per job, 20 % evaluation jobs,
  N = floor(2**U(12, 22)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEEDS = {"tiny": 1, "uniform": 2, "sedov": 3, "batch": 4, "serve": 5}


@dataclasses.dataclass
class Particles:
    """One SPH instance in structure-of-arrays form (host numpy arrays)."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    u: np.ndarray
    h: np.ndarray
    mass: float
    lo: tuple
    hi: tuple
    periodic: bool
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def dtype(self):
        return self.x.dtype

    def fields(self):
        return dict(x=self.x, y=self.y, z=self.z, vx=self.vx, vy=self.vy,
                    vz=self.vz, u=self.u, h=self.h)

    def astype(self, dtype) -> "Particles":
        f = {k: np.ascontiguousarray(v.astype(dtype)) for k, v in self.fields().items()}
        return Particles(**f, mass=self.mass, lo=self.lo, hi=self.hi,
                         periodic=self.periodic, name=self.name)

    def subset(self, idx) -> "Particles":
        f = {k: np.ascontiguousarray(v[idx]) for k, v in self.fields().items()}
        return Particles(**f, mass=self.mass, lo=self.lo, hi=self.hi,
                         periodic=self.periodic, name=self.name)


def _finish(pos, vel, u, h, mass, lo, hi, periodic, dtype, name):
    dt = np.dtype(dtype)
    return Particles(
        x=np.ascontiguousarray(pos[:, 0].astype(dt)),
        y=np.ascontiguousarray(pos[:, 1].astype(dt)),
        z=np.ascontiguousarray(pos[:, 2].astype(dt)),
        vx=np.ascontiguousarray(vel[:, 0].astype(dt)),
        vy=np.ascontiguousarray(vel[:, 1].astype(dt)),
        vz=np.ascontiguousarray(vel[:, 2].astype(dt)),
        u=np.ascontiguousarray(u.astype(dt)),
        h=np.ascontiguousarray(h.astype(dt)),
        mass=float(mass), lo=tuple(float(v) for v in lo),
        hi=tuple(float(v) for v in hi), periodic=bool(periodic), name=name)


def lattice(n1: int, seed: int, dtype=np.float32, jitter: float = 0.01,
            shuffle: bool = True, rho0: float = 1.0, hfact: float = 1.2) -> Particles:
    """Jittered cell-centred cubic lattice of n1**3 particles in [0,1)^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = n1 ** 3
    dx = 1.0 / n1
    ii = np.arange(n1, dtype=np.float64)
    gx, gy, gz = np.meshgrid(ii, ii, ii, indexing="ij")
    pos = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    pos = (pos + 0.5) * dx
    if jitter:
        pos += rng.uniform(-jitter, jitter, size=pos.shape) * dx
    if shuffle:
        pos = pos[rng.permutation(n)]
    vel = np.zeros_like(pos)
    u = np.ones(n)
    h = np.full(n, hfact * dx)
    return _finish(pos, vel, u, h, rho0 / n, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                   True, dtype, f"lattice{n1}")


def sedov(n1: int, seed: int, dtype=np.float32, energy: float = 1.0,
          u_floor: float = 1e-6, hfact: float = 1.2) -> Particles:
    """Sedov-like blast: lattice with E spread equally over r < 2*h0 of the centre."""
    p = lattice(n1, seed, dtype=np.float64, hfact=hfact)
    dx = 1.0 / n1
    h0 = hfact * dx
    r = np.sqrt((p.x - 0.5) ** 2 + (p.y - 0.5) ** 2 + (p.z - 0.5) ** 2)
    inj = r < 2.0 * h0
    n_inj = int(inj.sum())
    u = np.full(p.n, u_floor)
    u[inj] += energy / (n_inj * p.mass)
    p.u = u
    q = p.astype(dtype)
    q.name = f"sedov{n1}"
    return q


def plummer(n: int, seed: int, dtype=np.float32, a: float = 0.1,
            rmax: float = 1.0, hfact: float = 1.2) -> Particles:
    """Plummer sphere (a = 0.1, M = 1) truncated at rmax, isolated box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mcut = rmax ** 3 / (rmax ** 2 + a ** 2) ** 1.5
    X = rng.uniform(0.0, mcut, size=n)
    X = np.maximum(X, 1e-300)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    r = np.minimum(r, rmax)
    cth = rng.uniform(-1.0, 1.0, size=n)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    sth = np.sqrt(1.0 - cth ** 2)
    pos = np.stack([r * sth * np.cos(phi), r * sth * np.sin(phi), r * cth], axis=1)
    m = 1.0 / n
    rho_p = 3.0 / (4.0 * math.pi * a ** 3) * (1.0 + (r / a) ** 2) ** -2.5
    h = hfact * (m / rho_p) ** (1.0 / 3.0)
    vel = np.zeros_like(pos)
    u = np.ones(n)
    q = _finish(pos, vel, u, h, m, (0, 0, 0), (0, 0, 0), False, dtype, f"plummer{n}")
    # isolated: the box is the data's min/max in storage precision
    q.lo = (float(q.x.min()), float(q.y.min()), float(q.z.min()))
    q.hi = (float(q.x.max()), float(q.y.max()), float(q.z.max()))
    return q


def batch(seed: int = SEEDS["batch"], n_inst: int = 64, log2_lo: float = 12.0,
          log2_hi: float = 20.0, dtype=np.float32):
    """Uneven batch: N_i = floor(2**U(lo, hi)); alternate lattice / Plummer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(2.0 ** rng.uniform(log2_lo, log2_hi, size=n_inst)).astype(np.int64)
    out = []
    for k, n in enumerate(sizes):
        if k % 2 == 0:
            n1 = int(math.floor(round(n ** (1.0 / 3.0), 9)))
            while (n1 + 1) ** 3 <= n:
                n1 += 1
            while n1 ** 3 > n:
                n1 -= 1
            out.append(lattice(max(n1, 2), seed * 1000 + k, dtype=dtype))
        else:
            out.append(plummer(int(n), seed * 1000 + k, dtype=dtype))
    return out


def serve_trace(rate: float, n_jobs: int, seed: int = SEEDS["serve"],
                log2_lo: float = 12.0, log2_hi: float = 22.0):
    """Poisson arrival trace: list of (t_arrival, kind, nsteps, N, family)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
    kinds = np.where(rng.uniform(size=n_jobs) < 0.2, "eval", "step")
    steps = rng.integers(1, 11, size=n_jobs)
    sizes = np.floor(2.0 ** rng.uniform(log2_lo, log2_hi, size=n_jobs)).astype(np.int64)
    fam = np.where(rng.uniform(size=n_jobs) < 0.5, "lattice", "plummer")
    return [dict(t=float(t[i]), kind=str(kinds[i]), nsteps=int(steps[i]),
                 n=int(sizes[i]), family=str(fam[i])) for i in range(n_jobs)]
