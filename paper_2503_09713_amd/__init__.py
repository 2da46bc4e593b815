"""Python binding of ``libshsph.so``, the MI355X SPH hot path.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device memory comes from PyTorch tensors (``device='cuda'``); the
library never falls back to anything else and this module raises if the
library has not been built (``python -m paper_2503_09713_amd.build``).

Entry points mirror ``include/shsph.h``: ``Context.build_tree``,
``Context.density``, ``Context.force``, ``Context.step``,
``Context.get_info`` and ``Context.export_tree``; pooled instances and
batched passes (``instance_create``, ``step_batch``, ``eval_batch`` ...) and
the serving loop (``serve_start``, ``submit``, ``poll``, ``serve_drain`` ...).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshsph.so")
_lib = None

SHSPH_OK, SHSPH_EINVAL, SHSPH_ENOMEM, SHSPH_ENOCONV = 0, -1, -2, -3
SHSPH_ECAPACITY, SHSPH_EHIP, SHSPH_ESTATE = -4, -5, -6
ERRORS = {SHSPH_EINVAL: "EINVAL", SHSPH_ENOMEM: "ENOMEM", SHSPH_ENOCONV: "ENOCONV",
          SHSPH_ECAPACITY: "ECAPACITY", SHSPH_EHIP: "EHIP", SHSPH_ESTATE: "ESTATE"}
F32, F64 = 0, 1
NUM_STAGES = 12


class ShsphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("hfact", C.c_double), ("gamma", C.c_double), ("alpha_av", C.c_double),
                ("beta_av", C.c_double), ("beta_u", C.c_double), ("chi", C.c_double),
                ("lambda_", C.c_double), ("eps_h", C.c_double), ("c_cour", C.c_double),
                ("c_force", C.c_double), ("max_iter", C.c_int32), ("n_red", C.c_int32),
                ("max_restarts", C.c_int32), ("spread_slots", C.c_int32),
                ("stage1_serial", C.c_int32), ("stage2_mode", C.c_int32),
                ("kernel", C.c_int32), ("key_bits", C.c_int32), ("eps_v", C.c_double),
                ("max_reruns", C.c_int32), ("alpha_switch", C.c_int32),
                ("lambda_stiff", C.c_double), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("sigma_decay", C.c_double),
                ("force_split", C.c_int32), ("fused_density_force", C.c_int32),
                ("graph_batch", C.c_int32)]


KERNELS = {"M4": 0, "M5": 1, "M6": 2, "C2": 3, "C4": 4, "C6": 5}


class CParticles(C.Structure):
    _fields_ = [("n", C.c_int64), ("dtype", C.c_int32), ("periodic", C.c_int32),
                ("mass", C.c_double), ("lo", C.c_double * 3), ("hi", C.c_double * 3)] + \
               [(k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay",
                                          "az", "dudt", "rho", "omega")] + [("pid", C.c_void_p),
                                                                            ("alpha", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_leaf", C.c_int64), ("n_groups", C.c_int64),
                ("n_leaf_neigh", C.c_int64),
                ("n_neigh", C.c_int64), ("n_red", C.c_int32), ("restarts", C.c_int32),
                ("max_iter_seen", C.c_int32), ("n_noconv", C.c_int32), ("dt_cfl", C.c_double),
                ("dv_max", C.c_double), ("dv2_sum", C.c_double), ("v2_sum", C.c_double),
                ("reruns", C.c_int32), ("cache_capacity", C.c_int32),
                ("cfl_multiplier", C.c_double), ("graph_passes", C.c_int64),
                ("graph_aborts", C.c_int64), ("graph_abort_why", C.c_int32), ("pad1", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SERVE_CONTINUOUS, SERVE_ONE_AT_A_TIME = 0, 1
JOB_STEP, JOB_EVAL = 0, 1
JOB_STATES = {0: "pending", 1: "running", 2: "done", 3: "failed"}


class ServeConfig(C.Structure):
    _fields_ = [("budget_bytes", C.c_double), ("max_batch_particles", C.c_int64),
                ("max_batch", C.c_int32), ("policy", C.c_int32)]


class Job(C.Structure):
    _fields_ = [("handle", C.c_int64), ("init", C.c_void_p), ("kind", C.c_int32),
                ("nsteps", C.c_int32), ("dt", C.c_double), ("release", C.c_int32),
                ("reserved", C.c_int32)]


class JobStatus(C.Structure):
    _fields_ = [("state", C.c_int32), ("error", C.c_int32), ("handle", C.c_int64),
                ("steps_done", C.c_int32), ("passes", C.c_int32), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["state"] = JOB_STATES.get(d["state"], d["state"])
        return d


class ServeCounters(C.Structure):
    _fields_ = [("jobs_done", C.c_int64), ("jobs_failed", C.c_int64), ("passes", C.c_int64),
                ("peak_jobs", C.c_int64), ("particle_passes", C.c_double), ("busy_s", C.c_double),
                ("peak_bytes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_EXPORT_FIELDS = ["keys", "eps", "mu", "xi", "id", "mu_leaf", "lchild", "rchild", "endrange",
                  "lflag", "rflag", "parent", "bmin", "bmax", "hmax", "pbox", "plen", "group_off",
                  "group_leaves", "neigh_off", "neigh_list", "h_sorted", "h_cache"]


class TreeExport(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in _EXPORT_FIELDS]


def lib():
    """Load libshsph.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_09713_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, ip = C.c_void_p, C.c_int
    L.shsph_params_default.argtypes = [C.POINTER(Params)]
    L.shsph_params_default.restype = None
    L.shsph_create.argtypes = [ip, C.POINTER(Params), C.POINTER(vp)]
    L.shsph_destroy.argtypes = [vp]
    L.shsph_set_stream.argtypes = [vp, vp]
    L.shsph_set_params.argtypes = [vp, C.POINTER(Params)]
    L.shsph_get_params.argtypes = [vp, C.POINTER(Params)]
    L.shsph_last_error.argtypes = [vp]
    L.shsph_last_error.restype = C.c_char_p
    for fn in ("shsph_build_tree", "shsph_density", "shsph_force"):
        getattr(L, fn).argtypes = [vp, C.POINTER(CParticles)]
    L.shsph_step.argtypes = [vp, C.POINTER(CParticles), C.c_double, C.POINTER(C.c_double)]
    L.shsph_step_noalloc.argtypes = [vp, C.POINTER(CParticles), C.c_double, C.POINTER(C.c_double)]
    L.shsph_get_info.argtypes = [vp, C.POINTER(Info)]
    L.shsph_export_tree.argtypes = [vp, C.POINTER(TreeExport)]
    L.shsph_set_profiling.argtypes = [vp, ip]
    L.shsph_get_stage_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
    L.shsph_get_work.argtypes = [vp, C.POINTER(C.c_double)]
    L.shsph_stage_name.argtypes = [C.c_int32]
    L.shsph_stage_name.restype = C.c_char_p
    i64p, dp = C.POINTER(C.c_int64), C.POINTER(C.c_double)
    L.shsph_instance_create.argtypes = [vp, C.POINTER(CParticles), i64p]
    L.shsph_instance_destroy.argtypes = [vp, C.c_int64]
    L.shsph_instance_read.argtypes = [vp, C.c_int64, C.POINTER(CParticles)]
    L.shsph_instance_info.argtypes = [vp, C.c_int64, C.POINTER(Info)]
    L.shsph_step_batch.argtypes = [vp, i64p, C.c_int32, dp, dp]
    L.shsph_eval_batch.argtypes = [vp, i64p, C.c_int32]
    L.shsph_pool_usage.argtypes = [vp, i64p, i64p, i64p]
    L.shsph_autotune.argtypes = [vp, i64p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), dp]
    L.shsph_serve_start.argtypes = [vp, C.POINTER(ServeConfig)]
    L.shsph_submit.argtypes = [vp, C.POINTER(Job), C.POINTER(C.c_uint64)]
    L.shsph_poll.argtypes = [vp, C.c_uint64, C.POINTER(JobStatus)]
    L.shsph_serve_drain.argtypes = [vp, C.c_double]
    L.shsph_serve_stats.argtypes = [vp, C.POINTER(ServeCounters)]
    L.shsph_serve_stop.argtypes = [vp]
    L.shsph_footprint.argtypes = [vp, C.c_int64, C.c_int32, dp, dp]
    L.shsph_clock.argtypes = []
    L.shsph_clock.restype = C.c_double
    for fn in ("shsph_create", "shsph_destroy", "shsph_set_stream", "shsph_set_params",
               "shsph_get_params", "shsph_build_tree",
               "shsph_density", "shsph_force", "shsph_step",
               "shsph_get_info",
               "shsph_export_tree", "shsph_set_profiling", "shsph_get_stage_times",
               "shsph_get_work", "shsph_instance_create", "shsph_instance_destroy",
               "shsph_instance_read", "shsph_instance_info", "shsph_step_batch",
               "shsph_eval_batch", "shsph_pool_usage", "shsph_serve_start", "shsph_submit",
               "shsph_poll", "shsph_serve_drain", "shsph_serve_stats", "shsph_serve_stop",
               "shsph_footprint", "shsph_autotune"):
        getattr(L, fn).restype = ip
    _lib = L
    return L


def default_params() -> Params:
    p = Params()
    lib().shsph_params_default(C.byref(p))
    return p


class ParticleSet:
    """Device-resident SoA particle arrays (torch tensors) of one instance."""

    FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az", "dudt", "rho", "omega")

    def __init__(self, arrays: dict, mass: float, lo, hi, periodic: bool, device="cuda"):
        import torch
        self.torch = torch
        x = np.asarray(arrays["x"])
        self.dtype = x.dtype
        if self.dtype not in (np.float32, np.float64):
            raise TypeError(self.dtype)
        tdt = torch.float32 if self.dtype == np.float32 else torch.float64
        self.n = int(x.shape[0])
        self.t = {}
        for k in self.FIELDS:
            if k in arrays and arrays[k] is not None:
                a = np.ascontiguousarray(np.asarray(arrays[k], dtype=self.dtype))
                self.t[k] = torch.from_numpy(a).to(device)
            else:
                self.t[k] = torch.zeros(self.n, dtype=tdt, device=device)
        pid = arrays.get("pid")
        if pid is None:
            pid = np.arange(self.n, dtype=np.int32)
        self.t["pid"] = torch.from_numpy(np.ascontiguousarray(np.asarray(pid).astype(np.int32))).to(device)
        al = arrays.get("alpha")
        if al is not None:      # per-particle viscosity alpha (a scalar fills every particle)
            a = np.array(np.broadcast_to(np.asarray(al, dtype=self.dtype), (self.n,)))
            self.t["alpha"] = torch.from_numpy(a).to(device)
        self.mass = float(mass)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.periodic = bool(periodic)

    @classmethod
    def from_particles(cls, p, device="cuda", alpha=None):
        """From a ``gen.Particles``-like object (numpy fields, mass, box);
        alpha: optional per-particle viscosity alpha (array or scalar)."""
        f = dict(p.fields())
        if alpha is not None:
            f["alpha"] = alpha
        return cls(f, p.mass, p.lo, p.hi, p.periodic, device=device)

    def cstruct(self) -> CParticles:
        c = CParticles()
        c.n = self.n
        c.dtype = F32 if self.dtype == np.float32 else F64
        c.periodic = 1 if self.periodic else 0
        c.mass = self.mass
        c.lo[:] = self.lo
        c.hi[:] = self.hi
        for k in self.FIELDS:
            setattr(c, k, self.t[k].data_ptr())
        c.pid = self.t["pid"].data_ptr()
        c.alpha = self.t["alpha"].data_ptr() if "alpha" in self.t else None
        return c

    def host(self, *keys) -> dict:
        keys = keys or (self.FIELDS + ("pid",) + (("alpha",) if "alpha" in self.t else ()))
        out = {k: self.t[k].cpu().numpy() for k in keys}
        if "pid" in out:
            out["pid"] = out["pid"].view(np.uint32)
        return out


def _apply(params: Params, kw: dict) -> None:
    """Set fields of a Params from keyword arguments (kernel by name or id);
    an unknown name is an error."""
    names = {f for f, _ in Params._fields_}
    for k, v in kw.items():
        if k == "kernel" and isinstance(v, str):
            v = KERNELS[v]
        f = "lambda_" if k == "lambda" else k
        if f not in names:
            raise TypeError(f"unknown parameter {k!r}")
        setattr(params, f, v)


class Context:
    """A shsph context bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, params: Params | None = None, stream=None, **kw):
        L = lib()
        if params is None:
            params = default_params()
        _apply(params, kw)
        self.params = params
        h = C.c_void_p()
        rc = L.shsph_create(int(device), C.byref(params), C.byref(h))
        if rc != SHSPH_OK:
            raise ShsphError(rc, "shsph_create failed")
        self.h = h
        self.L = L
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self.set_stream(stream)

    def _check(self, rc: int, allow=()):
        if rc != SHSPH_OK and rc not in allow:
            raise ShsphError(rc, self.L.shsph_last_error(self.h).decode())
        return rc

    def set_params(self, **kw) -> None:
        """Change parameters of the context (shsph_set_params)."""
        p = Params()
        self._check(self.L.shsph_get_params(self.h, C.byref(p)))
        _apply(p, kw)
        self._check(self.L.shsph_set_params(self.h, C.byref(p)))
        self.params = p

    def set_stream(self, stream) -> None:
        self._check(self.L.shsph_set_stream(self.h, C.c_void_p(int(stream) if stream else 0)))

    def build_tree(self, ps: ParticleSet) -> None:
        self._cp = ps.cstruct()
        self._check(self.L.shsph_build_tree(self.h, C.byref(self._cp)))

    def density(self, ps: ParticleSet, allow_noconv: bool = False) -> int:
        self._cp = ps.cstruct()
        allow = (SHSPH_ENOCONV,) if allow_noconv else ()
        return self._check(self.L.shsph_density(self.h, C.byref(self._cp)), allow)

    def force(self, ps: ParticleSet) -> None:
        self._cp = ps.cstruct()
        self._check(self.L.shsph_force(self.h, C.byref(self._cp)))

    def step(self, ps: ParticleSet, dt: float = 0.0, want_dt: bool = False):
        self._cp = ps.cstruct()
        used = C.c_double(0.0)
        self._check(self.L.shsph_step(self.h, C.byref(self._cp), float(dt),
                                      C.byref(used) if want_dt else None))
        return used.value if want_dt else None

    def step_noalloc(self, ps: ParticleSet, dt: float = 0.0, want_dt: bool = False):
        """shsph_step_noalloc: the step with all device working memory in the
        library's static per-device scratch array (no allocation)."""
        self._cp = ps.cstruct()
        used = C.c_double(0.0)
        self._check(self.L.shsph_step_noalloc(self.h, C.byref(self._cp), float(dt),
                                              C.byref(used) if want_dt else None))
        return used.value if want_dt else None

    def get_info(self) -> dict:
        o = Info()
        self._check(self.L.shsph_get_info(self.h, C.byref(o)))
        return o.as_dict()

    def export_tree(self, dtype=np.float32, fields=None) -> dict:
        """Copy the last tree / caches to host numpy arrays."""
        info = self.get_info()
        n, nl, G = info["n"], info["n_leaf"], info["n_groups"]
        ni, nn = nl - 1, 2 * nl - 1
        e1, e2 = info["n_leaf_neigh"], info["n_neigh"]
        T = np.dtype(dtype)
        shapes = dict(keys=(n, np.uint64), eps=(n, np.uint32), mu=(n, np.uint64), xi=(n, np.uint8),
                      id=(nl + 1, np.uint32), mu_leaf=(nl, np.uint64), lchild=(ni, np.uint32),
                      rchild=(ni, np.uint32), endrange=(ni, np.uint32), lflag=(ni, np.uint8),
                      rflag=(ni, np.uint8), parent=(nn, np.uint32), bmin=((nn, 3), T),
                      bmax=((nn, 3), T), hmax=(nn, T), pbox=((nn, 6), np.uint32),
                      plen=(nn, np.int32), group_off=(G + 1, np.uint64),
                      group_leaves=(e1, np.uint32), neigh_off=(n + 1, np.uint64),
                      neigh_list=(e2, np.uint32), h_sorted=(n, T), h_cache=(n, T))
        want = fields or list(shapes)
        out, ex = {}, TreeExport()
        for k in want:
            shp, dt = shapes[k]
            a = np.zeros(shp, dt)
            out[k] = a
            setattr(ex, k, a.ctypes.data if a.size else None)
        self._check(self.L.shsph_export_tree(self.h, C.byref(ex)))
        return out

    def set_profiling(self, on: bool = True) -> None:
        self._check(self.L.shsph_set_profiling(self.h, 1 if on else 0))

    def stage_times(self) -> dict:
        """{stage: (total_ms, launches)} since profiling was turned on."""
        n = NUM_STAGES
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self._check(self.L.shsph_get_stage_times(self.h, ms, cnt, n))
        return {self.L.shsph_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(n)}

    def work(self) -> dict:
        """Work counted by the neighbour kernels since profiling was turned on."""
        w = (C.c_double * 6)()
        self._check(self.L.shsph_get_work(self.h, w))
        return dict(cache_tests=w[0], cache_prune_tests=w[1], density_pair_evals=w[2],
                    density_pairs_in_2h=w[3], force_entries=w[4], force_pairs=w[5])

    # ---------------------------------------------- pooled instances, batches
    def instance_create(self, ps: ParticleSet) -> int:
        """Copy ``ps`` into the context's instance pool; returns the handle."""
        cp = ps.cstruct()
        h = C.c_int64(0)
        self._check(self.L.shsph_instance_create(self.h, C.byref(cp), C.byref(h)))
        return h.value

    def instance_destroy(self, handle: int) -> None:
        self._check(self.L.shsph_instance_destroy(self.h, int(handle)))

    def instance_read(self, handle: int, out: ParticleSet) -> None:
        """Copy the pooled state (Morton order, ``pid`` = particle ids) into ``out``."""
        cp = out.cstruct()
        self._check(self.L.shsph_instance_read(self.h, int(handle), C.byref(cp)))

    def instance_info(self, handle: int) -> dict:
        o = Info()
        self._check(self.L.shsph_instance_info(self.h, int(handle), C.byref(o)))
        return o.as_dict()

    @staticmethod
    def _handles(handles):
        hs = list(int(h) for h in handles)
        return hs, (C.c_int64 * len(hs))(*hs)

    def step_batch(self, handles, dt=None, allow_noconv: bool = False):
        """One step of every listed instance in one batched pass; returns dt used."""
        hs, arr = self._handles(handles)
        dts = (C.c_double * len(hs))(*([0.0] * len(hs) if dt is None else
                                       [float(d) for d in (dt if hasattr(dt, "__len__") else [dt] * len(hs))]))
        used = (C.c_double * len(hs))()
        allow = (SHSPH_ENOCONV,) if allow_noconv else ()
        self._check(self.L.shsph_step_batch(self.h, arr, len(hs), dts, used), allow)
        return list(used)

    def eval_batch(self, handles, allow_noconv: bool = False) -> None:
        hs, arr = self._handles(handles)
        allow = (SHSPH_ENOCONV,) if allow_noconv else ()
        self._check(self.L.shsph_eval_batch(self.h, arr, len(hs)), allow)

    def autotune(self, handles) -> dict:
        """Pick leaf size (n_red), stage-2 walk and the force kernel's
        workgroup size (force_split) for batched passes of these instances."""
        hs, arr = self._handles(handles)
        nr, md, fs, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        self._check(self.L.shsph_autotune(self.h, arr, len(hs), C.byref(nr), C.byref(md),
                                          C.byref(fs), C.byref(ms)))
        self.params.n_red, self.params.stage2_mode = nr.value, md.value
        self.params.force_split = fs.value if fs.value else 1
        self.params.fused_density_force = 0 if fs.value else 1
        return dict(n_red=nr.value, stage2_mode=md.value, force_split=self.params.force_split,
                    fused_density_force=self.params.fused_density_force, pass_ms=ms.value)

    def pool_usage(self) -> dict:
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.L.shsph_pool_usage(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(particles=a.value, capacity=b.value, instances=c.value)

    # ------------------------------------------------------------- serving
    def serve_start(self, budget_bytes: float, max_batch: int = 256, policy: int = SERVE_CONTINUOUS,
                    max_batch_particles: int = 0) -> None:
        cfg = ServeConfig(float(budget_bytes), int(max_batch_particles), int(max_batch), int(policy))
        self._check(self.L.shsph_serve_start(self.h, C.byref(cfg)))
        self._keep = {}

    def submit(self, handle: int = 0, init: ParticleSet | None = None, kind: int = JOB_STEP,
               nsteps: int = 1, dt: float = 0.0, release: bool = False) -> int:
        """Queue a job; ``init`` (kept alive here until the job is admitted) brings a new instance."""
        cp = init.cstruct() if init is not None else None
        job = Job(int(handle), C.cast(C.pointer(cp), C.c_void_p) if cp is not None else None,
                  int(kind), int(nsteps), float(dt), 1 if release else 0, 0)
        t = C.c_uint64(0)
        self._check(self.L.shsph_submit(self.h, C.byref(job), C.byref(t)))
        if init is not None:
            self._keep[t.value] = init
        return t.value

    def poll(self, ticket: int) -> dict:
        st = JobStatus()
        self._check(self.L.shsph_poll(self.h, int(ticket), C.byref(st)))
        d = st.as_dict()
        if d["state"] != "pending":
            getattr(self, "_keep", {}).pop(int(ticket), None)
        return d

    def serve_drain(self, timeout_s: float = 600.0) -> None:
        self._check(self.L.shsph_serve_drain(self.h, float(timeout_s)))
        getattr(self, "_keep", {}).clear()

    def serve_wait(self, timeout_s: float) -> bool:
        """True when no job is pending or running (waits at most timeout_s)."""
        rc = self.L.shsph_serve_drain(self.h, float(timeout_s))
        if rc == SHSPH_ESTATE:
            return False
        self._check(rc)
        getattr(self, "_keep", {}).clear()
        return True

    def serve_stats(self) -> dict:
        o = ServeCounters()
        self._check(self.L.shsph_serve_stats(self.h, C.byref(o)))
        return o.as_dict()

    def serve_stop(self) -> None:
        self._check(self.L.shsph_serve_stop(self.h))
        getattr(self, "_keep", {}).clear()

    def footprint(self, n: int, dtype=np.float32):
        s, w = C.c_double(), C.c_double()
        self._check(self.L.shsph_footprint(self.h, int(n), F32 if np.dtype(dtype) == np.float32 else F64,
                                           C.byref(s), C.byref(w)))
        return s.value, w.value

    def clock(self) -> float:
        return self.L.shsph_clock()

    def close(self) -> None:
        if getattr(self, "h", None):
            self.L.shsph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def exported_symbols():
    """Names declared in include/shsph.h (for the ABI check)."""
    hdr = os.path.join(_HERE, "..", "include", "shsph.h")
    import re
    txt = open(hdr).read()
    return sorted(set(re.findall(r"\b(shsph_[a-z_]+)\s*\(", txt)))
