"""Python binding of libcosmica (ctypes; argument marshalling only).

Every step of the hot path runs in the HIP library ``libcosmica.so`` built from
``csrc/`` for gfx950; this module only packs workload dictionaries (see
``workloads.py``) into the C structs of ``include/cosmica.h`` and unpacks
results into numpy arrays.  There is no CPU fallback: if the library is
missing, :func:`load` raises.

PyTorch is optional plumbing: a torch stream can be handed to the context and
torch device tensors can receive a plan's results without a host copy.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcosmica.so")

NHIST = 129
MAX_REGIONS = 15
MAX_STEP_CAP = 16777215
MAX_ORBIT = 1024
MAX_JOBS = 1048576
MAX_REWEIGHT = 4096
MAX_LIS_KNOTS = 256
MAX_RANGE_BINS = 4096
STATIC_BYTES = 134217728
STATIC_MAX_JOBS = 256
STATIC_MAX_BINS = 8192
STATIC_MAX_ORBIT = 4096
MODEL_1D, MODEL_3D = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
PRECISION = {"fp64": PREC_FP64, "mixed": PREC_MIXED, PREC_FP64: PREC_FP64, PREC_MIXED: PREC_MIXED}

OK, EINVAL, ENOMEM, EDEVICE, EBUSY, ECANCELED, ESTEPCAP, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
ESCRATCH = -8

c_double_p = ctypes.POINTER(ctypes.c_double)
c_u32_p = ctypes.POINTER(ctypes.c_uint32)
c_u64_p = ctypes.POINTER(ctypes.c_uint64)


class Helio(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("n_regions", ctypes.c_int32),
        ("kappa0_cm2_s", ctypes.c_double * MAX_REGIONS),
        ("v_slow_km_s", ctypes.c_double * MAX_REGIONS),
        ("tilt_deg", ctypes.c_double * MAX_REGIONS),
        ("v_fast_km_s", ctypes.c_double), ("r_boundary_au", ctypes.c_double),
        ("r0_au", ctypes.c_double), ("theta0_rad", ctypes.c_double), ("phi0_rad", ctypes.c_double),
        ("b0_nT", ctypes.c_double), ("v_ref_km_s", ctypes.c_double),
        ("omega_rad_s", ctypes.c_double), ("kperp_over_kpar", ctypes.c_double),
        ("polarity", ctypes.c_int32), ("drift", ctypes.c_int32), ("hcs", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("dt_max_s", ctypes.c_double), ("dt_diff_frac", ctypes.c_double),
        ("dt_adv_frac", ctypes.c_double),
        ("r_boundary_nose_au", ctypes.c_double), ("nose_theta_rad", ctypes.c_double),
        ("nose_phi_rad", ctypes.c_double), ("heliosheath", ctypes.c_int32),
        ("reserved1", ctypes.c_int32), ("ts_nose_au", ctypes.c_double),
        ("ts_tail_au", ctypes.c_double), ("kappa0_hs_cm2_s", ctypes.c_double),
        ("v_hs_km_s", ctypes.c_double), ("tilt_hs_deg", ctypes.c_double),
    ]

# geometry fields that older job dictionaries may lack: a spherical heliosphere
_HELIO_DEFAULTS = {"r_boundary_nose_au": 0.0, "nose_theta_rad": 0.5 * np.pi, "nose_phi_rad": 0.0,
                   "heliosheath": 0, "ts_nose_au": 0.0, "ts_tail_au": 0.0,
                   "kappa0_hs_cm2_s": 0.0, "v_hs_km_s": 0.0, "tilt_hs_deg": 0.0}
REGION_HELIOSHEATH = 15


class Species(ctypes.Structure):
    _fields_ = [("mass_gev", ctypes.c_double), ("charge", ctypes.c_int32),
                ("mass_number", ctypes.c_int32), ("lis_norm", ctypes.c_double),
                ("lis_index", ctypes.c_double)]


class Job(ctypes.Structure):
    _fields_ = [("helio", ctypes.POINTER(Helio)), ("species", ctypes.POINTER(Species)),
                ("rigidity_gv", c_double_p), ("particles_per_bin", c_u32_p),
                ("n_bins", ctypes.c_int32), ("job_tag", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("step_cap", ctypes.c_uint32),
                ("bin_offset", ctypes.c_uint32), ("orbit", c_double_p),
                ("n_orbit", ctypes.c_uint32), ("formulation", ctypes.c_int32)]


class Exit(ctypes.Structure):
    _fields_ = [("P", ctypes.c_double), ("t", ctypes.c_double), ("r", ctypes.c_double),
                ("theta", ctypes.c_double), ("phi", ctypes.c_double),
                ("n", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("loss", ctypes.c_double)]


EXIT_DTYPE = np.dtype([("P", "<f8"), ("t", "<f8"), ("r", "<f8"), ("theta", "<f8"),
                       ("phi", "<f8"), ("n", "<u4"), ("flags", "<u4"), ("loss", "<f8")])
assert EXIT_DTYPE.itemsize == ctypes.sizeof(Exit)


class Result(ctypes.Structure):
    _fields_ = [("hist", c_u32_p), ("flux", c_double_p), ("flux_se", c_double_p),
                ("mean_exit_time_s", c_double_p), ("steps", c_u64_p),
                ("n_capped", c_u32_p), ("n_nan", c_u32_p), ("exits", ctypes.POINTER(Exit))]


class BinsDev(ctypes.Structure):
    _fields_ = [("hist", ctypes.c_void_p), ("flux", ctypes.c_void_p),
                ("flux_se", ctypes.c_void_p), ("mean_exit_time_s", ctypes.c_void_p),
                ("steps", ctypes.c_void_p), ("n_capped", ctypes.c_void_p),
                ("n_nan", ctypes.c_void_p)]


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("order", ctypes.c_int32)]


class Timings(ctypes.Structure):
    _fields_ = [("upload_ms", ctypes.c_double), ("propagate_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("download_ms", ctypes.c_double),
                ("steps", ctypes.c_uint64), ("particles", ctypes.c_uint64),
                ("grid_blocks", ctypes.c_int32), ("block", ctypes.c_int32)]


# exported symbols of include/cosmica.h and their C signatures
_SIGS = {
    "cosmica_abi_version": (ctypes.c_int, []),
    "cosmica_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "cosmica_validate_job": (ctypes.c_int, [ctypes.POINTER(Job)]),
    "cosmica_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                      ctypes.c_uint64, ctypes.c_void_p]),
    "cosmica_destroy": (None, [ctypes.c_void_p]),
    "cosmica_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_int32,
                                   ctypes.c_int, ctypes.POINTER(Result)]),
    "cosmica_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_int32,
                                           ctypes.c_int, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "cosmica_plan_execute": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BinsDev)]),
    "cosmica_plan_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Result)]),
    "cosmica_plan_info": (ctypes.c_int, [ctypes.c_void_p, c_u64_p, c_u64_p,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "cosmica_plan_destroy": (None, [ctypes.c_void_p]),
    "cosmica_plan_reweight": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_double, ctypes.c_double, c_double_p,
                                             c_double_p, c_double_p]),
    "cosmica_plan_exit_range": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, c_double_p,
                                               c_u32_p]),
    "cosmica_run_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_int32,
                                          ctypes.c_int, ctypes.POINTER(Result)]),
    "cosmica_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(Launch)]),
    "cosmica_get_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(Launch)]),
    "cosmica_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_char_p]),
    "cosmica_tune_jobs": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_int32,
                                         ctypes.c_int, ctypes.c_uint64, ctypes.c_char_p]),
    "cosmica_get_timings": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Timings)]),
    "cosmica_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_int,
                                      ctypes.POINTER(Result), c_u64_p]),
    "cosmica_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                    ctypes.POINTER(ctypes.c_int32)]),
    "cosmica_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32]),
    "cosmica_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "cosmica_request_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                             ctypes.POINTER(ctypes.c_int32)]),
    "cosmica_serve_stats": (ctypes.c_int, [ctypes.c_void_p, c_u64_p, c_u64_p, c_u64_p, c_u64_p]),
    "cosmica_probe_rng": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint32, c_u32_p, c_double_p,
                                         ctypes.POINTER(ctypes.c_float)]),
    "cosmica_probe_coeffs": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_int,
                                            ctypes.c_uint32, c_double_p, c_double_p]),
    "cosmica_probe_locate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_int,
                                            ctypes.c_uint32, c_double_p,
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
}

_lib = None


class CosmicaError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = load().cosmica_strerror(status).decode()
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


def load():
    """Loads libcosmica.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int, what: str, ok=(OK,)):
    if st not in ok:
        raise CosmicaError(st, what)
    return st


class _JobPack:
    """Keeps the ctypes storage of one job alive."""

    def __init__(self, job: dict):
        h = job["helio"]
        sp = job["species"]
        self.helio = Helio()
        for name, ctype in Helio._fields_:
            if name in ("reserved0", "reserved1"):
                continue
            v = h[name] if name in h else _HELIO_DEFAULTS[name]
            if name in ("kappa0_cm2_s", "v_slow_km_s", "tilt_deg"):
                arr = getattr(self.helio, name)
                for k, x in enumerate(v):
                    arr[k] = float(x)
            else:
                setattr(self.helio, name, v)
        self.species = Species(float(sp["mass_gev"]), int(sp["charge"]),
                               int(sp.get("mass_number", 0)), float(sp["lis_norm"]),
                               float(sp["lis_index"]))
        self.rig = np.ascontiguousarray(job["rigidity_gv"], dtype=np.float64)
        self.cnt = np.ascontiguousarray(job["particles_per_bin"], dtype=np.uint32)
        orbit = job.get("orbit")
        self.orbit = (np.ascontiguousarray(orbit, dtype=np.float64).reshape(-1, 3)
                      if orbit is not None and len(orbit) else np.zeros((0, 3)))
        self.job = Job(ctypes.pointer(self.helio), ctypes.pointer(self.species),
                       self.rig.ctypes.data_as(c_double_p), self.cnt.ctypes.data_as(c_u32_p),
                       len(self.rig), int(job["job_tag"]) & 0xffffffff,
                       int(job["seed"]) & (2**64 - 1), int(job.get("step_cap", 0)),
                       int(job.get("bin_offset", 0)),
                       self.orbit.ctypes.data_as(c_double_p) if len(self.orbit) else None,
                       len(self.orbit), int(job.get("formulation", 0)))
        self.n_bins = len(self.rig)
        self.total = int(self.cnt.sum())


class _ResultPack:
    """Host output buffers of one job."""

    def __init__(self, n_bins: int, total: int, exits: bool):
        self.hist = np.zeros((n_bins, NHIST), dtype=np.uint32)
        self.flux = np.zeros(n_bins)
        self.flux_se = np.zeros(n_bins)
        self.mean_exit_time_s = np.zeros(n_bins)
        self.steps = np.zeros(n_bins, dtype=np.uint64)
        self.n_capped = np.zeros(n_bins, dtype=np.uint32)
        self.n_nan = np.zeros(n_bins, dtype=np.uint32)
        self.exits = np.zeros(total, dtype=EXIT_DTYPE) if exits else None
        self.c = Result(self.hist.ctypes.data_as(c_u32_p), self.flux.ctypes.data_as(c_double_p),
                        self.flux_se.ctypes.data_as(c_double_p),
                        self.mean_exit_time_s.ctypes.data_as(c_double_p),
                        self.steps.ctypes.data_as(c_u64_p), self.n_capped.ctypes.data_as(c_u32_p),
                        self.n_nan.ctypes.data_as(c_u32_p),
                        self.exits.ctypes.data_as(ctypes.POINTER(Exit)) if exits else None)

    def as_dict(self) -> dict:
        d = {"hist": self.hist, "flux": self.flux, "flux_se": self.flux_se,
             "mean_exit_time_s": self.mean_exit_time_s, "steps": self.steps,
             "n_capped": self.n_capped, "n_nan": self.n_nan}
        if self.exits is not None:
            d["exits"] = self.exits
        return d


def validate_job(job: dict) -> int:
    """Host-only validation of one job (no device needed)."""
    p = _JobPack(job)
    return load().cosmica_validate_job(ctypes.byref(p.job))


class Plan:
    def __init__(self, engine: "Engine", handle, packs, precision):
        self.engine = engine
        self.handle = handle
        self.packs = packs
        self.precision = precision

    def info(self):
        tb, tp, nj = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int32()
        _check(load().cosmica_plan_info(self.handle, ctypes.byref(tb), ctypes.byref(tp),
                                        ctypes.byref(nj)), "plan_info")
        return {"bins": tb.value, "particles": tp.value, "jobs": nj.value}

    def execute(self, out: dict | None = None):
        """Enqueue propagation + reduction.  out: optional dict of torch device
        tensors (hist, flux, flux_se, mean_exit_time_s, steps, n_capped, n_nan)."""
        if out is None:
            _check(load().cosmica_plan_execute(self.handle, None), "plan_execute")
            return
        b = BinsDev(*[(out[k].data_ptr() if out.get(k) is not None else None)
                      for k, _ in BinsDev._fields_])
        _check(load().cosmica_plan_execute(self.handle, ctypes.byref(b)), "plan_execute")

    def read(self, exits: bool = False) -> list[dict]:
        res = [_ResultPack(p.n_bins, p.total, exits) for p in self.packs]
        arr = (Result * len(res))(*[r.c for r in res])
        self.last_status = _check(load().cosmica_plan_read(self.handle, arr), "plan_read",
                                  ok=(OK, ESTEPCAP))
        return [r.as_dict() for r in res]

    def reweight(self, lnP0: float, dlnP: float, lnJ) -> tuple[np.ndarray, np.ndarray]:
        """J_mod and its standard error for each tabulated spectrum (rows of
        lnJ: ln J at ln P = lnP0 + k dlnP) from the last execution's exits:
        arrays (n_lis, total_bins), bins in plan order."""
        lnJ = np.ascontiguousarray(np.atleast_2d(lnJ), dtype=np.float64)
        n_lis, n_knots = lnJ.shape
        nb = self.info()["bins"]
        flux = np.zeros((n_lis, nb))
        se = np.zeros((n_lis, nb))
        _check(load().cosmica_plan_reweight(self.handle, n_lis, n_knots, lnP0, dlnP,
                                            lnJ.ctypes.data_as(c_double_p),
                                            flux.ctypes.data_as(c_double_p),
                                            se.ctypes.data_as(c_double_p)), "plan_reweight")
        return flux, se

    def exit_range(self, n_hist: int) -> tuple[np.ndarray, np.ndarray]:
        """Per bin (plan order) the largest exit rigidity of the last execution
        and the counts of ln(P_ex/P0) in n_hist equal bins up to it:
        arrays (total_bins,), (total_bins, n_hist)."""
        nb = self.info()["bins"]
        pm = np.zeros(nb)
        hist = np.zeros((nb, n_hist), dtype=np.uint32)
        _check(load().cosmica_plan_exit_range(self.handle, n_hist,
                                              pm.ctypes.data_as(c_double_p),
                                              hist.ctypes.data_as(c_u32_p)), "plan_exit_range")
        return pm, hist

    def destroy(self):
        if self.handle:
            load().cosmica_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Ticket:
    def __init__(self, engine, ticket: int, jobpack: _JobPack, res: _ResultPack):
        self.engine = engine
        self.id = ticket
        self.jobpack = jobpack
        self.res = res

    def poll(self) -> tuple[bool, int]:
        d = ctypes.c_int32()
        st = load().cosmica_poll(self.engine.handle, self.id, ctypes.byref(d))
        return bool(d.value), st

    def wait(self, timeout_ms: int = -1) -> int:
        return load().cosmica_wait(self.engine.handle, self.id, timeout_ms)

    def cancel(self) -> int:
        return load().cosmica_cancel(self.engine.handle, self.id)

    def state(self) -> int:
        """0 waiting for admission, 1 on the device, 2 done."""
        s = ctypes.c_int32()
        _check(load().cosmica_request_state(self.engine.handle, self.id, ctypes.byref(s)),
               "request_state")
        return s.value

    def result(self) -> dict:
        return self.res.as_dict()


class Engine:
    """A cosmica context on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, stream=None):
        L = load()
        h = ctypes.c_void_p()
        s = None
        if stream is not None:  # torch.cuda.Stream or raw handle
            s = ctypes.c_void_p(getattr(stream, "cuda_stream", stream))
        _check(L.cosmica_create(ctypes.byref(h), device, hbm_budget_bytes, s), "create")
        self.handle = h

    def close(self):
        if self.handle:
            load().cosmica_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # batch
    def run(self, jobs, precision="mixed", exits: bool = False) -> list[dict]:
        jobs = [jobs] if isinstance(jobs, dict) else list(jobs)
        packs = [_JobPack(j) for j in jobs]
        res = [_ResultPack(p.n_bins, p.total, exits) for p in packs]
        jarr = (Job * len(packs))(*[p.job for p in packs])
        rarr = (Result * len(res))(*[r.c for r in res])
        self.last_status = _check(load().cosmica_run(self.handle, jarr, len(packs),
                                                     PRECISION[precision], rarr),
                                  "run", ok=(OK, ESTEPCAP))
        return [r.as_dict() for r in res]

    def run_static(self, jobs, precision="mixed", exits: bool = False) -> list[dict]:
        """cosmica_run_static: run without allocating device memory (buffers in
        the library's static per-GPU array; raises with ESCRATCH past its limits)."""
        jobs = [jobs] if isinstance(jobs, dict) else list(jobs)
        packs = [_JobPack(j) for j in jobs]
        res = [_ResultPack(p.n_bins, p.total, exits) for p in packs]
        jarr = (Job * len(packs))(*[p.job for p in packs])
        rarr = (Result * len(res))(*[r.c for r in res])
        self.last_status = _check(load().cosmica_run_static(self.handle, jarr, len(packs),
                                                            PRECISION[precision], rarr),
                                  "run_static", ok=(OK, ESTEPCAP))
        return [r.as_dict() for r in res]

    def plan(self, jobs, precision="mixed", exits: bool = False) -> Plan:
        jobs = [jobs] if isinstance(jobs, dict) else list(jobs)
        packs = [_JobPack(j) for j in jobs]
        jarr = (Job * len(packs))(*[p.job for p in packs])
        h = ctypes.c_void_p()
        _check(load().cosmica_plan_create(self.handle, jarr, len(packs), PRECISION[precision],
                                          1 if exits else 0, ctypes.byref(h)), "plan_create")
        return Plan(self, h, packs, precision)

    # launch shape / tuner / timings
    def set_launch(self, model, precision, block=256, blocks_per_cu=0, chunk=32, order=2):
        c = Launch(block, blocks_per_cu, chunk, order)
        _check(load().cosmica_set_launch(self.handle, model, PRECISION[precision], ctypes.byref(c)),
               "set_launch")

    def get_launch(self, model, precision) -> dict:
        c = Launch()
        _check(load().cosmica_get_launch(self.handle, model, PRECISION[precision], ctypes.byref(c)),
               "get_launch")
        return {"block": c.block, "blocks_per_cu": c.blocks_per_cu, "chunk": c.chunk,
                "order": c.order}

    def tune(self, model, precision, cache_path: str | None = None) -> dict:
        p = cache_path.encode() if cache_path else None
        _check(load().cosmica_tune(self.handle, model, PRECISION[precision], p), "tune")
        return self.get_launch(model, precision)

    def tune_jobs(self, jobs, precision, sample_particles: int,
                  cache_path: str | None = None) -> dict:
        """Tune on a down-scaled copy of the given jobs (all of one model)."""
        jobs = [jobs] if isinstance(jobs, dict) else list(jobs)
        packs = [_JobPack(j) for j in jobs]
        jarr = (Job * len(packs))(*[p.job for p in packs])
        p = cache_path.encode() if cache_path else None
        _check(load().cosmica_tune_jobs(self.handle, jarr, len(packs), PRECISION[precision],
                                        int(sample_particles), p), "tune_jobs")
        return self.get_launch(int(jobs[0]["helio"]["model"]), precision)

    def timings(self) -> dict:
        t = Timings()
        _check(load().cosmica_get_timings(self.handle, ctypes.byref(t)), "get_timings")
        return {k: getattr(t, k) for k, _ in Timings._fields_}

    # serving
    def submit(self, job: dict, precision="mixed", exits: bool = False) -> Ticket:
        p = _JobPack(job)
        r = _ResultPack(p.n_bins, p.total, exits)
        t = ctypes.c_uint64()
        _check(load().cosmica_submit(self.handle, ctypes.byref(p.job), PRECISION[precision],
                                     ctypes.byref(r.c), ctypes.byref(t)), "submit")
        return Ticket(self, t.value, p, r)

    def serve_stats(self) -> dict:
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(load().cosmica_serve_stats(self.handle, *[ctypes.byref(x) for x in v]),
               "serve_stats")
        return dict(zip(("queued", "resident", "particles_in_flight", "bytes_in_use"),
                        [x.value for x in v]))

    # diagnostics
    def probe_rng(self, seed: int, c0: int, c1: int, c2: int, c3: int, n: int):
        w = np.zeros((n, 4), dtype=np.uint32)
        z64 = np.zeros((n, 3))
        z32 = np.zeros((n, 3), dtype=np.float32)
        _check(load().cosmica_probe_rng(self.handle, seed & (2**64 - 1), c0, c1, c2, c3, n,
                                        w.ctypes.data_as(c_u32_p), z64.ctypes.data_as(c_double_p),
                                        z32.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "probe_rng")
        return w, z64, z32

    def probe_coeffs(self, job: dict, pts, precision="fp64") -> np.ndarray:
        p = _JobPack(job)
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 4)
        out = np.zeros((len(pts), 16))
        _check(load().cosmica_probe_coeffs(self.handle, ctypes.byref(p.job), PRECISION[precision],
                                           len(pts), pts.ctypes.data_as(c_double_p),
                                           out.ctypes.data_as(c_double_p)), "probe_coeffs")
        return out


    def probe_locate(self, job: dict, pts, precision="fp64"):
        """(region, outside) at points (r, theta, phi), decided on the device."""
        p = _JobPack(job)
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        region = np.zeros(len(pts), dtype=np.int32)
        outside = np.zeros(len(pts), dtype=np.int32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        _check(load().cosmica_probe_locate(self.handle, ctypes.byref(p.job), PRECISION[precision],
                                           len(pts), pts.ctypes.data_as(c_double_p),
                                           region.ctypes.data_as(i32p),
                                           outside.ctypes.data_as(i32p)), "probe_locate")
        return region, outside.astype(bool)


PROBE_FIELDS = ("Ar", "At", "Ap", "AP", "Brr", "Bpr", "Bpp", "Btt", "dt", "Hw", "vdr", "vdt",
                "vdp", "Krr", "Krp", "kpar")


def exported_symbols() -> list[str]:
    return sorted(_SIGS)
