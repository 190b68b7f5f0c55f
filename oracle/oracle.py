"""ctypes front-end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``oracle/liboracle.so`` (plain C, built with gcc
from ``cosmica_oracle.c``) and marshals the seeded workload dictionaries into
the oracle's own parameter struct.  No arithmetic of the method lives here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cosmica_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
NHIST = 129
MAXREG = 15


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, OpenMP, no fast-math, no FP contraction."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd, cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("n_regions", ctypes.c_int32),
        ("r_boundary_au", ctypes.c_double),
        ("r0_au", ctypes.c_double),
        ("theta0_rad", ctypes.c_double),
        ("phi0_rad", ctypes.c_double),
        ("kappa0_cm2_s", ctypes.c_double * MAXREG),
        ("v_slow_km_s", ctypes.c_double * MAXREG),
        ("tilt_deg", ctypes.c_double * MAXREG),
        ("v_fast_km_s", ctypes.c_double),
        ("b0_nT", ctypes.c_double),
        ("v_ref_km_s", ctypes.c_double),
        ("omega_rad_s", ctypes.c_double),
        ("kperp_over_kpar", ctypes.c_double),
        ("polarity", ctypes.c_int32),
        ("drift", ctypes.c_int32),
        ("hcs", ctypes.c_int32),
        ("flip_z2", ctypes.c_int32),
        ("dt_max_s", ctypes.c_double),
        ("dt_diff_frac", ctypes.c_double),
        ("dt_adv_frac", ctypes.c_double),
        ("mass_gev", ctypes.c_double),
        ("charge", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("lis_norm", ctypes.c_double),
        ("lis_index", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("job_tag", ctypes.c_uint32),
        ("step_cap", ctypes.c_uint32),
        ("r_boundary_nose_au", ctypes.c_double),
        ("nose_theta_rad", ctypes.c_double),
        ("nose_phi_rad", ctypes.c_double),
        ("heliosheath", ctypes.c_int32),
        ("pad1", ctypes.c_int32),
        ("ts_nose_au", ctypes.c_double),
        ("ts_tail_au", ctypes.c_double),
        ("kappa0_hs_cm2_s", ctypes.c_double),
        ("v_hs_km_s", ctypes.c_double),
        ("tilt_hs_deg", ctypes.c_double),
        ("orbit", ctypes.POINTER(ctypes.c_double)),
        ("n_orbit", ctypes.c_uint32),
        ("formulation", ctypes.c_int32),
    ]


class OrcExit(ctypes.Structure):
    _fields_ = [("P", ctypes.c_double), ("t", ctypes.c_double), ("r", ctypes.c_double),
                ("theta", ctypes.c_double), ("phi", ctypes.c_double),
                ("n", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("loss", ctypes.c_double)]


EXIT_DTYPE = np.dtype([("P", "<f8"), ("t", "<f8"), ("r", "<f8"), ("theta", "<f8"),
                       ("phi", "<f8"), ("n", "<u4"), ("flags", "<u4"), ("loss", "<f8")])
assert EXIT_DTYPE.itemsize == ctypes.sizeof(OrcExit)


class OrcCoeffs(ctypes.Structure):
    _fields_ = [
        ("region", ctypes.c_int32),
        ("V", ctypes.c_double), ("kpar", ctypes.c_double), ("kperp", ctypes.c_double),
        ("Krr", ctypes.c_double), ("Kpp", ctypes.c_double), ("Krp", ctypes.c_double),
        ("Ktt", ctypes.c_double), ("dKrr_dr", ctypes.c_double), ("dKrp_term", ctypes.c_double),
        ("Brr", ctypes.c_double), ("Bpr", ctypes.c_double), ("Bpp", ctypes.c_double),
        ("Btt", ctypes.c_double), ("Bmag_nT", ctypes.c_double), ("Gamma", ctypes.c_double),
        ("G", ctypes.c_double), ("Hw", ctypes.c_double), ("sign_qA", ctypes.c_double),
        ("vd", ctypes.c_double * 3), ("A", ctypes.c_double * 3), ("AP", ctypes.c_double),
        ("dt", ctypes.c_double),
    ]


class OrcBinResult(ctypes.Structure):
    _fields_ = [("hist", ctypes.c_uint32 * NHIST), ("flux", ctypes.c_double),
                ("flux_se", ctypes.c_double), ("mean_exit_time_s", ctypes.c_double),
                ("steps", ctypes.c_uint64), ("n_capped", ctypes.c_uint32),
                ("n_nan", ctypes.c_uint32), ("n_used", ctypes.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_philox4x32_10.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_uint32)]
        L.orc_normals.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32),
                                  ctypes.POINTER(ctypes.c_double)]
        L.orc_rng_block.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 5 + [
            ctypes.c_void_p, ctypes.c_void_p]
        L.orc_coeffs_3d.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.POINTER(OrcCoeffs)]
        L.orc_propagate.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_uint32, ctypes.c_double,
                                    ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                    ctypes.c_int]
        L.orc_propagate.restype = ctypes.c_int
        L.orc_advance.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint32),
                                  ctypes.c_uint32]
        L.orc_advance.restype = ctypes.c_int
        L.orc_reduce_bin.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_double, ctypes.c_void_p,
                                     ctypes.c_uint32, ctypes.POINTER(OrcBinResult)]
        L.orc_locate.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.POINTER(ctypes.c_int32)]
        L.orc_locate.restype = ctypes.c_int
        L.orc_reweight_bin.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_lis.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_double]
        L.orc_exit_range.argtypes = [ctypes.c_double, ctypes.c_void_p, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_lis.restype = ctypes.c_double
        _lib = L
    return _lib


def params(job: dict, **override) -> OrcParams:
    """Pack a workload job dictionary into the oracle's parameter struct."""
    h = dict(job["helio"])
    h.update({k: v for k, v in override.items() if k in h})
    sp = dict(job["species"])
    sp.update({k: v for k, v in override.items() if k in sp})
    p = OrcParams()
    p.model = int(h["model"])
    p.n_regions = int(h["n_regions"])
    p.r_boundary_au = h["r_boundary_au"]
    p.r0_au = h["r0_au"]
    p.theta0_rad = h["theta0_rad"]
    p.phi0_rad = h["phi0_rad"]
    for k in range(p.n_regions):
        p.kappa0_cm2_s[k] = h["kappa0_cm2_s"][k]
        p.v_slow_km_s[k] = h["v_slow_km_s"][k]
        p.tilt_deg[k] = h["tilt_deg"][k]
    p.v_fast_km_s = h["v_fast_km_s"]
    p.b0_nT = h["b0_nT"]
    p.v_ref_km_s = h["v_ref_km_s"]
    p.omega_rad_s = h["omega_rad_s"]
    p.kperp_over_kpar = h["kperp_over_kpar"]
    p.polarity = int(h["polarity"])
    p.drift = int(h["drift"])
    p.hcs = int(h["hcs"])
    p.flip_z2 = int(override.get("flip_z2", 0))
    p.dt_max_s = h["dt_max_s"]
    p.dt_diff_frac = h["dt_diff_frac"]
    p.dt_adv_frac = h["dt_adv_frac"]
    p.mass_gev = sp["mass_gev"]
    p.charge = int(sp["charge"])
    p.lis_norm = sp["lis_norm"]
    p.lis_index = sp["lis_index"]
    p.seed = int(override.get("seed", job["seed"])) & (2**64 - 1)
    p.job_tag = int(override.get("job_tag", job["job_tag"]))
    p.step_cap = int(override.get("step_cap", job.get("step_cap", 10_000_000)))
    p.r_boundary_nose_au = h.get("r_boundary_nose_au", 0.0)
    p.nose_theta_rad = h.get("nose_theta_rad", 0.5 * np.pi)
    p.nose_phi_rad = h.get("nose_phi_rad", 0.0)
    p.heliosheath = int(h.get("heliosheath", 0))
    p.ts_nose_au = h.get("ts_nose_au", 0.0)
    p.ts_tail_au = h.get("ts_tail_au", 0.0)
    p.kappa0_hs_cm2_s = h.get("kappa0_hs_cm2_s", 0.0)
    p.v_hs_km_s = h.get("v_hs_km_s", 0.0)
    p.tilt_hs_deg = h.get("tilt_hs_deg", 0.0)
    p.formulation = int(job.get("formulation", 0))
    orbit = job.get("orbit")
    if orbit is not None and len(orbit) > 0:
        arr = np.ascontiguousarray(orbit, dtype=np.float64).reshape(-1, 3)
        p._orbit_keep = arr  # the struct points into this array
        p.orbit = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.n_orbit = len(arr)
    return p


def philox(seed: int, ctr) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(ctypes.c_uint64(seed), c, o)
    return np.array(list(o), dtype=np.uint32)


def normals(seed: int, ctr) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    o = (ctypes.c_double * 4)()
    lib().orc_normals(ctypes.c_uint64(seed), c, o)
    return np.array(list(o))


def rng_block(seed: int, c0: int, c1: int, c2: int, c3: int, n: int):
    """Philox words (n, 4) and normals (n, 4) for counters (c0 + i, c1, c2, c3)."""
    w = np.zeros((n, 4), dtype=np.uint32)
    z = np.zeros((n, 4))
    lib().orc_rng_block(seed & (2**64 - 1), c0, c1, c2, c3, n, w.ctypes.data, z.ctypes.data)
    return w, z


def coeffs_3d(p: OrcParams, P, r, theta, phi) -> dict:
    c = OrcCoeffs()
    lib().orc_coeffs_3d(ctypes.byref(p), P, r, theta, phi, ctypes.byref(c))
    out = {}
    for name, _ in OrcCoeffs._fields_:
        v = getattr(c, name)
        out[name] = list(v) if name in ("vd", "A") else v
    return out


def propagate(p: OrcParams, bin_index: int, P0: float, count: int, first: int = 0,
              threads: int = 0) -> np.ndarray:
    out = np.zeros(count, dtype=EXIT_DTYPE)
    rc = lib().orc_propagate(ctypes.byref(p), bin_index, P0, first, count,
                             out.ctypes.data_as(ctypes.c_void_p), threads)
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    return out


def advance(p: OrcParams, bin_index: int, particle: int, state, n: int, max_steps: int):
    st = (ctypes.c_double * 5)(*state)
    nn = ctypes.c_uint32(n)
    done = lib().orc_advance(ctypes.byref(p), bin_index, particle, st, ctypes.byref(nn),
                             max_steps)
    return list(st), nn.value, bool(done)


def reduce_bin(p: OrcParams, P0: float, rec: np.ndarray) -> dict:
    rec = np.ascontiguousarray(rec, dtype=EXIT_DTYPE)
    r = OrcBinResult()
    lib().orc_reduce_bin(ctypes.byref(p), P0, rec.ctypes.data_as(ctypes.c_void_p), len(rec),
                         ctypes.byref(r))
    return {"hist": np.array(list(r.hist), dtype=np.uint32), "flux": r.flux,
            "flux_se": r.flux_se, "mean_exit_time_s": r.mean_exit_time_s, "steps": r.steps,
            "n_capped": r.n_capped, "n_nan": r.n_nan, "n_used": r.n_used}


def locate(p: OrcParams, r: float, theta: float, phi: float) -> tuple[bool, int]:
    """(outside the heliopause, parameter region) at a point."""
    k = ctypes.c_int32()
    out = lib().orc_locate(ctypes.byref(p), r, theta, phi, ctypes.byref(k))
    if out < 0:
        raise ValueError("oracle rejected the parameters")
    return bool(out), int(k.value)


def reweight_bin(p: OrcParams, P0: float, rec: np.ndarray, lnP0: float, dlnP: float,
                 lnJ: np.ndarray):
    """J_mod(P0) and its standard error for each tabulated spectrum (rows of lnJ)."""
    rec = np.ascontiguousarray(rec, dtype=EXIT_DTYPE)
    lnJ = np.ascontiguousarray(np.atleast_2d(lnJ), dtype=np.float64)
    n_lis, n_knots = lnJ.shape
    flux = np.zeros(n_lis)
    se = np.zeros(n_lis)
    lib().orc_reweight_bin(ctypes.byref(p), P0, rec.ctypes.data, len(rec), n_lis, n_knots,
                           lnP0, dlnP, lnJ.ctypes.data, flux.ctypes.data, se.ctypes.data)
    return flux, se


def exit_range(P0: float, rec: np.ndarray, n_hist: int):
    """(P_max, counts of ln(P_ex/P0) in n_hist equal bins over [0, ln(P_max/P0)])."""
    rec = np.ascontiguousarray(rec, dtype=EXIT_DTYPE)
    pm = ctypes.c_double()
    hist = np.zeros(n_hist, dtype=np.uint32)
    lib().orc_exit_range(P0, rec.ctypes.data, len(rec), n_hist, ctypes.byref(pm), hist.ctypes.data)
    return pm.value, hist


def lis(p: OrcParams, P: float) -> float:
    return lib().orc_lis(ctypes.byref(p), P)


def run_job(job: dict, threads: int = 0, bins=None, count=None, first: int = 0,
            **override) -> list[dict]:
    """Propagate and reduce every (or the selected) bin of a job.

    Returns one dict per bin with the exit records and the reduced results."""
    p = params(job, **override)
    out = []
    sel = range(len(job["rigidity_gv"])) if bins is None else bins
    for b in sel:
        P0 = job["rigidity_gv"][b]
        n = job["particles_per_bin"][b] if count is None else count
        # the bin's random streams are those of bin index bin_offset + b
        rec = propagate(p, int(job.get("bin_offset", 0)) + b, P0, n, first=first,
                        threads=threads)
        res = reduce_bin(p, P0, rec)
        res["records"] = rec
        res["bin"] = b
        res["P0"] = P0
        out.append(res)
    return out
