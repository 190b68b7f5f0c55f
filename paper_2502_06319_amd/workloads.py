"""Seeded synthetic inputs for the quasi-particle SDE engine.

This module only *draws and lists physical inputs* (heliosphere parameters in
cm^2/s, km/s, degrees, nT; species masses in GeV; rigidity bins in GV;
particle counts; RNG identities).  It holds none of the method's arithmetic:
unit conversions, coefficients and the integration live separately in the
GPU library and in the CPU oracle, and both consume these dictionaries.

The paper's own workloads (HelMod period parameters, Galprop LIS tables,
AMS-02 data; Sec. II.B, Sec. VII) are not available, so synthetic stand-ins
with the same structure are used: 15 radial shells of the inner heliosphere
(Sec. II.B), several isotopes, log-spaced rigidity checkpoints (Sec. VII), a
power-law LIS.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Rest masses [GeV] (CODATA 2018) and signed charges.
SPECIES = {
    "p": {"name": "p", "mass_gev": 0.93827208816, "charge": 1, "mass_number": 1},
    "He4": {"name": "He4", "mass_gev": 3.7273794066, "charge": 2, "mass_number": 4},
    "He3": {"name": "He3", "mass_gev": 2.80839160743, "charge": 2, "mass_number": 3},
    "e-": {"name": "e-", "mass_gev": 0.51099895e-3, "charge": -1, "mass_number": 0},
}
SPECIES_ORDER = ("p", "He4", "He3", "e-")

LIS_NORM = 1.9e4
LIS_INDEX = 2.78
STEP_CAP = 10_000_000


def log_bins(p_min: float, p_max: float, n: int) -> list[float]:
    """n rigidity checkpoints from p_min to p_max, log-spaced, endpoints included."""
    if n == 1:
        return [float(p_min)]
    return [float(p_min * (p_max / p_min) ** (i / (n - 1))) for i in range(n)]


def species(name: str) -> dict:
    s = dict(SPECIES[name])
    s["lis_norm"] = LIS_NORM
    s["lis_index"] = LIS_INDEX
    return s


def helio_1d(kappa0=1.5e22, v=400.0, r_boundary=100.0, dt_max=5e4) -> dict:
    """Spherically symmetric heliosphere with one shell (radial model)."""
    return {
        "model": 0,
        "n_regions": 1,
        "kappa0_cm2_s": [float(kappa0)],
        "v_slow_km_s": [float(v)],
        "tilt_deg": [0.0],
        "v_fast_km_s": float(v),
        "r_boundary_au": float(r_boundary),
        "r0_au": 1.0,
        "theta0_rad": math.pi / 2,
        "phi0_rad": 0.0,
        "b0_nT": 5.0,
        "v_ref_km_s": 400.0,
        "omega_rad_s": 2.66e-6,
        "kperp_over_kpar": 1.0,
        "polarity": 1,
        "drift": 0,
        "hcs": 0,
        "dt_max_s": float(dt_max),
        "dt_diff_frac": 0.02,
        "dt_adv_frac": 0.0,
        **SPHERICAL_NO_HELIOSHEATH,
    }


# Geometry fields of a spherical heliosphere without a heliosheath: the
# boundary's nose distance 0 means "equal to r_boundary_au".
SPHERICAL_NO_HELIOSHEATH = {
    "r_boundary_nose_au": 0.0,
    "nose_theta_rad": math.pi / 2,
    "nose_phi_rad": 0.0,
    "heliosheath": 0,
    "ts_nose_au": 0.0,
    "ts_tail_au": 0.0,
    "kappa0_hs_cm2_s": 0.0,
    "v_hs_km_s": 0.0,
    "tilt_hs_deg": 0.0,
}


def with_heliosheath(helio: dict, ts_nose, ts_tail, hp_nose, hp_tail, kappa0_hs, v_hs,
                     tilt_hs_deg, nose_theta=math.radians(95.0), nose_phi=0.0) -> dict:
    """A copy of a 3D heliosphere with a nose-squashed heliopause (distances
    hp_nose toward the nose, hp_tail toward the tail), a termination shock
    (ts_nose, ts_tail) and a heliosheath region between them."""
    h = copy.deepcopy(helio)
    assert h["model"] == 1
    h.update({"r_boundary_au": float(hp_tail), "r_boundary_nose_au": float(hp_nose),
              "nose_theta_rad": float(nose_theta), "nose_phi_rad": float(nose_phi),
              "heliosheath": 1, "ts_nose_au": float(ts_nose), "ts_tail_au": float(ts_tail),
              "kappa0_hs_cm2_s": float(kappa0_hs), "v_hs_km_s": float(v_hs),
              "tilt_hs_deg": float(tilt_hs_deg)})
    return h


def draw_heliosheath(rng: np.random.Generator, helio: dict) -> dict:
    """Synthetic heliosheath geometry for a drawn parameter set (stand-in for
    the HelMod geometry, which is not available): termination shock at
    U[80, 90] AU toward the nose and 1.2-1.4x that toward the tail; heliopause
    at U[115, 125] AU toward the nose and 1.3-1.5x that toward the tail; nose
    5 deg south of the solar equator at a uniform longitude from the injection
    point; heliosheath kappa0 ~ U[0.2, 1.0]e22 cm^2/s, wind U[100, 200] km/s,
    current-sheet tilt of the outermost shell."""
    ts_n = rng.uniform(80.0, 90.0)
    hp_n = rng.uniform(115.0, 125.0)
    return with_heliosheath(helio, ts_n, ts_n * rng.uniform(1.2, 1.4), hp_n,
                            hp_n * rng.uniform(1.3, 1.5), rng.uniform(0.2e22, 1.0e22),
                            rng.uniform(100.0, 200.0), helio["tilt_deg"][-1],
                            nose_theta=math.radians(95.0),
                            nose_phi=rng.uniform(0.0, 2.0 * math.pi))


def helio_3d(kappa0, v_slow, tilt_deg, polarity=1, r_boundary=120.0, drift=1, hcs=1,
             kperp_over_kpar=0.02, v_fast=760.0, dt_max=5e4, dt_adv_frac=0.1) -> dict:
    """Full 3D heliosphere: equal-width shells, each with (kappa0, Vslow, tilt)."""
    kappa0 = [float(x) for x in np.atleast_1d(kappa0)]
    v_slow = [float(x) for x in np.atleast_1d(v_slow)]
    tilt_deg = [float(x) for x in np.atleast_1d(tilt_deg)]
    n = len(kappa0)
    assert len(v_slow) == n and len(tilt_deg) == n and 1 <= n <= 15
    return {
        "model": 1,
        "n_regions": n,
        "kappa0_cm2_s": kappa0,
        "v_slow_km_s": v_slow,
        "tilt_deg": tilt_deg,
        "v_fast_km_s": float(v_fast),
        "r_boundary_au": float(r_boundary),
        "r0_au": 1.0,
        "theta0_rad": math.pi / 2,
        "phi0_rad": 0.0,
        "b0_nT": 5.0,
        "v_ref_km_s": 400.0,
        "omega_rad_s": 2.66e-6,
        "kperp_over_kpar": float(kperp_over_kpar),
        "polarity": int(polarity),
        "drift": int(drift),
        "hcs": int(hcs),
        "dt_max_s": float(dt_max),
        "dt_diff_frac": 0.02,
        "dt_adv_frac": float(dt_adv_frac),
        **SPHERICAL_NO_HELIOSHEATH,
    }


def draw_helio_3d(rng: np.random.Generator, polarity=None) -> dict:
    """One synthetic parameter set: 15 shells with kappa0 ~ U[0.5,3]e22 cm^2/s,
    Vslow ~ U[350,750] km/s, tilt ~ U[5,75] deg; polarity +-1 with equal odds
    unless given."""
    k0 = rng.uniform(0.5e22, 3.0e22, 15)
    vs = rng.uniform(350.0, 750.0, 15)
    tilt = rng.uniform(5.0, 75.0, 15)
    pol = int(polarity) if polarity is not None else (1 if rng.uniform() < 0.5 else -1)
    return helio_3d(k0, vs, tilt, polarity=pol)


def make_job(helio: dict, spec: dict, rigidities, counts, seed=42, job_tag=0) -> dict:
    rig = [float(x) for x in rigidities]
    cnt = [int(x) for x in np.broadcast_to(np.asarray(counts), (len(rig),))]
    return {
        "helio": copy.deepcopy(helio),
        "species": dict(spec),
        "rigidity_gv": rig,
        "particles_per_bin": cnt,
        "seed": int(seed),
        "job_tag": int(job_tag),
        "step_cap": STEP_CAP,
    }


# --------------------------------------------------------------------------
# The five workloads (config 1..5).
# --------------------------------------------------------------------------

def c1_job(particles_per_bin=1024, seed=42) -> dict:
    """Radial model, protons, R=100 AU, V=400 km/s, kappa0=1.5e22 cm^2/s, no drift;
    8 log-spaced rigidities 0.5-20 GV; 1,024 particles per bin; Philox seed 42."""
    return make_job(helio_1d(), species("p"), log_bins(0.5, 20.0, 8), particles_per_bin,
                    seed=seed, job_tag=0)


def c2_helio(seed=42) -> dict:
    rng = np.random.default_rng(seed)
    return draw_helio_3d(rng, polarity=1)


def c2_job(particles_per_bin=5000, seed=42, n_bins=20) -> dict:
    """Full 3D model, protons, A>0, one 15-shell parameter set drawn with seed 42;
    20 log-spaced rigidities 0.1-100 GV; 5,000 particles per bin."""
    return make_job(c2_helio(seed), species("p"), log_bins(0.1, 100.0, n_bins),
                    particles_per_bin, seed=seed, job_tag=0)


def c4_jobs(seed=42, n_sets=64, species_names=SPECIES_ORDER, n_bins=30,
            n_min=500, n_max=20000, count_scale=1.0) -> list[dict]:
    """Batched workload: n_sets parameter sets x species x n_bins rigidities
    0.1-100 GV, particles per bin log-uniform in [n_min, n_max]."""
    rng = np.random.default_rng(seed)
    sets = [draw_helio_3d(rng) for _ in range(n_sets)]
    bins = log_bins(0.1, 100.0, n_bins)
    jobs = []
    tag = 0
    for h in sets:
        for sp in species_names:
            n = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_bins)))
            n = np.maximum(1, np.rint(n * count_scale)).astype(int)
            jobs.append(make_job(h, species(sp), bins, n, seed=seed, job_tag=tag))
            tag += 1
    return jobs


def c2_heliosheath_job(particles_per_bin=5000, seed=42, n_bins=20) -> dict:
    """The config-2 job in a nose-squashed heliosphere with a heliosheath
    (geometry drawn with seed + 1)."""
    job = c2_job(particles_per_bin, seed, n_bins)
    job["helio"] = draw_heliosheath(np.random.default_rng(seed + 1), job["helio"])
    return job


def c4_heliosheath_jobs(seed=42, **kw) -> list[dict]:
    """The batched workload with a heliosheath geometry drawn per parameter
    set (seed + 1 stream, so the shells, species and counts are unchanged)."""
    jobs = c4_jobs(seed=seed, **kw)
    rng = np.random.default_rng(seed + 1)
    n_species = len(kw.get("species_names", SPECIES_ORDER))
    for i in range(0, len(jobs), n_species):
        h = draw_heliosheath(rng, jobs[i]["helio"])
        for j in jobs[i:i + n_species]:
            j["helio"] = copy.deepcopy(h)
    return jobs


def kepler_orbit(n, a_au, ecc, incl_deg, arg_peri_deg=0.0, node_deg=0.0) -> np.ndarray:
    """n positions (r [AU], theta, phi) at equal time steps along a heliocentric
    Kepler orbit (semi-major axis a, eccentricity, inclination to the solar
    equator, argument of perihelion, longitude of the ascending node)."""
    M = 2.0 * math.pi * (np.arange(n) + 0.5) / n  # mean anomaly, equal times
    E = M.copy()
    for _ in range(50):  # Newton on E - e sin E = M
        E = E - (E - ecc * np.sin(E) - M) / (1.0 - ecc * np.cos(E))
    nu = 2.0 * np.arctan2(math.sqrt(1 + ecc) * np.sin(E / 2), math.sqrt(1 - ecc) * np.cos(E / 2))
    r = a_au * (1.0 - ecc * np.cos(E))
    u = nu + math.radians(arg_peri_deg)  # argument of latitude
    i, Om = math.radians(incl_deg), math.radians(node_deg)
    x = r * (np.cos(Om) * np.cos(u) - np.sin(Om) * np.sin(u) * np.cos(i))
    y = r * (np.sin(Om) * np.cos(u) + np.cos(Om) * np.sin(u) * np.cos(i))
    z = r * np.sin(u) * np.sin(i)
    th = np.arccos(np.clip(z / r, -1.0, 1.0))
    ph = np.mod(np.arctan2(y, x), 2.0 * math.pi)
    return np.stack([r, th, ph], 1)


def earth_orbit(n=12) -> np.ndarray:
    """One year of the Earth's orbit: a = 1 AU, e = 0.0167, 7.25 deg to the
    solar equator."""
    return kepler_orbit(n, 1.0, 0.0167, 7.25)


def ulysses_like_orbit(n=24) -> np.ndarray:
    """A polar out-of-ecliptic orbit like Ulysses' (a = 3.37 AU, e = 0.603,
    79 deg to the solar equator; perihelion 1.34 AU, aphelion 5.4 AU)."""
    return kepler_orbit(n, 3.37, 0.603, 79.1, arg_peri_deg=-90.0)


def with_orbit(job: dict, orbit) -> dict:
    """A copy of a job whose particles are split over the orbit positions
    (particle i of every bin starts at position i mod len(orbit))."""
    j = copy.deepcopy(job)
    j["orbit"] = np.ascontiguousarray(orbit, dtype=np.float64).reshape(-1, 3).tolist()
    return j


def c4_orbit_jobs(seed=42, n_orbit=24, **kw) -> list[dict]:
    """The batched workload seen from a Ulysses-like polar orbit."""
    orbit = ulysses_like_orbit(n_orbit)
    return [with_orbit(j, orbit) for j in c4_jobs(seed=seed, **kw)]


def c5_requests(seed=42, rate_hz=5.0, duration_s=600.0, n_min=1000, n_max=100000,
                bins_min=10, bins_max=50, count_scale=1.0, max_requests=None) -> list[dict]:
    """Poisson stream of spectrum requests.  Each carries one random parameter set
    and species, U{bins_min..bins_max} rigidity bins over 0.1-100 GV and
    log-uniform [n_min, n_max] particles per bin; each has its own seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    i = 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s or (max_requests is not None and i >= max_requests):
            break
        h = draw_helio_3d(rng)
        sp = SPECIES_ORDER[int(rng.integers(0, len(SPECIES_ORDER)))]
        nb = int(rng.integers(bins_min, bins_max + 1))
        n = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), nb)))
        n = np.maximum(1, np.rint(n * count_scale)).astype(int)
        req_seed = int(rng.integers(1, 2**63 - 1))
        job = make_job(h, species(sp), log_bins(0.1, 100.0, nb), n, seed=req_seed, job_tag=i)
        reqs.append({"arrival_s": t, "job": job})
        i += 1
    return reqs


def total_particles(jobs) -> int:
    return int(sum(sum(j["particles_per_bin"]) for j in jobs))
