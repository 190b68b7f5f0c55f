"""Parameter scans and spectrum fits on the engine.

The use the paper closes on (Sec. VIII): heliospheric parameters are found by
fitting simulated spectra to observed ones, averaging many simulation fits.  A
scan runs every point of a grid of heliosphere parameters as one batched plan
(one persistent launch), then re-weights the stored exit records with a
family of local interstellar spectra (cosmica_plan_reweight): G parameter
points and S spectra cost G propagations, not G * S.

Host-side orchestration only: the propagation, reduction and re-weighting run
in the HIP library.
"""
from __future__ import annotations

import copy
import itertools
import math
from dataclasses import dataclass

import numpy as np

from . import cosmica as C


def power_law_tables(norms, indices, lnP0=math.log(0.05), dlnP=0.25, n_knots=40):
    """ln J tables of power laws J = norm P^-index on the knots
    ln P = lnP0 + k dlnP (exact in log-log interpolation)."""
    lnP = lnP0 + dlnP * np.arange(n_knots)
    rows = [math.log(n) - g * lnP for n, g in itertools.product(norms, indices)]
    return np.array(rows), lnP0, dlnP


def _apply(helio: dict, point: dict) -> dict:
    h = copy.deepcopy(helio)
    for k, v in point.items():
        if k == "kappa0_scale":  # every shell's kappa0, and the heliosheath's
            h["kappa0_cm2_s"] = [x * v for x in h["kappa0_cm2_s"]]
            if h.get("heliosheath", 0):
                h["kappa0_hs_cm2_s"] *= v
        elif k == "tilt_deg":  # one tilt for every shell
            h["tilt_deg"] = [float(v)] * len(h["tilt_deg"])
        else:
            h[k] = v
    return h


@dataclass
class ScanResult:
    points: list[dict]       # grid points, in job order
    lis: np.ndarray          # the ln J tables (n_lis, n_knots)
    flux: np.ndarray         # (n_points, n_lis, n_bins)
    flux_se: np.ndarray
    rigidity_gv: np.ndarray  # (n_bins,)


def scan(engine: C.Engine, base_job: dict, grid: dict, lis_tables, precision="mixed",
         seed=None) -> ScanResult:
    """Run base_job at every point of the Cartesian grid {field: values} (fields
    of the heliosphere, plus kappa0_scale), as one plan, and re-weight every
    point with each spectrum of lis_tables = (lnJ rows, lnP0, dlnP)."""
    lnJ, lnP0, dlnP = lis_tables
    keys = list(grid)
    points = [dict(zip(keys, vals)) for vals in itertools.product(*(grid[k] for k in keys))]
    jobs = []
    for i, pt in enumerate(points):
        j = copy.deepcopy(base_job)
        j["helio"] = _apply(base_job["helio"], pt)
        j["job_tag"] = i
        if seed is not None:
            j["seed"] = seed
        jobs.append(j)
    plan = engine.plan(jobs, precision)
    try:
        plan.execute()
        plan.read()
        flux, se = plan.reweight(lnP0, dlnP, lnJ)
    finally:
        plan.destroy()
    nb = len(base_job["rigidity_gv"])
    n = len(points)
    # plan bins are job-major: [lis, point * nb + b] -> [point, lis, b]
    flux = flux.reshape(len(lnJ), n, nb).transpose(1, 0, 2)
    se = se.reshape(len(lnJ), n, nb).transpose(1, 0, 2)
    return ScanResult(points, np.asarray(lnJ), flux, se, np.asarray(base_job["rigidity_gv"]))


def fit(result: ScanResult, observed, observed_err, lis_params=None) -> dict:
    """chi^2 of every (grid point, spectrum) against an observed spectrum (same
    rigidities), with the simulation's own standard error added in quadrature;
    the best pair, and the average of the parameters weighted by
    exp(-(chi^2 - chi^2_min)/2) over all fits.  lis_params: optional
    (n_lis, k) array of the spectra's parameters, averaged likewise."""
    obs = np.asarray(observed, dtype=float)
    err2 = np.asarray(observed_err, dtype=float) ** 2
    chi2 = (((result.flux - obs) ** 2) / (err2 + result.flux_se ** 2)).sum(axis=2)
    g, l = np.unravel_index(int(np.argmin(chi2)), chi2.shape)
    w = np.exp(-(chi2 - chi2[g, l]) / 2.0)
    w /= w.sum()
    out = {"chi2": chi2, "best_point": result.points[g], "best_lis": int(l),
           "chi2_min": float(chi2[g, l]), "ndof": obs.size}
    mean, sd = {}, {}
    for k in result.points[0]:
        vals = np.array([p[k] for p in result.points], dtype=float)
        m = float((w.sum(axis=1) * vals).sum())
        mean[k] = m
        sd[k] = math.sqrt(max(0.0, float((w.sum(axis=1) * (vals - m) ** 2).sum())))
    if lis_params is not None:
        lp = np.asarray(lis_params, dtype=float).reshape(chi2.shape[1], -1)
        wl = w.sum(axis=0)
        m = (wl[:, None] * lp).sum(axis=0)
        mean["lis"] = m.tolist()
        sd["lis"] = np.sqrt((wl[:, None] * (lp - m) ** 2).sum(axis=0)).tolist()
    out["mean"], out["sd"] = mean, sd
    return out
