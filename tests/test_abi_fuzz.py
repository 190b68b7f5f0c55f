"""Property tests of the host-side job validation (no device): whatever the
fields hold (NaN, infinities, negatives, zero, huge values), cosmica_validate_job
returns OK or EINVAL without faulting, and every job it accepts satisfies the
rules the header states for the fields drawn here."""
import copy
import math

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_2502_06319_amd import cosmica as C
from paper_2502_06319_amd import workloads as W

ODD = st.sampled_from([0.0, -0.0, -1.0, 1e-300, 1e300, math.inf, -math.inf, math.nan])
VAL = st.one_of(ODD, st.floats(min_value=-1e6, max_value=1e6, allow_nan=False))

HELIO_FIELDS = ["r_boundary_au", "r0_au", "theta0_rad", "phi0_rad", "v_fast_km_s", "b0_nT",
                "v_ref_km_s", "omega_rad_s", "kperp_over_kpar", "dt_max_s", "dt_diff_frac",
                "dt_adv_frac", "r_boundary_nose_au", "ts_nose_au", "ts_tail_au",
                "kappa0_hs_cm2_s", "v_hs_km_s", "tilt_hs_deg", "nose_theta_rad", "nose_phi_rad"]
_BASE = W.c2_job(particles_per_bin=4, n_bins=3)


def _finite_pos(x):
    return math.isfinite(x) and x > 0


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(field=st.sampled_from(HELIO_FIELDS), value=VAL, heliosheath=st.booleans(),
       model=st.sampled_from([0, 1]))
def test_helio_fields(field, value, heliosheath, model):
    job = copy.deepcopy(_BASE)
    if heliosheath:
        job["helio"] = W.with_heliosheath(job["helio"], 85.0, 100.0, 110.0, 140.0, 0.5e22, 150.0,
                                          20.0)
    h = job["helio"]
    h["model"] = model  # a radial model with a heliosheath must be refused
    h[field] = value
    st_ = C.validate_job(job)
    assert st_ in (C.OK, C.EINVAL)
    if st_ == C.OK:
        assert model == 1 or not heliosheath
        assert _finite_pos(h["r_boundary_au"]) and _finite_pos(h["r0_au"])
        assert h["r0_au"] < h["r_boundary_au"]
        assert _finite_pos(h["dt_max_s"]) and _finite_pos(h["dt_diff_frac"])
        if model == 1:
            assert 0.0 < h["theta0_rad"] < math.pi
            assert 0.0 < h["kperp_over_kpar"] <= 1.0
            assert math.isfinite(h["omega_rad_s"]) and h["omega_rad_s"] >= 0.0


@settings(max_examples=200, deadline=None)
@given(values=st.lists(VAL, min_size=15, max_size=15), which=st.sampled_from(
    ["kappa0_cm2_s", "v_slow_km_s", "tilt_deg"]))
def test_region_tables(values, which):
    job = copy.deepcopy(_BASE)
    job["helio"][which] = values
    st_ = C.validate_job(job)
    assert st_ in (C.OK, C.EINVAL)
    if st_ == C.OK:
        v = np.array(values)
        if which == "kappa0_cm2_s":
            assert np.all(np.isfinite(v) & (v > 0))
        elif which == "v_slow_km_s":
            assert np.all(np.isfinite(v) & (v > 0))  # drift is on in this job
        else:
            assert np.all(np.isfinite(v) & (v >= 0) & (v < 90))


@settings(max_examples=200, deadline=None)
@given(rig=st.lists(VAL, min_size=1, max_size=6),
       cnt=st.lists(st.integers(min_value=0, max_value=2**32 - 1), min_size=1, max_size=6),
       mass=VAL, charge=st.integers(min_value=-3, max_value=3), norm=VAL, index=VAL,
       step_cap=st.integers(min_value=0, max_value=2**32 - 1))
def test_bins_species_and_caps(rig, cnt, mass, charge, norm, index, step_cap):
    n = min(len(rig), len(cnt))
    job = copy.deepcopy(_BASE)
    job["rigidity_gv"] = rig[:n]
    job["particles_per_bin"] = cnt[:n]
    job["species"] = dict(job["species"], mass_gev=mass, charge=charge, lis_norm=norm,
                          lis_index=index)
    job["step_cap"] = step_cap
    st_ = C.validate_job(job)
    assert st_ in (C.OK, C.EINVAL)
    if st_ == C.OK:
        assert all(_finite_pos(x) for x in rig[:n])
        assert all(c >= 1 for c in cnt[:n]) and sum(cnt[:n]) < 2**32
        assert math.isfinite(mass) and mass >= 0 and charge != 0
        assert _finite_pos(norm) and math.isfinite(index)
        assert step_cap <= C.MAX_STEP_CAP


@settings(max_examples=150, deadline=None)
@given(orbit=st.lists(st.tuples(VAL, VAL, VAL), min_size=1, max_size=5),
       formulation=st.integers(min_value=-2, max_value=3))
def test_orbits_and_formulation(orbit, formulation):
    job = W.with_orbit(copy.deepcopy(_BASE), [list(p) for p in orbit])
    job["formulation"] = formulation
    st_ = C.validate_job(job)
    assert st_ in (C.OK, C.EINVAL)
    if st_ == C.OK:
        assert formulation in (0, 1)
        for r, th, ph in orbit:
            assert _finite_pos(r) and r < job["helio"]["r_boundary_au"]
            assert 0.0 < th < math.pi and math.isfinite(ph)
