/* Drives the host-side logic of libcosmica that needs no device (job
 * validation, error strings, NULL handles, a context on a missing device),
 * for builds whose host code carries the address and undefined-behaviour
 * sanitizers. */
#include <stdio.h>
#include <string.h>

#include "cosmica.h"

static cosmica_helio helio(void)
{
    cosmica_helio h;
    memset(&h, 0, sizeof(h));
    h.model = COSMICA_MODEL_3D;
    h.n_regions = 15;
    h.r_boundary_au = 120.0;
    h.r0_au = 1.0;
    h.theta0_rad = 1.5707963267948966;
    for (int k = 0; k < 15; ++k) {
        h.kappa0_cm2_s[k] = 1.5e22;
        h.v_slow_km_s[k] = 400.0;
        h.tilt_deg[k] = 30.0;
    }
    h.v_fast_km_s = 760.0;
    h.b0_nT = 5.0;
    h.v_ref_km_s = 400.0;
    h.omega_rad_s = 2.66e-6;
    h.kperp_over_kpar = 0.02;
    h.polarity = 1;
    h.drift = 1;
    h.hcs = 1;
    h.dt_max_s = 5e4;
    h.dt_diff_frac = 0.02;
    h.dt_adv_frac = 0.1;
    return h;
}

int main(void)
{
    int bad = 0;
    cosmica_helio h = helio();
    cosmica_species sp = {0.93827208816, 1, 1, 1.9e4, 2.78};
    double rig[3] = {0.5, 2.0, 10.0};
    uint32_t cnt[3] = {10, 20, 30};
    double orbit[6] = {1.0, 1.5, 0.0, 5.0, 0.5, 1.0};
    cosmica_job j;
    memset(&j, 0, sizeof(j));
    j.helio = &h;
    j.species = &sp;
    j.rigidity_gv = rig;
    j.particles_per_bin = cnt;
    j.n_bins = 3;
    j.seed = 42;
    bad |= cosmica_validate_job(&j) != COSMICA_OK;
    j.orbit = orbit;
    j.n_orbit = 2;
    j.formulation = 1;
    bad |= cosmica_validate_job(&j) != COSMICA_OK;
    /* rejected: each alone */
    cosmica_job b = j;
    b.n_bins = 0;
    bad |= cosmica_validate_job(&b) != COSMICA_EINVAL;
    b = j;
    b.formulation = 2;
    bad |= cosmica_validate_job(&b) != COSMICA_EINVAL;
    b = j;
    b.n_orbit = COSMICA_MAX_ORBIT + 1;
    bad |= cosmica_validate_job(&b) != COSMICA_EINVAL;
    b = j;
    b.orbit = NULL;
    bad |= cosmica_validate_job(&b) != COSMICA_EINVAL;
    cosmica_helio hb = h;
    hb.kappa0_cm2_s[7] = -1.0;
    b = j;
    b.helio = &hb;
    bad |= cosmica_validate_job(&b) != COSMICA_EINVAL;
    hb = h;
    hb.heliosheath = 1;  /* no shock distances */
    bad |= cosmica_validate_job(&b) != COSMICA_EINVAL;
    hb = h;
    hb.omega_rad_s = 0.0;
    hb.v_slow_km_s[3] = 0.0;
    hb.drift = 0;
    hb.hcs = 0;
    bad |= cosmica_validate_job(&b) != COSMICA_EINVAL;
    bad |= cosmica_validate_job(NULL) != COSMICA_EINVAL;
    /* strings, NULL handles */
    for (int s = 0; s >= -8; --s) bad |= cosmica_strerror((cosmica_status)s) == NULL;
    bad |= cosmica_abi_version() < 4;
    bad |= cosmica_plan_execute(NULL, NULL) != COSMICA_EINVAL;
    bad |= cosmica_plan_read(NULL, NULL) != COSMICA_EINVAL;
    bad |= cosmica_plan_reweight(NULL, 1, 2, 0.0, 1.0, rig, NULL, NULL) != COSMICA_EINVAL;
    bad |= cosmica_plan_exit_range(NULL, 8, NULL, NULL) != COSMICA_EINVAL;
    cosmica_plan_destroy(NULL);
    cosmica_destroy(NULL);
    /* a context: on a machine without the device this fails cleanly */
    cosmica_ctx* ctx = NULL;
    const cosmica_status st = cosmica_create(&ctx, 0, 0, NULL);
    if (st == COSMICA_OK)
        cosmica_destroy(ctx);
    else
        bad |= ctx != NULL;
    printf(bad ? "failed\n" : "library host code ok\n");
    return bad;
}
