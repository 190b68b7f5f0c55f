/* Drives every oracle entry point on small inputs, for builds with the
 * address and undefined-behaviour sanitizers (host code only). */
#include <stdio.h>
#include <string.h>

#include "cosmica_oracle.h"

static void helio_3d(orc_params* p)
{
    memset(p, 0, sizeof(*p));
    p->model = 1;
    p->n_regions = 15;
    p->r_boundary_au = 100.0;
    p->r0_au = 1.0;
    p->theta0_rad = 1.5707963267948966;
    for (int k = 0; k < 15; ++k) {
        p->kappa0_cm2_s[k] = 1.5e22;
        p->v_slow_km_s[k] = 400.0;
        p->tilt_deg[k] = 30.0;
    }
    p->v_fast_km_s = 760.0;
    p->b0_nT = 5.0;
    p->v_ref_km_s = 400.0;
    p->omega_rad_s = 2.66e-6;
    p->kperp_over_kpar = 0.02;
    p->polarity = -1;
    p->drift = 1;
    p->hcs = 1;
    p->dt_max_s = 5e4;
    p->dt_diff_frac = 0.02;
    p->dt_adv_frac = 0.1;
    p->mass_gev = 0.93827208816;
    p->charge = 1;
    p->lis_norm = 1.9e4;
    p->lis_index = 2.78;
    p->seed = 42;
    p->step_cap = 200000;
}

static int run(const orc_params* p, const char* what)
{
    enum { N = 24 };
    orc_exit rec[N];
    orc_bin_result res;
    double lnJ[2 * 8], flux[2], se[2], pmax;
    uint32_t hist[16];
    for (int k = 0; k < 8; ++k) {
        lnJ[k] = 9.9 - 2.7 * (-3.0 + 0.5 * k);
        lnJ[8 + k] = 9.5 - 3.0 * (-3.0 + 0.5 * k);
    }
    if (orc_propagate(p, 0, 2.0, 0, N, rec, 1) != 0) {
        printf("%s: propagate failed\n", what);
        return 1;
    }
    orc_reduce_bin(p, 2.0, rec, N, &res);
    orc_reweight_bin(p, 2.0, rec, N, 2, 8, -3.0, 0.5, lnJ, flux, se);
    orc_exit_range(2.0, rec, N, 16, &pmax, hist);
    printf("%s: J %.4e se %.2e reweighted %.4e max %.3f\n", what, res.flux, res.flux_se, flux[1],
           pmax);
    return 0;
}

int main(void)
{
    orc_params p;
    int bad = 0;
    uint32_t ctr[4] = {1, 2, 3, 4}, w[4];
    double z[4];
    orc_philox4x32_10(42, ctr, w);
    orc_normals(42, ctr, z);

    helio_3d(&p);
    bad |= run(&p, "3d momentum");
    p.formulation = 1;
    bad |= run(&p, "3d energy");
    p.formulation = 0;
    p.r_boundary_nose_au = 80.0;
    p.heliosheath = 1;
    p.ts_nose_au = 60.0;
    p.ts_tail_au = 70.0;
    p.kappa0_hs_cm2_s = 5e21;
    p.v_hs_km_s = 150.0;
    p.tilt_hs_deg = 30.0;
    bad |= run(&p, "3d heliosheath");
    const double orbit[6] = {1.0, 1.2, 0.0, 3.0, 0.6, 2.0};
    p.orbit = orbit;
    p.n_orbit = 2;
    bad |= run(&p, "3d orbit");
    helio_3d(&p);
    p.model = 0;
    p.n_regions = 1;
    bad |= run(&p, "radial");
    p.step_cap = 3;
    bad |= run(&p, "radial capped");
    double state[5] = {1.0, 1.5, 0.0, 2.0, 0.0};
    uint32_t n = 0;
    (void)orc_advance(&p, 0, 0, state, &n, 2);
    p.n_regions = 0;  /* invalid: rejected, nothing written */
    orc_exit rec[1];
    if (orc_propagate(&p, 0, 2.0, 0, 1, rec, 1) != -1) bad = 1;
    printf(bad ? "failed\n" : "oracle ok\n");
    return bad;
}
