/*
 * cosmica_oracle.h -- plain FP64 CPU oracle for the backward-in-time SDE
 * integration of heliospheric cosmic-ray quasi-particles (COSMICA, arXiv
 * 2502.06319).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference that
 * the GPU path is compared against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source,
 * header, table or helper with the HIP library; both sides only consume the
 * same seeded physical inputs.
 *
 * What it computes (paper sections / equations):
 *   - the momentum form of the Parker transport equation, Eq.(5), written in
 *     the backward Kolmogorov form of Eq.(2) (Sec. III), integrated as the
 *     Ito SDE of Eq.(3) with the Euler-Maruyama scheme (Sec. III);
 *   - the adiabatic term A_P = (2/3)(V/r)P of Eq.(6) with no loss term (L=0);
 *   - the exit-rigidity histogram and the LIS-weighted modulated flux of
 *     Eq.(4) (Sec. III, Sec. IV.A);
 *   - random numbers from the Philox4x32-10 counter-based generator cited in
 *     Sec. IV.A (Salmon et al., SC'11), written from that paper;
 *   - optionally the heliosphere squashed toward its nose with a heliosheath
 *     beyond the termination shock (Sec. II.B), with its shape as a reading.
 * Every coefficient the paper leaves to its external references is a stated
 * reading marked as such; the formulas are the ones spelled out
 * next to each function below.
 *
 * Units inside the oracle: AU, s, GV, GeV.  Inputs arrive in the physical units
 * of the workload description (cm^2/s, km/s, degrees, nT, rad/s, GeV).
 */
#ifndef COSMICA_ORACLE_H
#define COSMICA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_REGIONS 15
#define ORC_NHIST 129 /* 128 log-ratio bins over [0,3) decades + overflow */

typedef struct {
    int32_t model;            /* 0: radial 1D model, 1: full 3D model */
    int32_t n_regions;        /* 1..15 equal-width radial shells */
    double r_boundary_au;     /* absorbing spherical boundary */
    double r0_au, theta0_rad, phi0_rad; /* injection point */
    double kappa0_cm2_s[ORC_MAX_REGIONS];
    double v_slow_km_s[ORC_MAX_REGIONS];
    double tilt_deg[ORC_MAX_REGIONS];
    double v_fast_km_s;       /* wind outside the slow band (3D) */
    double b0_nT;             /* |B| at 1 AU on the ecliptic for v_ref */
    double v_ref_km_s;        /* wind speed that fixes the B normalisation */
    double omega_rad_s;       /* solar rotation rate */
    double kperp_over_kpar;   /* kappa_perp / kappa_par (3D) */
    int32_t polarity;         /* A = +1 or -1 */
    int32_t drift;            /* 1: gradient-curvature drift on */
    int32_t hcs;              /* 1: wavy current sheet (field reversal + sheet drift) */
    int32_t flip_z2;          /* test hook: use -z2 for the theta noise (mirror test) */
    double dt_max_s;
    double dt_diff_frac;      /* dt <= frac * r^2 / kappa */
    double dt_adv_frac;       /* 3D: dt <= frac * r / |A_det|; <= 0 disables */
    double mass_gev;          /* rest mass of the nucleus / particle */
    int32_t charge;           /* Z, signed */
    int32_t pad0;
    double lis_norm, lis_index; /* J_LIS(P) = norm * P^-index */
    uint64_t seed;            /* Philox key */
    uint32_t job_tag;         /* fourth Philox counter word */
    uint32_t step_cap;        /* particles still inside after this many steps are flagged */
    /* Nose-squashed heliosphere with a heliosheath (3D model only; Sec. II.B
     * names the two regions and the squashing but gives no shape, so all of
     * this is a READING).  The heliopause and the termination shock are each a
     * sphere whose centre sits behind the Sun, on the side opposite the nose
     * direction (nose_theta, nose_phi); each is fixed by its distances from the
     * Sun toward the nose and toward the tail.  r_boundary_au above is the
     * heliopause's tail distance. */
    double r_boundary_nose_au; /* heliopause toward the nose; <= 0: r_boundary_au (spherical) */
    double nose_theta_rad, nose_phi_rad;
    int32_t heliosheath;      /* 1: termination shock and heliosheath region */
    int32_t pad1;
    double ts_nose_au, ts_tail_au; /* termination shock distances */
    /* heliosheath region: diffusion coefficient, one wind speed (no fast/slow
     * band), current-sheet tilt */
    double kappa0_hs_cm2_s, v_hs_km_s, tilt_hs_deg;
    /* Moving detection point (Sec. IV.A: the sample of a bin is divided among
     * the positions of a spacecraft orbit).  READING: n_orbit positions sampled
     * at equal time steps along the orbit, orbit[3k..3k+2] = (r [AU], theta,
     * phi); particle i starts at position i mod n_orbit.  n_orbit = 0: every
     * particle starts at (r0_au, theta0_rad, phi0_rad). */
    const double* orbit;
    uint32_t n_orbit;
    /* 0: momentum form, Eq.(5) with L = 0 (Sec. VI, Version 6).  1: energy
     * form, Eq.(1) (the form of Versions 0-3), whose backward SDE carries the
     * loss term of Eq.(2) and the exponential weight of Eq.(4); 3D model only. */
    int32_t formulation;
} orc_params;

enum { ORC_FLAG_CAPPED = 1, ORC_FLAG_NAN = 2 };

typedef struct {
    double P;      /* exit rigidity [GV] */
    double t;      /* backward time to exit [s] */
    double r, theta, phi;
    uint32_t n;    /* number of Euler-Maruyama steps */
    uint32_t flags;
    double loss;   /* energy form: sum of L ds along the path; 0 in the momentum form */
} orc_exit;

/* Local SDE coefficients of the 3D model at one point, for unit-level pins. */
typedef struct {
    int32_t region;
    double V;                 /* local wind speed [AU/s] */
    double kpar, kperp;       /* [AU^2/s] */
    double Krr, Kpp, Krp, Ktt;  /* physical components of the symmetric tensor */
    double dKrr_dr;           /* d/dr K_rr */
    double dKrp_term;         /* (1/r) d/dr (r K_rphi) */
    double Brr, Bpr, Bpp, Btt;  /* B with B B^T = 2K (lower triangular in (r,phi)) */
    double Bmag_nT;           /* |B| */
    double Gamma;             /* Parker spiral: tan of the winding angle */
    double G;                 /* kappa_A / sqrt(1+Gamma^2) [AU^2/s] */
    double Hw;                /* field-polarity factor across the current sheet */
    double sign_qA;           /* sign(Z) * A */
    double vd[3];             /* total drift velocity, physical (r, theta, phi) [AU/s] */
    double A[3];              /* drift of the SDE: dr, dtheta, dphi per unit time */
    double AP;                /* dP/ds [GV/s] */
    double dt;                /* time step [s] */
} orc_coeffs;

/* Philox4x32-10 of (key = seed, counter ctr[4]) -> out[4]. */
void orc_philox4x32_10(uint64_t seed, const uint32_t ctr[4], uint32_t out[4]);

/* Four standard normals from one Philox block (two Box-Muller pairs). */
void orc_normals(uint64_t seed, const uint32_t ctr[4], double z[4]);

/* Loops of the two calls above over counters (c0 + i, c1, c2, c3), i < n:
 * words[4i..4i+3] and z[4i..4i+3] (either may be NULL). */
void orc_rng_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t n,
                   uint32_t* words, double* z);

/* Where a point lies: returns 1 if it is outside the heliopause (the exit
 * test), else 0; *region receives the parameter region used there (0..n-1 the
 * radial shells, n_regions the heliosheath). */
int orc_locate(const orc_params* p, double r, double theta, double phi, int32_t* region);

/* Local 3D coefficients at (P, r, theta, phi). */
void orc_coeffs_3d(const orc_params* p, double P, double r, double theta, double phi,
                   orc_coeffs* out);

/* Propagate particles first..first+count-1 of one rigidity bin to the boundary.
 * out[i] receives particle first+i.  n_threads <= 0 uses OpenMP's default.
 * Returns 0, or -1 on invalid parameters. */
int orc_propagate(const orc_params* p, uint32_t bin_index, double P0_gv,
                  uint32_t first, uint32_t count, orc_exit* out, int n_threads);

/* Propagate one particle, stopping early after max_steps (checkpoint test):
 * state in/out is (r, theta, phi, P, t, n); returns 1 if it exited. */
int orc_advance(const orc_params* p, uint32_t bin_index, uint32_t particle,
                double state[5], uint32_t* n, uint32_t max_steps);

/* Per-bin results of Eq.(4): momentum form with f = J/P^2 (Sec. VI, Version 6);
 * energy form with U = 4 pi p^2 f / v transported and the exponential loss
 * weight, which gives J_mod(P0) = mean(beta0 / beta_ex J_LIS(P_ex) exp(-loss)). */
typedef struct {
    uint32_t hist[ORC_NHIST];
    double flux;        /* J_mod(P0) */
    double flux_se;     /* Monte Carlo standard error of J_mod */
    double mean_exit_time_s;
    uint64_t steps;     /* total EM steps of the bin */
    uint32_t n_capped;
    uint32_t n_nan;
    uint32_t n_used;
} orc_bin_result;

void orc_reduce_bin(const orc_params* p, double P0_gv, const orc_exit* rec, uint32_t n,
                    orc_bin_result* res);

/* J_LIS of the parameters at rigidity P [GV]. */
double orc_lis(const orc_params* p, double P_gv);

/* Re-weighting of stored exit records with other local interstellar spectra
 * (the weight of Eq.(4) with another LIS; the paths do not depend on it).
 * Each of n_lis spectra is tabulated as ln J at n_knots points
 * ln P = lnP0 + k dlnP; between knots ln J is linear in ln P and beyond the
 * ends the end segments are extended (READING: the format of tabulated LIS
 * such as Galprop's, interpolated in log-log).  lnJ[l * n_knots + k];
 * flux[l], flux_se[l] receive the bin's J_mod(P0) and its standard error for
 * spectrum l (momentum or energy form as p->formulation). */
void orc_reweight_bin(const orc_params* p, double P0_gv, const orc_exit* rec, uint32_t n,
                      uint32_t n_lis, uint32_t n_knots, double lnP0, double dlnP,
                      const double* lnJ, double* flux, double* flux_se);

/* Exit histogram over the range the exits reach (Sec. IV.A: the largest exit
 * energy of the sample sets the histogram's binning).  READING: equal-width
 * bins in ln(P_ex / P0) over [0, ln(P_max / P0)], P_max the largest exit
 * rigidity of the bin's used records; the record at P_max falls in the last
 * bin; with P_max = P0 every record falls in bin 0.  Capped and non-finite
 * records are left out.  *p_max receives P_max (0 if no record is used);
 * hist[0..n_hist-1] the counts. */
void orc_exit_range(double P0_gv, const orc_exit* rec, uint32_t n, uint32_t n_hist, double* p_max,
                    uint32_t* hist);

#ifdef __cplusplus
}
#endif
#endif
