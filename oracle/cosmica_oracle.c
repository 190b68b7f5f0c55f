/*
 * cosmica_oracle.c -- plain FP64 CPU oracle (test infrastructure only).
 *
 * A slow, scalar, obviously-correct rendering of the method of COSMICA
 * (arXiv 2502.06319): quasi-particles are integrated backward in time with the
 * Euler-Maruyama scheme (Sec. III, Eq.(3)) through the SDE equivalent to the
 * momentum-form Parker equation (Eq.(5), Eq.(6); L = 0), until they leave the
 * heliosphere; their exit rigidities are then histogrammed and LIS-weighted
 * (Eq.(4), with J = f P^2 from Sec. VI).
 *
 * Nothing here is blocked, fused or reordered for speed: one particle at a
 * time, one step at a time, libm transcendentals, doubles everywhere.  OpenMP
 * only spreads independent particles over host threads.
 *
 * The paper defers every SDE coefficient to an external reference.  The
 * coefficients below are derived from Eq.(5) in heliocentric spherical
 * coordinates (r, theta = colatitude, phi) with a Parker-spiral field; each
 * modelling choice the paper does not fix is marked READING.
 */
#include "cosmica_oracle.h"

#include <math.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double ORC_PI = 3.14159265358979323846;
static const double AU_CM = 1.495978707e13; /* IAU 2012 astronomical unit */
static const double AU_M = 1.495978707e11;
static const double AU_KM = 1.495978707e8;
static const double C_LIGHT_M_S = 299792458.0;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11), the generator named in Sec. IV.A.  Each round   */
/* multiplies counter words 0 and 2 by the two round multipliers, and the    */
/* new words are (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1,        */
/* lo(M0*x0)); the key is bumped by the two Weyl constants between rounds.   */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(uint64_t seed, const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t k0 = (uint32_t)(seed & 0xffffffffu);
    uint32_t k1 = (uint32_t)(seed >> 32);
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)(p1 & 0xffffffffu);
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)(p0 & 0xffffffffu);
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Uniform in (0,1): the top 23 bits of a word, centred in their cell:
 * u = (floor(x / 2^9) + 1/2) * 2^-23.  Every such value is exact in both
 * binary32 and binary64 (READING: the paper only says one random float is
 * drawn per step). */
static double uniform01(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * 0x1p-23;
}

/* Box-Muller on the two uniform pairs (u0,u1), (u2,u3). */
void orc_normals(uint64_t seed, const uint32_t ctr[4], double z[4])
{
    uint32_t x[4];
    orc_philox4x32_10(seed, ctr, x);
    double u0 = uniform01(x[0]), u1 = uniform01(x[1]);
    double u2 = uniform01(x[2]), u3 = uniform01(x[3]);
    double rho0 = sqrt(-2.0 * log(u0));
    double rho2 = sqrt(-2.0 * log(u2));
    z[0] = rho0 * cos(2.0 * ORC_PI * u1);
    z[1] = rho0 * sin(2.0 * ORC_PI * u1);
    z[2] = rho2 * cos(2.0 * ORC_PI * u3);
    z[3] = rho2 * sin(2.0 * ORC_PI * u3);
}

void orc_rng_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t n,
                   uint32_t* words, double* z)
{
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t ctr[4] = {c0 + i, c1, c2, c3};
        if (words) orc_philox4x32_10(seed, ctr, words + 4 * (size_t)i);
        if (z) orc_normals(seed, ctr, z + 4 * (size_t)i);
    }
}

/* ------------------------------------------------------------------------ */
/* Per-job constants in internal units.                                      */
/* ------------------------------------------------------------------------ */
/* Parameter regions: the radial shells 0..nreg-1 and, when the heliosheath
 * is on, the heliosheath as entry nreg. */
#define ORC_REGION_SLOTS (ORC_MAX_REGIONS + 1)

typedef struct {
    int nreg;
    double Rb, shell;
    double Rb_nose;                /* heliopause toward the nose (== Rb: spherical) */
    int hs;                        /* heliosheath on */
    double ts_nose, ts_tail;       /* termination shock */
    double nose[3];                /* unit vector toward the nose */
    double k0[ORC_REGION_SLOTS];    /* kappa0 [AU^2/s] */
    double vs[ORC_REGION_SLOTS];    /* slow wind [AU/s] */
    double vf[ORC_REGION_SLOTS];    /* fast wind [AU/s] */
    double alpha[ORC_REGION_SLOTS]; /* tilt [rad] */
    double tana[ORC_REGION_SLOTS];
    double Br0;                    /* radial field at 1 AU [nT] */
    double absZ, mass;
    double sqA;                    /* sign(Z) * A */
} derived;

static int derive(const orc_params* p, derived* d)
{
    if (p->n_regions < 1 || p->n_regions > ORC_MAX_REGIONS) return -1;
    if (!(p->r_boundary_au > p->r0_au) || !(p->r0_au > 0.0)) return -1;
    if (p->charge == 0 || !(p->mass_gev >= 0.0)) return -1;
    d->nreg = p->n_regions;
    d->Rb = p->r_boundary_au;
    d->Rb_nose = p->r_boundary_nose_au > 0.0 ? p->r_boundary_nose_au : p->r_boundary_au;
    if (!(d->Rb_nose <= d->Rb) || !(d->Rb_nose > p->r0_au)) return -1;
    d->hs = p->heliosheath != 0;
    if (p->model == 0 && (d->hs || d->Rb_nose != d->Rb)) return -1; /* 3D only */
    if (p->formulation != 0 && (p->formulation != 1 || p->model == 0)) return -1;
    d->ts_nose = p->ts_nose_au;
    d->ts_tail = p->ts_tail_au;
    if (d->hs && !(d->ts_nose > p->r0_au && d->ts_nose <= d->ts_tail)) return -1;
    d->nose[0] = sin(p->nose_theta_rad) * cos(p->nose_phi_rad);
    d->nose[1] = sin(p->nose_theta_rad) * sin(p->nose_phi_rad);
    d->nose[2] = cos(p->nose_theta_rad);
    /* READING: the shells split the inner heliosphere radially in equal widths
     * up to the boundary's (with a heliosheath: the termination shock's) nose
     * distance; beyond it the last shell holds up to that surface. */
    d->shell = (d->hs ? d->ts_nose : d->Rb_nose) / (double)p->n_regions;
    for (int k = 0; k < p->n_regions; ++k) {
        d->k0[k] = p->kappa0_cm2_s[k] / (AU_CM * AU_CM);
        d->vs[k] = p->v_slow_km_s[k] / AU_KM;
        d->vf[k] = p->v_fast_km_s / AU_KM;
        d->alpha[k] = p->tilt_deg[k] * ORC_PI / 180.0;
        d->tana[k] = tan(d->alpha[k]);
    }
    if (d->hs) {
        const int k = p->n_regions;
        d->k0[k] = p->kappa0_hs_cm2_s / (AU_CM * AU_CM);
        d->vs[k] = p->v_hs_km_s / AU_KM;
        d->vf[k] = p->v_hs_km_s / AU_KM;
        d->alpha[k] = p->tilt_hs_deg * ORC_PI / 180.0;
        d->tana[k] = tan(d->alpha[k]);
    }
    /* READING: b0 is |B| at 1 AU on the ecliptic for a wind of v_ref, so the
     * radial component there is b0 / sqrt(1 + (Omega * 1 AU / v_ref)^2). */
    double gE = (p->v_ref_km_s > 0.0) ? p->omega_rad_s * AU_KM / p->v_ref_km_s : 0.0;
    d->Br0 = p->b0_nT / sqrt(1.0 + gE * gE);
    d->absZ = fabs((double)p->charge);
    d->mass = p->mass_gev;
    d->sqA = (double)((p->charge > 0) ? 1 : -1) * (double)p->polarity;
    return 0;
}

static int shell_of(const derived* d, double r)
{
    int k = (int)floor(r / d->shell);
    if (k > d->nreg - 1) k = d->nreg - 1;
    if (k < 0) k = 0;
    return k;
}

/* READING: a heliospheric surface with distances Rn toward the nose and Rt
 * toward the tail is the sphere of radius (Rn + Rt)/2 centred (Rt - Rn)/2
 * behind the Sun, against the nose direction; with Rn == Rt it is the sphere
 * of radius Rt about the Sun.  A point is outside when its distance from the
 * centre is at least the radius. */
static int outside_surface(const derived* d, double Rn, double Rt, double r, double th,
                           double ph)
{
    if (Rn == Rt) return r >= Rt;
    double a = 0.5 * (Rn + Rt);
    double delta = 0.5 * (Rt - Rn);
    double x = r * sin(th) * cos(ph) + delta * d->nose[0];
    double y = r * sin(th) * sin(ph) + delta * d->nose[1];
    double z = r * cos(th) + delta * d->nose[2];
    return x * x + y * y + z * z >= a * a;
}

/* Parameter region at a point: the heliosheath beyond the termination shock,
 * else the radial shell. */
static int region_of(const derived* d, double r, double th, double ph)
{
    if (d->hs && outside_surface(d, d->ts_nose, d->ts_tail, r, th, ph)) return d->nreg;
    return shell_of(d, r);
}

static int outside_heliopause(const derived* d, double r, double th, double ph)
{
    return outside_surface(d, d->Rb_nose, d->Rb, r, th, ph);
}

/* Particle speed over c for rigidity P: pc = |Z| P, E = sqrt((pc)^2 + M^2). */
static double beta_of(const derived* d, double P)
{
    double pc = d->absZ * P;
    return pc / sqrt(pc * pc + d->mass * d->mass);
}

/* ------------------------------------------------------------------------ */
/* 3D coefficients.  K is given in the local orthonormal frame (e_r, e_theta, */
/* e_phi); the field direction is b = (e_r - Gamma e_phi) / sqrt(1+Gamma^2)   */
/* with Gamma = Omega r sin(theta) / V (Parker spiral, V locally constant).  */
/* The Ito drift of the backward SDE is A^i = (1/sqrt g) d_j(sqrt g K^ij)    */
/* - V^i - v_d^i in coordinates (r, theta, phi), sqrt g = r^2 sin(theta),     */
/* and B B^T = 2K; dP = (1/3)(div V) P ds = (2V/3r) P ds (Eq.(6)).            */
/* ------------------------------------------------------------------------ */
static void coeffs3d(const orc_params* p, const derived* d, double P, double r,
                     double th, double ph, orc_coeffs* c)
{
    int k = region_of(d, r, th, ph);
    double st = sin(th), ct = cos(th);
    double cot = ct / st;
    /* READING: slow wind inside the band |latitude| <= tilt of the region,
     * fast wind outside it (the heliosheath has one speed for both). */
    double lam = 0.5 * ORC_PI - th;
    double V = (fabs(lam) <= d->alpha[k]) ? d->vs[k] : d->vf[k];
    double beta = beta_of(d, P);
    double kpar = d->k0[k] * beta * P;
    double kperp = p->kperp_over_kpar * kpar;
    double dk = kpar - kperp;

    /* Parker-spiral geometry, written so that V = 0 (no spiral, drift off)
     * stays finite: g = 1/(1+Gamma^2), Gg = Gamma g, GGg = Gamma^2 g. */
    double w = p->omega_rad_s * r * st;
    double D = V * V + w * w;
    double g = V * V / D;
    double Gg = V * w / D;
    double GGg = w * w / D;

    c->region = k;
    c->V = V;
    c->kpar = kpar;
    c->kperp = kperp;
    c->Krr = kperp + dk * g;
    c->Kpp = kpar - dk * g;
    c->Krp = -dk * Gg;
    c->Ktt = kperp;
    /* kappa is constant inside a shell (READING: shell jumps are not
     * differentiated); Gamma is proportional to r, so
     * d/dr g = -2 Gamma^2 g^2 / r and (1/r) d/dr (r Gamma g) = 2 Gamma g^2 / r. */
    c->dKrr_dr = -2.0 * dk * GGg * g / r;
    c->dKrp_term = -2.0 * dk * Gg * g / r;
    /* Closed-form Cholesky factor of 2K in the (r, phi) block; the block has
     * determinant kpar * kperp. */
    c->Brr = sqrt(2.0 * c->Krr);
    c->Bpr = 2.0 * c->Krp / c->Brr;
    c->Bpp = sqrt(2.0 * kpar * kperp / c->Krr);
    c->Btt = sqrt(2.0 * c->Ktt);

    c->Gamma = 0.0;
    c->G = 0.0;
    c->Hw = 1.0;
    c->sign_qA = d->sqA;
    c->Bmag_nT = 0.0;
    c->vd[0] = c->vd[1] = c->vd[2] = 0.0;
    if (V > 0.0) {
        double Gam = w / V;
        double opg = 1.0 + Gam * Gam;
        c->Gamma = Gam;
        c->Bmag_nT = d->Br0 / (r * r) * sqrt(opg);
    }
    if (p->drift && V > 0.0) {
        double Gam = c->Gamma;
        double opg = 1.0 + Gam * Gam;
        double gg = 1.0 / opg;
        double Bmag = c->Bmag_nT;
        /* Weak-scattering drift coefficient kappa_A = beta P / (3 |B|), from
         * P in GV and B in nT to AU^2/s (READING: no drift reduction). */
        double kA = beta * P * 1e18 / (3.0 * Bmag) / (AU_M * AU_M);
        double G = kA / sqrt(opg);
        c->G = G;
        double Hw = 1.0;
        double vcs_r = 0.0, vcs_t = 0.0, vcs_p = 0.0;
        if (p->hcs) {
            /* READING: static wavy current sheet
             * theta_cs = pi/2 - atan(tan(alpha) sin(phi + Omega r / Vs)), the
             * field reverses across it with the smooth profile
             * Hw = tanh((theta_cs - theta) / Delta), Delta = 2 r_L / r. */
            double vsk = d->vs[k];
            double tana = d->tana[k];
            double chi = ph + p->omega_rad_s * r / vsk;
            double sc = sin(chi), cc = cos(chi);
            double th_cs = 0.5 * ORC_PI - atan(tana * sc);
            double u = th_cs - th;
            double rL = P * 1e9 / (C_LIGHT_M_S * Bmag * 1e-9) / AU_M; /* Larmor radius [AU] */
            double Delta = 2.0 * rL / r;
            Hw = tanh(u / Delta);
            double Hp = 1.0 - Hw * Hw;
            double cs = -tana * cc / (1.0 + tana * tana * sc * sc); /* d theta_cs / d chi */
            double gr = cs * p->omega_rad_s / vsk;                    /* d theta_cs / dr */
            double gph = cs / (r * st);                               /* (1/(r sin)) d theta_cs / dphi */
            /* grad Hw = (Hp/Delta) (grad u - u grad ln Delta), with
             * grad ln Delta = (g/r, -Gamma^2 cot(theta) g / r, 0); the sheet
             * drift is grad Hw x W with W = G (1, 0, -Gamma). */
            double f = Hp / Delta * G;
            vcs_r = f * (Gam / r - u * Gam * Gam * Gam * cot * gg / r);
            vcs_t = f * (gph + gr * Gam - u * Gam * gg / r);
            vcs_p = f * (1.0 / r - u * Gam * Gam * cot * gg / r);
        }
        c->Hw = Hw;
        /* Gradient-curvature drift Hw * curl(W), W = G (1, 0, -Gamma). */
        double vgc_r = Hw * (-2.0 * G * (p->omega_rad_s / V) * ct * gg);
        double vgc_t = Hw * (2.0 * G * Gam * (2.0 + Gam * Gam) * gg / r);
        double vgc_p = Hw * (2.0 * G * Gam * Gam * cot * gg / r);
        c->vd[0] = d->sqA * (vgc_r + vcs_r);
        c->vd[1] = d->sqA * (vgc_t + vcs_t);
        c->vd[2] = d->sqA * (vgc_p + vcs_p);
    }

    c->A[0] = 2.0 * c->Krr / r + c->dKrr_dr - V - c->vd[0];
    c->A[1] = c->Ktt * cot / (r * r) - c->vd[1] / r;
    c->A[2] = (c->dKrp_term - c->vd[2]) / (r * st);
    c->AP = 2.0 * V * P / (3.0 * r);

    /* READING: time step min(dt_max, f_diff r^2/kpar, f_adv r/|A_det|) --
     * the advective limit follows the Kruells-type condition of Sec. IV.A. */
    double dt = p->dt_max_s;
    double d1 = p->dt_diff_frac * r * r / kpar;
    if (d1 < dt) dt = d1;
    if (p->dt_adv_frac > 0.0) {
        double a_r = c->A[0], a_t = r * c->A[1], a_p = r * st * c->A[2];
        double a2 = a_r * a_r + a_t * a_t + a_p * a_p;
        if (a2 > 0.0) {
            double d2 = p->dt_adv_frac * r / sqrt(a2);
            if (d2 < dt) dt = d2;
        }
    }
    c->dt = dt;
}

int orc_locate(const orc_params* p, double r, double theta, double phi, int32_t* region)
{
    derived d;
    *region = -1;
    if (derive(p, &d) != 0) return -1;
    if (p->model == 0) {
        *region = shell_of(&d, r);
        return r >= d.Rb;
    }
    *region = region_of(&d, r, theta, phi);
    return outside_heliopause(&d, r, theta, phi);
}

void orc_coeffs_3d(const orc_params* p, double P, double r, double theta, double phi,
                   orc_coeffs* out)
{
    derived d;
    memset(out, 0, sizeof(*out));
    if (derive(p, &d) != 0) return;
    coeffs3d(p, &d, P, r, theta, phi, out);
}

/* ------------------------------------------------------------------------ */
/* One Euler-Maruyama step (Sec. III).  The Philox counter of step n of       */
/* particle i of bin b is (n, i, b, job_tag).                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    double r, th, ph, P, t;
    uint32_t n;
    double T, lam; /* energy form: kinetic energy [GeV] and the loss integral */
} pstate;

static void step1d(const orc_params* p, const derived* d, uint32_t bin, uint32_t particle,
                   pstate* s)
{
    uint32_t ctr[4] = {s->n, particle, bin, p->job_tag};
    double z[4];
    orc_normals(p->seed, ctr, z);
    int k = shell_of(d, s->r);
    double beta = beta_of(d, s->P);
    double kap = d->k0[k] * beta * s->P;
    double V = d->vs[k];
    /* dr = (2 kappa / r - V) ds + sqrt(2 kappa) dW  (radial part of Eq.(3)) */
    double Ar = 2.0 * kap / s->r - V;
    double Brr = sqrt(2.0 * kap);
    double AP = 2.0 * V * s->P / (3.0 * s->r);
    double dt = p->dt_max_s;
    double d1 = p->dt_diff_frac * s->r * s->r / kap;
    if (d1 < dt) dt = d1;
    double sdt = sqrt(dt);
    double r1 = s->r + Ar * dt + Brr * z[0] * sdt;
    double P1 = s->P + AP * dt;
    if (r1 < 0.0) r1 = -r1; /* READING: reflection at the origin */
    s->r = r1;
    s->P = P1;
    s->t = s->t + dt;
    s->n = s->n + 1;
}

static void step3d(const orc_params* p, const derived* d, uint32_t bin, uint32_t particle,
                   pstate* s)
{
    uint32_t ctr[4] = {s->n, particle, bin, p->job_tag};
    double z[4];
    orc_normals(p->seed, ctr, z);
    double z2 = p->flip_z2 ? -z[2] : z[2];
    orc_coeffs c;
    coeffs3d(p, d, s->P, s->r, s->th, s->ph, &c);
    double dt = c.dt;
    double sdt = sqrt(dt);
    double st = sin(s->th);
    double r1 = s->r + c.A[0] * dt + c.Brr * z[0] * sdt;
    double th1 = s->th + c.A[1] * dt + c.Btt * z2 * sdt / s->r;
    double ph1 = s->ph + c.A[2] * dt + (c.Bpr * z[0] + c.Bpp * z[1]) * sdt / (s->r * st);
    double P1 = s->P + c.AP * dt;
    /* READING: reflections keep (r, theta, phi) a valid spherical triple. */
    if (r1 < 0.0) {
        r1 = -r1;
        th1 = ORC_PI - th1;
        ph1 = ph1 + ORC_PI;
    }
    if (th1 < 0.0) {
        th1 = -th1;
        ph1 = ph1 + ORC_PI;
    }
    th1 = fmod(th1, 2.0 * ORC_PI);
    if (th1 > ORC_PI) {
        th1 = 2.0 * ORC_PI - th1;
        ph1 = ph1 + ORC_PI;
    }
    ph1 = fmod(ph1, 2.0 * ORC_PI);
    if (ph1 < 0.0) ph1 += 2.0 * ORC_PI;
    s->r = r1;
    s->th = th1;
    s->ph = ph1;
    s->P = P1;
    s->t = s->t + dt;
    s->n = s->n + 1;
}

/* ------------------------------------------------------------------------ */
/* Energy form, Eq.(1).  Written for the backward Kolmogorov form of Eq.(2),  */
/* the spatial terms are those of the momentum form (diffusion, convection,   */
/* drift); the energy term (1/3)(div V) d(alpha T U)/dT splits into the       */
/* advection (1/3)(div V) alpha T dU/dT and a term proportional to U, which   */
/* with the -(div V) U of the convective divergence is the loss               */
/*   L = (div V) [1 - (1/3) d(alpha T)/dT],  d(alpha T)/dT = 1 + (M/(T+M))^2, */
/* alpha = (T + 2M)/(T + M), T the kinetic energy of the particle and M its   */
/* rest energy (per nucleon both, or both per particle: alpha is a ratio).    */
/* So dT = (1/3)(div V) alpha T ds, and each step adds L ds to the exponent   */
/* of Eq.(4).  div V = 2V/r for the radial wind.                              */
/* ------------------------------------------------------------------------ */
static double rigidity_of_T(const derived* d, double T)
{
    return sqrt(T * (T + 2.0 * d->mass)) / d->absZ;
}

static void step3d_energy(const orc_params* p, const derived* d, uint32_t bin,
                          uint32_t particle, pstate* s)
{
    uint32_t ctr[4] = {s->n, particle, bin, p->job_tag};
    double z[4];
    orc_normals(p->seed, ctr, z);
    double z2 = p->flip_z2 ? -z[2] : z[2];
    double P = rigidity_of_T(d, s->T);
    orc_coeffs c;
    coeffs3d(p, d, P, s->r, s->th, s->ph, &c);
    double dt = c.dt;
    double sdt = sqrt(dt);
    double st = sin(s->th);
    double M = d->mass;
    double divV = 2.0 * c.V / s->r;
    double alpha = (s->T + 2.0 * M) / (s->T + M);
    double dalphaT = 1.0 + (M / (s->T + M)) * (M / (s->T + M));
    double AT = divV / 3.0 * alpha * s->T;
    double L = divV * (1.0 - dalphaT / 3.0);
    double r1 = s->r + c.A[0] * dt + c.Brr * z[0] * sdt;
    double th1 = s->th + c.A[1] * dt + c.Btt * z2 * sdt / s->r;
    double ph1 = s->ph + c.A[2] * dt + (c.Bpr * z[0] + c.Bpp * z[1]) * sdt / (s->r * st);
    double T1 = s->T + AT * dt;
    if (r1 < 0.0) {
        r1 = -r1;
        th1 = ORC_PI - th1;
        ph1 = ph1 + ORC_PI;
    }
    if (th1 < 0.0) {
        th1 = -th1;
        ph1 = ph1 + ORC_PI;
    }
    th1 = fmod(th1, 2.0 * ORC_PI);
    if (th1 > ORC_PI) {
        th1 = 2.0 * ORC_PI - th1;
        ph1 = ph1 + ORC_PI;
    }
    ph1 = fmod(ph1, 2.0 * ORC_PI);
    if (ph1 < 0.0) ph1 += 2.0 * ORC_PI;
    s->r = r1;
    s->th = th1;
    s->ph = ph1;
    s->T = T1;
    s->P = rigidity_of_T(d, T1);
    s->lam = s->lam + L * dt;
    s->t = s->t + dt;
    s->n = s->n + 1;
}

/* Runs steps until exit (r >= R_b), NaN, the step cap, or max_steps more steps.
 * Returns 1 exited, 0 still inside, 2 capped, 3 NaN. */
static int run(const orc_params* p, const derived* d, uint32_t bin, uint32_t particle,
               pstate* s, uint64_t max_steps)
{
    for (uint64_t i = 0; i < max_steps; ++i) {
        if (s->n >= p->step_cap) return 2;
        if (p->model == 0)
            step1d(p, d, bin, particle, s);
        else if (p->formulation == 1)
            step3d_energy(p, d, bin, particle, s);
        else
            step3d(p, d, bin, particle, s);
        if (isnan(s->r) || isnan(s->P)) return 3;
        /* READING: exit at the first step that ends outside; no crossing
         * interpolation */
        if (p->model == 0 ? s->r >= d->Rb : outside_heliopause(d, s->r, s->th, s->ph)) return 1;
    }
    return 0;
}

int orc_propagate(const orc_params* p, uint32_t bin_index, double P0_gv, uint32_t first,
                  uint32_t count, orc_exit* out, int n_threads)
{
    derived d;
    if (derive(p, &d) != 0 || !(P0_gv > 0.0)) return -1;
    /* every orbit position lies inside the heliopause */
    for (uint32_t k = 0; k < p->n_orbit; ++k) {
        const double* q = p->orbit + 3 * (size_t)k;
        int32_t reg;
        if (!(q[0] > 0.0) || !(q[1] > 0.0) || !(q[1] < ORC_PI)) return -1;
        if (orc_locate(p, q[0], q[1], q[2], &reg) != 0) return -1;
    }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < (int64_t)count; ++i) {
        uint32_t particle = first + (uint32_t)i;
        pstate s = {p->r0_au, p->theta0_rad, p->phi0_rad, P0_gv, 0.0, 0u, 0.0, 0.0};
        /* kinetic energy from rigidity: E^2 = (Z P)^2 + M^2 */
        s.T = sqrt(d.absZ * P0_gv * d.absZ * P0_gv + d.mass * d.mass) - d.mass;
        if (p->n_orbit > 0) {
            const double* q = p->orbit + 3 * (size_t)(particle % p->n_orbit);
            s.r = q[0];
            s.th = q[1];
            s.ph = q[2];
        }
        int rc = run(p, &d, bin_index, particle, &s, UINT64_MAX);
        orc_exit* e = &out[i];
        e->P = s.P;
        e->t = s.t;
        e->r = s.r;
        e->theta = s.th;
        e->phi = s.ph;
        e->n = s.n;
        e->flags = (rc == 2) ? ORC_FLAG_CAPPED : (rc == 3) ? ORC_FLAG_NAN : 0u;
        e->loss = s.lam;
    }
    return 0;
}

int orc_advance(const orc_params* p, uint32_t bin_index, uint32_t particle, double state[5],
                uint32_t* n, uint32_t max_steps)
{
    derived d;
    if (derive(p, &d) != 0 || p->formulation != 0) return -1; /* momentum form only */
    pstate s = {state[0], state[1], state[2], state[3], state[4], *n, 0.0, 0.0};
    int rc = run(p, &d, bin_index, particle, &s, max_steps);
    state[0] = s.r;
    state[1] = s.th;
    state[2] = s.ph;
    state[3] = s.P;
    state[4] = s.t;
    *n = s.n;
    return rc == 1 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Eq.(4) in the momentum form: L = 0, f = J / P^2 is the transported         */
/* quantity, so each quasi-particle carries w = J_LIS(P_ex) / P_ex^2 and      */
/* J_mod(P0) = P0^2 * mean(w) (READING: "proportional to" read as the sample  */
/* mean over the N particles of the bin).                                     */
/* ------------------------------------------------------------------------ */
double orc_lis(const orc_params* p, double P_gv)
{
    return p->lis_norm * pow(P_gv, -p->lis_index);
}

/* Contribution of one exit record to J_mod(P0): momentum form
 * P0^2 J_LIS(P_ex) / P_ex^2 (f conserved); energy form, where U = 4 pi p^2 f / v
 * is transported with the loss weight, beta0 / beta_ex J_LIS(P_ex) exp(-loss). */
static double contribution(const orc_params* p, const derived* d, double P0, const orc_exit* e)
{
    if (p->formulation == 1)
        return beta_of(d, P0) / beta_of(d, e->P) * orc_lis(p, e->P) * exp(-e->loss);
    return P0 * P0 * (orc_lis(p, e->P) / (e->P * e->P));
}

void orc_reduce_bin(const orc_params* p, double P0_gv, const orc_exit* rec, uint32_t n,
                    orc_bin_result* res)
{
    memset(res, 0, sizeof(*res));
    derived d;
    if (derive(p, &d) != 0) return;
    double sw = 0.0, st = 0.0;
    uint32_t used = 0;
    for (uint32_t i = 0; i < n; ++i) {
        res->steps += rec[i].n;
        if (rec[i].flags & ORC_FLAG_CAPPED) {
            res->n_capped++;
            continue;
        }
        if (rec[i].flags & ORC_FLAG_NAN) {
            res->n_nan++;
            continue;
        }
        double P = rec[i].P;
        sw += contribution(p, &d, P0_gv, &rec[i]);
        st += rec[i].t;
        used++;
        /* histogram of log10(P_ex / P0) over [0, 3) in 128 bins + overflow */
        double x = 128.0 * log10(P / P0_gv) / 3.0;
        int j = (int)floor(x);
        if (j < 0) j = 0;
        if (j > 128) j = 128;
        res->hist[j]++;
    }
    res->n_used = used;
    if (used > 0) {
        double N = (double)used;
        res->flux = sw / N;
        res->mean_exit_time_s = st / N;
        if (used > 1) {
            /* standard error of the mean contribution: two-pass sample variance */
            double mean = sw / N, ss = 0.0;
            for (uint32_t i = 0; i < n; ++i) {
                if (rec[i].flags & (ORC_FLAG_CAPPED | ORC_FLAG_NAN)) continue;
                double dw = contribution(p, &d, P0_gv, &rec[i]) - mean;
                ss += dw * dw;
            }
            res->flux_se = sqrt(ss / (N - 1.0) / N);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Re-weighting with tabulated spectra: ln J linear in ln P between knots,   */
/* end segments extended.                                                     */
/* ------------------------------------------------------------------------ */
static double table_lis(uint32_t n_knots, double lnP0, double dlnP, const double* lnJ,
                        double P)
{
    double x = (log(P) - lnP0) / dlnP;
    int k = (int)floor(x);
    if (k < 0) k = 0;
    if (k > (int)n_knots - 2) k = (int)n_knots - 2;
    double f = x - (double)k;
    return exp(lnJ[k] + f * (lnJ[k + 1] - lnJ[k]));
}

void orc_reweight_bin(const orc_params* p, double P0_gv, const orc_exit* rec, uint32_t n,
                      uint32_t n_lis, uint32_t n_knots, double lnP0, double dlnP,
                      const double* lnJ, double* flux, double* flux_se)
{
    derived d;
    if (derive(p, &d) != 0 || n_knots < 2) return;
    const double b0 = beta_of(&d, P0_gv);
    for (uint32_t l = 0; l < n_lis; ++l) {
        const double* t = lnJ + (size_t)l * n_knots;
        double sw = 0.0;
        uint32_t used = 0;
        for (uint32_t i = 0; i < n; ++i) {
            if (rec[i].flags & (ORC_FLAG_CAPPED | ORC_FLAG_NAN)) continue;
            double P = rec[i].P, J = table_lis(n_knots, lnP0, dlnP, t, P);
            sw += p->formulation == 1 ? b0 / beta_of(&d, P) * J * exp(-rec[i].loss)
                                      : P0_gv * P0_gv * (J / (P * P));
            used++;
        }
        flux[l] = used ? sw / (double)used : 0.0;
        flux_se[l] = 0.0;
        if (used > 1) {
            double mean = sw / (double)used, ss = 0.0;
            for (uint32_t i = 0; i < n; ++i) {
                if (rec[i].flags & (ORC_FLAG_CAPPED | ORC_FLAG_NAN)) continue;
                double P = rec[i].P, J = table_lis(n_knots, lnP0, dlnP, t, P);
                double w = p->formulation == 1 ? b0 / beta_of(&d, P) * J * exp(-rec[i].loss)
                                               : P0_gv * P0_gv * (J / (P * P));
                ss += (w - mean) * (w - mean);
            }
            flux_se[l] = sqrt(ss / ((double)used - 1.0) / (double)used);
        }
    }
}

/* The largest exit rigidity, then the counts of ln(P / P0) in n_hist equal
 * bins up to it (the bin index is floor(n_hist x / x_max), x = ln(P / P0),
 * clamped to the last bin). */
void orc_exit_range(double P0_gv, const orc_exit* rec, uint32_t n, uint32_t n_hist, double* p_max,
                    uint32_t* hist)
{
    double pm = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        if (rec[i].flags & (ORC_FLAG_CAPPED | ORC_FLAG_NAN)) continue;
        if (rec[i].P > pm) pm = rec[i].P;
    }
    *p_max = pm;
    for (uint32_t k = 0; k < n_hist; ++k) hist[k] = 0;
    if (n_hist == 0 || pm == 0.0) return;
    const double xmax = log(pm / P0_gv);
    for (uint32_t i = 0; i < n; ++i) {
        if (rec[i].flags & (ORC_FLAG_CAPPED | ORC_FLAG_NAN)) continue;
        uint32_t k = 0;
        if (xmax > 0.0) {
            const double x = log(rec[i].P / P0_gv);
            const double f = floor((double)n_hist * x / xmax);
            k = f <= 0.0 ? 0u : (f >= (double)n_hist ? n_hist - 1 : (uint32_t)f);
        }
        hist[k] += 1;
    }
}
