/*
 * cosmica.h -- C ABI of the MI355X (gfx950) quasi-particle SDE engine.
 *
 * The library integrates independent cosmic-ray quasi-particles backward in
 * time through the stochastic differential equations equivalent to the
 * momentum-form Parker transport equation (arXiv 2502.06319: Eq.(5), its
 * backward Kolmogorov form Eq.(2) and SDE form Eq.(3), Sec. III), one
 * Euler-Maruyama step at a time, until each leaves the heliosphere; exit
 * rigidities are histogrammed and weighted by the local interstellar spectrum
 * into modulated spectra (Eq.(4) with J = f P^2 and L = 0, Sec. VI "Version 6").
 *
 * Every function returns a cosmica_status (0 = success, negative = error) unless
 * stated otherwise.  All structs are plain C, little-endian, with explicit
 * padding; cosmica_abi_version() identifies the layout.
 *
 * Ownership: the caller owns every input and output buffer.  The library copies
 * inputs before returning from cosmica_run / cosmica_plan_create /
 * cosmica_submit.  Only opaque handles (cosmica_ctx, cosmica_plan) are
 * allocated by the library, and each has a matching destroy call.
 * Errors: COSMICA_EINVAL is returned before anything is written to outputs;
 * after COSMICA_EDEVICE outputs are undefined.  A context is not thread-safe
 * except for cosmica_poll / cosmica_cancel / cosmica_wait /
 * cosmica_request_state, which may be called from any thread while the serving
 * worker runs.
 */
#ifndef COSMICA_H
#define COSMICA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COSMICA_ABI_VERSION 5
#define COSMICA_MAX_REGIONS 15 /* radial shells of the inner heliosphere (Sec. II.B) */
#define COSMICA_REGION_HELIOSHEATH 15 /* region index of the heliosheath */
#define COSMICA_NHIST 129      /* 128 bins of log10(P_ex/P0) over [0,3) + overflow */
#define COSMICA_MAX_STEP_CAP 16777215u
#define COSMICA_MAX_ORBIT 1024 /* positions of a moving detection point */
#define COSMICA_MAX_JOBS 1048576 /* jobs in one plan or cosmica_run call */

typedef enum {
    COSMICA_OK = 0,
    COSMICA_EINVAL = -1,    /* invalid argument; nothing written */
    COSMICA_ENOMEM = -2,    /* device memory exhausted or over the HBM budget */
    COSMICA_EDEVICE = -3,   /* HIP runtime / kernel failure */
    COSMICA_EBUSY = -4,     /* serving queue full */
    COSMICA_ECANCELED = -5, /* the request was cancelled */
    COSMICA_ESTEPCAP = -6,  /* warning: results written, some particles hit the step cap */
    COSMICA_ENOTFOUND = -7, /* unknown ticket */
    COSMICA_ESCRATCH = -8   /* cosmica_run_static: the work does not fit its static array */
} cosmica_status;

typedef enum { COSMICA_MODEL_1D = 0, COSMICA_MODEL_3D = 1 } cosmica_model;
typedef enum { COSMICA_PREC_FP64 = 0, COSMICA_PREC_MIXED = 1 } cosmica_precision;

/* Heliosphere parameters in physical units.
 * model 1D: radial SDE dr = (2k/r - V) ds + sqrt(2k) dW, dP = (2V/3r) P ds with
 *   k = kappa0 beta P / 1 GV of the shell containing r and V its v_slow.
 * model 3D: spherical (r, theta colatitude, phi); Parker-spiral field with
 *   |B| = b0 at 1 AU on the ecliptic for a wind of v_ref; diffusion tensor with
 *   k_par = kappa0 beta P / 1 GV along the field and kperp_over_kpar * k_par across
 *   it; wind v_slow inside |latitude| <= tilt, v_fast outside; gradient-curvature
 *   drift (drift=1) and a wavy current sheet of the shell's tilt (hcs=1).
 * The inner heliosphere is split into n_regions equal-width shells out to
 * r_boundary_au (Sec. II.B); each shell has its own kappa0, v_slow and tilt.
 * 3D only: the heliosphere can be squashed toward its nose and carry a
 * heliosheath (Sec. II.B names both regions and the squashing; the shape is
 * this library's reading).  The heliopause and the termination shock are each
 * a sphere whose centre sits behind the Sun, against the nose direction
 * (nose_theta_rad, nose_phi_rad), fixed by its distances from the Sun toward the
 * nose and toward the tail; r_boundary_au is then the heliopause's tail
 * distance.  A point is outside a surface with distances Rn, Rt when
 * r^2 + (Rt - Rn) r cos(psi) >= Rn Rt, psi its angle from the nose.  With a
 * heliosheath the shells span the inner heliosphere up to the shock's nose
 * distance, and beyond the shock the heliosheath's own kappa0, wind (one speed,
 * no fast/slow band) and current-sheet tilt apply.  The shock is a parameter
 * discontinuity like the shell edges, not a source of acceleration.  With
 * r_boundary_nose_au = 0 and heliosheath = 0 the heliosphere is the sphere of
 * radius r_boundary_au. */
typedef struct {
    int32_t model;           /* cosmica_model */
    int32_t n_regions;       /* 1..15 */
    double kappa0_cm2_s[COSMICA_MAX_REGIONS]; /* > 0 */
    double v_slow_km_s[COSMICA_MAX_REGIONS];  /* >= 0 (> 0 when drift or hcs) */
    double tilt_deg[COSMICA_MAX_REGIONS];     /* [0, 90) */
    double v_fast_km_s;      /* >= 0 (> 0 for 3D with drift) */
    double r_boundary_au;    /* absorbing boundary, > r0 */
    double r0_au, theta0_rad, phi0_rad; /* injection point; theta0 in (0, pi) for 3D */
    double b0_nT;            /* > 0 when drift */
    double v_ref_km_s;       /* > 0 when drift */
    double omega_rad_s;      /* solar rotation, >= 0 (> 0 if any 3D wind speed is 0) */
    double kperp_over_kpar;  /* (0, 1] */
    int32_t polarity;        /* +1 or -1 */
    int32_t drift;           /* 0 or 1 */
    int32_t hcs;             /* 0 or 1 (requires drift) */
    int32_t reserved0;
    double dt_max_s;         /* > 0 */
    double dt_diff_frac;     /* > 0: dt <= frac r^2 / k_par */
    double dt_adv_frac;      /* >= 0: 3D, dt <= frac r / |A|; 0 disables */
    double r_boundary_nose_au; /* 0 (spherical), or heliopause toward the nose in (r0, r_boundary_au] */
    double nose_theta_rad, nose_phi_rad; /* nose direction (colatitude, longitude) */
    int32_t heliosheath;     /* 0 or 1 (3D only) */
    int32_t reserved1;
    double ts_nose_au, ts_tail_au; /* termination shock: r0 < ts_nose <= ts_tail */
    double kappa0_hs_cm2_s;  /* heliosheath kappa0, > 0 */
    double v_hs_km_s;        /* heliosheath wind, >= 0 (> 0 when drift) */
    double tilt_hs_deg;      /* heliosheath current-sheet tilt, [0, 90) */
} cosmica_helio;

/* Particle species: rigidity P = pc/(|Z| e) [GV] (Sec. VI); LIS J(P) = lis_norm P^-lis_index. */
typedef struct {
    double mass_gev;         /* rest mass, >= 0 */
    int32_t charge;          /* Z, signed, != 0 */
    int32_t mass_number;     /* informational */
    double lis_norm;         /* > 0 */
    double lis_index;
} cosmica_species;

/* One spectrum request: a (heliosphere, species) pair at n_bins initial rigidities.
 * Random numbers of step n of particle i of bin b come from Philox4x32-10 with
 * key = seed and counter (n, i, bin_offset + b, job_tag), so results do not depend
 * on batching, scheduling or device. */
typedef struct {
    const cosmica_helio* helio;
    const cosmica_species* species;
    const double* rigidity_gv;          /* n_bins initial rigidities, > 0 */
    const uint32_t* particles_per_bin;  /* n_bins counts, >= 1 */
    int32_t n_bins;                     /* >= 1 */
    uint32_t job_tag;
    uint64_t seed;
    uint32_t step_cap;                  /* 1..COSMICA_MAX_STEP_CAP; 0 selects 10^7 */
    uint32_t bin_offset;                /* bin b draws the streams of bin bin_offset + b, so
                                           the bins of one spectrum can be split over jobs
                                           (or devices) with identical results */
    /* Moving detection point (Sec. IV.A: the sample is divided among the
     * positions of a spacecraft orbit, so the flux integrates over the
     * mission): n_orbit positions at equal time steps, orbit[3k..3k+2] =
     * (r [AU], theta, phi); particle i of every bin starts at position
     * i mod n_orbit, and each bin's flux is the mean over all its particles.
     * Positions lie inside the heliopause, theta in (0, pi); n_orbit <=
     * COSMICA_MAX_ORBIT.  n_orbit = 0 (orbit may be NULL): every particle
     * starts at the heliosphere's (r0_au, theta0_rad, phi0_rad).  The library
     * copies the positions. */
    const double* orbit;
    uint32_t n_orbit;
    /* 0: momentum form of the transport equation, Eq.(5) (Sec. VI, Version
     * 6; L = 0).  1: energy form, Eq.(1) (Versions 0-3), 3D only: the state
     * carries the kinetic energy T with dT = (1/3)(div V) alpha T ds,
     * alpha = (T + 2M)/(T + M), and the loss L = (div V)[1 - (1/3)
     * d(alpha T)/dT] summed into the exponential weight of Eq.(4); the bin's
     * flux is the mean of beta0/beta_ex J_LIS(P_ex) exp(-loss). */
    int32_t formulation;
} cosmica_job;

/* Per-particle exit record (optional output, for checks). */
typedef struct {
    double P;       /* exit rigidity [GV] */
    double t;       /* backward time to exit [s] */
    double r, theta, phi;
    uint32_t n;     /* Euler-Maruyama steps */
    uint32_t flags; /* 1 = hit the step cap, 2 = non-finite state */
    double loss;    /* energy form: the summed L ds of Eq.(4); 0 in the momentum form */
} cosmica_exit;

/* Host output buffers of one job; each array has n_bins entries (hist has
 * n_bins * COSMICA_NHIST).  Any pointer may be NULL to skip that output.
 * exits, if not NULL, receives sum(particles_per_bin) records in bin order. */
typedef struct {
    uint32_t* hist;
    double* flux;             /* J_mod(P0) = P0^2 <J_LIS(P_ex)/P_ex^2> */
    double* flux_se;          /* Monte Carlo standard error of flux */
    double* mean_exit_time_s;
    uint64_t* steps;          /* EM steps summed over the bin */
    uint32_t* n_capped;
    uint32_t* n_nan;
    cosmica_exit* exits;
} cosmica_result;

/* Device output buffers of a plan: arrays over all bins of all jobs of the plan,
 * jobs in submission order, bins in order (hist: total_bins * COSMICA_NHIST).
 * Device pointers (e.g. from torch); any may be NULL to skip. */
typedef struct {
    uint32_t* hist;
    double* flux;
    double* flux_se;
    double* mean_exit_time_s;
    uint64_t* steps;
    uint32_t* n_capped;
    uint32_t* n_nan;
} cosmica_bins_dev;

/* Launch shape of the persistent propagation kernel. */
typedef struct {
    int32_t block;          /* threads per workgroup: 64, 128 or 256 */
    int32_t blocks_per_cu;  /* resident workgroups requested per compute unit (1..32) */
    int32_t chunk;          /* refill chunk: particles handed out per queue grab (>= 1) */
    int32_t order;          /* 0: bins in submission order; 1: largest bins first;
                             * 2: most expected steps per particle first (the
                             * library's estimate from the drift sign sign(Z) A, the
                             * shells' mean tilt and the rigidity; ties largest
                             * first), from the first execution on; serving orders
                             * each request's own bins so.  Results never depend on
                             * the order */
} cosmica_launch;

/* Timings of the last cosmica_run / cosmica_plan_execute, from HIP events on
 * the context's stream [ms]. */
typedef struct {
    double upload_ms;
    double propagate_ms;
    double reduce_ms;
    double download_ms;
    uint64_t steps;          /* EM steps of the last execution */
    uint64_t particles;
    int32_t grid_blocks;
    int32_t block;
} cosmica_timings;

typedef struct cosmica_ctx cosmica_ctx;
typedef struct cosmica_plan cosmica_plan;

/* Layout version of this header (COSMICA_ABI_VERSION). */
int cosmica_abi_version(void);

/* Human-readable name of a status code; never NULL, static storage. */
const char* cosmica_strerror(cosmica_status status);

/* Checks one job against the validation rules without touching a device.
 * Returns COSMICA_OK or COSMICA_EINVAL. */
cosmica_status cosmica_validate_job(const cosmica_job* job);

/* Opens a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory the context may hold (0 = 90% of the device's free memory).  Device
 * blocks freed by finished runs and plans stay with the context (up to a
 * quarter of the budget) for reuse by allocations of the same size, and are
 * given back first when an allocation would exceed the budget.
 * hip_stream: a hipStream_t to run on, or NULL for a stream the context owns.
 * *out receives the handle (NULL on error). */
cosmica_status cosmica_create(cosmica_ctx** out, int device, uint64_t hbm_budget_bytes,
                              void* hip_stream);

/* Stops the serving worker, frees all device memory and the handle. NULL is a no-op. */
void cosmica_destroy(cosmica_ctx* ctx);

/* Blocking batch run: all jobs are packed into one flat work queue and
 * integrated by one persistent launch per model (1D / 3D), then reduced per bin
 * (Sec. IV.A: propagation, histogramming, LIS weighting).  results[j] receives
 * job j; 1 <= n_jobs <= COSMICA_MAX_JOBS, else COSMICA_EINVAL.  Returns
 * COSMICA_ESTEPCAP (results valid) if any particle hit its cap. */
cosmica_status cosmica_run(cosmica_ctx* ctx, const cosmica_job* jobs, int32_t n_jobs,
                           cosmica_precision precision, cosmica_result* results);

/* Plans: the same work as cosmica_run, split so the inputs stay resident in
 * device memory and executions can be repeated and timed.
 * cosmica_plan_create uploads the job tables and reserves exit records
 * (ENOMEM when over the context's budget); want_exits != 0 also keeps the
 * per-particle (r, theta, phi) for cosmica_plan_read. */
cosmica_status cosmica_plan_create(cosmica_ctx* ctx, const cosmica_job* jobs, int32_t n_jobs,
                                   cosmica_precision precision, int32_t want_exits,
                                   cosmica_plan** out);

/* Enqueues propagation + reduction on the context's stream and returns without
 * waiting.  out == NULL keeps results in plan-owned device memory (read them
 * with cosmica_plan_read); otherwise results go to the given device buffers. */
cosmica_status cosmica_plan_execute(cosmica_plan* plan, const cosmica_bins_dev* out);

/* Waits for the plan's last execution and copies its plan-owned results into
 * results[0..n_jobs-1] (host buffers).  Returns COSMICA_ESTEPCAP as cosmica_run. */
cosmica_status cosmica_plan_read(cosmica_plan* plan, cosmica_result* results);

/* Sizes of a plan: total bins, total particles, number of jobs. */
cosmica_status cosmica_plan_info(const cosmica_plan* plan, uint64_t* total_bins,
                                 uint64_t* total_particles, int32_t* n_jobs);

/* Re-weights the exit records of the plan's last execution with n_lis other
 * local interstellar spectra: the paths do not depend on the spectrum, which
 * only enters the weight of Eq.(4) (the parameter-fitting use of Sec. VIII).
 * Each spectrum is tabulated as ln J at n_knots points ln P = lnP0 + k dlnP
 * (P in GV); ln J is linear in ln P between knots and the end segments are
 * extended.  lnJ: host, n_lis * n_knots (spectrum-major).  flux, flux_se: host,
 * n_lis * total_bins, [l * total_bins + b] with bins in plan order (either may
 * be NULL): J_mod(P0) and its standard error for spectrum l, in each job's
 * formulation.  EINVAL if the plan has not been executed, n_lis is outside
 * 1..COSMICA_MAX_REWEIGHT, n_knots outside 2..COSMICA_MAX_LIS_KNOTS, dlnP <= 0
 * or a table value is not finite.  Blocking; it holds n_lis * (n_knots + 2 *
 * total_bins) doubles of device memory for the call (ENOMEM beyond the
 * context's budget). */
#define COSMICA_MAX_REWEIGHT 4096
#define COSMICA_MAX_LIS_KNOTS 256
cosmica_status cosmica_plan_reweight(cosmica_plan* plan, uint32_t n_lis, uint32_t n_knots,
                                     double lnP0, double dlnP, const double* lnJ, double* flux,
                                     double* flux_se);

/* Exit histograms over the range the exits reach, as the paper bins them
 * (Sec. IV.A: the largest exit energy of the sample sets the binning), from
 * the plan's last execution: for each bin, p_max = its largest exit rigidity
 * [GV] (0 if no exit is used) and n_hist counts of ln(P_ex / P0) in equal
 * bins over [0, ln(p_max / P0)] (the exit at p_max in the last bin; with no
 * energy change every exit in bin 0).  Capped and non-finite exits are left
 * out, as in the modulated flux.  p_max: host, total_bins; hist: host,
 * total_bins * n_hist, bin-major, bins in plan order (either may be NULL).
 * EINVAL if the plan has not been executed or n_hist is outside
 * 1..COSMICA_MAX_RANGE_BINS.  Blocking.  The fixed log-ratio histogram of
 * cosmica_result is the default binning; this one is the paper's. */
#define COSMICA_MAX_RANGE_BINS 4096
cosmica_status cosmica_plan_exit_range(cosmica_plan* plan, uint32_t n_hist, double* p_max,
                                       uint32_t* hist);

void cosmica_plan_destroy(cosmica_plan* plan);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cosmica_run
 * with every device buffer -- job and region tables, work queue, exit records,
 * per-bin results -- carved from one array of COSMICA_STATIC_BYTES that the
 * library holds on each GPU it runs on, from the first cosmica_create on that
 * GPU until the process ends.  The call allocates no memory, on the device or
 * the host (its host staging is set aside by cosmica_create).  Arguments,
 * results (bit for bit) and errors are those of cosmica_run; in addition
 * COSMICA_ESCRATCH, before anything is written, when the work exceeds the
 * limits: n_jobs <= COSMICA_STATIC_MAX_JOBS, total bins <=
 * COSMICA_STATIC_MAX_BINS, orbit positions of all jobs <=
 * COSMICA_STATIC_MAX_ORBIT, and the buffers within the array (about 20 B per
 * particle, 28 B in the energy form, 80 B more when exits are requested, plus
 * ~600 B per bin and ~1.4 KB per job).  The array keeps the last call's
 * contents; calls on one GPU share it and would race, so the library runs
 * them one at a time (a call waits for the previous one to return). */
#define COSMICA_STATIC_BYTES 134217728ull /* 128 MiB per GPU */
#define COSMICA_STATIC_MAX_JOBS 256
#define COSMICA_STATIC_MAX_BINS 8192
#define COSMICA_STATIC_MAX_ORBIT 4096
cosmica_status cosmica_run_static(cosmica_ctx* ctx, const cosmica_job* jobs, int32_t n_jobs,
                                  cosmica_precision precision, cosmica_result* results);

/* Launch shape used for (model, precision); the defaults come from the
 * autotuner cache when one was loaded, else built-in values (256 threads, full
 * residency, 32-particle chunks, order 2). */
cosmica_status cosmica_set_launch(cosmica_ctx* ctx, cosmica_model model,
                                  cosmica_precision precision, const cosmica_launch* cfg);
cosmica_status cosmica_get_launch(cosmica_ctx* ctx, cosmica_model model,
                                  cosmica_precision precision, cosmica_launch* cfg);

/* Times a calibration batch over candidate launch shapes and keeps the fastest
 * for (model, precision) (the paper's warps-per-block sweep, Sec. VI "Version 2",
 * generalised).  cache_path, if not NULL, is read first (a hit skips the sweep)
 * and updated afterwards; the cache key includes the device architecture and
 * a digest of the kernel and runtime sources the library was built from.  A
 * candidate replaces the best shape so far only when more than 1% faster. */
cosmica_status cosmica_tune(cosmica_ctx* ctx, cosmica_model model, cosmica_precision precision,
                            const char* cache_path);

/* The same sweep on a sample of the caller's own workload: every k-th of
 * jobs[0..n_jobs-1] (all of one model; k odd, about total / sample_particles),
 * whole, so bins keep their sizes, seeds and tags.  Cache handling as
 * cosmica_tune. */
cosmica_status cosmica_tune_jobs(cosmica_ctx* ctx, const cosmica_job* jobs, int32_t n_jobs,
                                 cosmica_precision precision, uint64_t sample_particles,
                                 const char* cache_path);

/* Section timings of the last execution. */
cosmica_status cosmica_get_timings(cosmica_ctx* ctx, cosmica_timings* out);

/* Serving (continuous batching).  cosmica_submit copies the job and queues it;
 * a worker thread admits queued jobs while the device-memory footprint of
 * resident particle state + exit records stays within the budget, and runs the
 * persistent kernel in bounded slices so that newly admitted jobs join the
 * particles already in flight.  The result buffers must stay valid until the
 * ticket is done.  *ticket receives a positive id.
 *
 * The worker enqueues each slice before it reads what the previous one did, so
 * a job is seen to be finished one slice after its last particle exits and is
 * handed over after the next one (a slice lasts COSMICA_SLICE_MS).  Results
 * are the same, bit for bit, as cosmica_run of the job alone.  Environment,
 * read at every slice:
 *   COSMICA_SLICE_MS     slice length on the device clock, default 6 (ms);
 *   COSMICA_SLICE_STEPS  if set, a slice also ends after that many steps of
 *                        each wave (tests use it to force many slices);
 * and when a context first serves a (model, precision):
 *   COSMICA_SERVE_POOL   exit records of the admission pool, in particles
 *                        (default 2^28, at most a 20th of the budget not in use);
 *   COSMICA_SERVE_RING   initial entries of the device work queue, a power of
 *                        two from 64 to 2^26 (default 2^20); it grows as needed. */
cosmica_status cosmica_submit(cosmica_ctx* ctx, const cosmica_job* job,
                              cosmica_precision precision, cosmica_result* result,
                              uint64_t* ticket);

/* *done = 1 once the ticket's results are in its buffers (status of the job is
 * returned: COSMICA_OK, COSMICA_ESTEPCAP or COSMICA_ECANCELED), else 0. */
cosmica_status cosmica_poll(cosmica_ctx* ctx, uint64_t ticket, int32_t* done);

/* Blocks until the ticket is done or timeout_ms elapses (< 0: no limit); returns
 * the job's status as cosmica_poll does, or COSMICA_EBUSY on timeout. */
cosmica_status cosmica_wait(cosmica_ctx* ctx, uint64_t ticket, int32_t timeout_ms);

/* Cancels a queued or running ticket; its particles are dropped at the next slice. */
cosmica_status cosmica_cancel(cosmica_ctx* ctx, uint64_t ticket);

/* *state = 0 while the ticket waits for admission, 1 while its particles are on
 * the device, 2 once it is done (finished, failed or cancelled).  For load
 * shedding: cancelling a ticket in state 0 costs the device nothing.  Returns
 * COSMICA_ENOTFOUND for an unknown ticket.  Thread-safe like cosmica_poll. */
cosmica_status cosmica_request_state(cosmica_ctx* ctx, uint64_t ticket, int32_t* state);

/* Serving counters: jobs queued, jobs resident, particles parked between
 * slices (as of the last slice the worker has read), device bytes the context
 * holds (live and kept for reuse). */
cosmica_status cosmica_serve_stats(cosmica_ctx* ctx, uint64_t* queued, uint64_t* resident,
                                   uint64_t* particles_in_flight, uint64_t* bytes_in_use);

/* Diagnostics of single hot-path steps, for parity checks against an
 * independent implementation.
 * cosmica_probe_rng: Philox4x32-10 words of key = seed, counters
 *   (c0 + i, c1, c2, c3) for i < n (words: 4n, may be NULL), and the normals
 *   z0, z1, z2 the integrator draws from them in FP64 (z64: 3n) and in FP32
 *   (z32: 3n) (Sec. IV.A random numbers; Box-Muller).  Host buffers.
 * cosmica_probe_coeffs: local 3D SDE coefficients of job->helio/species at
 *   n points pts[4i..4i+3] = (P [GV], r [AU], theta, phi); out[16i..16i+15] =
 *   (A_r, A_theta, A_phi, A_P, B_rr, B_phir, B_phiphi, B_thth, dt, Hw, vd_r,
 *   vd_theta, vd_phi, K_rr, K_rphi, k_par) in AU, s, GV (Eq.(3), Eq.(5),
 *   Eq.(6)).  Host buffers. */
cosmica_status cosmica_probe_rng(cosmica_ctx* ctx, uint64_t seed, uint32_t c0, uint32_t c1,
                                 uint32_t c2, uint32_t c3, uint32_t n, uint32_t* words,
                                 double* z64, float* z32);
cosmica_status cosmica_probe_coeffs(cosmica_ctx* ctx, const cosmica_job* job,
                                    cosmica_precision precision, uint32_t n, const double* pts,
                                    double* out);
/* cosmica_probe_locate: where n points pts[3i..3i+2] = (r [AU], theta, phi)
 *   lie for job->helio (Sec. II.B regions), decided by the integrator's own
 *   device code in the given precision: region[i] = the parameter region (0..
 *   n_regions-1 the shells, 15 the heliosheath), outside[i] = 1 if the point is
 *   beyond the heliopause (the exit test), else 0.  Host buffers. */
cosmica_status cosmica_probe_locate(cosmica_ctx* ctx, const cosmica_job* job,
                                    cosmica_precision precision, uint32_t n, const double* pts,
                                    int32_t* region, int32_t* outside);

#ifdef __cplusplus
}
#endif
#endif
