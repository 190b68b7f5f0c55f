// engine.hpp -- device-side tables shared by the HIP kernels and the host
// runtime of libcosmica (internal; not part of the C ABI).
//
// Units on the device: AU, s, GV.  The runtime converts the physical inputs of
// cosmica.h once per job; kernels only read these tables.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cosmica {

constexpr int kMaxRegions = 15;
constexpr int kRegionStride = 16;  // region-table entries reserved per job
constexpr int kRegionHeliosheath = 15;  // the heliosheath's entry
constexpr int kNHist = 129;
constexpr uint32_t kFlagCapped = 1u;
constexpr uint32_t kFlagNaN = 2u;
constexpr int kFlagShift = 24;  // exit word = n | flags << 24 (n < 2^24)

// Per-job constants.  R is the bulk precision of the kernel (float for the
// mixed kernel, double for the plain FP64 one); r, t, P and the geometry of the
// boundary are always double.
template <typename R>
struct alignas(16) JobDev {
    uint32_t seed_lo, seed_hi, job_tag, step_cap;
    int32_t nreg, drift, hcs, shaped;  // shaped: nose-squashed boundary or heliosheath
    double rb;         // heliopause nose distance: every r >= rb may be outside [AU]
    double inv_shell;  // n_regions / (extent of the shells) [1/AU]
    double r0, th0, ph0;
    double rb_tail;    // heliopause tail distance: every r >= rb_tail is outside
    // Surfaces with nose / tail distances Rn, Rt: outside when
    // r^2 + (Rt - Rn) r cos(psi) >= Rn Rt (psi: angle from the nose).
    double hp_d2, hp_prod;       // heliopause: Rt - Rn, Rn Rt
    double ts_nose, ts_tail;     // termination shock (ts_nose = +inf: no heliosheath)
    double ts_d2, ts_prod;
    uint32_t orbit_off, n_orbit;  // moving detection point: first entry and count (0: r0, th0, ph0)
    int32_t energy, pad_e;        // 1: energy form (state T and the loss integral)
    double mass;                  // rest energy [GeV], for T <-> P
    R sin_tn, cos_tn, ph_n, pad_n;  // nose direction: sin, cos of its colatitude; longitude
    R vf;          // fast wind [AU/s]
    R omega;       // solar rotation [rad/s]
    R kperp_frac;  // f = kappa_perp / kappa_par
    R omf;         // 1 - f
    R sqf2;        // 2 sqrt(f)
    R twof;        // 2 f
    R gcoef;       // kappa_A / sqrt(1+G^2) = gcoef * beta * P * r^2 / (1+G^2)
    R hb;          // 1/Delta = hb sqrt(1+G^2) / (r P): B_r(1 AU) / (2 x Larmor coefficient)
    R abs_z, mass2;
    R sqA;         // sign(Z) * polarity
    R dt_max, diff_frac, adv_frac;
};

// One parameter region (a radial shell, or the heliosheath): kappa0 [AU^2/s],
// slow wind [AU/s], tilt [rad], tan(tilt), omega / slow wind [rad/AU], fast
// wind [AU/s]; om_rev = omega / (2 pi slow wind) [revolutions/AU] in FP64, the
// current sheet's phase per AU (32 B per entry in binary32, 64 B in binary64).
template <typename R>
struct alignas(16) RegionDev {
    R k0, vs, alpha, tana, om_vs, vf;
    double om_rev;
};
static_assert(sizeof(RegionDev<float>) == 32 && sizeof(RegionDev<double>) == 64,
              "region entries: two 16-byte loads in binary32");

// One position of a moving detection point.
struct alignas(16) OrbitDev {
    double r, th, ph, pad;
};

// One (job, rigidity bin) segment of the flat work index.
struct alignas(16) SegmentDev {
    double P0;
    uint32_t job, bin, count, out_offset;
    uint32_t pad0, pad1;
};

// A refill chunk: particles [first, first+count) of segment seg.
struct alignas(16) ChunkDev {
    uint32_t seg, first, count, pad0;
};

struct alignas(16) LisDev {
    double norm, index;
    double abs_z, mass;  // for beta in the energy form's weight
    int32_t energy, pad0, pad1, pad2;
};

// Parked particles of a serving slice, one array per field (lane i of a wave
// writes entry base + i, so every store is contiguous): full state, bit-exact
// on resume.  T and the loss integral belong to the energy form.
struct ParkDev {
    double *r, *P, *t, *th, *ph, *T, *lam;
    uint32_t *n, *seg, *pid;
};

// The lists a serving slice works on, in device memory (one descriptor per
// slice parity, written once): what the previous slice parked and left
// unissued comes back first; this slice parks its own into the other lists.
struct SliceDev {
    ParkDev resume;
    ParkDev suspend;
    const uint32_t* n_resume;     // count of resume
    uint32_t* resume_head;        // cursor over resume
    uint32_t* suspend_count;
    const ChunkDev* left_in;      // chunk remainders of the previous slice
    const uint32_t* n_left_in;    // their count
    uint32_t* left_in_head;       // cursor over left_in
    ChunkDev* leftover;           // chunk remainders a wave holds when this slice ends
    uint32_t* leftover_count;
    uint32_t* overflow;           // set to 1 if suspend or leftover would overflow
    uint32_t park_cap;            // entries of suspend
    uint32_t left_cap;            // entries of leftover
};

template <typename R>
struct PropArgs {
    const JobDev<R>* jobs;
    const RegionDev<R>* regions;  // jobs * kRegionStride
    const OrbitDev* orbit;        // orbit positions, indexed by JobDev::orbit_off
    const SegmentDev* segs;
    // refill queue: positions [*head, q_tail) are still to be issued, position
    // c at chunks[c & q_mask] (a ring buffer when q_mask + 1 is its size)
    const ChunkDev* chunks;
    unsigned long long* head;
    uint64_t q_tail, q_mask;
    // exit records, indexed by segment out_offset + particle
    double* exP;
    double* exT;
    uint32_t* exNF;
    double* exL;   // energy form: summed loss per particle (nullptr without energy-form jobs)
    double* exR;   // optional (nullptr)
    double* exTh;
    double* exPh;
    const SliceDev* slice;        // serving slices (nullptr: one whole pass)
    uint32_t step_budget;         // steps per wave per launch (0xffffffff: unlimited)
    uint64_t slice_ticks;         // launch length in device wall-clock ticks (0: unlimited)
    uint32_t uniform_key;         // 1: every job of the launch has the Philox key below
    uint32_t shaped;              // 1: some job of the launch has a squashed boundary or a heliosheath
    uint32_t energy;              // 1: some job of the launch is in the energy form
    uint32_t key_lo, key_hi;
    const uint32_t* job_cancel;   // optional per-job cancel flags
    uint32_t* job_done;           // optional per-job count of finished particles
};

// End of a serving slice (one workgroup, after the propagation kernel):
// resume entries and chunk remainders of the previous slice that no wave
// claimed move to this slice's lists (those of cancelled jobs are dropped),
// the queue head is clamped to the slice's tail (waves that found the queue
// empty advanced it past), and the next slice's counters are cleared.
struct CloseArgs {
    SliceDev sl;  // the slice's lists: resume / left_in in, suspend / leftover out
    unsigned long long* head;
    uint64_t q_tail;
    const SegmentDev* segs;
    const uint32_t* job_cancel;
    uint32_t* next_counters;  // 4 words cleared at the end
};

struct ReduceArgs {
    const SegmentDev* segs;
    const LisDev* lis;  // per job
    const double* exP;
    const double* exT;
    const uint32_t* exNF;
    const double* exL;  // energy form: summed loss (may be null without energy-form jobs)
    uint32_t seg_base;  // first segment of this launch
    uint32_t* hist;     // per segment: kNHist (may be null)
    double* flux;
    double* flux_se;
    double* mean_t;
    uint64_t* steps;
    uint32_t* n_capped;
    uint32_t* n_nan;
    uint32_t out_base;  // output index of segment seg_base
};

// Re-weighting of exit records with tabulated spectra.
constexpr int kReweightGroup = 16;  // spectra per workgroup
constexpr int kMaxLisKnots = 256;
struct ReweightArgs {
    const SegmentDev* segs;
    const LisDev* lis;
    const double* exP;
    const uint32_t* exNF;
    const double* exL;  // energy form (may be null without energy-form jobs)
    const double* lnJ;  // n_lis * n_knots
    uint32_t n_lis, n_knots;
    double lnP0, dlnP;
    uint32_t seg_base, out_base, total_bins, pad0;
    double* flux;       // n_lis * total_bins
    double* flux_se;
};

// Exit histogram over the reached range: per bin the largest used exit
// rigidity and the counts of ln(P_ex / P0) in n_hist equal bins up to it.
constexpr int kMaxRangeBins = 4096;
struct RangeArgs {
    const SegmentDev* segs;
    const double* exP;
    const uint32_t* exNF;
    uint32_t n_hist, seg_base, out_base, total_bins;
    double* p_max;   // total_bins
    uint32_t* hist;  // total_bins * n_hist
};

// An exit record in the layout of cosmica_exit, so records can be copied
// straight into a caller's array.
struct ExitRecDev {
    double P, t, r, th, ph;
    uint32_t n, flags;
    double loss;
};

// Launchers (kernels.hip).
hipError_t launch_propagate_3d_mixed(const PropArgs<float>& a, int grid, int block, hipStream_t s);
hipError_t launch_propagate_3d_fp64(const PropArgs<double>& a, int grid, int block, hipStream_t s);
hipError_t launch_propagate_1d_mixed(const PropArgs<float>& a, int grid, int block, hipStream_t s);
hipError_t launch_propagate_1d_fp64(const PropArgs<double>& a, int grid, int block, hipStream_t s);
hipError_t occupancy_propagate(int model, int prec, int block, int shaped, int energy, int ukey,
                               int* blocks_per_cu);
hipError_t launch_reduce(const ReduceArgs& a, uint32_t n_segs, hipStream_t s);
hipError_t launch_reweight(const ReweightArgs& a, uint32_t n_segs, hipStream_t s);
hipError_t launch_exit_range(const RangeArgs& a, uint32_t n_segs, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint32_t n, hipStream_t s);
hipError_t launch_slice_close(const CloseArgs& a, hipStream_t s);
// Exit records [0, n) from the per-field arrays (L, R, Th, Ph may be null: 0).
hipError_t launch_pack_exits(const double* P, const double* T, const uint32_t* NF,
                             const double* L, const double* R, const double* Th,
                             const double* Ph, uint32_t n, ExitRecDev* out, hipStream_t s);

// Diagnostics: raw Philox words and normals for counters (i, c1, c2, c3),
// i = c0 .. c0+n-1; coefficients at given points.
hipError_t launch_probe_rng(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                            uint32_t c3, uint32_t n, uint32_t* words, double* z64, float* z32,
                            hipStream_t s);
hipError_t launch_probe_coeffs_fp64(const JobDev<double>* job, const RegionDev<double>* reg,
                                    const double* pts, uint32_t n, double* out, hipStream_t s);
hipError_t launch_probe_coeffs_mixed(const JobDev<float>* job, const RegionDev<float>* reg,
                                     const double* pts, uint32_t n, double* out, hipStream_t s);
constexpr int kProbeOut = 16;
hipError_t launch_probe_locate_fp64(const JobDev<double>* job, const RegionDev<double>* reg,
                                    const double* pts, uint32_t n, int32_t* region,
                                    int32_t* outside, hipStream_t s);
hipError_t launch_probe_locate_mixed(const JobDev<float>* job, const RegionDev<float>* reg,
                                     const double* pts, uint32_t n, int32_t* region,
                                     int32_t* outside, hipStream_t s);

}  // namespace cosmica
