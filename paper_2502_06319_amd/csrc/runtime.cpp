// runtime.cpp -- host runtime of libcosmica: the C ABI of include/cosmica.h.
//
// Validation, unit conversion into device tables, the flat work index
// (jobs x rigidity bins x particles, cut into refill chunks), persistent
// launches, per-bin reduction, HIP-event timings, the launch-shape tuner and
// the continuous-batching server.
#include "cosmica.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"

using namespace cosmica;

namespace {

static_assert(sizeof(ExitRecDev) == sizeof(cosmica_exit) &&
                  offsetof(ExitRecDev, n) == offsetof(cosmica_exit, n) &&
                  offsetof(ExitRecDev, loss) == offsetof(cosmica_exit, loss),
              "device exit records use the layout of cosmica_exit");

// Physical constants of the unit conversion (AU: IAU 2012).
constexpr double kAuCm = 1.495978707e13;
constexpr double kAuKm = 1.495978707e8;
constexpr double kAuM = 1.495978707e11;
constexpr double kLightMs = 299792458.0;
constexpr double kPiH = 3.141592653589793238462643383279502884;
constexpr uint32_t kDefaultStepCap = 10000000u;

#define HIP_TRY(expr)                                        \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) {                              \
            last_hip_error() = e_;                           \
            return COSMICA_EDEVICE;                          \
        }                                                    \
    } while (0)

hipError_t& last_hip_error()
{
    static thread_local hipError_t e = hipSuccess;
    return e;
}

// ---------------------------------------------------------------------------
// Validated, self-contained copy of a job.
// ---------------------------------------------------------------------------
struct JobCopy {
    cosmica_helio helio;
    cosmica_species species;
    std::vector<double> rig;
    std::vector<uint32_t> cnt;
    uint64_t seed = 0;
    uint32_t tag = 0;
    uint32_t cap = kDefaultStepCap;
    uint32_t bin_offset = 0;
    uint64_t total = 0;
    std::vector<double> orbit;  // 3 per position
    int formulation = 0;        // 0 momentum form, 1 energy form
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// The fields of a job the device tables are made from: a view of either a
// caller's cosmica_job or a JobCopy, so tables can be made without a copy.
struct JobHead {
    const cosmica_helio* helio;
    const cosmica_species* species;
    uint64_t seed;
    uint32_t tag, cap, n_orbit;
    int formulation;
};

JobHead head_of(const cosmica_job& j)
{
    return JobHead{j.helio, j.species, j.seed, j.job_tag,
                   j.step_cap == 0 ? kDefaultStepCap : j.step_cap, j.n_orbit, j.formulation};
}

// A point strictly inside the heliopause (the squashed surface of cosmica.h
// for a 3D heliosphere with a nose distance, else the sphere r_boundary_au).
bool inside_heliopause(const cosmica_helio& h, double r, double th, double ph)
{
    const double rt = h.r_boundary_au;
    const double rn = h.r_boundary_nose_au > 0.0 ? h.r_boundary_nose_au : rt;
    if (h.model != COSMICA_MODEL_3D || rn == rt) return r < rt;
    const double cpsi = std::sin(th) * std::sin(h.nose_theta_rad) * std::cos(ph - h.nose_phi_rad) +
                        std::cos(th) * std::cos(h.nose_theta_rad);
    return r * r + (rt - rn) * r * cpsi < rn * rt;
}

cosmica_status validate(const cosmica_job* j)
{
    if (j == nullptr || j->helio == nullptr || j->species == nullptr) return COSMICA_EINVAL;
    if (j->n_bins < 1 || j->rigidity_gv == nullptr || j->particles_per_bin == nullptr)
        return COSMICA_EINVAL;
    const cosmica_helio& h = *j->helio;
    const cosmica_species& s = *j->species;
    if (h.model != COSMICA_MODEL_1D && h.model != COSMICA_MODEL_3D) return COSMICA_EINVAL;
    if (h.n_regions < 1 || h.n_regions > COSMICA_MAX_REGIONS) return COSMICA_EINVAL;
    if (!finite_pos(h.r_boundary_au) || !finite_pos(h.r0_au) || !(h.r0_au < h.r_boundary_au))
        return COSMICA_EINVAL;
    if (!finite_pos(h.dt_max_s) || !finite_pos(h.dt_diff_frac)) return COSMICA_EINVAL;
    if (!std::isfinite(h.dt_adv_frac) || h.dt_adv_frac < 0.0) return COSMICA_EINVAL;
    if (h.drift != 0 && h.drift != 1) return COSMICA_EINVAL;
    if (h.hcs != 0 && h.hcs != 1) return COSMICA_EINVAL;
    if (h.hcs == 1 && h.drift != 1) return COSMICA_EINVAL;
    if (h.polarity != 1 && h.polarity != -1) return COSMICA_EINVAL;
    const bool drift = h.model == COSMICA_MODEL_3D && h.drift == 1;
    for (int k = 0; k < h.n_regions; ++k) {
        if (!finite_pos(h.kappa0_cm2_s[k])) return COSMICA_EINVAL;
        if (!std::isfinite(h.v_slow_km_s[k]) || h.v_slow_km_s[k] < 0.0) return COSMICA_EINVAL;
        if (drift && !(h.v_slow_km_s[k] > 0.0)) return COSMICA_EINVAL;
        if (!std::isfinite(h.tilt_deg[k]) || h.tilt_deg[k] < 0.0 || !(h.tilt_deg[k] < 90.0))
            return COSMICA_EINVAL;
    }
    // nose-squashed heliopause and heliosheath (3D only)
    const bool nosed = h.r_boundary_nose_au != 0.0;
    if (h.heliosheath != 0 && h.heliosheath != 1) return COSMICA_EINVAL;
    if ((nosed || h.heliosheath == 1) && h.model != COSMICA_MODEL_3D) return COSMICA_EINVAL;
    if (nosed && (!finite_pos(h.r_boundary_nose_au) || !(h.r_boundary_nose_au <= h.r_boundary_au) ||
                  !(h.r0_au < h.r_boundary_nose_au)))
        return COSMICA_EINVAL;
    if ((nosed || h.heliosheath == 1) &&
        (!std::isfinite(h.nose_theta_rad) || !std::isfinite(h.nose_phi_rad)))
        return COSMICA_EINVAL;
    if (h.heliosheath == 1) {
        if (!finite_pos(h.ts_nose_au) || !std::isfinite(h.ts_tail_au) || !(h.r0_au < h.ts_nose_au) ||
            !(h.ts_nose_au <= h.ts_tail_au))
            return COSMICA_EINVAL;
        if (!finite_pos(h.kappa0_hs_cm2_s)) return COSMICA_EINVAL;
        if (!std::isfinite(h.v_hs_km_s) || h.v_hs_km_s < 0.0) return COSMICA_EINVAL;
        if (drift && !(h.v_hs_km_s > 0.0)) return COSMICA_EINVAL;
        if (!std::isfinite(h.tilt_hs_deg) || h.tilt_hs_deg < 0.0 || !(h.tilt_hs_deg < 90.0))
            return COSMICA_EINVAL;
    }
    if (h.model == COSMICA_MODEL_3D) {
        if (!std::isfinite(h.v_fast_km_s) || h.v_fast_km_s < 0.0) return COSMICA_EINVAL;
        if (drift && !(h.v_fast_km_s > 0.0)) return COSMICA_EINVAL;
        if (!(h.theta0_rad > 0.0) || !(h.theta0_rad < kPiH)) return COSMICA_EINVAL;
        if (!std::isfinite(h.phi0_rad)) return COSMICA_EINVAL;
        if (!std::isfinite(h.omega_rad_s) || h.omega_rad_s < 0.0) return COSMICA_EINVAL;
        // the spiral weights V^2 / (V^2 + (Omega r sin theta)^2) need V > 0 or Omega > 0
        if (h.omega_rad_s == 0.0) {
            bool calm = !(h.v_fast_km_s > 0.0) || (h.heliosheath == 1 && !(h.v_hs_km_s > 0.0));
            for (int k = 0; k < h.n_regions; ++k) calm = calm || !(h.v_slow_km_s[k] > 0.0);
            if (calm) return COSMICA_EINVAL;
        }
        if (!(h.kperp_over_kpar > 0.0) || !(h.kperp_over_kpar <= 1.0)) return COSMICA_EINVAL;
        if (drift && (!finite_pos(h.b0_nT) || !finite_pos(h.v_ref_km_s))) return COSMICA_EINVAL;
    }
    if (!std::isfinite(s.mass_gev) || s.mass_gev < 0.0 || s.charge == 0) return COSMICA_EINVAL;
    if (!finite_pos(s.lis_norm) || !std::isfinite(s.lis_index)) return COSMICA_EINVAL;
    if (j->step_cap > COSMICA_MAX_STEP_CAP) return COSMICA_EINVAL;
    uint64_t total = 0;
    for (int b = 0; b < j->n_bins; ++b) {
        if (!finite_pos(j->rigidity_gv[b])) return COSMICA_EINVAL;
        if (j->particles_per_bin[b] < 1) return COSMICA_EINVAL;
        total += j->particles_per_bin[b];
    }
    if (total >= (1ull << 32)) return COSMICA_EINVAL;
    if ((uint64_t)j->bin_offset + (uint64_t)j->n_bins > (1ull << 32)) return COSMICA_EINVAL;
    // formulation: momentum (any model) or energy (3D)
    if (j->formulation != 0 && j->formulation != 1) return COSMICA_EINVAL;
    if (j->formulation == 1 && h.model != COSMICA_MODEL_3D) return COSMICA_EINVAL;
    // moving detection point: positions inside the heliopause
    if (j->n_orbit > COSMICA_MAX_ORBIT || (j->n_orbit > 0 && j->orbit == nullptr))
        return COSMICA_EINVAL;
    for (uint32_t k = 0; k < j->n_orbit; ++k) {
        const double* q = j->orbit + 3 * (size_t)k;
        if (!finite_pos(q[0]) || !std::isfinite(q[1]) || !std::isfinite(q[2])) return COSMICA_EINVAL;
        if (h.model == COSMICA_MODEL_3D && (!(q[1] > 0.0) || !(q[1] < kPiH))) return COSMICA_EINVAL;
        if (!inside_heliopause(h, q[0], q[1], q[2])) return COSMICA_EINVAL;
    }
    return COSMICA_OK;
}

// A job whose heliopause is squashed or that has a heliosheath needs the
// propagation kernel that tests those surfaces.
bool helio_shaped(const cosmica_helio& h)
{
    return h.model == COSMICA_MODEL_3D &&
           (h.heliosheath == 1 || (h.r_boundary_nose_au > 0.0 && h.r_boundary_nose_au != h.r_boundary_au));
}

bool job_shaped(const JobCopy& jc) { return helio_shaped(jc.helio); }

JobCopy copy_job(const cosmica_job* j)
{
    JobCopy c;
    c.helio = *j->helio;
    c.species = *j->species;
    c.rig.assign(j->rigidity_gv, j->rigidity_gv + j->n_bins);
    c.cnt.assign(j->particles_per_bin, j->particles_per_bin + j->n_bins);
    c.seed = j->seed;
    c.tag = j->job_tag;
    c.cap = j->step_cap == 0 ? kDefaultStepCap : j->step_cap;
    c.bin_offset = j->bin_offset;
    for (uint32_t n : c.cnt) c.total += n;
    if (j->n_orbit > 0) c.orbit.assign(j->orbit, j->orbit + 3 * (size_t)j->n_orbit);
    c.formulation = j->formulation;
    return c;
}

JobHead head_of(const JobCopy& c)
{
    return JobHead{&c.helio, &c.species, c.seed, c.tag, c.cap, (uint32_t)(c.orbit.size() / 3),
                   c.formulation};
}

// Physical inputs -> device constants in AU, s, GV.
template <typename R>
void make_tables(const JobHead& jc, JobDev<R>* J, RegionDev<R>* reg, LisDev* lis)
{
    const cosmica_helio& h = *jc.helio;
    const cosmica_species& s = *jc.species;
    std::memset(J, 0, sizeof(*J));
    J->seed_lo = (uint32_t)(jc.seed & 0xffffffffu);
    J->seed_hi = (uint32_t)(jc.seed >> 32);
    J->job_tag = jc.tag;
    J->step_cap = jc.cap;
    J->nreg = h.n_regions;
    J->drift = h.model == COSMICA_MODEL_3D ? h.drift : 0;
    J->hcs = h.model == COSMICA_MODEL_3D ? h.hcs : 0;
    // heliopause: nose and tail distances (equal for a sphere); termination
    // shock only with a heliosheath
    const bool hs = h.model == COSMICA_MODEL_3D && h.heliosheath == 1;
    const double rb_nose = h.r_boundary_nose_au > 0.0 ? h.r_boundary_nose_au : h.r_boundary_au;
    J->rb = rb_nose;
    J->rb_tail = h.r_boundary_au;
    J->hp_d2 = h.r_boundary_au - rb_nose;
    J->hp_prod = rb_nose * h.r_boundary_au;
    J->ts_nose = hs ? h.ts_nose_au : HUGE_VAL;
    J->ts_tail = hs ? h.ts_tail_au : HUGE_VAL;
    J->ts_d2 = hs ? h.ts_tail_au - h.ts_nose_au : 0.0;
    J->ts_prod = hs ? h.ts_nose_au * h.ts_tail_au : 0.0;
    J->shaped = (hs || rb_nose != h.r_boundary_au) ? 1 : 0;
    J->n_orbit = jc.n_orbit;
    J->orbit_off = 0;  // set where the positions are placed
    J->energy = jc.formulation == 1 ? 1 : 0;
    J->mass = s.mass_gev;
    J->sin_tn = (R)std::sin(h.nose_theta_rad);
    J->cos_tn = (R)std::cos(h.nose_theta_rad);
    const double phn = std::fmod(h.nose_phi_rad, 2.0 * kPiH);
    J->ph_n = (R)(phn < 0.0 ? phn + 2.0 * kPiH : phn);
    // the shells split the inner heliosphere up to the shock's (or else the
    // heliopause's) nose distance
    J->inv_shell = (double)h.n_regions / (hs ? h.ts_nose_au : rb_nose);
    J->r0 = h.r0_au;
    J->th0 = h.theta0_rad;
    J->ph0 = h.phi0_rad;
    J->vf = (R)(h.v_fast_km_s / kAuKm);
    J->omega = (R)h.omega_rad_s;
    J->kperp_frac = (R)h.kperp_over_kpar;
    J->omf = (R)(1.0 - h.kperp_over_kpar);
    J->sqf2 = (R)(2.0 * std::sqrt(h.kperp_over_kpar));
    J->twof = (R)(2.0 * h.kperp_over_kpar);
    // |B| at 1 AU on the ecliptic is b0 for a wind of v_ref: B_r(1 AU) = b0 / sqrt(1 + Gamma_E^2)
    double br0 = h.b0_nT;
    if (h.v_ref_km_s > 0.0) {
        const double gE = h.omega_rad_s * kAuKm / h.v_ref_km_s;
        br0 = h.b0_nT / std::sqrt(1.0 + gE * gE);
    }
    // kappa_A = beta P / (3 |B|) [GV, nT -> AU^2/s], |B| = br0 / r^2 * sqrt(1 + Gamma^2)
    J->gcoef = br0 > 0.0 ? (R)(1e18 / (3.0 * br0 * kAuM * kAuM)) : (R)0;
    // sheet half-width Delta = 2 r_L / r with r_L = P / (c |B|) [GV, nT -> AU]
    const double rlcoef = 1e18 / (kLightMs * kAuM);
    J->hb = (R)(br0 / (2.0 * rlcoef));
    if (J->drift == 0) {
        // the field strength matters only to the drift, and cosmica.h leaves
        // b0_nT and v_ref_km_s unchecked without it; the binary32 kernel
        // evaluates the drift terms for every job (times a zero drift sign),
        // so they must stay finite
        J->gcoef = (R)0;
        J->hb = (R)0;
    }
    J->abs_z = (R)std::fabs((double)s.charge);
    J->mass2 = (R)(s.mass_gev * s.mass_gev);
    J->sqA = (R)((s.charge > 0 ? 1.0 : -1.0) * (double)h.polarity);
    J->dt_max = (R)h.dt_max_s;
    J->diff_frac = (R)h.dt_diff_frac;
    J->adv_frac = h.model == COSMICA_MODEL_3D ? (R)h.dt_adv_frac : (R)0;
    for (int k = 0; k < kRegionStride; ++k) {
        RegionDev<R>& g = reg[k];
        std::memset(&g, 0, sizeof(g));
        const int kk = k < h.n_regions ? k : h.n_regions - 1;
        const bool sheath = hs && k == kRegionHeliosheath;
        // the heliosheath has one wind speed for both bands
        const double vs = (sheath ? h.v_hs_km_s : h.v_slow_km_s[kk]) / kAuKm;
        const double vf = (sheath ? h.v_hs_km_s : h.v_fast_km_s) / kAuKm;
        const double alpha = (sheath ? h.tilt_hs_deg : h.tilt_deg[kk]) * kPiH / 180.0;
        const double k0 = sheath ? h.kappa0_hs_cm2_s : h.kappa0_cm2_s[kk];
        g.k0 = (R)(k0 / (kAuCm * kAuCm));
        g.vs = (R)vs;
        g.vf = (R)vf;
        g.alpha = (R)alpha;
        g.tana = (R)std::tan(alpha);
        g.om_vs = vs > 0.0 ? (R)(h.omega_rad_s / vs) : (R)0;
        g.om_rev = vs > 0.0 ? h.omega_rad_s / (2.0 * kPiH * vs) : 0.0;
    }
    lis->norm = s.lis_norm;
    lis->index = s.lis_index;
    lis->abs_z = std::fabs((double)s.charge);
    lis->mass = s.mass_gev;
    lis->energy = jc.formulation == 1 ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Device memory accounted against the context budget.
// ---------------------------------------------------------------------------
struct Pool;

}  // namespace

struct Req;
struct ServeGroup;
struct ServeHost;

// The device array behind cosmica_run_static: file scope, so each GPU the
// library runs on holds one copy from module load until the process ends.
// In host code its name only stands in for the symbol: every use goes through
// the address hipGetSymbolAddress returned for the device (static_base).
static __device__ __align__(256) unsigned char scratch[COSMICA_STATIC_BYTES];

namespace {

constexpr int kStaticDevices = 64;
std::mutex g_static_mu;                         // guards g_static_base
void* g_static_base[kStaticDevices] = {};       // device address of `scratch`, per device
std::mutex g_static_call_mu[kStaticDevices];    // one cosmica_run_static per device at a time

// Looks up the array's address on `device` once (the device must be current).
void static_setup(int device)
{
    if (device < 0 || device >= kStaticDevices) return;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_base[device] != nullptr) return;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p != nullptr)
        g_static_base[device] = p;
    else
        (void)hipGetLastError();  // cosmica_run_static then reports COSMICA_EDEVICE
}

void* static_base(int device)
{
    if (device < 0 || device >= kStaticDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_static_mu);
    return g_static_base[device];
}

// Host staging of cosmica_run_static, set aside when a context is created so
// that the call itself allocates nothing (~1.9 MB).
constexpr uint32_t kStaticMaxChunks = 65536;
struct StaticHost {
    alignas(64) unsigned char jobs[COSMICA_STATIC_MAX_JOBS * sizeof(JobDev<double>)];
    alignas(64) unsigned char regions[COSMICA_STATIC_MAX_JOBS * kRegionStride *
                                      sizeof(RegionDev<double>)];
    LisDev lis[COSMICA_STATIC_MAX_JOBS];
    uint32_t seg_first[COSMICA_STATIC_MAX_JOBS];
    OrbitDev orbit[COSMICA_STATIC_MAX_ORBIT];
    SegmentDev segs[COSMICA_STATIC_MAX_BINS];
    double cost[COSMICA_STATIC_MAX_BINS];
    uint32_t ids[COSMICA_STATIC_MAX_BINS];
    uint32_t ncap[COSMICA_STATIC_MAX_BINS];
    ChunkDev chunks[kStaticMaxChunks];
};

}  // namespace

struct cosmica_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t budget = 0;
    std::atomic<uint64_t> in_use{0};  // live and cached device bytes
    // Freed device blocks kept for reuse by an allocation of the same size
    // (repeated runs and plans of one shape allocate alike); counted in in_use
    // and released first when an allocation would exceed the budget.
    std::mutex cache_mu;
    std::multimap<size_t, void*> cache;
    std::atomic<uint64_t> cached{0};
    int num_cus = 0;
    int wall_khz = 0;  // rate of the device's constant-rate clock [kHz]
    std::string arch;
    cosmica_launch launch[2][2];
    cosmica_timings timings{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // steps of the last execution: device array and its length
    const uint64_t* last_steps = nullptr;
    uint32_t last_nsteps = 0;
    bool timings_pending = false;
    // serving
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    bool worker_started = false;
    uint64_t next_ticket = 1;
    std::deque<Req*> queued;
    std::map<uint64_t, std::unique_ptr<Req>> reqs;
    std::unique_ptr<ServeGroup> groups[2][2];
    hipStream_t serve_stream = nullptr;
    std::unique_ptr<ServeHost> serve_host;  // the worker's pinned buffers and events
    cosmica_status serve_error = COSMICA_OK;
    std::unique_ptr<StaticHost> stat;  // host staging of cosmica_run_static
    cosmica_ctx() = default;
    ~cosmica_ctx();  // defined once the serving types are complete
};

namespace {

// Returns cached blocks to the device until `need` more bytes fit the budget
// (all of them for need = ~0).
void cache_trim(cosmica_ctx* ctx, uint64_t need)
{
    std::lock_guard<std::mutex> lk(ctx->cache_mu);
    while (!ctx->cache.empty() && (need == ~0ull || ctx->in_use.load() + need > ctx->budget)) {
        auto it = std::prev(ctx->cache.end());  // largest first
        (void)hipFree(it->second);
        ctx->in_use.fetch_sub(it->first);
        ctx->cached -= it->first;
        ctx->cache.erase(it);
    }
}

cosmica_status dalloc(cosmica_ctx* ctx, size_t bytes, void** p)
{
    *p = nullptr;
    if (bytes == 0) return COSMICA_OK;
    bytes = (bytes + 255) & ~(size_t)255;
    {
        std::lock_guard<std::mutex> lk(ctx->cache_mu);
        auto it = ctx->cache.find(bytes);
        if (it != ctx->cache.end()) {
            *p = it->second;
            ctx->cached -= bytes;
            ctx->cache.erase(it);
            return COSMICA_OK;
        }
    }
    if (ctx->in_use.load() + bytes > ctx->budget) cache_trim(ctx, bytes);
    const uint64_t cur = ctx->in_use.fetch_add(bytes);
    if (cur + bytes > ctx->budget) {
        ctx->in_use.fetch_sub(bytes);
        return COSMICA_ENOMEM;
    }
    if (hipMalloc(p, bytes) != hipSuccess) {
        ctx->in_use.fetch_sub(bytes);
        *p = nullptr;
        (void)hipGetLastError();
        return COSMICA_ENOMEM;
    }
    return COSMICA_OK;
}

// The caller has waited for every use of the block: it is kept for reuse
// (up to a quarter of the budget in cached blocks), else given back.
void dfree(cosmica_ctx* ctx, void* p, size_t bytes)
{
    if (p == nullptr) return;
    bytes = (bytes + 255) & ~(size_t)255;
    {
        std::lock_guard<std::mutex> lk(ctx->cache_mu);
        if (ctx->cached.load() + bytes <= ctx->budget / 4) {
            ctx->cache.emplace(bytes, p);
            ctx->cached += bytes;
            return;
        }
    }
    (void)hipFree(p);
    ctx->in_use.fetch_sub(bytes);
}

// A set of device allocations freed together.
struct DevSet {
    cosmica_ctx* ctx = nullptr;
    std::vector<std::pair<void*, size_t>> blocks;
    explicit DevSet(cosmica_ctx* c) : ctx(c) {}
    ~DevSet() { release(); }
    void release()
    {
        // blocks go back to the context's cache: first let every copy or
        // kernel enqueued on the context's stream finish with them
        if (!blocks.empty()) (void)hipStreamSynchronize(ctx->stream);
        for (auto& b : blocks) dfree(ctx, b.first, b.second);
        blocks.clear();
    }
    template <typename T>
    cosmica_status alloc(T** p, size_t n)
    {
        void* q = nullptr;
        cosmica_status st = dalloc(ctx, n * sizeof(T), &q);
        if (st != COSMICA_OK) return st;
        if (q) blocks.emplace_back(q, n * sizeof(T));
        *p = (T*)q;
        return COSMICA_OK;
    }
};

// Expected Euler-Maruyama steps per particle of one (job, bin), used only to
// order the work queue.  Particles whose drift runs against the Parker
// spiral's polarity (sign(Z) A < 0, Eq.(3)'s drift term) ride the wavy current
// sheet: 10^3-10^5 steps, more the wavier the sheet, so the shells' mean tilt
// sets their cost; the others take 300-600 steps, weakly dependent on
// rigidity.  The coefficients are a least-squares fit of the logarithm of the
// measured mean steps per bin of the batched workload (64 parameter sets x 4
// species x 30 bins, seed 42); on an independent draw of that workload
// (seed 43) the estimate ranks the bins with a Spearman correlation of 0.93.
// A wrong estimate costs time only: results do not depend on the queue order.
double expected_steps(const cosmica_helio& h, const cosmica_species& sp, double P0)
{
    if (h.model != COSMICA_MODEL_3D) return 1.0;
    const double lp = std::log(P0);
    const int sq = sp.charge > 0 ? 1 : -1;
    if (h.drift == 1 && h.hcs == 1 && sq * h.polarity < 0) {
        double tilt = 0.0;
        for (int k = 0; k < h.n_regions; ++k) tilt += h.tilt_deg[k];
        tilt /= (double)h.n_regions;
        return std::exp(3.697 + 0.0365 * lp + 0.0201 * lp * lp + 6.653 * tilt / 45.0);
    }
    return std::exp(5.825 - 0.0657 * lp + 0.0489 * lp * lp);
}

// Chunks of every segment of a model group, in the requested order: 0 as
// given, 1 largest segments first, 2 highest expected steps per particle first
// (cost: one value per segment; ties and a missing cost fall back to 1).
// Particles are independent and their random numbers do not depend on the
// schedule, so the order changes only the time to drain the queue: starting
// the longest paths first keeps them out of the end-of-launch tail.
void make_chunks(const std::vector<SegmentDev>& segs, const std::vector<uint32_t>& seg_ids,
                 int chunk, int order, std::vector<ChunkDev>* out,
                 const std::vector<double>* cost = nullptr)
{
    std::vector<uint32_t> ids = seg_ids;
    if (order == 2 && cost != nullptr)
        std::stable_sort(ids.begin(), ids.end(), [&](uint32_t a, uint32_t b) {
            if ((*cost)[a] != (*cost)[b]) return (*cost)[a] > (*cost)[b];
            return segs[a].count > segs[b].count;
        });
    else if (order >= 1)
        std::stable_sort(ids.begin(), ids.end(),
                         [&](uint32_t a, uint32_t b) { return segs[a].count > segs[b].count; });
    const uint32_t c = (uint32_t)std::max(1, chunk);
    for (uint32_t s : ids) {
        for (uint32_t f = 0; f < segs[s].count; f += c) {
            ChunkDev ch;
            ch.seg = s;
            ch.first = f;
            ch.count = std::min(c, segs[s].count - f);
            ch.pad0 = 0;
            out->push_back(ch);
        }
    }
}

int grid_for(cosmica_ctx* ctx, int model, int prec, const cosmica_launch& L, uint64_t lanes_wanted,
             bool shaped, bool energy, bool ukey)
{
    int occ = 0;
    if (occupancy_propagate(model, prec, L.block, shaped ? 1 : 0, energy ? 1 : 0, ukey ? 1 : 0,
                            &occ) !=
            hipSuccess ||
        occ < 1)
        occ = 1;
    int bpc = L.blocks_per_cu > 0 ? std::min(L.blocks_per_cu, occ) : occ;
    uint64_t grid = (uint64_t)ctx->num_cus * (uint64_t)bpc;
    const uint64_t need = (lanes_wanted + (uint64_t)L.block - 1) / (uint64_t)L.block;
    if (need < grid) grid = std::max<uint64_t>(1, need);
    return (int)grid;
}

bool launch_ok(const cosmica_launch& L)
{
    return (L.block == 64 || L.block == 128 || L.block == 256) &&
           L.blocks_per_cu >= 0 && L.blocks_per_cu <= 32 && L.chunk >= 1 &&
           L.order >= 0 && L.order <= 2;
}

template <typename R>
hipError_t launch_model(int model, const PropArgs<R>& a, int grid, int block, hipStream_t s);
template <>
hipError_t launch_model<float>(int model, const PropArgs<float>& a, int grid, int block,
                               hipStream_t s)
{
    return model == 1 ? launch_propagate_3d_mixed(a, grid, block, s)
                      : launch_propagate_1d_mixed(a, grid, block, s);
}
template <>
hipError_t launch_model<double>(int model, const PropArgs<double>& a, int grid, int block,
                                hipStream_t s)
{
    return model == 1 ? launch_propagate_3d_fp64(a, grid, block, s)
                      : launch_propagate_1d_fp64(a, grid, block, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// Plans.
// ---------------------------------------------------------------------------
struct cosmica_plan {
    cosmica_ctx* ctx = nullptr;
    int prec = 0;
    bool want_exits = false;
    std::vector<JobCopy> jobs;
    std::vector<SegmentDev> segs;
    std::vector<uint32_t> seg_first;  // first segment of each job
    uint64_t total_particles = 0;
    uint64_t model_particles[2] = {0, 0};
    std::vector<ChunkDev> chunks_h[2];
    DevSet mem;
    void* jobs_d = nullptr;
    void* regions_d = nullptr;
    LisDev* lis_d = nullptr;
    OrbitDev* orbit_d = nullptr;
    SegmentDev* segs_d = nullptr;
    ChunkDev* chunks_d[2] = {nullptr, nullptr};
    uint32_t* counters_d = nullptr;  // 8 words: the queue heads of the two models (64-bit each)
    double* exP = nullptr;
    double* exT = nullptr;
    uint32_t* exNF = nullptr;
    double* exR = nullptr;
    double* exTh = nullptr;
    double* exPh = nullptr;
    // plan-owned results
    uint32_t* hist = nullptr;
    double* flux = nullptr;
    double* se = nullptr;
    double* mt = nullptr;
    uint64_t* steps = nullptr;
    uint32_t* ncap = nullptr;
    uint32_t* nnan = nullptr;
    bool executed = false;
    bool own_out = true;
    bool uniform_key = false;  // every job has the same seed
    bool shaped = false;       // some job has a squashed heliopause or a heliosheath
    bool energy = false;       // some job is in the energy form
    double* exL = nullptr;     // energy form: summed loss per particle
    uint64_t key = 0;
    explicit cosmica_plan(cosmica_ctx* c) : ctx(c), mem(c) {}
};

namespace {

template <typename R>
cosmica_status upload_tables(cosmica_plan* p)
{
    const size_t nj = p->jobs.size();
    std::vector<JobDev<R>> jh(nj);
    std::vector<RegionDev<R>> rh(nj * kRegionStride);
    std::vector<LisDev> lh(nj);
    std::vector<OrbitDev> oh;
    for (size_t j = 0; j < nj; ++j) {
        make_tables<R>(head_of(p->jobs[j]), &jh[j], &rh[j * kRegionStride], &lh[j]);
        jh[j].orbit_off = (uint32_t)oh.size();
        const std::vector<double>& o = p->jobs[j].orbit;
        for (size_t k = 0; k + 2 < o.size(); k += 3) oh.push_back(OrbitDev{o[k], o[k + 1], o[k + 2], 0.0});
    }
    JobDev<R>* jd = nullptr;
    RegionDev<R>* rd = nullptr;
    cosmica_status st;
    if (!oh.empty()) {
        if ((st = p->mem.alloc(&p->orbit_d, oh.size())) != COSMICA_OK) return st;
        HIP_TRY(hipMemcpyAsync(p->orbit_d, oh.data(), oh.size() * sizeof(OrbitDev),
                               hipMemcpyHostToDevice, p->ctx->stream));
    }
    if ((st = p->mem.alloc(&jd, nj)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&rd, rh.size())) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->lis_d, nj)) != COSMICA_OK) return st;
    HIP_TRY(hipMemcpyAsync(jd, jh.data(), nj * sizeof(JobDev<R>), hipMemcpyHostToDevice,
                           p->ctx->stream));
    HIP_TRY(hipMemcpyAsync(rd, rh.data(), rh.size() * sizeof(RegionDev<R>),
                           hipMemcpyHostToDevice, p->ctx->stream));
    HIP_TRY(hipMemcpyAsync(p->lis_d, lh.data(), nj * sizeof(LisDev), hipMemcpyHostToDevice,
                           p->ctx->stream));
    // the host tables are pageable and local: the copies must be complete
    HIP_TRY(hipStreamSynchronize(p->ctx->stream));
    p->jobs_d = jd;
    p->regions_d = rd;
    return COSMICA_OK;
}

// Device buffers of one propagation + reduction pass (a plan's, or the static
// array's for cosmica_run_static).
struct PassDev {
    const void* jobs;
    const void* regions;
    const OrbitDev* orbit;
    const SegmentDev* segs;
    const ChunkDev* chunks[2];  // the refill queues of the radial and 3D groups
    uint32_t n_chunks[2];
    uint64_t model_particles[2];
    uint32_t* counters;  // 8 words, zeroed: the queue heads of the two models (64-bit each)
    double *exP, *exT, *exL, *exR, *exTh, *exPh;
    uint32_t* exNF;
    bool uniform_key, shaped, energy;
    uint64_t key;
    int prec;
};

template <typename R>
cosmica_status execute_prop(cosmica_ctx* ctx, const PassDev& d)
{
    for (int model = 0; model < 2; ++model) {
        const uint32_t nch = d.n_chunks[model];
        if (nch == 0) continue;
        const cosmica_launch& L = ctx->launch[model][d.prec];
        PropArgs<R> a;
        std::memset(&a, 0, sizeof(a));
        a.jobs = (const JobDev<R>*)d.jobs;
        a.regions = (const RegionDev<R>*)d.regions;
        a.orbit = d.orbit;
        a.segs = d.segs;
        a.chunks = d.chunks[model];
        a.head = (unsigned long long*)(d.counters + 2 * model);
        a.q_tail = nch;
        a.q_mask = ~0ull;
        a.exP = d.exP;
        a.exT = d.exT;
        a.exNF = d.exNF;
        a.exR = d.exR;
        a.exTh = d.exTh;
        a.exPh = d.exPh;
        // one whole pass: nothing parked, nothing left over (the serving fields
        // stay null)
        a.step_budget = 0xffffffffu;
        a.slice_ticks = 0;
        a.job_cancel = nullptr;
        a.job_done = nullptr;
        a.uniform_key = d.uniform_key ? 1u : 0u;
        a.shaped = d.shaped ? 1u : 0u;
        a.energy = d.energy ? 1u : 0u;
        a.exL = d.exL;
        a.key_lo = (uint32_t)(d.key & 0xffffffffu);
        a.key_hi = (uint32_t)(d.key >> 32);
        const int grid =
            grid_for(ctx, model, d.prec, L, d.model_particles[model], d.shaped, d.energy, d.uniform_key);
        ctx->timings.grid_blocks = grid;
        ctx->timings.block = L.block;
        HIP_TRY(launch_model<R>(model, a, grid, L.block, ctx->stream));
    }
    return COSMICA_OK;
}

PassDev pass_of(const cosmica_plan* p)
{
    PassDev d;
    d.jobs = p->jobs_d;
    d.regions = p->regions_d;
    d.orbit = p->orbit_d;
    d.segs = p->segs_d;
    for (int m = 0; m < 2; ++m) {
        d.chunks[m] = p->chunks_d[m];
        d.n_chunks[m] = (uint32_t)p->chunks_h[m].size();
        d.model_particles[m] = p->model_particles[m];
    }
    d.counters = p->counters_d;
    d.exP = p->exP;
    d.exT = p->exT;
    d.exL = p->exL;
    d.exR = p->exR;
    d.exTh = p->exTh;
    d.exPh = p->exPh;
    d.exNF = p->exNF;
    d.uniform_key = p->uniform_key;
    d.shaped = p->shaped;
    d.energy = p->energy;
    d.key = p->key;
    d.prec = p->prec;
    return d;
}

}  // namespace

extern "C" {

int cosmica_abi_version(void) { return COSMICA_ABI_VERSION; }

const char* cosmica_strerror(cosmica_status s)
{
    switch (s) {
    case COSMICA_OK: return "ok";
    case COSMICA_EINVAL: return "invalid argument";
    case COSMICA_ENOMEM: return "out of device memory or over the HBM budget";
    case COSMICA_EDEVICE: return "HIP device error";
    case COSMICA_EBUSY: return "serving queue full";
    case COSMICA_ECANCELED: return "request cancelled";
    case COSMICA_ESTEPCAP: return "some particles reached the step cap";
    case COSMICA_ENOTFOUND: return "unknown ticket";
    case COSMICA_ESCRATCH: return "the work exceeds the static array of cosmica_run_static";
    }
    return "unknown status";
}

cosmica_status cosmica_validate_job(const cosmica_job* job) { return validate(job); }

cosmica_status cosmica_create(cosmica_ctx** out, int device, uint64_t hbm_budget_bytes,
                              void* hip_stream)
{
    if (out == nullptr) return COSMICA_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return COSMICA_EDEVICE;
    }
    if (device < 0 || device >= ndev) return COSMICA_EINVAL;
    HIP_TRY(hipSetDevice(device));
    auto ctx = std::make_unique<cosmica_ctx>();
    ctx->device = device;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    ctx->num_cus = prop.multiProcessorCount;
    if (hipDeviceGetAttribute(&ctx->wall_khz, hipDeviceAttributeWallClockRate, device) !=
            hipSuccess ||
        ctx->wall_khz <= 0) {
        (void)hipGetLastError();
        ctx->wall_khz = 0;  // slices then end by their step budget only
    }
    ctx->arch = prop.gcnArchName;
    // set-up of cosmica_run_static: its host staging, and (once per device)
    // the device address of its array
    ctx->stat.reset(new (std::nothrow) StaticHost);
    if (!ctx->stat) return COSMICA_ENOMEM;
    static_setup(device);
    size_t freeb = 0, totalb = 0;
    HIP_TRY(hipMemGetInfo(&freeb, &totalb));
    ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)freeb);
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    for (int i = 0; i < 4; ++i) HIP_TRY(hipEventCreate(&ctx->ev[i]));
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 2; ++q) ctx->launch[m][q] = cosmica_launch{256, 0, 32, 2};
    *out = ctx.release();
    return COSMICA_OK;
}

// the kernels address a job's region entries by a 32-bit byte offset
static_assert((uint64_t)COSMICA_MAX_JOBS * kRegionStride * sizeof(RegionDev<double>) <= (1ull << 32),
              "region offsets must fit 32 bits");

cosmica_status cosmica_plan_create(cosmica_ctx* ctx, const cosmica_job* jobs, int32_t n_jobs,
                                   cosmica_precision precision, int32_t want_exits,
                                   cosmica_plan** out)
{
    if (ctx == nullptr || out == nullptr || jobs == nullptr || n_jobs < 1 ||
        n_jobs > COSMICA_MAX_JOBS)
        return COSMICA_EINVAL;
    if (precision != COSMICA_PREC_FP64 && precision != COSMICA_PREC_MIXED) return COSMICA_EINVAL;
    *out = nullptr;
    uint64_t total = 0;
    for (int j = 0; j < n_jobs; ++j) {
        if (validate(&jobs[j]) != COSMICA_OK) return COSMICA_EINVAL;
        for (int b = 0; b < jobs[j].n_bins; ++b) total += jobs[j].particles_per_bin[b];
    }
    if (total >= (1ull << 32)) return COSMICA_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    auto p = std::make_unique<cosmica_plan>(ctx);
    p->prec = precision;
    p->want_exits = want_exits != 0;
    p->total_particles = total;
    std::vector<uint32_t> ids[2];
    std::vector<double> cost;  // expected steps per particle of each segment
    uint32_t off = 0;
    for (int j = 0; j < n_jobs; ++j) {
        p->jobs.push_back(copy_job(&jobs[j]));
        const JobCopy& jc = p->jobs.back();
        const int model = jc.helio.model;
        p->seg_first.push_back((uint32_t)p->segs.size());
        for (size_t b = 0; b < jc.rig.size(); ++b) {
            SegmentDev s;
            std::memset(&s, 0, sizeof(s));
            s.P0 = jc.rig[b];
            s.job = (uint32_t)j;
            s.bin = jc.bin_offset + (uint32_t)b;
            s.count = jc.cnt[b];
            s.out_offset = off;
            off += jc.cnt[b];
            ids[model].push_back((uint32_t)p->segs.size());
            p->model_particles[model] += jc.cnt[b];
            p->segs.push_back(s);
            cost.push_back(expected_steps(jc.helio, jc.species, jc.rig[b]));
        }
    }
    for (int m = 0; m < 2; ++m) {
        const cosmica_launch& L = ctx->launch[m][precision];
        make_chunks(p->segs, ids[m], L.chunk, L.order, &p->chunks_h[m], &cost);
    }
    p->key = p->jobs[0].seed;
    p->uniform_key = true;
    for (const JobCopy& jc : p->jobs) p->uniform_key &= jc.seed == p->key;
    for (const JobCopy& jc : p->jobs) p->shaped |= job_shaped(jc);
    for (const JobCopy& jc : p->jobs) p->energy |= jc.formulation == 1;
    cosmica_status st = precision == COSMICA_PREC_MIXED ? upload_tables<float>(p.get())
                                                         : upload_tables<double>(p.get());
    if (st != COSMICA_OK) return st;
    const size_t ns = p->segs.size();
    if ((st = p->mem.alloc(&p->segs_d, ns)) != COSMICA_OK) return st;
    for (int m = 0; m < 2; ++m)
        if (!p->chunks_h[m].empty() &&
            (st = p->mem.alloc(&p->chunks_d[m], p->chunks_h[m].size())) != COSMICA_OK)
            return st;
    if ((st = p->mem.alloc(&p->counters_d, 8)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->exP, total)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->exT, total)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->exNF, total)) != COSMICA_OK) return st;
    if (p->energy && (st = p->mem.alloc(&p->exL, total)) != COSMICA_OK) return st;
    if (p->want_exits) {
        if ((st = p->mem.alloc(&p->exR, total)) != COSMICA_OK) return st;
        if ((st = p->mem.alloc(&p->exTh, total)) != COSMICA_OK) return st;
        if ((st = p->mem.alloc(&p->exPh, total)) != COSMICA_OK) return st;
    }
    if ((st = p->mem.alloc(&p->hist, ns * kNHist)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->flux, ns)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->se, ns)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->mt, ns)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->steps, ns)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->ncap, ns)) != COSMICA_OK) return st;
    if ((st = p->mem.alloc(&p->nnan, ns)) != COSMICA_OK) return st;
    HIP_TRY(hipMemcpyAsync(p->segs_d, p->segs.data(), ns * sizeof(SegmentDev),
                           hipMemcpyHostToDevice, ctx->stream));
    for (int m = 0; m < 2; ++m)
        if (!p->chunks_h[m].empty())
            HIP_TRY(hipMemcpyAsync(p->chunks_d[m], p->chunks_h[m].data(),
                                   p->chunks_h[m].size() * sizeof(ChunkDev),
                                   hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *out = p.release();
    return COSMICA_OK;
}

cosmica_status cosmica_plan_execute(cosmica_plan* p, const cosmica_bins_dev* out)
{
    if (p == nullptr) return COSMICA_EINVAL;
    cosmica_ctx* ctx = p->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
    HIP_TRY(launch_fill_u32(p->counters_d, 0u, 8, ctx->stream));
    const PassDev d = pass_of(p);
    cosmica_status st = p->prec == COSMICA_PREC_MIXED ? execute_prop<float>(ctx, d)
                                                       : execute_prop<double>(ctx, d);
    if (st != COSMICA_OK) return st;
    HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
    ReduceArgs r;
    std::memset(&r, 0, sizeof(r));
    r.segs = p->segs_d;
    r.lis = p->lis_d;
    r.exP = p->exP;
    r.exT = p->exT;
    r.exNF = p->exNF;
    r.exL = p->exL;
    r.seg_base = 0;
    r.out_base = 0;
    if (out == nullptr) {
        r.hist = p->hist;
        r.flux = p->flux;
        r.flux_se = p->se;
        r.mean_t = p->mt;
        r.steps = p->steps;
        r.n_capped = p->ncap;
        r.n_nan = p->nnan;
    } else {
        r.hist = out->hist;
        r.flux = out->flux;
        r.flux_se = out->flux_se;
        r.mean_t = out->mean_exit_time_s;
        r.steps = out->steps ? out->steps : p->steps;
        r.n_capped = out->n_capped;
        r.n_nan = out->n_nan;
    }
    HIP_TRY(launch_reduce(r, (uint32_t)p->segs.size(), ctx->stream));
    // the plan keeps the step counts (the context's timings sum them)
    if (r.steps != p->steps)
        HIP_TRY(hipMemcpyAsync(p->steps, r.steps, p->segs.size() * 8, hipMemcpyDeviceToDevice,
                               ctx->stream));
    HIP_TRY(hipEventRecord(ctx->ev[2], ctx->stream));
    p->executed = true;
    p->own_out = out == nullptr;
    ctx->last_steps = r.steps;
    ctx->last_nsteps = (uint32_t)p->segs.size();
    ctx->timings_pending = true;
    ctx->timings.particles = p->total_particles;
    ctx->timings.upload_ms = 0.0;
    ctx->timings.download_ms = 0.0;
    return COSMICA_OK;
}

static cosmica_status finish_timings(cosmica_ctx* ctx)
{
    if (!ctx->timings_pending) return COSMICA_OK;
    HIP_TRY(hipEventSynchronize(ctx->ev[2]));
    float a = 0.f, b = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]));
    HIP_TRY(hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]));
    ctx->timings.propagate_ms = a;
    ctx->timings.reduce_ms = b;
    if (ctx->last_steps && ctx->last_nsteps) {
        std::vector<uint64_t> s(ctx->last_nsteps);
        HIP_TRY(hipMemcpy(s.data(), ctx->last_steps, s.size() * sizeof(uint64_t),
                          hipMemcpyDeviceToHost));
        uint64_t t = 0;
        for (uint64_t v : s) t += v;
        ctx->timings.steps = t;
    }
    ctx->timings_pending = false;
    return COSMICA_OK;
}

cosmica_status cosmica_plan_read(cosmica_plan* p, cosmica_result* results)
{
    if (p == nullptr || results == nullptr) return COSMICA_EINVAL;
    if (!p->executed || !p->own_out) return COSMICA_EINVAL;
    cosmica_ctx* ctx = p->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    cosmica_status st = finish_timings(ctx);
    if (st != COSMICA_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t ns = p->segs.size();
    std::vector<uint32_t> hist(ns * kNHist), ncap(ns), nnan(ns);
    std::vector<double> flux(ns), se(ns), mt(ns);
    std::vector<uint64_t> steps(ns);
    HIP_TRY(hipMemcpy(hist.data(), p->hist, hist.size() * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(flux.data(), p->flux, ns * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(se.data(), p->se, ns * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(mt.data(), p->mt, ns * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(steps.data(), p->steps, ns * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ncap.data(), p->ncap, ns * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(nnan.data(), p->nnan, ns * 4, hipMemcpyDeviceToHost));
    bool capped = false;
    bool need_exits = false;
    for (size_t j = 0; j < p->jobs.size(); ++j) need_exits |= results[j].exits != nullptr;
    std::vector<double> eP, eT, eR, eTh, ePh, eL;
    std::vector<uint32_t> eNF;
    if (need_exits) {
        const size_t n = p->total_particles;
        eP.resize(n);
        eT.resize(n);
        eNF.resize(n);
        HIP_TRY(hipMemcpy(eP.data(), p->exP, n * 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(eT.data(), p->exT, n * 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(eNF.data(), p->exNF, n * 4, hipMemcpyDeviceToHost));
        if (p->exL) {
            eL.resize(n);
            HIP_TRY(hipMemcpy(eL.data(), p->exL, n * 8, hipMemcpyDeviceToHost));
        }
        if (p->want_exits) {
            eR.resize(n);
            eTh.resize(n);
            ePh.resize(n);
            HIP_TRY(hipMemcpy(eR.data(), p->exR, n * 8, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(eTh.data(), p->exTh, n * 8, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(ePh.data(), p->exPh, n * 8, hipMemcpyDeviceToHost));
        }
    }
    for (size_t j = 0; j < p->jobs.size(); ++j) {
        const cosmica_result& R = results[j];
        const uint32_t s0 = p->seg_first[j];
        const size_t nb = p->jobs[j].rig.size();
        for (size_t b = 0; b < nb; ++b) {
            const size_t s = s0 + b;
            if (R.hist) std::memcpy(R.hist + b * kNHist, &hist[s * kNHist], kNHist * 4);
            if (R.flux) R.flux[b] = flux[s];
            if (R.flux_se) R.flux_se[b] = se[s];
            if (R.mean_exit_time_s) R.mean_exit_time_s[b] = mt[s];
            if (R.steps) R.steps[b] = steps[s];
            if (R.n_capped) R.n_capped[b] = ncap[s];
            if (R.n_nan) R.n_nan[b] = nnan[s];
            capped |= ncap[s] > 0;
        }
        if (R.exits) {
            const uint32_t base = p->segs[s0].out_offset;
            for (uint64_t i = 0; i < p->jobs[j].total; ++i) {
                cosmica_exit& e = R.exits[i];
                const size_t o = base + i;
                e.P = eP[o];
                e.t = eT[o];
                e.n = eNF[o] & ((1u << kFlagShift) - 1u);
                e.flags = eNF[o] >> kFlagShift;
                e.r = p->want_exits ? eR[o] : 0.0;
                e.theta = p->want_exits ? eTh[o] : 0.0;
                e.phi = p->want_exits ? ePh[o] : 0.0;
                e.loss = p->jobs[j].formulation == 1 ? eL[o] : 0.0;
            }
        }
    }
    ctx->timings.download_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return capped ? COSMICA_ESTEPCAP : COSMICA_OK;
}

cosmica_status cosmica_plan_info(const cosmica_plan* p, uint64_t* total_bins,
                                 uint64_t* total_particles, int32_t* n_jobs)
{
    if (p == nullptr) return COSMICA_EINVAL;
    if (total_bins) *total_bins = p->segs.size();
    if (total_particles) *total_particles = p->total_particles;
    if (n_jobs) *n_jobs = (int32_t)p->jobs.size();
    return COSMICA_OK;
}

static_assert(kMaxLisKnots == COSMICA_MAX_LIS_KNOTS, "LDS table size and the ABI limit agree");

cosmica_status cosmica_plan_reweight(cosmica_plan* p, uint32_t n_lis, uint32_t n_knots,
                                     double lnP0, double dlnP, const double* lnJ, double* flux,
                                     double* flux_se)
{
    if (p == nullptr || lnJ == nullptr || n_lis < 1 || n_lis > COSMICA_MAX_REWEIGHT ||
        n_knots < 2 || n_knots > (uint32_t)kMaxLisKnots || !std::isfinite(lnP0) ||
        !finite_pos(dlnP) || !p->executed)
        return COSMICA_EINVAL;
    for (size_t i = 0; i < (size_t)n_lis * n_knots; ++i)
        if (!std::isfinite(lnJ[i])) return COSMICA_EINVAL;
    cosmica_ctx* ctx = p->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    const uint32_t nb = (uint32_t)p->segs.size();
    DevSet m(ctx);
    double* tab = nullptr;
    double* fd = nullptr;
    double* sd = nullptr;
    cosmica_status st;
    const size_t nout = (size_t)n_lis * nb;
    if ((st = m.alloc(&tab, (size_t)n_lis * n_knots)) != COSMICA_OK) return st;
    if ((st = m.alloc(&fd, nout)) != COSMICA_OK) return st;
    if ((st = m.alloc(&sd, nout)) != COSMICA_OK) return st;
    HIP_TRY(hipMemcpyAsync(tab, lnJ, (size_t)n_lis * n_knots * 8, hipMemcpyHostToDevice,
                           ctx->stream));
    ReweightArgs a;
    std::memset(&a, 0, sizeof(a));
    a.segs = p->segs_d;
    a.lis = p->lis_d;
    a.exP = p->exP;
    a.exNF = p->exNF;
    a.exL = p->exL;
    a.lnJ = tab;
    a.n_lis = n_lis;
    a.n_knots = n_knots;
    a.lnP0 = lnP0;
    a.dlnP = dlnP;
    a.seg_base = 0;
    a.out_base = 0;
    a.total_bins = nb;
    a.flux = fd;
    a.flux_se = sd;
    HIP_TRY(launch_reweight(a, nb, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (flux) HIP_TRY(hipMemcpy(flux, fd, nout * 8, hipMemcpyDeviceToHost));
    if (flux_se) HIP_TRY(hipMemcpy(flux_se, sd, nout * 8, hipMemcpyDeviceToHost));
    return COSMICA_OK;
}

cosmica_status cosmica_plan_exit_range(cosmica_plan* p, uint32_t n_hist, double* p_max,
                                       uint32_t* hist)
{
    static_assert(kMaxRangeBins == COSMICA_MAX_RANGE_BINS, "range histogram limit");
    if (p == nullptr || n_hist < 1 || n_hist > COSMICA_MAX_RANGE_BINS || !p->executed)
        return COSMICA_EINVAL;
    cosmica_ctx* ctx = p->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    const uint32_t nb = (uint32_t)p->segs.size();
    DevSet m(ctx);
    double* pm = nullptr;
    uint32_t* h = nullptr;
    cosmica_status st;
    if ((st = m.alloc(&pm, nb)) != COSMICA_OK) return st;
    if ((st = m.alloc(&h, (size_t)nb * n_hist)) != COSMICA_OK) return st;
    RangeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.segs = p->segs_d;
    a.exP = p->exP;
    a.exNF = p->exNF;
    a.n_hist = n_hist;
    a.seg_base = 0;
    a.out_base = 0;
    a.total_bins = nb;
    a.p_max = pm;
    a.hist = h;
    HIP_TRY(launch_exit_range(a, nb, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (p_max) HIP_TRY(hipMemcpy(p_max, pm, (size_t)nb * 8, hipMemcpyDeviceToHost));
    if (hist) HIP_TRY(hipMemcpy(hist, h, (size_t)nb * n_hist * 4, hipMemcpyDeviceToHost));
    return COSMICA_OK;
}

void cosmica_plan_destroy(cosmica_plan* p)
{
    if (p == nullptr) return;
    (void)hipSetDevice(p->ctx->device);
    (void)hipStreamSynchronize(p->ctx->stream);
    if (p->ctx->last_nsteps && (p->ctx->last_steps == p->steps)) {
        (void)finish_timings(p->ctx);
        p->ctx->last_steps = nullptr;
        p->ctx->last_nsteps = 0;
    }
    delete p;
}

cosmica_status cosmica_run(cosmica_ctx* ctx, const cosmica_job* jobs, int32_t n_jobs,
                           cosmica_precision precision, cosmica_result* results)
{
    if (ctx == nullptr || jobs == nullptr || results == nullptr || n_jobs < 1 ||
        n_jobs > COSMICA_MAX_JOBS)
        return COSMICA_EINVAL;
    bool want = false;
    for (int j = 0; j < n_jobs; ++j) want |= results[j].exits != nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    cosmica_plan* p = nullptr;
    cosmica_status st = cosmica_plan_create(ctx, jobs, n_jobs, precision, want ? 1 : 0, &p);
    if (st != COSMICA_OK) return st;
    const double up =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st = cosmica_plan_execute(p, nullptr);
    if (st == COSMICA_OK) {
        st = cosmica_plan_read(p, results);
        ctx->timings.upload_ms = up;
    }
    cosmica_plan_destroy(p);
    return st;
}

}  // extern "C"

namespace {

// Byte offsets of cosmica_run_static's buffers within the static array.
struct StaticLayout {
    size_t jobs, regions, lis, orbit, segs, chunks, counters;
    size_t exP, exT, exNF, exL, exR, exTh, exPh, exits;
    size_t hist, flux, se, mt, steps, ncap, nnan;
    size_t total;
};

StaticLayout static_layout(int prec, uint32_t n_jobs, uint32_t n_bins, uint32_t n_orbit,
                           uint32_t n_chunks, uint64_t n, bool energy, bool exits)
{
    StaticLayout L;
    size_t at = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = at;
        at += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t jb = prec == COSMICA_PREC_MIXED ? sizeof(JobDev<float>) : sizeof(JobDev<double>);
    const size_t rb = prec == COSMICA_PREC_MIXED ? sizeof(RegionDev<float>) : sizeof(RegionDev<double>);
    L.jobs = carve(n_jobs * jb);
    L.regions = carve((size_t)n_jobs * kRegionStride * rb);
    L.lis = carve(n_jobs * sizeof(LisDev));
    L.orbit = carve(n_orbit * sizeof(OrbitDev));
    L.segs = carve(n_bins * sizeof(SegmentDev));
    L.chunks = carve(n_chunks * sizeof(ChunkDev));
    L.counters = carve(8 * sizeof(uint32_t));
    L.exP = carve(n * 8);
    L.exT = carve(n * 8);
    L.exNF = carve(n * 4);
    L.exL = carve(energy ? n * 8 : 0);
    L.exR = carve(exits ? n * 8 : 0);
    L.exTh = carve(exits ? n * 8 : 0);
    L.exPh = carve(exits ? n * 8 : 0);
    L.exits = carve(exits ? n * sizeof(ExitRecDev) : 0);
    L.hist = carve((size_t)n_bins * kNHist * 4);
    L.flux = carve(n_bins * 8);
    L.se = carve(n_bins * 8);
    L.mt = carve(n_bins * 8);
    L.steps = carve(n_bins * 8);
    L.ncap = carve(n_bins * 4);
    L.nnan = carve(n_bins * 4);
    L.total = at;
    return L;
}

template <typename R>
cosmica_status run_static(cosmica_ctx* ctx, const cosmica_job* jobs, uint32_t n_jobs, int prec,
                          cosmica_result* results)
{
    StaticHost& H = *ctx->stat;
    // sizes of the work
    uint32_t n_bins = 0, n_orbit = 0;
    uint64_t total = 0, model_particles[2] = {0, 0};
    bool energy = false, shaped = false, exits = false, ukey = true;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        const cosmica_job& J = jobs[j];
        n_bins += (uint32_t)J.n_bins;
        n_orbit += J.n_orbit;
        for (int b = 0; b < J.n_bins; ++b) {
            total += J.particles_per_bin[b];
            model_particles[J.helio->model] += J.particles_per_bin[b];
        }
        energy |= J.formulation == 1;
        shaped |= helio_shaped(*J.helio);
        exits |= results[j].exits != nullptr;
        ukey &= J.seed == jobs[0].seed;
        if (n_bins > COSMICA_STATIC_MAX_BINS || n_orbit > COSMICA_STATIC_MAX_ORBIT)
            return COSMICA_ESCRATCH;
    }
    if (total >= (1ull << 32)) return COSMICA_EINVAL;
    // segments (jobs x bins) and their expected steps per particle
    uint32_t off = 0, ns = 0;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        const cosmica_job& J = jobs[j];
        H.seg_first[j] = ns;
        for (int b = 0; b < J.n_bins; ++b, ++ns) {
            SegmentDev& g = H.segs[ns];
            std::memset(&g, 0, sizeof(g));
            g.P0 = J.rigidity_gv[b];
            g.job = j;
            g.bin = J.bin_offset + (uint32_t)b;
            g.count = J.particles_per_bin[b];
            g.out_offset = off;
            off += J.particles_per_bin[b];
            H.cost[ns] = expected_steps(*J.helio, *J.species, J.rigidity_gv[b]);
        }
    }
    // refill chunks of each model group in the launch's queue order; the chunk
    // is enlarged where needed to keep the queue within the staging (the
    // results do not depend on the chunk size)
    const uint64_t room = kStaticMaxChunks - COSMICA_STATIC_MAX_BINS;
    uint32_t nc = 0, first[2] = {0, 0}, nch[2] = {0, 0};
    for (int m = 0; m < 2; ++m) {
        const cosmica_launch& L = ctx->launch[m][prec];
        const uint32_t c =
            (uint32_t)std::max<uint64_t>((uint64_t)std::max(1, L.chunk), (total + room - 1) / room);
        uint32_t k = 0;
        for (uint32_t i = 0; i < ns; ++i)
            if (jobs[H.segs[i].job].helio->model == m) H.ids[k++] = i;
        const SegmentDev* sg = H.segs;
        const double* cost = H.cost;
        if (L.order == 2)
            std::sort(H.ids, H.ids + k, [&](uint32_t a, uint32_t b) {
                if (cost[a] != cost[b]) return cost[a] > cost[b];
                if (sg[a].count != sg[b].count) return sg[a].count > sg[b].count;
                return a < b;
            });
        else if (L.order == 1)
            std::sort(H.ids, H.ids + k, [&](uint32_t a, uint32_t b) {
                if (sg[a].count != sg[b].count) return sg[a].count > sg[b].count;
                return a < b;
            });
        first[m] = nc;
        for (uint32_t i = 0; i < k; ++i) {
            const uint32_t seg = H.ids[i];
            for (uint32_t f = 0; f < sg[seg].count; f += c) {
                ChunkDev& ch = H.chunks[nc++];
                ch.seg = seg;
                ch.first = f;
                ch.count = std::min(c, sg[seg].count - f);
                ch.pad0 = 0;
            }
        }
        nch[m] = nc - first[m];
    }
    const StaticLayout Lo = static_layout(prec, n_jobs, n_bins, n_orbit, nc, total, energy, exits);
    if (Lo.total > COSMICA_STATIC_BYTES) return COSMICA_ESCRATCH;
    // device tables
    JobDev<R>* jh = (JobDev<R>*)H.jobs;
    RegionDev<R>* rh = (RegionDev<R>*)H.regions;
    uint32_t o = 0;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        make_tables<R>(head_of(jobs[j]), &jh[j], &rh[(size_t)j * kRegionStride], &H.lis[j]);
        jh[j].orbit_off = o;
        for (uint32_t k = 0; k < jobs[j].n_orbit; ++k, ++o) {
            const double* q = jobs[j].orbit + 3 * (size_t)k;
            H.orbit[o] = OrbitDev{q[0], q[1], q[2], 0.0};
        }
    }

    HIP_TRY(hipSetDevice(ctx->device));
    unsigned char* base = (unsigned char*)static_base(ctx->device);
    if (base == nullptr) return COSMICA_EDEVICE;
    std::lock_guard<std::mutex> lk(g_static_call_mu[ctx->device]);
    hipStream_t st = ctx->stream;
    const auto t0 = std::chrono::steady_clock::now();
    auto at = [&](size_t offset) { return (void*)(base + offset); };
    HIP_TRY(hipMemcpyAsync(at(Lo.jobs), jh, n_jobs * sizeof(JobDev<R>), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(at(Lo.regions), rh, (size_t)n_jobs * kRegionStride * sizeof(RegionDev<R>),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(at(Lo.lis), H.lis, n_jobs * sizeof(LisDev), hipMemcpyHostToDevice, st));
    if (n_orbit)
        HIP_TRY(hipMemcpyAsync(at(Lo.orbit), H.orbit, n_orbit * sizeof(OrbitDev),
                               hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(at(Lo.segs), H.segs, n_bins * sizeof(SegmentDev), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(at(Lo.chunks), H.chunks, nc * sizeof(ChunkDev), hipMemcpyHostToDevice, st));
    // the array keeps the last call's contents: the queue cursors start at
    // zero, and momentum-form particles leave the loss records unwritten
    HIP_TRY(launch_fill_u32((uint32_t*)at(Lo.counters), 0u, 8, st));
    if (energy) HIP_TRY(launch_fill_u32((uint32_t*)at(Lo.exL), 0u, (uint32_t)(2 * total), st));
    const double up =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();

    PassDev d;
    d.jobs = at(Lo.jobs);
    d.regions = at(Lo.regions);
    d.orbit = (const OrbitDev*)at(Lo.orbit);
    d.segs = (const SegmentDev*)at(Lo.segs);
    for (int m = 0; m < 2; ++m) {
        d.chunks[m] = (const ChunkDev*)at(Lo.chunks) + first[m];
        d.n_chunks[m] = nch[m];
        d.model_particles[m] = model_particles[m];
    }
    d.counters = (uint32_t*)at(Lo.counters);
    d.exP = (double*)at(Lo.exP);
    d.exT = (double*)at(Lo.exT);
    d.exNF = (uint32_t*)at(Lo.exNF);
    d.exL = energy ? (double*)at(Lo.exL) : nullptr;
    d.exR = exits ? (double*)at(Lo.exR) : nullptr;
    d.exTh = exits ? (double*)at(Lo.exTh) : nullptr;
    d.exPh = exits ? (double*)at(Lo.exPh) : nullptr;
    d.uniform_key = ukey;
    d.shaped = shaped;
    d.energy = energy;
    d.key = jobs[0].seed;
    d.prec = prec;
    HIP_TRY(hipEventRecord(ctx->ev[0], st));
    cosmica_status s = execute_prop<R>(ctx, d);
    if (s != COSMICA_OK) return s;
    HIP_TRY(hipEventRecord(ctx->ev[1], st));
    ReduceArgs r;
    std::memset(&r, 0, sizeof(r));
    r.segs = d.segs;
    r.lis = (const LisDev*)at(Lo.lis);
    r.exP = d.exP;
    r.exT = d.exT;
    r.exNF = d.exNF;
    r.exL = d.exL;
    r.seg_base = 0;
    r.out_base = 0;
    r.hist = (uint32_t*)at(Lo.hist);
    r.flux = (double*)at(Lo.flux);
    r.flux_se = (double*)at(Lo.se);
    r.mean_t = (double*)at(Lo.mt);
    r.steps = (uint64_t*)at(Lo.steps);
    r.n_capped = (uint32_t*)at(Lo.ncap);
    r.n_nan = (uint32_t*)at(Lo.nnan);
    HIP_TRY(launch_reduce(r, n_bins, st));
    HIP_TRY(hipEventRecord(ctx->ev[2], st));
    ExitRecDev* ex = (ExitRecDev*)at(Lo.exits);
    if (exits)
        HIP_TRY(launch_pack_exits(d.exP, d.exT, d.exNF, d.exL, d.exR, d.exTh, d.exPh,
                                  (uint32_t)total, ex, st));
    HIP_TRY(hipStreamSynchronize(st));
    // results straight into the caller's buffers (a job's bins and particles
    // are contiguous)
    const auto t1 = std::chrono::steady_clock::now();
    HIP_TRY(hipMemcpy(H.ncap, r.n_capped, n_bins * 4, hipMemcpyDeviceToHost));
    bool capped = false;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        const cosmica_result& R_ = results[j];
        const uint32_t s0 = H.seg_first[j];
        const size_t nb = (size_t)jobs[j].n_bins;
        if (R_.hist)
            HIP_TRY(hipMemcpy(R_.hist, r.hist + (size_t)s0 * kNHist, nb * kNHist * 4,
                              hipMemcpyDeviceToHost));
        if (R_.flux) HIP_TRY(hipMemcpy(R_.flux, r.flux + s0, nb * 8, hipMemcpyDeviceToHost));
        if (R_.flux_se) HIP_TRY(hipMemcpy(R_.flux_se, r.flux_se + s0, nb * 8, hipMemcpyDeviceToHost));
        if (R_.mean_exit_time_s)
            HIP_TRY(hipMemcpy(R_.mean_exit_time_s, r.mean_t + s0, nb * 8, hipMemcpyDeviceToHost));
        if (R_.steps) HIP_TRY(hipMemcpy(R_.steps, r.steps + s0, nb * 8, hipMemcpyDeviceToHost));
        if (R_.n_nan) HIP_TRY(hipMemcpy(R_.n_nan, r.n_nan + s0, nb * 4, hipMemcpyDeviceToHost));
        if (R_.n_capped) std::memcpy(R_.n_capped, H.ncap + s0, nb * 4);
        for (size_t b = 0; b < nb; ++b) capped |= H.ncap[s0 + b] > 0;
        if (R_.exits) {
            uint64_t n = 0;
            for (size_t b = 0; b < nb; ++b) n += jobs[j].particles_per_bin[b];
            HIP_TRY(hipMemcpy(R_.exits, ex + H.segs[s0].out_offset, n * sizeof(ExitRecDev),
                              hipMemcpyDeviceToHost));
        }
    }
    ctx->last_steps = r.steps;
    ctx->last_nsteps = n_bins;
    ctx->timings_pending = true;
    ctx->timings.particles = total;
    ctx->timings.upload_ms = up;
    ctx->timings.download_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
    return capped ? COSMICA_ESTEPCAP : COSMICA_OK;
}

}  // namespace

extern "C" {

cosmica_status cosmica_run_static(cosmica_ctx* ctx, const cosmica_job* jobs, int32_t n_jobs,
                                  cosmica_precision precision, cosmica_result* results)
{
    if (ctx == nullptr || jobs == nullptr || results == nullptr || n_jobs < 1) return COSMICA_EINVAL;
    if (precision != COSMICA_PREC_FP64 && precision != COSMICA_PREC_MIXED) return COSMICA_EINVAL;
    for (int j = 0; j < n_jobs && j < COSMICA_MAX_JOBS; ++j)
        if (validate(&jobs[j]) != COSMICA_OK) return COSMICA_EINVAL;
    if (n_jobs > COSMICA_STATIC_MAX_JOBS) return COSMICA_ESCRATCH;
    if (!ctx->stat) return COSMICA_EDEVICE;
    return precision == COSMICA_PREC_MIXED
               ? run_static<float>(ctx, jobs, (uint32_t)n_jobs, precision, results)
               : run_static<double>(ctx, jobs, (uint32_t)n_jobs, precision, results);
}

cosmica_status cosmica_set_launch(cosmica_ctx* ctx, cosmica_model model,
                                  cosmica_precision precision, const cosmica_launch* cfg)
{
    if (ctx == nullptr || cfg == nullptr || (model != 0 && model != 1) ||
        (precision != 0 && precision != 1) || !launch_ok(*cfg))
        return COSMICA_EINVAL;
    ctx->launch[model][precision] = *cfg;
    return COSMICA_OK;
}

cosmica_status cosmica_get_launch(cosmica_ctx* ctx, cosmica_model model,
                                  cosmica_precision precision, cosmica_launch* cfg)
{
    if (ctx == nullptr || cfg == nullptr || (model != 0 && model != 1) ||
        (precision != 0 && precision != 1))
        return COSMICA_EINVAL;
    *cfg = ctx->launch[model][precision];
    return COSMICA_OK;
}

cosmica_status cosmica_get_timings(cosmica_ctx* ctx, cosmica_timings* out)
{
    if (ctx == nullptr || out == nullptr) return COSMICA_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    cosmica_status st = finish_timings(ctx);
    if (st != COSMICA_OK) return st;
    *out = ctx->timings;
    return COSMICA_OK;
}

cosmica_status cosmica_probe_rng(cosmica_ctx* ctx, uint64_t seed, uint32_t c0, uint32_t c1,
                                 uint32_t c2, uint32_t c3, uint32_t n, uint32_t* words,
                                 double* z64, float* z32)
{
    if (ctx == nullptr || n == 0) return COSMICA_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    DevSet m(ctx);
    uint32_t* w = nullptr;
    double* a = nullptr;
    float* b = nullptr;
    cosmica_status st;
    if (words && (st = m.alloc(&w, 4 * (size_t)n)) != COSMICA_OK) return st;
    if (z64 && (st = m.alloc(&a, 3 * (size_t)n)) != COSMICA_OK) return st;
    if (z32 && (st = m.alloc(&b, 3 * (size_t)n)) != COSMICA_OK) return st;
    HIP_TRY(launch_probe_rng((uint32_t)seed, (uint32_t)(seed >> 32), c0, c1, c2, c3, n, w, a, b,
                             ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (words) HIP_TRY(hipMemcpy(words, w, 16 * (size_t)n, hipMemcpyDeviceToHost));
    if (z64) HIP_TRY(hipMemcpy(z64, a, 24 * (size_t)n, hipMemcpyDeviceToHost));
    if (z32) HIP_TRY(hipMemcpy(z32, b, 12 * (size_t)n, hipMemcpyDeviceToHost));
    return COSMICA_OK;
}

cosmica_status cosmica_probe_coeffs(cosmica_ctx* ctx, const cosmica_job* job,
                                    cosmica_precision precision, uint32_t n, const double* pts,
                                    double* out)
{
    if (ctx == nullptr || pts == nullptr || out == nullptr || n == 0) return COSMICA_EINVAL;
    if (validate(job) != COSMICA_OK || job->helio->model != COSMICA_MODEL_3D) return COSMICA_EINVAL;
    if (precision != COSMICA_PREC_FP64 && precision != COSMICA_PREC_MIXED) return COSMICA_EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
        const double* q = pts + 4 * (size_t)i;
        if (!finite_pos(q[0]) || !finite_pos(q[1]) || !(q[2] > 0.0) || !(q[2] < kPiH) ||
            !std::isfinite(q[3]))
            return COSMICA_EINVAL;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    const JobCopy jc = copy_job(job);
    DevSet m(ctx);
    double* pd = nullptr;
    double* od = nullptr;
    cosmica_status st;
    if ((st = m.alloc(&pd, 4 * (size_t)n)) != COSMICA_OK) return st;
    if ((st = m.alloc(&od, (size_t)kProbeOut * n)) != COSMICA_OK) return st;
    HIP_TRY(hipMemcpy(pd, pts, 32 * (size_t)n, hipMemcpyHostToDevice));
    LisDev lis;
    if (precision == COSMICA_PREC_FP64) {
        JobDev<double> J;
        std::vector<RegionDev<double>> R(kRegionStride);
        make_tables<double>(head_of(jc), &J, R.data(), &lis);
        JobDev<double>* jd = nullptr;
        RegionDev<double>* rd = nullptr;
        if ((st = m.alloc(&jd, 1)) != COSMICA_OK) return st;
        if ((st = m.alloc(&rd, kRegionStride)) != COSMICA_OK) return st;
        HIP_TRY(hipMemcpy(jd, &J, sizeof(J), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(rd, R.data(), R.size() * sizeof(R[0]), hipMemcpyHostToDevice));
        HIP_TRY(launch_probe_coeffs_fp64(jd, rd, pd, n, od, ctx->stream));
    } else {
        JobDev<float> J;
        std::vector<RegionDev<float>> R(kRegionStride);
        make_tables<float>(head_of(jc), &J, R.data(), &lis);
        JobDev<float>* jd = nullptr;
        RegionDev<float>* rd = nullptr;
        if ((st = m.alloc(&jd, 1)) != COSMICA_OK) return st;
        if ((st = m.alloc(&rd, kRegionStride)) != COSMICA_OK) return st;
        HIP_TRY(hipMemcpy(jd, &J, sizeof(J), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(rd, R.data(), R.size() * sizeof(R[0]), hipMemcpyHostToDevice));
        HIP_TRY(launch_probe_coeffs_mixed(jd, rd, pd, n, od, ctx->stream));
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(out, od, 8 * (size_t)kProbeOut * n, hipMemcpyDeviceToHost));
    return COSMICA_OK;
}

cosmica_status cosmica_probe_locate(cosmica_ctx* ctx, const cosmica_job* job,
                                    cosmica_precision precision, uint32_t n, const double* pts,
                                    int32_t* region, int32_t* outside)
{
    if (ctx == nullptr || pts == nullptr || region == nullptr || outside == nullptr || n == 0)
        return COSMICA_EINVAL;
    if (validate(job) != COSMICA_OK || job->helio->model != COSMICA_MODEL_3D) return COSMICA_EINVAL;
    if (precision != COSMICA_PREC_FP64 && precision != COSMICA_PREC_MIXED) return COSMICA_EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
        const double* q = pts + 3 * (size_t)i;
        if (!(q[0] >= 0.0) || !std::isfinite(q[0]) || !(q[1] >= 0.0) || !(q[1] <= kPiH) ||
            !(q[2] >= 0.0) || !(q[2] < 2.0 * kPiH))
            return COSMICA_EINVAL;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    const JobCopy jc = copy_job(job);
    DevSet m(ctx);
    double* pd = nullptr;
    int32_t* rd_out = nullptr;
    int32_t* od = nullptr;
    cosmica_status st;
    if ((st = m.alloc(&pd, 3 * (size_t)n)) != COSMICA_OK) return st;
    if ((st = m.alloc(&rd_out, n)) != COSMICA_OK) return st;
    if ((st = m.alloc(&od, n)) != COSMICA_OK) return st;
    HIP_TRY(hipMemcpy(pd, pts, 24 * (size_t)n, hipMemcpyHostToDevice));
    LisDev lis;
    if (precision == COSMICA_PREC_FP64) {
        JobDev<double> J;
        std::vector<RegionDev<double>> R(kRegionStride);
        make_tables<double>(head_of(jc), &J, R.data(), &lis);
        JobDev<double>* jd = nullptr;
        RegionDev<double>* rg = nullptr;
        if ((st = m.alloc(&jd, 1)) != COSMICA_OK) return st;
        if ((st = m.alloc(&rg, kRegionStride)) != COSMICA_OK) return st;
        HIP_TRY(hipMemcpy(jd, &J, sizeof(J), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(rg, R.data(), R.size() * sizeof(R[0]), hipMemcpyHostToDevice));
        HIP_TRY(launch_probe_locate_fp64(jd, rg, pd, n, rd_out, od, ctx->stream));
    } else {
        JobDev<float> J;
        std::vector<RegionDev<float>> R(kRegionStride);
        make_tables<float>(head_of(jc), &J, R.data(), &lis);
        JobDev<float>* jd = nullptr;
        RegionDev<float>* rg = nullptr;
        if ((st = m.alloc(&jd, 1)) != COSMICA_OK) return st;
        if ((st = m.alloc(&rg, kRegionStride)) != COSMICA_OK) return st;
        HIP_TRY(hipMemcpy(jd, &J, sizeof(J), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(rg, R.data(), R.size() * sizeof(R[0]), hipMemcpyHostToDevice));
        HIP_TRY(launch_probe_locate_mixed(jd, rg, pd, n, rd_out, od, ctx->stream));
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(region, rd_out, 4 * (size_t)n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(outside, od, 4 * (size_t)n, hipMemcpyDeviceToHost));
    return COSMICA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Launch-shape tuner: the warps-per-block sweep of the paper (Sec. VI,
// Version 2) widened to workgroup size, resident workgroups per CU and the
// refill chunk, timed on a calibration batch.
// ---------------------------------------------------------------------------
namespace {

struct Calib {
    cosmica_helio helio;
    cosmica_species species;
    std::vector<double> rig;
    std::vector<uint32_t> cnt;
    cosmica_job job;
};

void make_calibration(int model, uint32_t per_bin, Calib* c)
{
    std::memset(&c->helio, 0, sizeof(c->helio));
    cosmica_helio& h = c->helio;
    h.model = model;
    h.n_regions = model == 1 ? 15 : 1;
    for (int k = 0; k < h.n_regions; ++k) {
        // a smooth, deterministic spread of shell parameters
        h.kappa0_cm2_s[k] = 1.0e22 + 1.0e21 * (double)(k % 7);
        h.v_slow_km_s[k] = 380.0 + 20.0 * (double)(k % 5);
        h.tilt_deg[k] = 15.0 + 3.0 * (double)k;
    }
    h.v_fast_km_s = 760.0;
    h.r_boundary_au = model == 1 ? 120.0 : 100.0;
    h.r0_au = 1.0;
    h.theta0_rad = 0.5 * kPiH;
    h.phi0_rad = 0.0;
    h.b0_nT = 5.0;
    h.v_ref_km_s = 400.0;
    h.omega_rad_s = 2.66e-6;
    h.kperp_over_kpar = model == 1 ? 0.02 : 1.0;
    h.polarity = 1;
    h.drift = model == 1 ? 1 : 0;
    h.hcs = model == 1 ? 1 : 0;
    h.dt_max_s = 5e4;
    h.dt_diff_frac = 0.02;
    h.dt_adv_frac = model == 1 ? 0.1 : 0.0;
    c->species = cosmica_species{0.93827208816, 1, 1, 1.9e4, 2.78};
    const int nb = 16;
    c->rig.resize(nb);
    c->cnt.assign(nb, per_bin);
    for (int b = 0; b < nb; ++b) c->rig[b] = 0.1 * std::pow(1000.0, (double)b / (nb - 1));
    c->job = cosmica_job{&c->helio, &c->species, c->rig.data(), c->cnt.data(), nb, 0u, 12345ull,
                         0u, 0u};  // tag 0, seed 12345, default cap, bin offset 0
}

#ifndef COSMICA_KERNEL_ID
#define COSMICA_KERNEL_ID "unversioned"
#endif

// Device architecture plus the digest of the kernel source the library was
// built from: a launch shape tuned for other kernel code is not reused.
std::string tune_key(cosmica_ctx* ctx, int model, int prec)
{
    std::string a = ctx->arch + "@" + COSMICA_KERNEL_ID;
    for (char& ch : a)
        if (ch == ' ') ch = '_';
    return a + " " + std::to_string(model) + " " + std::to_string(prec);
}

bool cache_lookup(const char* path, const std::string& key, cosmica_launch* L)
{
    if (path == nullptr) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string arch;
        int m, q;
        cosmica_launch c;
        double rate;
        if (!(is >> arch >> m >> q >> c.block >> c.blocks_per_cu >> c.chunk >> c.order >> rate))
            continue;
        if (arch + " " + std::to_string(m) + " " + std::to_string(q) == key && launch_ok(c)) {
            *L = c;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const cosmica_launch& L, double rate)
{
    if (path == nullptr) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {
            std::istringstream is(line);
            std::string arch;
            int m, q;
            if (!(is >> arch >> m >> q)) continue;
            if (arch + " " + std::to_string(m) + " " + std::to_string(q) != key)
                keep.push_back(line);
        }
    }
    std::ofstream f(path, std::ios::trunc);
    for (auto& l : keep) f << l << "\n";
    f << key << " " << L.block << " " << L.blocks_per_cu << " " << L.chunk << " " << L.order
      << " " << rate << "\n";
}

}  // namespace

namespace {

// Steps/s of one launch shape on a calibration batch (second of two runs).
cosmica_status time_shape(cosmica_ctx* ctx, const cosmica_job* jobs, int n_jobs, int model,
                          int precision, const cosmica_launch& c, double* rate)
{
    ctx->launch[model][precision] = c;
    cosmica_plan* p = nullptr;
    cosmica_status st = cosmica_plan_create(ctx, jobs, n_jobs, (cosmica_precision)precision, 0, &p);
    if (st != COSMICA_OK) return st;
    *rate = 0.0;
    for (int rep = 0; rep < 2 && st == COSMICA_OK; ++rep) {
        st = cosmica_plan_execute(p, nullptr);
        cosmica_timings t;
        if (st == COSMICA_OK) st = cosmica_get_timings(ctx, &t);
        if (st == COSMICA_OK && rep == 1 && t.propagate_ms > 0.0)
            *rate = (double)t.steps / (t.propagate_ms * 1e-3);
    }
    cosmica_plan_destroy(p);
    return st;
}

// Coordinate sweep: workgroup size, then resident workgroups per CU, then the
// refill chunk, then the queue order, each from the best shape so far.
cosmica_status sweep(cosmica_ctx* ctx, const cosmica_job* jobs, int n_jobs, int model,
                     int precision, const char* cache_path)
{
    const std::string key = tune_key(ctx, model, precision);
    const cosmica_launch saved = ctx->launch[model][precision];
    // Start from full residency, 32-particle chunks and queue order 2 (long
    // paths kept out of the tail); the other orders are tried last.  Timings
    // of one shape vary by about 1% from run to run as the device warms, so
    // another shape replaces the best only when it is more than 1% faster.
    cosmica_launch best{256, 0, 32, 2};
    double best_rate = -1.0;
    auto consider = [&](const cosmica_launch& c) -> cosmica_status {
        if (!launch_ok(c)) return COSMICA_OK;
        double rate = 0.0;
        cosmica_status st = time_shape(ctx, jobs, n_jobs, model, precision, c, &rate);
        if (st != COSMICA_OK) return st;
        if (best_rate < 0.0 || rate > 1.01 * best_rate) {
            best_rate = rate;
            best = c;
        }
        return COSMICA_OK;
    };
    cosmica_status st = COSMICA_OK;
    for (int blk : {256, 128, 64})
        if ((st = consider(cosmica_launch{blk, 0, best.chunk, best.order})) != COSMICA_OK) break;
    if (st == COSMICA_OK) {
        int occ = 0;
        bool shaped_jobs = false, energy_jobs = false, one_key = true;
        for (int j = 0; j < n_jobs; ++j) {
            shaped_jobs |= job_shaped(copy_job(&jobs[j]));
            energy_jobs |= jobs[j].formulation == 1;
            one_key &= jobs[j].seed == jobs[0].seed;
        }
        if (occupancy_propagate(model, precision, best.block, shaped_jobs ? 1 : 0,
                                energy_jobs ? 1 : 0, one_key ? 1 : 0, &occ) != hipSuccess ||
            occ < 1)
            occ = 1;
        const cosmica_launch base = best;
        for (int bpc : {occ - occ / 4, occ / 2})
            if (bpc >= 1 && bpc < occ &&
                (st = consider(cosmica_launch{base.block, bpc, base.chunk, base.order})) != COSMICA_OK)
                break;
    }
    if (st == COSMICA_OK) {
        const cosmica_launch base = best;
        for (int ch : {32, 128, 512, 1024}) {
            if (ch == base.chunk) continue;
            st = consider(cosmica_launch{base.block, base.blocks_per_cu, ch, base.order});
            if (st != COSMICA_OK) break;
        }
    }
    if (st == COSMICA_OK) {
        const cosmica_launch base = best;
        for (int o = 0; o <= 2 && st == COSMICA_OK; ++o)
            if (o != base.order)
                st = consider(cosmica_launch{base.block, base.blocks_per_cu, base.chunk, o});
    }
    if (st != COSMICA_OK) {
        ctx->launch[model][precision] = saved;
        return st;
    }
    ctx->launch[model][precision] = best;
    cache_store(cache_path, key, best, best_rate);
    return COSMICA_OK;
}

}  // namespace

extern "C" cosmica_status cosmica_tune(cosmica_ctx* ctx, cosmica_model model,
                                       cosmica_precision precision, const char* cache_path)
{
    if (ctx == nullptr || (model != 0 && model != 1) || (precision != 0 && precision != 1))
        return COSMICA_EINVAL;
    cosmica_launch L;
    if (cache_lookup(cache_path, tune_key(ctx, model, precision), &L)) {
        ctx->launch[model][precision] = L;
        return COSMICA_OK;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    // about two resident waves' worth of particles per SIMD at full occupancy
    const uint64_t lanes = (uint64_t)ctx->num_cus * 4 * 64 * 8;
    Calib cal;
    make_calibration(model, (uint32_t)std::max<uint64_t>(64, 2 * lanes / 16), &cal);
    return sweep(ctx, &cal.job, 1, model, precision, cache_path);
}

extern "C" cosmica_status cosmica_tune_jobs(cosmica_ctx* ctx, const cosmica_job* jobs,
                                            int32_t n_jobs, cosmica_precision precision,
                                            uint64_t sample_particles, const char* cache_path)
{
    if (ctx == nullptr || jobs == nullptr || n_jobs < 1 || sample_particles < 1 ||
        (precision != 0 && precision != 1))
        return COSMICA_EINVAL;
    uint64_t total = 0;
    for (int j = 0; j < n_jobs; ++j) {
        if (validate(&jobs[j]) != COSMICA_OK) return COSMICA_EINVAL;
        if (jobs[j].helio->model != jobs[0].helio->model) return COSMICA_EINVAL;
        for (int b = 0; b < jobs[j].n_bins; ++b) total += jobs[j].particles_per_bin[b];
    }
    const int model = jobs[0].helio->model;
    cosmica_launch L;
    if (cache_lookup(cache_path, tune_key(ctx, model, precision), &L)) {
        ctx->launch[model][precision] = L;
        return COSMICA_OK;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    // every k-th whole job (k odd, so a batch ordered set x species keeps all
    // species), bins at their full sizes: the sample keeps the refill-chunk and
    // job-mixing structure of the real batch
    uint64_t k = (uint64_t)std::llround((double)total / (double)sample_particles);
    if (k < 1) k = 1;
    if (k > 1 && k % 2 == 0) ++k;
    std::vector<cosmica_job> sample;
    for (int j = 0; j < n_jobs; j += (int)k) sample.push_back(jobs[j]);
    return sweep(ctx, sample.data(), (int)sample.size(), model, precision, cache_path);
}

// ---------------------------------------------------------------------------
// Serving: continuous batching over bounded slices of the persistent kernel.
// Requests are admitted while their exit records fit in the device pool; the
// particles of every admitted request share the same launches, and particles
// still inside at the end of a slice are parked (bit-exact) and resumed first
// in the next one.  The work queue, the parked particles and every cursor over
// them stay on the device, so the worker enqueues a group's next slice before
// it reads what the previous one did, and the device runs slices back to back.
// ---------------------------------------------------------------------------
struct Req {
    uint64_t ticket = 0;
    JobCopy job;
    int prec = 0;
    int model = 0;
    cosmica_result res{};
    int state = 0;  // 0 queued, 1 resident, 2 done
    cosmica_status status = COSMICA_OK;
    bool cancel = false;
    bool cancel_sent = false;
    int slot = -1;
    uint64_t ex0 = 0;
    uint64_t ring_end = 0;      // queue position just past the request's last chunk
    uint64_t first_slice = 0;   // first slice of its group that can hold its particles
    uint64_t cancel_slice = 0;  // first slice of its group that sees its cancel flag
    // reduced results on their way to the host, and the event that ends the copy
    unsigned char* staged = nullptr;
    hipEvent_t staged_ev = nullptr;
};

// Pinned host memory and events of the serving worker.
struct ServeHost {
    // Uploads go through two pinned arenas used by alternate rounds of the
    // worker.  The uploads of round i are enqueued before round i's slices,
    // and round i+1 waits for those slices, so round i+2 finds arena i % 2 free.
    static constexpr size_t kArenaBytes = 16u << 20;
    unsigned char* arena[2] = {nullptr, nullptr};
    int cur = 0;
    size_t used = 0;
    // per finished request: its reduced bins (at most kBinsPerSlot of them)
    static constexpr size_t kResultBytes = 40960;
    std::vector<unsigned char*> blocks, free_blocks;
    std::vector<hipEvent_t> events, free_events;
    hipEvent_t round_ev[2] = {nullptr, nullptr};
    std::vector<Req*> finishing;  // results being copied to the host
    ~ServeHost()
    {
        for (unsigned char* a : arena)
            if (a) (void)hipHostFree(a);
        for (unsigned char* b : blocks) (void)hipHostFree(b);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipEvent_t e : round_ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct ServeGroup {
    static constexpr uint32_t kSlots = 256;
    static constexpr uint32_t kBinsPerSlot = 64;
    // Control words on the device: the queue head (64-bit), per slice parity p
    // the words at kCtlPark + 4 p: [particles parked, chunk remainders, resume
    // cursor, remainder cursor]; an overflow flag; finished particles per slot.
    // A slice of parity p resumes the lists of parity 1 - p and writes those of
    // parity p; its closing kernel clears the counters of parity 1 - p.
    static constexpr uint32_t kCtlPark = 4, kCtlOverflow = 12, kCtlDone = 16;
    static constexpr uint32_t kCtlWords = kCtlDone + kSlots;
    int model = 0, prec = 0;
    cosmica_ctx* ctx = nullptr;
    DevSet mem;
    void* jobs_d = nullptr;
    void* regions_d = nullptr;
    LisDev* lis_d = nullptr;
    OrbitDev* orbit_d = nullptr;  // kSlots * COSMICA_MAX_ORBIT positions
    uint32_t* cancel_d = nullptr;
    SegmentDev* segs_d = nullptr;
    uint32_t* ctl_d = nullptr;
    uint32_t* snap_h = nullptr;  // pinned: the control words after each slice, by parity
    // Work queue of the admitted requests' chunks: a ring of ring_cap (a power
    // of two) entries on the device, position c at c & (ring_cap - 1).  The host
    // appends at q_tail; the device advances the head.  q_head is the head as
    // of the last slice the worker has read (a lower bound of the device's).
    ChunkDev* ring_d = nullptr;
    uint64_t ring_cap = 0;
    uint64_t q_head = 0, q_tail = 0;
    uint64_t seq = 0;            // slices enqueued
    uint64_t in_flight = 0;      // particles parked after the last slice read
    uint64_t pool_cap = 0;
    double* exL = nullptr;  // energy form: allocated when the first energy-form request arrives
    double* exP = nullptr;
    double* exT = nullptr;
    uint32_t* exNF = nullptr;
    ParkDev park[2] = {};
    uint32_t park_cap = 0;
    ChunkDev* left_d[2] = {nullptr, nullptr};
    uint32_t left_cap = 0;
    SliceDev slice_h[2] = {};    // the lists of a slice of each parity
    SliceDev* slice_d = nullptr;  // the same on the device
    uint32_t* r_hist = nullptr;
    double* r_flux = nullptr;
    double* r_se = nullptr;
    double* r_mt = nullptr;
    uint64_t* r_steps = nullptr;
    uint32_t* r_ncap = nullptr;
    uint32_t* r_nnan = nullptr;
    std::vector<int> free_slots;
    std::vector<SegmentDev> segs_h;
    std::map<uint64_t, uint64_t> free_ranges;  // offset -> length of free pool ranges
    std::vector<Req*> resident;
    std::vector<Req*> releasing;               // cancelled, freed once none of their work is left
    int grid = 0, block = 256;
    int grid_var[4] = {0, 0, 0, 0};  // by (shaped | 2 energy)
    explicit ServeGroup(cosmica_ctx* c) : ctx(c), mem(c) {}
    ~ServeGroup()
    {
        if (snap_h) (void)hipHostFree(snap_h);
    }
    static uint32_t park_word(int parity, int k) { return kCtlPark + 4u * (uint32_t)parity + (uint32_t)k; }
};

cosmica_ctx::~cosmica_ctx() = default;

namespace {

// A serving slice ends after COSMICA_SLICE_MS milliseconds (default 6; the
// device's constant-rate clock, read by every wave) or, if set, after
// COSMICA_SLICE_STEPS steps of each wave, whichever comes first.
uint32_t slice_steps()
{
    const char* e = std::getenv("COSMICA_SLICE_STEPS");
    long v = e ? std::strtol(e, nullptr, 10) : 0;
    return v > 0 ? (uint32_t)std::min<long>(v, 0xfffffffel) : 0xffffffffu;
}

uint64_t slice_ticks(const cosmica_ctx* ctx)
{
    const char* e = std::getenv("COSMICA_SLICE_MS");
    double ms = e ? std::strtod(e, nullptr) : 0.0;
    if (!(ms > 0.0)) ms = 6.0;
    if (ctx->wall_khz <= 0) return 0;
    return std::max<uint64_t>(1, (uint64_t)(ms * (double)ctx->wall_khz));
}

uint64_t pool_particles(cosmica_ctx* ctx)
{
    const char* e = std::getenv("COSMICA_SERVE_POOL");
    long long v = e ? std::strtoll(e, nullptr, 10) : 0;
    uint64_t want = v > 0 ? (uint64_t)v : (256ull << 20);
    const uint64_t used = ctx->in_use.load() - ctx->cached.load();  // cached blocks give way
    const uint64_t room = ctx->budget > used + (512ull << 20) ? ctx->budget - used - (512ull << 20) : 0;
    return std::min<uint64_t>(want, room / 20);
}

// Initial entries of a group's work-queue ring: COSMICA_SERVE_RING (a power of
// two, 64 to 2^26), default 2^20 (16 MB); it doubles as admission needs.
uint64_t ring_initial()
{
    const char* e = std::getenv("COSMICA_SERVE_RING");
    long long v = e ? std::strtoll(e, nullptr, 10) : 0;
    if (v < 64 || v > (1ll << 26) || (v & (v - 1)) != 0) return 1ull << 20;
    return (uint64_t)v;
}

cosmica_status serve_host_init(cosmica_ctx* ctx)
{
    auto H = std::make_unique<ServeHost>();
    for (int i = 0; i < 2; ++i) {
        HIP_TRY(hipHostMalloc((void**)&H->arena[i], ServeHost::kArenaBytes, hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&H->round_ev[i], hipEventDisableTiming));
    }
    ctx->serve_host = std::move(H);
    return COSMICA_OK;
}

// Copies host bytes to the device on the serving stream, staged in the
// current round's pinned arena (the source may go away at once).
cosmica_status upload(cosmica_ctx* ctx, void* dst, const void* src, size_t bytes)
{
    if (bytes == 0) return COSMICA_OK;
    ServeHost& H = *ctx->serve_host;
    hipStream_t s = ctx->serve_stream;
    if (bytes > ServeHost::kArenaBytes) {
        HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // pageable source
        return COSMICA_OK;
    }
    size_t off = (H.used + 255) & ~(size_t)255;
    if (off + bytes > ServeHost::kArenaBytes) {
        // every copy enqueued so far is done: both arenas are free
        HIP_TRY(hipStreamSynchronize(s));
        off = 0;
    }
    unsigned char* p = H.arena[H.cur] + off;
    std::memcpy(p, src, bytes);
    H.used = off + bytes;
    HIP_TRY(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, s));
    return COSMICA_OK;
}

template <typename R>
cosmica_status group_alloc_tables(ServeGroup* g)
{
    JobDev<R>* jd = nullptr;
    RegionDev<R>* rd = nullptr;
    cosmica_status st;
    if ((st = g->mem.alloc(&jd, ServeGroup::kSlots)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&rd, (size_t)ServeGroup::kSlots * kRegionStride)) != COSMICA_OK)
        return st;
    g->jobs_d = jd;
    g->regions_d = rd;
    return COSMICA_OK;
}

cosmica_status park_alloc(ServeGroup* g, ParkDev* pk)
{
    const size_t n = g->park_cap;
    unsigned char* b = nullptr;
    cosmica_status st = g->mem.alloc(&b, n * (7 * sizeof(double) + 3 * sizeof(uint32_t)));
    if (st != COSMICA_OK) return st;
    double* d = (double*)b;
    pk->r = d;
    pk->P = d + n;
    pk->t = d + 2 * n;
    pk->th = d + 3 * n;
    pk->ph = d + 4 * n;
    pk->T = d + 5 * n;
    pk->lam = d + 6 * n;
    uint32_t* u = (uint32_t*)(d + 7 * n);
    pk->n = u;
    pk->seg = u + n;
    pk->pid = u + 2 * n;
    return COSMICA_OK;
}

cosmica_status group_create(cosmica_ctx* ctx, int model, int prec, ServeGroup** out)
{
    auto g = std::make_unique<ServeGroup>(ctx);
    g->model = model;
    g->prec = prec;
    cosmica_status st = prec == 1 ? group_alloc_tables<float>(g.get())
                                  : group_alloc_tables<double>(g.get());
    if (st != COSMICA_OK) return st;
    const uint32_t S = ServeGroup::kSlots, B = ServeGroup::kBinsPerSlot;
    if ((st = g->mem.alloc(&g->lis_d, S)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->orbit_d, (size_t)S * COSMICA_MAX_ORBIT)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->cancel_d, S)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->segs_d, (size_t)S * B)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->ctl_d, ServeGroup::kCtlWords)) != COSMICA_OK) return st;
    HIP_TRY(hipHostMalloc((void**)&g->snap_h, 2 * ServeGroup::kCtlWords * sizeof(uint32_t),
                          hipHostMallocDefault));
    const cosmica_launch& L = ctx->launch[model][prec];
    g->block = L.block;
    // serving launches run the per-lane-key variants (each request has its own seed)
    g->grid = grid_for(ctx, model, prec, L, ~0ull >> 8, false, false, false);
    // slices with a squashed heliosphere or the energy form run the kernel
    // variants for them; the parking lists are sized for the largest grid
    for (int v = 1; v < 4; ++v)
        g->grid_var[v] =
            std::min(g->grid, grid_for(ctx, model, prec, L, ~0ull >> 8, v & 1, v & 2, false));
    g->grid_var[0] = g->grid;
    g->park_cap = (uint32_t)g->grid * (uint32_t)g->block;
    for (int p = 0; p < 2; ++p)
        if ((st = park_alloc(g.get(), &g->park[p])) != COSMICA_OK) return st;
    g->left_cap = g->park_cap / 64 + 64;  // one remainder per wave
    for (int p = 0; p < 2; ++p)
        if ((st = g->mem.alloc(&g->left_d[p], g->left_cap)) != COSMICA_OK) return st;
    for (int p = 0; p < 2; ++p) {
        const int o = p ^ 1;
        SliceDev& v = g->slice_h[p];
        uint32_t* c = g->ctl_d;
        v.resume = g->park[o];
        v.suspend = g->park[p];
        v.n_resume = c + ServeGroup::park_word(o, 0);
        v.resume_head = c + ServeGroup::park_word(p, 2);
        v.suspend_count = c + ServeGroup::park_word(p, 0);
        v.left_in = g->left_d[o];
        v.n_left_in = c + ServeGroup::park_word(o, 1);
        v.left_in_head = c + ServeGroup::park_word(p, 3);
        v.leftover = g->left_d[p];
        v.leftover_count = c + ServeGroup::park_word(p, 1);
        v.overflow = c + ServeGroup::kCtlOverflow;
        v.park_cap = g->park_cap;
        v.left_cap = g->left_cap;
    }
    if ((st = g->mem.alloc(&g->slice_d, 2)) != COSMICA_OK) return st;
    HIP_TRY(hipMemcpy(g->slice_d, g->slice_h, sizeof(g->slice_h), hipMemcpyHostToDevice));
    if ((st = g->mem.alloc(&g->r_hist, (size_t)B * kNHist)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->r_flux, B)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->r_se, B)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->r_mt, B)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->r_steps, B)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->r_ncap, B)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->r_nnan, B)) != COSMICA_OK) return st;
    g->pool_cap = pool_particles(ctx);
    if (g->pool_cap < 1024) return COSMICA_ENOMEM;
    if ((st = g->mem.alloc(&g->exP, g->pool_cap)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->exT, g->pool_cap)) != COSMICA_OK) return st;
    if ((st = g->mem.alloc(&g->exNF, g->pool_cap)) != COSMICA_OK) return st;
    g->ring_cap = ring_initial();
    if ((st = dalloc(ctx, g->ring_cap * sizeof(ChunkDev), (void**)&g->ring_d)) != COSMICA_OK)
        return st;
    g->free_ranges[0] = g->pool_cap;
    for (int s = (int)S - 1; s >= 0; --s) g->free_slots.push_back(s);
    g->segs_h.resize((size_t)S * B);
    HIP_TRY(launch_fill_u32(g->cancel_d, 0u, S, ctx->serve_stream));
    HIP_TRY(launch_fill_u32(g->ctl_d, 0u, ServeGroup::kCtlWords, ctx->serve_stream));
    *out = g.release();
    return COSMICA_OK;
}

bool pool_take(ServeGroup* g, uint64_t n, uint64_t* off)
{
    for (auto it = g->free_ranges.begin(); it != g->free_ranges.end(); ++it) {
        if (it->second >= n) {
            *off = it->first;
            const uint64_t rest = it->second - n, start = it->first + n;
            g->free_ranges.erase(it);
            if (rest) g->free_ranges[start] = rest;
            return true;
        }
    }
    return false;
}

void pool_give(ServeGroup* g, uint64_t off, uint64_t n)
{
    auto it = g->free_ranges.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != g->free_ranges.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        g->free_ranges.erase(nx);
    }
    if (it != g->free_ranges.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            g->free_ranges.erase(it);
        }
    }
}

// Appends chunks at the queue's tail.  When the ring could overflow, the
// worker waits for the device, reads its head and, if still short of room,
// moves the queued entries to a ring twice as large (same positions).
cosmica_status ring_append(ServeGroup* g, const std::vector<ChunkDev>& ch)
{
    cosmica_ctx* ctx = g->ctx;
    hipStream_t s = ctx->serve_stream;
    const uint64_t n = ch.size();
    if (n == 0) return COSMICA_OK;
    if (g->q_tail + n - g->q_head > g->ring_cap) {
        HIP_TRY(hipStreamSynchronize(s));
        uint64_t head = 0;
        HIP_TRY(hipMemcpy(&head, g->ctl_d, sizeof(head), hipMemcpyDeviceToHost));
        g->q_head = head;
        const uint64_t live = g->q_tail - g->q_head;
        if (live + n > g->ring_cap) {
            uint64_t cap = g->ring_cap;
            while (live + n > cap / 2) cap *= 2;
            ChunkDev* dst = nullptr;
            cosmica_status st = dalloc(ctx, cap * sizeof(ChunkDev), (void**)&dst);
            if (st != COSMICA_OK) return st;
            for (uint64_t pos = g->q_head; pos < g->q_tail;) {
                const uint64_t from = pos & (g->ring_cap - 1), to = pos & (cap - 1);
                const uint64_t len =
                    std::min({g->q_tail - pos, g->ring_cap - from, cap - to});
                HIP_TRY(hipMemcpyAsync(dst + to, g->ring_d + from, len * sizeof(ChunkDev),
                                       hipMemcpyDeviceToDevice, s));
                pos += len;
            }
            HIP_TRY(hipStreamSynchronize(s));
            dfree(ctx, g->ring_d, g->ring_cap * sizeof(ChunkDev));
            g->ring_d = dst;
            g->ring_cap = cap;
        }
    }
    for (uint64_t k = 0; k < n;) {
        const uint64_t at = (g->q_tail + k) & (g->ring_cap - 1);
        const uint64_t len = std::min(n - k, g->ring_cap - at);
        cosmica_status st = upload(ctx, g->ring_d + at, ch.data() + k, len * sizeof(ChunkDev));
        if (st != COSMICA_OK) return st;
        k += len;
    }
    g->q_tail += n;
    return COSMICA_OK;
}

template <typename R>
cosmica_status upload_slot(ServeGroup* g, Req* q)
{
    JobDev<R> J;
    RegionDev<R> reg[kRegionStride];
    LisDev lis;
    make_tables<R>(head_of(q->job), &J, reg, &lis);
    cosmica_ctx* ctx = g->ctx;
    const int slot = q->slot;
    J.orbit_off = (uint32_t)slot * COSMICA_MAX_ORBIT;
    std::vector<OrbitDev> oh;
    const std::vector<double>& o = q->job.orbit;
    for (size_t k = 0; k + 2 < o.size(); k += 3) oh.push_back(OrbitDev{o[k], o[k + 1], o[k + 2], 0.0});
    cosmica_status st;
    if ((st = upload(ctx, g->orbit_d + J.orbit_off, oh.data(), oh.size() * sizeof(OrbitDev))) !=
        COSMICA_OK)
        return st;
    if ((st = upload(ctx, (JobDev<R>*)g->jobs_d + slot, &J, sizeof(J))) != COSMICA_OK) return st;
    if ((st = upload(ctx, (RegionDev<R>*)g->regions_d + (size_t)slot * kRegionStride, reg,
                     sizeof(reg))) != COSMICA_OK)
        return st;
    if ((st = upload(ctx, g->lis_d + slot, &lis, sizeof(lis))) != COSMICA_OK) return st;
    const size_t s0 = (size_t)slot * ServeGroup::kBinsPerSlot;
    return upload(ctx, g->segs_d + s0, &g->segs_h[s0], q->job.rig.size() * sizeof(SegmentDev));
}

// Admit queued requests (FIFO) while a slot and a contiguous exit-record range fit.
cosmica_status admit(cosmica_ctx* ctx)
{
    hipStream_t s = ctx->serve_stream;
    while (!ctx->queued.empty()) {
        Req* q = ctx->queued.front();
        if (q->cancel) {
            ctx->queued.pop_front();
            q->state = 2;
            q->status = COSMICA_ECANCELED;
            ctx->cv.notify_all();
            continue;
        }
        std::unique_ptr<ServeGroup>& gp = ctx->groups[q->model][q->prec];
        if (!gp) {
            ServeGroup* g = nullptr;
            cosmica_status st = group_create(ctx, q->model, q->prec, &g);
            if (st != COSMICA_OK) return st;
            gp.reset(g);
        }
        ServeGroup* g = gp.get();
        if (g->free_slots.empty()) break;
        uint64_t off = 0;
        if (q->job.total > g->pool_cap) {  // can never fit
            ctx->queued.pop_front();
            q->state = 2;
            q->status = COSMICA_ENOMEM;
            ctx->cv.notify_all();
            continue;
        }
        if (q->job.formulation == 1 && g->exL == nullptr) {
            cosmica_status st = g->mem.alloc(&g->exL, g->pool_cap);
            if (st != COSMICA_OK) {  // no room for the energy form's loss records
                ctx->queued.pop_front();
                q->state = 2;
                q->status = st;
                ctx->cv.notify_all();
                continue;
            }
        }
        if (!pool_take(g, q->job.total, &off)) break;
        ctx->queued.pop_front();
        q->slot = g->free_slots.back();
        g->free_slots.pop_back();
        q->ex0 = off;
        const size_t s0 = (size_t)q->slot * ServeGroup::kBinsPerSlot;
        uint64_t o = off;
        std::vector<uint32_t> ids;
        for (size_t b = 0; b < q->job.rig.size(); ++b) {
            SegmentDev& sg = g->segs_h[s0 + b];
            std::memset(&sg, 0, sizeof(sg));
            sg.P0 = q->job.rig[b];
            sg.job = (uint32_t)q->slot;
            sg.bin = q->job.bin_offset + (uint32_t)b;
            sg.count = q->job.cnt[b];
            sg.out_offset = (uint32_t)o;
            o += q->job.cnt[b];
            ids.push_back((uint32_t)(s0 + b));
        }
        // the request's own bins, longest expected paths first (order 2), so its
        // latency is not set by a long path that started last; requests stay
        // first come, first served
        const cosmica_launch& L = ctx->launch[q->model][q->prec];
        std::vector<double> cost(g->segs_h.size(), 0.0);
        for (size_t b = 0; b < q->job.rig.size(); ++b)
            cost[s0 + b] = expected_steps(q->job.helio, q->job.species, q->job.rig[b]);
        std::vector<ChunkDev> chunks;
        make_chunks(g->segs_h, ids, L.chunk, L.order, &chunks, &cost);
        cosmica_status st = q->prec == 1 ? upload_slot<float>(g, q) : upload_slot<double>(g, q);
        if (st != COSMICA_OK) return st;
        // the slot's counters start again (stream-ordered after every slice
        // enqueued so far, before the request's first one)
        HIP_TRY(launch_fill_u32(g->ctl_d + ServeGroup::kCtlDone + q->slot, 0u, 1, s));
        HIP_TRY(launch_fill_u32(g->cancel_d + q->slot, 0u, 1, s));
        if ((st = ring_append(g, chunks)) != COSMICA_OK) return st;
        q->ring_end = g->q_tail;
        q->first_slice = g->seq;
        q->state = 1;
        g->resident.push_back(q);
    }
    return COSMICA_OK;
}

// Enqueues one slice of a group: the propagation kernel, the closing kernel,
// and the copy of the control words to the host.
template <typename R>
cosmica_status launch_slice(ServeGroup* g)
{
    cosmica_ctx* ctx = g->ctx;
    hipStream_t s = ctx->serve_stream;
    const int p = (int)(g->seq & 1u), o = p ^ 1;
    uint32_t* c = g->ctl_d;
    PropArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.jobs = (const JobDev<R>*)g->jobs_d;
    a.regions = (const RegionDev<R>*)g->regions_d;
    a.orbit = g->orbit_d;
    a.segs = g->segs_d;
    a.chunks = g->ring_d;
    a.head = (unsigned long long*)c;
    a.q_tail = g->q_tail;
    a.q_mask = g->ring_cap - 1;
    a.exP = g->exP;
    a.exT = g->exT;
    a.exNF = g->exNF;
    a.exL = g->exL;
    a.slice = g->slice_d + p;
    a.step_budget = slice_steps();
    a.slice_ticks = slice_ticks(ctx);
    if (a.step_budget == 0xffffffffu && a.slice_ticks == 0) a.step_budget = 2048u;
    a.job_cancel = g->cancel_d;
    a.job_done = c + ServeGroup::kCtlDone;
    // every request holding a slot may have particles in this slice
    for (const Req* q : g->resident) a.shaped |= job_shaped(q->job) ? 1u : 0u;
    for (const Req* q : g->releasing) a.shaped |= job_shaped(q->job) ? 1u : 0u;
    for (const Req* q : g->resident) a.energy |= q->job.formulation == 1 ? 1u : 0u;
    for (const Req* q : g->releasing) a.energy |= q->job.formulation == 1 ? 1u : 0u;
    // The variants for a squashed heliosphere or the energy form may fit fewer
    // lanes than the previous slice parked particles: the closing kernel
    // carries what no wave claimed over to the next slice.
    const int grid = g->grid_var[(a.shaped ? 1 : 0) | (a.energy ? 2 : 0)];
    HIP_TRY(launch_model<R>(g->model, a, grid, g->block, s));
    CloseArgs k;
    std::memset(&k, 0, sizeof(k));
    k.sl = g->slice_h[p];
    k.head = a.head;
    k.q_tail = g->q_tail;
    k.segs = g->segs_d;
    k.job_cancel = g->cancel_d;
    k.next_counters = c + ServeGroup::park_word(o, 0);
    HIP_TRY(launch_slice_close(k, s));
    HIP_TRY(hipMemcpyAsync(g->snap_h + (size_t)p * ServeGroup::kCtlWords, c,
                           ServeGroup::kCtlWords * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    ++g->seq;
    return COSMICA_OK;
}

void release(ServeGroup* g, Req* q)
{
    pool_give(g, q->ex0, q->job.total);
    g->free_slots.push_back(q->slot);
    q->slot = -1;
}

// Enqueues the reduction of a finished request's bins and the copy of its
// results to pinned memory; the slot and the exit records go back at once
// (what is enqueued later on the stream runs after these copies).
cosmica_status finish_request(ServeGroup* g, Req* q)
{
    cosmica_ctx* ctx = g->ctx;
    ServeHost& H = *ctx->serve_host;
    hipStream_t s = ctx->serve_stream;
    const uint32_t nb = (uint32_t)q->job.rig.size();
    ReduceArgs r;
    std::memset(&r, 0, sizeof(r));
    r.segs = g->segs_d;
    r.lis = g->lis_d;
    r.exP = g->exP;
    r.exT = g->exT;
    r.exNF = g->exNF;
    r.exL = g->exL;
    r.seg_base = (uint32_t)q->slot * ServeGroup::kBinsPerSlot;
    r.out_base = 0;
    r.hist = g->r_hist;
    r.flux = g->r_flux;
    r.flux_se = g->r_se;
    r.mean_t = g->r_mt;
    r.steps = g->r_steps;
    r.n_capped = g->r_ncap;
    r.n_nan = g->r_nnan;
    HIP_TRY(launch_reduce(r, nb, s));
    if (H.free_blocks.empty()) {
        unsigned char* b = nullptr;
        HIP_TRY(hipHostMalloc((void**)&b, ServeHost::kResultBytes, hipHostMallocDefault));
        H.blocks.push_back(b);
        H.free_blocks.push_back(b);
    }
    if (H.free_events.empty()) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        H.events.push_back(e);
        H.free_events.push_back(e);
    }
    q->staged = H.free_blocks.back();
    H.free_blocks.pop_back();
    q->staged_ev = H.free_events.back();
    H.free_events.pop_back();
    unsigned char* b = q->staged;
    HIP_TRY(hipMemcpyAsync(b, g->r_hist, (size_t)nb * kNHist * 4, hipMemcpyDeviceToHost, s));
    b += (size_t)nb * kNHist * 4;
    const void* src8[4] = {g->r_flux, g->r_se, g->r_mt, g->r_steps};
    for (const void* p : src8) {
        HIP_TRY(hipMemcpyAsync(b, p, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
        b += (size_t)nb * 8;
    }
    HIP_TRY(hipMemcpyAsync(b, g->r_ncap, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
    b += (size_t)nb * 4;
    HIP_TRY(hipMemcpyAsync(b, g->r_nnan, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(q->staged_ev, s));
    const cosmica_result& R = q->res;
    if (R.exits) {
        // exit records go straight to the caller's (pageable) array
        HIP_TRY(hipStreamSynchronize(s));
        const size_t n = q->job.total;
        std::vector<double> P(n), T(n), Ls(n, 0.0);
        std::vector<uint32_t> NF(n);
        HIP_TRY(hipMemcpy(P.data(), g->exP + q->ex0, n * 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(T.data(), g->exT + q->ex0, n * 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(NF.data(), g->exNF + q->ex0, n * 4, hipMemcpyDeviceToHost));
        if (q->job.formulation == 1)
            HIP_TRY(hipMemcpy(Ls.data(), g->exL + q->ex0, n * 8, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < n; ++i) {
            cosmica_exit& e = R.exits[i];
            e.P = P[i];
            e.t = T[i];
            e.loss = Ls[i];
            e.r = e.theta = e.phi = 0.0;
            e.n = NF[i] & ((1u << kFlagShift) - 1u);
            e.flags = NF[i] >> kFlagShift;
        }
    }
    release(g, q);
    H.finishing.push_back(q);
    return COSMICA_OK;
}

// Hands the staged results of finished requests to their callers: those whose
// copies are done (all of them, waiting, if wait is set).
cosmica_status deliver(cosmica_ctx* ctx, bool wait)
{
    ServeHost& H = *ctx->serve_host;
    for (auto it = H.finishing.begin(); it != H.finishing.end();) {
        Req* q = *it;
        hipError_t e = wait ? hipEventSynchronize(q->staged_ev) : hipEventQuery(q->staged_ev);
        if (e == hipErrorNotReady) {
            ++it;
            continue;
        }
        if (e != hipSuccess) return COSMICA_EDEVICE;
        const uint32_t nb = (uint32_t)q->job.rig.size();
        const cosmica_result& R = q->res;
        const unsigned char* b = q->staged;
        if (R.hist) std::memcpy(R.hist, b, (size_t)nb * kNHist * 4);
        b += (size_t)nb * kNHist * 4;
        double* dst8[3] = {R.flux, R.flux_se, R.mean_exit_time_s};
        for (double* d : dst8) {
            if (d) std::memcpy(d, b, (size_t)nb * 8);
            b += (size_t)nb * 8;
        }
        if (R.steps) std::memcpy(R.steps, b, (size_t)nb * 8);
        b += (size_t)nb * 8;
        const uint32_t* ncap = (const uint32_t*)b;
        if (R.n_capped) std::memcpy(R.n_capped, ncap, (size_t)nb * 4);
        b += (size_t)nb * 4;
        if (R.n_nan) std::memcpy(R.n_nan, b, (size_t)nb * 4);
        bool capped = false;
        for (uint32_t k = 0; k < nb; ++k) capped |= ncap[k] > 0;
        q->status = capped ? COSMICA_ESTEPCAP : COSMICA_OK;
        q->state = 2;
        H.free_blocks.push_back(q->staged);
        H.free_events.push_back(q->staged_ev);
        q->staged = nullptr;
        q->staged_ev = nullptr;
        it = H.finishing.erase(it);
        ctx->cv.notify_all();
    }
    return COSMICA_OK;
}

// What slice `seq` of a group did, from its copy of the control words:
// requests whose particles have all exited are finished, and cancelled ones
// are freed once none of their work is left on the device.
cosmica_status read_slice(ServeGroup* g, uint64_t seq)
{
    const int p = (int)(seq & 1u);
    const uint32_t* c = g->snap_h + (size_t)p * ServeGroup::kCtlWords;
    if (c[ServeGroup::kCtlOverflow] != 0u) return COSMICA_EDEVICE;
    g->q_head = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
    g->in_flight = c[ServeGroup::park_word(p, 0)];
    for (auto it = g->resident.begin(); it != g->resident.end();) {
        Req* q = *it;
        if (q->first_slice <= seq && c[ServeGroup::kCtlDone + q->slot] >= q->job.total) {
            cosmica_status st = finish_request(g, q);
            if (st != COSMICA_OK) return st;
            it = g->resident.erase(it);
        } else {
            ++it;
        }
    }
    // A slice that sees a cancel flag drops the request's parked particles and
    // chunk remainders (claimed or not), and every chunk issued from then on;
    // so after such a slice, with the head past the request's last chunk,
    // nothing of it is left.
    for (auto it = g->releasing.begin(); it != g->releasing.end();) {
        Req* q = *it;
        if (q->cancel_slice <= seq && g->q_head >= q->ring_end) {
            release(g, q);
            it = g->releasing.erase(it);
        } else {
            ++it;
        }
    }
    return COSMICA_OK;
}

void serve_loop(cosmica_ctx* ctx)
{
    (void)hipSetDevice(ctx->device);
    ServeHost& H = *ctx->serve_host;
    std::vector<std::pair<ServeGroup*, uint64_t>> prev, cur;  // (group, slice) per round
    uint64_t round = 0;
    std::unique_lock<std::mutex> lk(ctx->mu);
    while (!ctx->stop) {
        H.cur = (int)(round & 1u);
        H.used = 0;
        cosmica_status st = admit(ctx);
        if (st != COSMICA_OK) {
            ctx->serve_error = st;
            break;
        }
        std::vector<ServeGroup*> active;
        for (int m = 0; m < 2; ++m)
            for (int q = 0; q < 2; ++q) {
                ServeGroup* g = ctx->groups[m][q].get();
                if (g == nullptr) continue;
                // cancellations: a flag on the device, set before the next slice
                for (auto it = g->resident.begin(); it != g->resident.end();) {
                    Req* r = *it;
                    if (r->cancel && !r->cancel_sent) {
                        if (launch_fill_u32(g->cancel_d + r->slot, 1u, 1, ctx->serve_stream) !=
                            hipSuccess)
                            ctx->serve_error = COSMICA_EDEVICE;
                        r->cancel_sent = true;
                        r->cancel_slice = g->seq;
                        r->state = 2;
                        r->status = COSMICA_ECANCELED;
                        g->releasing.push_back(r);
                        it = g->resident.erase(it);
                        ctx->cv.notify_all();
                    } else {
                        ++it;
                    }
                }
                if (!g->resident.empty() || !g->releasing.empty()) active.push_back(g);
            }
        if (ctx->serve_error != COSMICA_OK) break;
        if (active.empty() && prev.empty()) {
            if (!H.finishing.empty()) {
                lk.unlock();
                const hipError_t e = hipStreamSynchronize(ctx->serve_stream);
                lk.lock();
                if (e != hipSuccess || (st = deliver(ctx, false)) != COSMICA_OK) {
                    ctx->serve_error = COSMICA_EDEVICE;
                    break;
                }
                continue;
            }
            ctx->cv.wait(lk, [&] { return ctx->stop || !ctx->queued.empty(); });
            continue;
        }
        lk.unlock();
        bool ok = true;
        cur.clear();
        for (ServeGroup* g : active) {
            st = g->prec == 1 ? launch_slice<float>(g) : launch_slice<double>(g);
            ok &= st == COSMICA_OK;
            cur.emplace_back(g, g->seq - 1);
        }
        // the device now holds this round's slices: read what the previous
        // round's did while they run
        if (ok && hipEventRecord(H.round_ev[round & 1u], ctx->serve_stream) != hipSuccess) ok = false;
        if (ok && !prev.empty() && hipEventSynchronize(H.round_ev[(round - 1) & 1u]) != hipSuccess)
            ok = false;
        lk.lock();
        if (!ok) {
            ctx->serve_error = COSMICA_EDEVICE;
            break;
        }
        // results copied after the previous round's slices are next in the
        // stream (this round's slices queue behind them): a short wait
        if ((st = deliver(ctx, true)) != COSMICA_OK) {
            ctx->serve_error = st;
            break;
        }
        for (auto& gs : prev)
            if ((st = read_slice(gs.first, gs.second)) != COSMICA_OK) {
                ctx->serve_error = st;
                ok = false;
                break;
            }
        if (!ok) break;
        prev.swap(cur);
        ++round;
    }
    // results already on their way are handed over; whatever is left fails so
    // waiters return
    if (ctx->serve_error == COSMICA_OK) (void)deliver(ctx, true);
    for (auto& kv : ctx->reqs)
        if (kv.second->state != 2) {
            kv.second->state = 2;
            kv.second->status = ctx->serve_error != COSMICA_OK ? ctx->serve_error
                                                               : COSMICA_ECANCELED;
        }
    ctx->cv.notify_all();
}

}  // namespace

extern "C" {

cosmica_status cosmica_submit(cosmica_ctx* ctx, const cosmica_job* job,
                              cosmica_precision precision, cosmica_result* result,
                              uint64_t* ticket)
{
    if (ctx == nullptr || result == nullptr || ticket == nullptr) return COSMICA_EINVAL;
    if (precision != COSMICA_PREC_FP64 && precision != COSMICA_PREC_MIXED) return COSMICA_EINVAL;
    if (validate(job) != COSMICA_OK || job->n_bins > (int)ServeGroup::kBinsPerSlot)
        return COSMICA_EINVAL;
    auto q = std::make_unique<Req>();
    q->job = copy_job(job);
    q->prec = precision;
    q->model = job->helio->model;
    q->res = *result;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->serve_error != COSMICA_OK) return ctx->serve_error;
    if (ctx->queued.size() >= 100000) return COSMICA_EBUSY;
    if (!ctx->worker_started) {
        if (hipSetDevice(ctx->device) != hipSuccess ||
            hipStreamCreateWithFlags(&ctx->serve_stream, hipStreamNonBlocking) != hipSuccess)
            return COSMICA_EDEVICE;
        if (serve_host_init(ctx) != COSMICA_OK) {
            (void)hipStreamDestroy(ctx->serve_stream);
            ctx->serve_stream = nullptr;
            return COSMICA_EDEVICE;
        }
        ctx->worker = std::thread(serve_loop, ctx);
        ctx->worker_started = true;
    }
    q->ticket = ctx->next_ticket++;
    *ticket = q->ticket;
    ctx->queued.push_back(q.get());
    ctx->reqs[q->ticket] = std::move(q);
    ctx->cv.notify_all();
    return COSMICA_OK;
}

cosmica_status cosmica_poll(cosmica_ctx* ctx, uint64_t ticket, int32_t* done)
{
    if (ctx == nullptr || done == nullptr) return COSMICA_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->reqs.find(ticket);
    if (it == ctx->reqs.end()) return COSMICA_ENOTFOUND;
    *done = it->second->state == 2 ? 1 : 0;
    return *done ? it->second->status : COSMICA_OK;
}

cosmica_status cosmica_wait(cosmica_ctx* ctx, uint64_t ticket, int32_t timeout_ms)
{
    if (ctx == nullptr) return COSMICA_EINVAL;
    std::unique_lock<std::mutex> lk(ctx->mu);
    auto it = ctx->reqs.find(ticket);
    if (it == ctx->reqs.end()) return COSMICA_ENOTFOUND;
    Req* q = it->second.get();
    auto pred = [&] { return q->state == 2; };
    if (timeout_ms < 0)
        ctx->cv.wait(lk, pred);
    else if (!ctx->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
        return COSMICA_EBUSY;
    return q->status;
}

cosmica_status cosmica_cancel(cosmica_ctx* ctx, uint64_t ticket)
{
    if (ctx == nullptr) return COSMICA_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->reqs.find(ticket);
    if (it == ctx->reqs.end()) return COSMICA_ENOTFOUND;
    if (it->second->state != 2) it->second->cancel = true;
    ctx->cv.notify_all();
    return COSMICA_OK;
}

cosmica_status cosmica_request_state(cosmica_ctx* ctx, uint64_t ticket, int32_t* state)
{
    if (ctx == nullptr || state == nullptr) return COSMICA_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->reqs.find(ticket);
    if (it == ctx->reqs.end()) return COSMICA_ENOTFOUND;
    *state = it->second->state;
    return COSMICA_OK;
}

cosmica_status cosmica_serve_stats(cosmica_ctx* ctx, uint64_t* queued, uint64_t* resident,
                                   uint64_t* particles_in_flight, uint64_t* bytes_in_use)
{
    if (ctx == nullptr) return COSMICA_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    uint64_t res = 0, fl = 0;
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 2; ++q)
            if (ctx->groups[m][q]) {
                res += ctx->groups[m][q]->resident.size();
                fl += ctx->groups[m][q]->in_flight;
            }
    if (queued) *queued = ctx->queued.size();
    if (resident) *resident = res;
    if (particles_in_flight) *particles_in_flight = fl;
    if (bytes_in_use) *bytes_in_use = ctx->in_use.load();
    return COSMICA_OK;
}

void cosmica_destroy(cosmica_ctx* ctx)
{
    if (ctx == nullptr) return;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->stop = true;
        ctx->cv.notify_all();
    }
    if (ctx->worker.joinable()) ctx->worker.join();
    (void)hipSetDevice(ctx->device);
    if (ctx->serve_stream) (void)hipStreamSynchronize(ctx->serve_stream);
    (void)hipStreamSynchronize(ctx->stream);
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 2; ++q) {
            ServeGroup* g = ctx->groups[m][q].get();
            if (g && g->ring_d) dfree(ctx, g->ring_d, g->ring_cap * sizeof(ChunkDev));
            ctx->groups[m][q].reset();
        }
    if (ctx->serve_stream) (void)hipStreamDestroy(ctx->serve_stream);
    for (int i = 0; i < 4; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    cache_trim(ctx, ~0ull);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // extern "C"
