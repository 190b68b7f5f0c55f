// kernels.hip -- gfx950 kernels of libcosmica.
//
// propagate<R, 3D>: persistent Euler-Maruyama integrator of the backward SDE
//   (arXiv 2502.06319, Eq.(3) applied to Eq.(5) with A_P of Eq.(6), Sec. III),
//   one lane per quasi-particle (Sec. IV.A).  Lanes whose particle left the
//   heliosphere are refilled from a flat work queue at the next step; each
//   wave takes a whole refill chunk with one atomic and hands its particles to
//   its idle lanes by ballot rank, so waves stay full until the queue drains.
//   R = double is the plain FP64 path; R = float is the mixed path (bulk FP32
//   with the hardware transcendentals, r / t / P accumulated in FP64).
//   Variants per launch: surface tests (nose-squashed heliosphere with a
//   heliosheath, Sec. II.B) and the energy form (Eq.(1), with the loss of
//   Eq.(4)).
// reduce: one workgroup per rigidity bin; LDS-privatised exit histogram and
//   fixed-order FP64 sums of the LIS weights (Eq.(4): J = f P^2 with L = 0 in
//   the momentum form, the loss weight in the energy form).
// reweight: the same sums for many tabulated spectra over stored exits.
//
// No MFMA: the work is per-particle scalar arithmetic, bound by VALU issue
// and the transcendental unit.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "engine.hpp"

namespace cosmica {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kTwoPi = 6.283185307179586476925286766559005768;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11 -- the generator of Sec. IV.A).  Written
// for gfx950: each 32x32->64 product is one v_mad_u64_u32 and each three-way
// XOR one v_bitop3_b32, so a round is two of each.
// ---------------------------------------------------------------------------
// a ^ b ^ c: truth table 0x96 sets the output bit where an odd number of the
// three input bits is set.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint32_t k0, uint32_t k1, uint32_t c0,
                                               uint32_t c1, uint32_t c2, uint32_t c3)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(m1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(m0 >> 32), c3, k1);
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// Precision traits.  float: gfx950 hardware ops (v_rcp/v_sqrt/v_rsq/v_log/
// v_exp/v_sin/v_cos; sin/cos take revolutions).  double: IEEE FP64 library.
// ---------------------------------------------------------------------------
template <typename R>
struct Mth;

template <>
struct Mth<float> {
    // Floors that keep binary32 finite at the poles (where theta can round onto
    // float(pi) and the hardware sine returns exactly 0) and at r -> 0.
    static constexpr float kSinFloor = 1e-7f;
    static constexpr float kRFloor = 1e-6f;
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    // sin(2 pi x), cos(2 pi x)
    static __device__ __forceinline__ void sincos_rev(float x, float* s, float* c)
    {
        *s = __builtin_amdgcn_sinf(x);
        *c = __builtin_amdgcn_cosf(x);
    }
    static __device__ __forceinline__ void sincos_rad(float x, float* s, float* c)
    {
        sincos_rev(x * 0.159154943091895336f, s, c);
    }
    static __device__ __forceinline__ float cos_rad(float x)
    {
        return __builtin_amdgcn_cosf(x * 0.159154943091895336f);
    }
    static __device__ __forceinline__ float atan(float x) { return ::atanf(x); }
    // tanh x and (1 - tanh^2 x) / 4 for x = x4 / 4, both from e = e^(-2|x|) in
    // [0, 1]: tanh|x| = (1 - e) / (1 + e) and 1 - tanh^2 x = 4 e / (1 + e)^2.  The
    // second keeps its relative accuracy where tanh x -> +-1 (1 - tanh^2 would
    // cancel there: at tanh x = 0.9999997 binary32 leaves it ~20 % off);
    // |x4| = inf gives exactly +-1 and 0.  The caller's x4 carries the 4 that
    // the second result drops (one multiply fewer).
    static __device__ __forceinline__ void tanh_sech2_x4(float x4, float* t, float* s2_4)
    {
        const float e = __builtin_amdgcn_exp2f(-0.721347520444482f * fabsf(x4));
        const float q = __builtin_amdgcn_rcpf(1.0f + e);
        const float eq = e * q;
        *t = __builtin_copysignf(q - eq, x4);
        *s2_4 = eq * q;
    }
    // x - 2 pi floor(x / 2 pi): in [0, 2 pi) up to one rounding
    static __device__ __forceinline__ float fmod2pi(float x)
    {
        return x - (float)kTwoPi * floorf(x * 0.159154943091895336f);
    }
};

template <>
struct Mth<double> {
    static constexpr double kSinFloor = 0.0;  // FP64 needs no floors
    static constexpr double kRFloor = 0.0;
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    static __device__ __forceinline__ void sincos_rad(double x, double* s, double* c)
    {
        ::sincos(x, s, c);
    }
    static __device__ __forceinline__ double cos_rad(double x) { return ::cos(x); }
    static __device__ __forceinline__ double atan(double x) { return ::atan(x); }
    static __device__ __forceinline__ void tanh_sech2_x4(double x, double* t, double* s2)
    {
        // binary64: x is the argument itself (no factor 4; see load_job)
        *t = ::tanh(x);
        *s2 = 1.0 - *t * *t;
    }
    static __device__ __forceinline__ double fmod2pi(double x) { return ::fmod(x, kTwoPi); }
};

// Uniform in (0,1): (floor(x / 2^9) + 1/2) * 2^-23, exact in binary32 and
// binary64.  In binary32 it is built from the bits: 1 + floor(x/2^9) 2^-23 has
// the 23 bits as mantissa, and subtracting 1 - 2^-24 is exact.  The pattern
// 0x3F800000 | (x >> 9) is one v_alignbit_b32: the 64-bit pair (0x7F, x)
// shifted right by 9.
__device__ __forceinline__ float uniform_f32(uint32_t x)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9u)) - 0.99999994039535522f;
}
__device__ __forceinline__ double uniform_f64(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * 1.1920928955078125e-07;
}

// Box-Muller: z0, z1 from (u0, u1), z2 from (u2, u3).
template <typename R, int NZ>
__device__ __forceinline__ void normals(uint32_t k0, uint32_t k1, uint32_t n, uint32_t pid,
                                        uint32_t bin, uint32_t tag, R* z)
{
    const uint4 x = philox4x32_10(k0, k1, n, pid, bin, tag);
    if constexpr (std::is_same<R, float>::value) {
        // sqrt(-2 ln u) = sqrt(log2(u) * (-2 ln 2))
        const float rho0 = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(uniform_f32(x.x)) *
                                                  -1.38629436111989061f);
        if (NZ == 1) {
            z[0] = rho0 * __builtin_amdgcn_cosf(uniform_f32(x.y));
        } else {
            const float u1 = uniform_f32(x.y);
            const float rho2 = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(uniform_f32(x.z)) *
                                                      -1.38629436111989061f);
            z[0] = rho0 * __builtin_amdgcn_cosf(u1);
            z[1] = rho0 * __builtin_amdgcn_sinf(u1);
            z[2] = rho2 * __builtin_amdgcn_cosf(uniform_f32(x.w));
        }
    } else {
        const double rho0 = ::sqrt(-2.0 * ::log(uniform_f64(x.x)));
        if (NZ == 1) {
            z[0] = rho0 * ::cospi(2.0 * uniform_f64(x.y));
        } else {
            double s1, c1;
            ::sincospi(2.0 * uniform_f64(x.y), &s1, &c1);
            const double rho2 = ::sqrt(-2.0 * ::log(uniform_f64(x.z)));
            z[0] = rho0 * c1;
            z[1] = rho0 * s1;
            z[2] = rho2 * ::cospi(2.0 * uniform_f64(x.w));
        }
    }
}

// ---------------------------------------------------------------------------
// Particle state and one step.
// ---------------------------------------------------------------------------
template <typename R>
struct PState {
    double r, P, t;
    R th, ph;
    uint32_t n;
    double T, lam;  // energy form: kinetic energy [GeV] and the summed loss
};

// Local SDE coefficients of the 3D model (see cosmica.h for the model).
template <typename R>
struct Coef3 {
    R Ar, At, Ap, AP;      // drift of the SDE (r, theta, phi per unit time), dP/ds
    R V;                   // local wind speed
    R Brr, Bpr, Bpp, Btt;  // B with B B^T = 2K
    R dt;
    R invr, invst;         // 1/r, 1/sin(theta) of the step
    R Hw, vdr, vdt, vdp, Krr, Krp, kpar;
};

// Per-lane copy of a job's constants, loaded once when a lane takes a
// particle: the step then reads only its shell entry from memory, however
// many jobs the lanes of a wave belong to.
template <typename R>
struct JobReg {
    R omega, kfrac, omf, sqf2, twof, gcoef, hb, abs_z, mass2, sqA, dt_max, diff_frac,
        adv_frac;
    double rb, inv_shell;
    double rb_tail, ts_nose, ts_tail;  // used by the kernels of squashed heliospheres
    R mass;                             // rest energy, used by the energy form
    int32_t energy;
    uint32_t seed_lo, seed_hi, job_tag, step_cap;
    int32_t nreg, drift;
    R sheet_off;  // 0 with the current sheet, +inf without it (then Hw = 1)
    R v_nodrift;  // 0 with drift, 1 without (keeps Gamma finite where V = 0)
};

template <typename R>
__device__ __forceinline__ JobReg<R> load_job(const JobDev<R>& J)
{
    JobReg<R> o;
    o.omega = J.omega;
    o.kfrac = J.kperp_frac;
    o.omf = J.omf;
    o.sqf2 = J.sqf2;
    o.twof = J.twof;
    o.gcoef = J.gcoef;
    // binary32: 1/Delta carries a factor 4 that the sheet factor drops
    // (Mth<float>::tanh_sech2_x4)
    o.hb = std::is_same<R, float>::value ? J.hb * (R)4 : J.hb;
    o.abs_z = J.abs_z;
    o.mass2 = J.mass2;
    o.sqA = J.sqA;
    o.dt_max = J.dt_max;
    o.diff_frac = J.diff_frac;
    o.adv_frac = J.adv_frac > (R)0 ? J.adv_frac : (R)__builtin_huge_valf();
    o.rb = J.rb;
    o.inv_shell = J.inv_shell;
    o.rb_tail = J.rb_tail;
    o.mass = (R)J.mass;
    o.energy = J.energy;
    o.ts_nose = J.ts_nose;
    o.ts_tail = J.ts_tail;
    o.seed_lo = J.seed_lo;
    o.seed_hi = J.seed_hi;
    o.job_tag = J.job_tag;
    o.step_cap = J.step_cap;
    o.nreg = J.nreg;
    o.drift = J.drift;
    o.sheet_off = J.hcs ? (R)0 : (R)__builtin_huge_valf();
    o.v_nodrift = J.drift ? (R)0 : (R)1;
    if (!J.drift) o.sqA = (R)0;
    return o;
}

// Shell index of r (r >= 0 after the reflections), clamped to the last shell.
template <typename R>
__device__ __forceinline__ int region_of(const JobReg<R>& J, double r)
{
    const int k = (int)(r * J.inv_shell);
    return k < J.nreg - 1 ? k : J.nreg - 1;
}

// Side of a heliospheric surface with distances Rn toward the nose and Rt
// toward the tail (Sec. II.B squashing; the sphere of radius (Rn + Rt)/2
// centred (Rt - Rn)/2 behind the Sun): outside when
// r^2 + (Rt - Rn) r cos(psi) >= Rn Rt, psi the angle from the nose.  Called
// only for Rn <= r < Rt, where the answer depends on the direction.
template <typename R>
__device__ __forceinline__ bool outside_surface(const JobDev<R>& G, double d2, double prod,
                                                double r, R th, R ph)
{
    using M = Mth<R>;
    R st, ct;
    M::sincos_rad(th, &st, &ct);
    const R cpsi = st * G.sin_tn * M::cos_rad(ph - G.ph_n) + ct * G.cos_tn;
    return r * r + (d2 * r) * (double)cpsi >= prod;
}

// Parameter region at a point: the heliosheath beyond the termination shock,
// else the shell of r.  Without SHAPED the heliosphere is a sphere with no
// heliosheath.  jd: the lane's job entry, read only near the shock.
template <typename R, bool SHAPED>
__device__ __forceinline__ int region_at(const JobReg<R>& J, const JobDev<R>* __restrict__ jd,
                                         double r, R th, R ph)
{
    int k = region_of(J, r);
    if (SHAPED && r >= J.ts_nose) {
        if (r >= J.ts_tail || outside_surface(*jd, jd->ts_d2, jd->ts_prod, r, th, ph))
            k = kRegionHeliosheath;
    }
    return k;
}

// Exit test: beyond the heliopause.  A NaN r counts as outside, so a
// non-finite particle also leaves the step loop.
template <typename R, bool SHAPED>
__device__ __forceinline__ bool outside_boundary(const JobReg<R>& J,
                                                 const JobDev<R>* __restrict__ jd, double r,
                                                 R th, R ph)
{
    bool out = !(r < J.rb);
    if (SHAPED && out && r < J.rb_tail) out = outside_surface(*jd, jd->hp_d2, jd->hp_prod, r, th, ph);
    return out;
}

// Local coefficients, written to share every common factor:
//   g = 1/(1+Gamma^2) = V^2/(V^2+w^2), Gamma g = V w/(V^2+w^2), Gamma^2 g = 1 - g
//   (w = Omega r sin(theta)), B from one reciprocal square root of 2 K_rr with
//   B_phiphi = 2 sqrt(kperp/kpar) kpar / sqrt(2 K_rr), B_thth = sqrt(2 kperp).
template <typename R, bool FULL>
__device__ __forceinline__ void coeffs3d(const JobReg<R>& J, const RegionDev<R>& g, double rd,
                                         R P, R th, R ph, Coef3<R>& c)
{
    using M = Mth<R>;
    const R r0 = (R)rd;
    const R r = r0 > M::kRFloor ? r0 : M::kRFloor;
    R st, ct;
    M::sincos_rad(th, &st, &ct);
    st = st > M::kSinFloor ? st : M::kSinFloor;
    const R invr = M::rcp(r);
    const R invst = M::rcp(st);
    const R cot = ct * invst;
    const R irs = invr * invst;
    // wind: slow inside |latitude| <= tilt of the shell, fast outside
    const R lam = (R)(0.5 * kPi) - th;
    const R V = (fabs(lam) <= g.alpha) ? g.vs : g.vf;
    // diffusion tensor: k_par along b ~ (1, 0, -Gamma), k_perp across
    const R pc = J.abs_z * P;
    const R beta = pc * M::rsqrt(pc * pc + J.mass2);
    const R bP = beta * P;
    const R kpar = g.k0 * bP;
    const R kperp = J.kfrac * kpar;
    const R dk = J.omf * kpar;
    const R w = (J.omega * r) * st;  // corotation speed; Gamma = w / V
    const R V2 = V * V;
    const R invD = M::rcp(w * w + V2);
    const R gq = V2 * invD;          // 1 / (1 + Gamma^2)
    const R Gg = (V * invD) * w;     // Gamma / (1 + Gamma^2)
    const R GGg = (R)1.0 - gq;       // Gamma^2 / (1 + Gamma^2)
    const R Krr = dk * gq + kperp;
    const R Krp = -dk * Gg;
    // d/dr K_rr and (1/r) d/dr (r K_rphi), Gamma proportional to r
    const R q = ((R)-2.0 * dk * invr) * gq;
    const R dKrr = q * GGg;
    const R dKrp = q * Gg;
    const R rr = r * r;

    R vdr = 0, vdt = 0, vdp = 0, Hw = 1;
    // binary32: computed for every lane, with sqA = 0 and a unit wind speed in
    // Gamma for jobs without drift (whose wind may be zero), so no branch
    if (std::is_same<R, float>::value || J.drift) {
        const R invV = M::rcp(V + J.v_nodrift);
        const R Gam = w * invV;
        const R Gam2 = Gam * Gam;
        // kappa_A / sqrt(1 + Gamma^2) with kappa_A = beta P / (3 |B|)
        const R G = (J.gcoef * bP) * (rr * gq);
        const R Gcot = Gam * cot;
        const R G2cot = Gam * Gcot;
        R vcr, vct, vcp;
        {
            // wavy sheet: latitude atan(tan(alpha) sin(phi + Omega r / Vs)),
            // polarity factor tanh((theta_cs - theta) / Delta), Delta = 2 r_L / r
            R sc, cc;
            if constexpr (std::is_same<R, float>::value) {
                // The phase Omega r / Vs reaches hundreds of radians, where a
                // binary32 ulp is a visible part of the sheet's width: it is
                // formed from the binary64 r and reduced to one revolution in
                // binary64, so the sine sees [0, 2) revolutions at any wind speed.
                const float frac = (float)__builtin_amdgcn_fract(g.om_rev * rd);  // v_fract_f64
                M::sincos_rev(fmaf(ph, 0.159154943091895336f, frac), &sc, &cc);
            } else {
                M::sincos_rad(g.om_vs * r + ph, &sc, &cc);
            }
            const R y = g.tana * sc;
            const R u = lam - M::atan(y);
            // 1/Delta = r |B| / (2 r_L coefficient P), |B| = br0 sqrt(1+Gamma^2) / r^2
            // (in binary32 times 4, and Hp below over 4: their product is exact)
            const R invDelta = (J.hb * M::sqrt((R)1.0 + Gam2)) * (invr * M::rcp(P));
            // without the sheet the argument is +inf: Hw = 1, Hp = 0, no sheet drift
            R Hp;
            M::tanh_sech2_x4(u * invDelta + J.sheet_off, &Hw, &Hp);
            const R cs = (-g.tana * cc) * M::rcp(y * y + (R)1.0);
            const R gr = cs * g.om_vs;  // d theta_cs / dr
            const R gph = cs * irs;     // (1/(r sin)) d theta_cs / dphi
            // grad Hw x W, grad Hw = (Hp/Delta)(grad u - u grad ln Delta)
            const R f = (Hp * invDelta) * G;
            const R ug = (u * gq) * invr;
            vcr = f * (-ug * (Gam * G2cot) + Gam * invr);
            vct = f * (Gam * (gr - ug) + gph);
            vcp = f * (-ug * G2cot + invr);
        }
        // gradient-curvature drift Hw curl(G (1, 0, -Gamma)):
        // 2 G g / r (-Gamma cot, Gamma (2 + Gamma^2), Gamma^2 cot)
        const R hA = Hw * (((G + G) * gq) * invr);
        vdr = J.sqA * (-hA * Gcot + vcr);
        vdt = J.sqA * ((hA * Gam) * (Gam2 + (R)2.0) + vct);
        vdp = J.sqA * (hA * G2cot + vcp);
    }
    c.Ar = ((Krr + Krr) * invr + dKrr) - V - vdr;
    c.At = invr * ((kperp * cot) * invr - vdt);
    c.Ap = (dKrp - vdp) * irs;
    c.AP = ((V * P) * invr) * (R)(2.0 / 3.0);
    c.V = V;
    // time step: min(dt_max, f_diff r^2 / k_par, f_adv r / |A_det|); fmin keeps
    // the running value when a limit is NaN, like the comparison d < dt would
    R dt = J.dt_max;
    const R d1 = (J.diff_frac * rr) * M::rcp(kpar);
    dt = fmin(d1, dt);
    {
        // adv_frac is +inf when the limit is off, and a2 = 0 gives d2 = inf too
        const R at = r * c.At;
        const R ap = (r * st) * c.Ap;
        const R a2 = c.Ar * c.Ar + (at * at + ap * ap);
        const R d2 = (J.adv_frac * r) * M::rsqrt(a2);
        dt = fmin(d2, dt);
    }
    c.dt = dt;
    const R tK = Krr + Krr;
    const R rs = M::rsqrt(tK);
    c.Brr = tK * rs;
    c.Bpr = (Krp + Krp) * rs;
    c.Bpp = (J.sqf2 * kpar) * rs;
    c.Btt = M::sqrt(J.twof * kpar);
    c.invr = invr;
    c.invst = invst;
    if (FULL) {
        c.Hw = Hw;
        c.vdr = vdr;
        c.vdt = vdt;
        c.vdp = vdp;
        c.Krr = Krr;
        c.Krp = Krp;
        c.kpar = kpar;
    }
}

// Energy form (Eq.(1), rearranged into the backward form of Eq.(2)): the
// kinetic energy T advances with dT = (1/3)(div V) alpha T ds, alpha =
// (T + 2M)/(T + M), and each step adds L ds to the exponent of Eq.(4),
// L = (div V)[1 - (1/3) d(alpha T)/dT] with d(alpha T)/dT = 1 + (M/(T+M))^2;
// div V = 2V/r.  The spatial part is the momentum form's at the rigidity
// P = sqrt(T (T + 2M)) / |Z|.
__device__ __forceinline__ double rigidity_of_T(double T, double M, double abs_z)
{
    return ::sqrt(T * (T + 2.0 * M)) / abs_z;
}

// A lane's view of its job's region entries: the table's base, the same for
// every lane, and the byte offset of the job's first entry, so the per-step
// load is the base plus one 32-bit offset.
template <typename R>
struct RegionRef {
    const RegionDev<R>* base;
    uint32_t off;
    __device__ __forceinline__ RegionDev<R> at(int k) const
    {
        return *(const RegionDev<R>*)((const char*)base +
                                      (off + (uint32_t)k * (uint32_t)sizeof(RegionDev<R>)));
    }
};

// phi outside [0, 2 pi) (or NaN).  In binary32 one unsigned compare of the
// bits: non-negative floats order like their bit patterns, and every negative
// one (sign bit set) lies above the pattern of 2 pi.
__device__ __forceinline__ bool outside_turn(float x)
{
    return __float_as_uint(x) >= __float_as_uint((float)kTwoPi);
}
__device__ __forceinline__ bool outside_turn(double x) { return !(x >= 0.0 && x < kTwoPi); }

// One EM step of the 3D model.  The caller tests for the exit.
template <typename R, bool UKEY, bool SHAPED, bool ENERGY>
__device__ __forceinline__ void step3d(const JobReg<R>& J, const JobDev<R>* __restrict__ jd,
                                       const RegionRef<R> reg, PState<R>& s,
                                       uint32_t pid, uint32_t bin, uint32_t k0, uint32_t k1)
{
    using M = Mth<R>;
    R z[3];
    normals<R, 3>(UKEY ? k0 : J.seed_lo, UKEY ? k1 : J.seed_hi, s.n, pid, bin, J.job_tag, z);
    const RegionDev<R> g = reg.at(region_at<R, SHAPED>(J, jd, s.r, s.th, s.ph));
    const bool efo = ENERGY && J.energy != 0;
    R Pc = (R)s.P;  // the rigidity the coefficients see
    if (efo) {
        if constexpr (std::is_same<R, float>::value) {
            // the rigidity of T; binary32 suffices there
            const float T = (float)s.T;
            Pc = M::sqrt(T * (T + 2.0f * J.mass)) * M::rcp(J.abs_z);
        } else {
            Pc = rigidity_of_T(s.T, J.mass, (double)J.abs_z);
        }
    }
    Coef3<R> c;
    coeffs3d<R, false>(J, g, s.r, Pc, s.th, s.ph, c);
    const R dt = c.dt;
    const R sdt = M::sqrt(dt);
    double r1;
    R th1, ph1;
    double P1;
    if constexpr (std::is_same<R, float>::value) {
        // binary32 increments, accumulated into the binary64 r, P, t
        const float sdi = sdt * c.invr;
        r1 = s.r + (double)((c.Brr * z[0]) * sdt + c.Ar * dt);
        th1 = (c.Btt * z[2]) * sdi + (c.At * dt + s.th);
        ph1 = (c.Bpr * z[0] + c.Bpp * z[1]) * (sdi * c.invst) + (c.Ap * dt + s.ph);
        P1 = s.P + (double)(c.AP * dt);
    } else {
        // same association of terms as a plain left-to-right evaluation
        r1 = s.r + c.Ar * dt + c.Brr * z[0] * sdt;
        th1 = s.th + c.At * dt + c.Btt * z[2] * sdt * c.invr;
        ph1 = s.ph + c.Ap * dt + (c.Bpr * z[0] + c.Bpp * z[1]) * sdt * (c.invr * c.invst);
        P1 = s.P + c.AP * dt;
    }
    // reflections through the origin and the poles are rare: a wave branches
    // to them only when one of its lanes needs them
    if (__builtin_amdgcn_ballot_w64(r1 < 0.0) != 0) {
        __asm__ volatile("");  // keeps the block a branch instead of selects
        if (r1 < 0.0) {
            r1 = -r1;
            th1 = (R)kPi - th1;
            ph1 = ph1 + (R)kPi;
        }
    }
    if (__builtin_amdgcn_ballot_w64(th1 < (R)0) != 0) {
        __asm__ volatile("");
        if (th1 < (R)0) {
            th1 = -th1;
            ph1 = ph1 + (R)kPi;
        }
    }
    if (th1 > (R)kPi) {
        th1 = M::fmod2pi(th1);
        if (th1 > (R)kPi) {
            th1 = (R)kTwoPi - th1;
            ph1 = ph1 + (R)kPi;
        }
    }
    if (outside_turn(ph1)) {
        ph1 = M::fmod2pi(ph1);
        if (ph1 < (R)0) ph1 = ph1 + (R)kTwoPi;
    }
    if (efo) {
        // (1/3) div V, alpha T and the loss at the start of the step
        const R T = (R)s.T, Mr = J.mass;
        const R divV3 = ((R)2.0 / (R)3.0) * c.V * c.invr;
        const R ie = M::rcp(T + Mr);
        const R alphaT = ((T + (R)2.0 * Mr) * ie) * T;
        const R me = Mr * ie;
        const R L = divV3 * ((R)2.0 - me * me);  // (div V) (1 - (1 + me^2) / 3)
        s.T = s.T + (double)(divV3 * alphaT * dt);
        s.lam = s.lam + (double)(L * dt);
        P1 = s.P;  // the rigidity is refreshed from T when the particle leaves
    }
    s.r = r1;
    s.th = th1;
    s.ph = ph1;
    s.P = P1;
    s.t = s.t + (double)dt;
    s.n = s.n + 1u;
}

// One EM step of the radial model: dr = (2k/r - V) ds + sqrt(2k) dW.
template <typename R, bool UKEY>
__device__ __forceinline__ void step1d(const JobReg<R>& J, const RegionRef<R> reg,
                                       PState<R>& s, uint32_t pid, uint32_t bin, uint32_t k0,
                                       uint32_t k1)
{
    using M = Mth<R>;
    R z[1];
    normals<R, 1>(UKEY ? k0 : J.seed_lo, UKEY ? k1 : J.seed_hi, s.n, pid, bin, J.job_tag, z);
    const RegionDev<R> g = reg.at(region_of(J, s.r));
    const R r0 = (R)s.r;
    const R r = r0 > M::kRFloor ? r0 : M::kRFloor;
    const R P = (R)s.P;
    const R invr = M::rcp(r);
    const R pc = J.abs_z * P;
    const R beta = pc * M::rsqrt(pc * pc + J.mass2);
    const R kap = g.k0 * beta * P;
    const R V = g.vs;
    const R Ar = (R)2.0 * kap * invr - V;
    const R Brr = M::sqrt((R)2.0 * kap);
    const R AP = (R)(2.0 / 3.0) * V * P * invr;
    R dt = J.dt_max;
    const R d1 = J.diff_frac * r * r * M::rcp(kap);
    dt = fmin(d1, dt);
    const R sdt = M::sqrt(dt);
    double r1 = s.r + (double)(Ar * dt) + (double)(Brr * z[0] * sdt);
    const double P1 = s.P + (double)(AP * dt);
    if (r1 < 0.0) r1 = -r1;
    s.r = r1;
    s.P = P1;
    s.t = s.t + (double)dt;
    s.n = s.n + 1u;
}

// ---------------------------------------------------------------------------
// Persistent propagation kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// The binary32 energy-form variants are held to 128 VGPRs (4 waves per SIMD).
template <typename R, bool M3D, bool UKEY, bool SHAPED, bool ENERGY>
__global__ void __launch_bounds__(256, ((std::is_same<R, float>::value && M3D) ? (ENERGY ? 4 : 1) : 1))
k_propagate(const PropArgs<R> a)
{
    const uint32_t lane = __lane_id();
    PState<R> s = {0.0, 0.0, 0.0, (R)0, (R)0, 0u, 0.0, 0.0};
    uint32_t pid = 0, bin = 0, job = 0, out = 0, seg = 0;
    JobReg<R> J = {};
    RegionRef<R> reg = {a.regions, 0u};
    const JobDev<R>* jd = a.jobs;  // the lane's job entry (surface constants)
    bool active = false;
    // steps this wave has taken in this launch (wave-uniform), counted against
    // a.step_budget when the launch is a slice; a slice also ends at a time
    // every wave reads from the device's constant-rate clock, so the waves stop
    // together instead of the slice waiting for its slowest wave's budget
    uint32_t wave_steps = 0;
    // a serving slice parks into the lists of its descriptor
    const SliceDev* sv = a.slice;
    const bool sliced = sv != nullptr && (a.step_budget != 0xffffffffu || a.slice_ticks != 0);
    const uint64_t t_stop =
        a.slice_ticks != 0 ? (uint64_t)wall_clock64() + a.slice_ticks : ~(uint64_t)0;

    // wave-uniform refill cursors
    uint32_t c_seg = 0, c_next = 0, c_end = 0;
    // the counts of a slice's resume and remainder lists are read where they are
    // used (kept live across the kernel they would cost registers)
    bool resume_open = sv != nullptr;
    bool left_open = sv != nullptr;
    bool queue_open = true;
    bool launch_open = true;  // false once this wave used its step budget

    for (;;) {
        uint64_t need = __ballot(!active);
        // 1) suspended particles of earlier slices come back first
        while (need != 0 && resume_open && launch_open) {
            uint32_t base = 0;
            const uint32_t cnt = (uint32_t)__popcll(need);
            if (lane == 0) base = atomicAdd(sv->resume_head, cnt);
            base = wave_uniform(base);
            // (a count past the list's capacity only follows an overflow,
            // which the host reports as an error)
            const uint32_t n_resume = min(*sv->n_resume, sv->park_cap);
            if (base >= n_resume) {
                resume_open = false;
                break;
            }
            const uint32_t rank = lane_rank(need);
            if (!active && base + rank < n_resume) {
                // kernels without the energy form leave T and the loss unread
                const uint32_t i = base + rank;
                const ParkDev& q = sv->resume;
                s.r = q.r[i];
                s.P = q.P[i];
                s.t = q.t[i];
                s.th = (R)q.th[i];
                s.ph = (R)q.ph[i];
                s.n = q.n[i];
                seg = q.seg[i];
                pid = q.pid[i];
                const SegmentDev sg = a.segs[seg];
                job = sg.job;
                bin = sg.bin;
                out = sg.out_offset + pid;
                J = load_job(a.jobs[job]);
                if (ENERGY) {
                    // momentum-form particles may have been parked by a kernel
                    // that did not store T and the loss
                    s.T = J.energy ? q.T[i] : 0.0;
                    s.lam = J.energy ? q.lam[i] : 0.0;
                }
                jd = a.jobs + job;
                reg.off = job * (uint32_t)(kRegionStride * sizeof(RegionDev<R>));
                active = true;
            }
            need = __ballot(!active);
        }
        // 2) new particles from the chunk queue
        while (need != 0 && !resume_open && queue_open && launch_open) {
            if (c_next == c_end) {
                // remainders the previous slice left unissued go first
                ChunkDev ch;
                bool got = false;
                if (left_open) {
                    uint32_t c = 0;
                    if (lane == 0) c = atomicAdd(sv->left_in_head, 1u);
                    c = wave_uniform(c);
                    if (c < min(*sv->n_left_in, sv->left_cap)) {
                        ch = sv->left_in[c];
                        got = true;
                    } else {
                        left_open = false;
                    }
                }
                if (!got) {
                    unsigned long long c = 0;
                    if (lane == 0) c = atomicAdd(a.head, 1ull);
                    c = ((unsigned long long)wave_uniform((uint32_t)(c >> 32)) << 32) |
                        wave_uniform((uint32_t)c);
                    if (c >= a.q_tail) {
                        queue_open = false;
                        break;
                    }
                    ch = a.chunks[c & a.q_mask];
                }
                c_seg = wave_uniform(ch.seg);
                c_next = wave_uniform(ch.first);
                c_end = c_next + wave_uniform(ch.count);
            }
            const SegmentDev sg = a.segs[c_seg];
            const uint32_t avail = c_end - c_next;
            const uint32_t rank = lane_rank(need);
            if (!active && rank < avail) {
                const JobDev<R>& Jd = a.jobs[sg.job];
                seg = c_seg;
                pid = c_next + rank;
                job = sg.job;
                bin = sg.bin;
                out = sg.out_offset + pid;
                J = load_job(Jd);
                jd = a.jobs + job;
                reg.off = job * (uint32_t)(kRegionStride * sizeof(RegionDev<R>));
                if (Jd.n_orbit == 0) {
                    s.r = Jd.r0;
                    s.th = (R)Jd.th0;
                    s.ph = (R)Jd.ph0;
                } else {
                    // moving detection point: particle i starts at position i mod n
                    const OrbitDev o = a.orbit[Jd.orbit_off + pid % Jd.n_orbit];
                    s.r = o.r;
                    s.th = (R)o.th;
                    s.ph = (R)o.ph;
                }
                s.P = sg.P0;
                s.t = 0.0;
                s.n = 0u;
                if (ENERGY) {
                    // kinetic energy from rigidity: E^2 = (Z P)^2 + M^2
                    const double pc = (double)J.abs_z * sg.P0;
                    s.T = ::sqrt(pc * pc + Jd.mass * Jd.mass) - Jd.mass;
                    s.lam = 0.0;
                }
                active = true;
            }
            const uint32_t cnt = (uint32_t)__popcll(need);
            c_next += cnt < avail ? cnt : avail;
            need = __ballot(!active);
        }
        if (!__any(active)) {
            // hand back the unissued rest of this wave's chunk (nothing of a
            // cancelled job)
            if (c_next < c_end && lane == 0 && sv != nullptr &&
                !(a.job_cancel != nullptr && a.job_cancel[a.segs[c_seg].job] != 0u)) {
                const uint32_t slot = atomicAdd(sv->leftover_count, 1u);
                if (slot < sv->left_cap) {
                    ChunkDev ch;
                    ch.seg = c_seg;
                    ch.first = c_next;
                    ch.count = c_end - c_next;
                    ch.pad0 = 0;
                    sv->leftover[slot] = ch;
                } else {
                    *sv->overflow = 1u;
                }
            }
            break;
        }

        // a cancelled job's particles are dropped without a record
        if (active && a.job_cancel != nullptr && a.job_cancel[job] != 0u) active = false;
        if (!__any(active)) continue;

        // Advance the active lanes in lockstep until one of them leaves (boundary
        // crossing, non-finite state or step cap) or the slice is over.  The loop
        // carries only the particle state, so it stays in place; why a lane left
        // is worked out afterwards from its state.  SK: the Philox key (k0, k1)
        // is the same for every active lane and sits in scalar registers.
        // SL: the launch is a serving slice (budget and clock checks).
        bool slice_over = false;
        uint32_t k0 = a.key_lo, k1 = a.key_hi;
        auto lockstep = [&](auto sk, auto sl) {
            constexpr bool SK = decltype(sk)::value;
            constexpr bool SL = decltype(sl)::value;
            // Where the loop sits in memory sets its issue rate: with the same
            // instructions, the binary32 3D loops measured from 0.6% to 7% slower
            // at other offsets within a 64-byte line than at byte 48 (a line
            // boundary, then 11 four-byte s_nop, run once per entry: the loop's
            // own first instruction follows them).
            if constexpr (M3D && std::is_same<R, float>::value)
                __asm__ volatile(".p2align 6\n.rept 11\ns_nop 0\n.endr");
            for (;;) {
                bool leave = false;
                if (active) {
                    if (M3D)
                        step3d<R, SK, SHAPED, ENERGY>(J, jd, reg, s, pid, bin, k0, k1);
                    else
                        step1d<R, SK>(J, reg, s, pid, bin, k0, k1);
                    leave = outside_boundary<R, SHAPED>(J, jd, s.r, s.th, s.ph) ||
                            s.n >= J.step_cap;
                }
                ++wave_steps;
                if constexpr (SL) {
                    if (wave_steps >= a.step_budget ||
                        ((wave_steps & 15u) == 0u && (uint64_t)wall_clock64() >= t_stop))
                        slice_over = true;
                    if (__any(leave) || slice_over) break;
                } else {
                    if (__any(leave)) break;
                }
            }
        };
        auto keyed = [&](auto sl) {
            if constexpr (UKEY) {
                lockstep(std::true_type{}, sl);
            } else {
                // Jobs of a launch may carry different seeds, but a wave's lanes
                // often hold particles of one job (a refill chunk is one bin):
                // then the key schedule runs on the scalar unit too.
                const uint64_t act = __ballot(active);
                const int first = (int)__builtin_ctzll(act);
                k0 = (uint32_t)__builtin_amdgcn_readlane((int)J.seed_lo, first);
                k1 = (uint32_t)__builtin_amdgcn_readlane((int)J.seed_hi, first);
                if (__all(!active || (J.seed_lo == k0 && J.seed_hi == k1)))
                    lockstep(std::true_type{}, sl);
                else
                    lockstep(std::false_type{}, sl);
            }
        };
        if (sliced)
            keyed(std::true_type{});
        else
            keyed(std::false_type{});
        const bool outside = active && outside_boundary<R, SHAPED>(J, jd, s.r, s.th, s.ph);
        const bool bad_T = ENERGY && !(s.T == s.T);
        if (active && (outside || !(s.P == s.P) || bad_T || s.n >= J.step_cap)) {
            uint32_t flags = 0;
            if (!(s.r == s.r) || !(s.P == s.P) || bad_T)
                flags = kFlagNaN;
            else if (!outside)
                flags = kFlagCapped;
            if (ENERGY && J.energy) {
                s.P = rigidity_of_T(s.T, jd->mass, (double)J.abs_z);
                a.exL[out] = s.lam;
            }
            a.exP[out] = s.P;
            a.exT[out] = s.t;
            a.exNF[out] = s.n | (flags << kFlagShift);
            if (a.exR != nullptr) {
                a.exR[out] = s.r;
                a.exTh[out] = (double)s.th;
                a.exPh[out] = (double)s.ph;
            }
            if (a.job_done != nullptr) atomicAdd(&a.job_done[job], 1u);
            active = false;
        }
        if (slice_over) {
            // slice over (wave-uniform): park the wave's particles in
            // consecutive entries for the next launch and stop taking work
            const uint64_t parked = __ballot(active);
            if (parked != 0) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(sv->suspend_count, (uint32_t)__popcll(parked));
                base = wave_uniform(base);
                const uint32_t i = base + lane_rank(parked);
                const ParkDev& q = sv->suspend;
                if (active && i < sv->park_cap) {
                    q.r[i] = s.r;
                    q.P[i] = s.P;
                    q.t[i] = s.t;
                    q.th[i] = (double)s.th;
                    q.ph[i] = (double)s.ph;
                    q.n[i] = s.n;
                    q.seg[i] = seg;
                    q.pid[i] = pid;
                    // an energy-form particle is only ever parked by a launch of
                    // the energy-form kernel, so only that kernel stores T and
                    // the loss
                    if (ENERGY) {
                        q.T[i] = s.T;
                        q.lam[i] = s.lam;
                    }
                } else if (active) {
                    *sv->overflow = 1u;
                }
                active = false;
            }
            launch_open = false;
        }
    }
}

template <typename R, bool M3D, bool SHAPED, bool ENERGY>
static void launch_keyed(const PropArgs<R>& a, int grid, int block, hipStream_t s)
{
    // one Philox key for the whole launch: the key schedule runs on the scalar unit
    if (a.uniform_key)
        hipLaunchKernelGGL((k_propagate<R, M3D, true, SHAPED, ENERGY>), dim3(grid), dim3(block),
                           0, s, a);
    else
        hipLaunchKernelGGL((k_propagate<R, M3D, false, SHAPED, ENERGY>), dim3(grid), dim3(block),
                           0, s, a);
}

template <typename R, bool M3D>
static hipError_t launch_prop(const PropArgs<R>& a, int grid, int block, hipStream_t s)
{
    // squashed heliopause / heliosheath tests, and the energy form, only where a
    // job of the launch needs them
    if constexpr (M3D) {
        if (a.shaped && a.energy)
            launch_keyed<R, M3D, true, true>(a, grid, block, s);
        else if (a.shaped)
            launch_keyed<R, M3D, true, false>(a, grid, block, s);
        else if (a.energy)
            launch_keyed<R, M3D, false, true>(a, grid, block, s);
        else
            launch_keyed<R, M3D, false, false>(a, grid, block, s);
    } else {
        launch_keyed<R, M3D, false, false>(a, grid, block, s);
    }
    return hipGetLastError();
}

hipError_t launch_propagate_3d_mixed(const PropArgs<float>& a, int grid, int block, hipStream_t s)
{
    return launch_prop<float, true>(a, grid, block, s);
}
hipError_t launch_propagate_3d_fp64(const PropArgs<double>& a, int grid, int block, hipStream_t s)
{
    return launch_prop<double, true>(a, grid, block, s);
}
hipError_t launch_propagate_1d_mixed(const PropArgs<float>& a, int grid, int block, hipStream_t s)
{
    return launch_prop<float, false>(a, grid, block, s);
}
hipError_t launch_propagate_1d_fp64(const PropArgs<double>& a, int grid, int block, hipStream_t s)
{
    return launch_prop<double, false>(a, grid, block, s);
}

template <typename R, bool M3D, bool SHAPED, bool ENERGY>
static void keyed_variants(const void** f)
{
    f[0] = (const void*)&k_propagate<R, M3D, false, SHAPED, ENERGY>;
    f[1] = (const void*)&k_propagate<R, M3D, true, SHAPED, ENERGY>;
}

template <typename R>
static void model3d_variants(int shaped, int energy, const void** f)
{
    if (shaped && energy)
        keyed_variants<R, true, true, true>(f);
    else if (shaped)
        keyed_variants<R, true, true, false>(f);
    else if (energy)
        keyed_variants<R, true, false, true>(f);
    else
        keyed_variants<R, true, false, false>(f);
}

hipError_t occupancy_propagate(int model, int prec, int block, int shaped, int energy, int ukey,
                               int* blocks_per_cu)
{
    const void* f[2] = {nullptr, nullptr};
    if (model == 1 && prec == 1)
        model3d_variants<float>(shaped, energy, f);
    else if (model == 1 && prec == 0)
        model3d_variants<double>(shaped, energy, f);
    else if (model == 0 && prec == 1)
        keyed_variants<float, false, false, false>(f);
    else if (model == 0 && prec == 0)
        keyed_variants<double, false, false, false>(f);
    else
        return hipErrorInvalidValue;
    // the variant the launch runs: one Philox key for the launch (f[1]) or a
    // key per lane (f[0])
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f[ukey ? 1 : 0], block, 0);
    if (e != hipSuccess) return e;
    *blocks_per_cu = n;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Per-bin reduction.
// ---------------------------------------------------------------------------
constexpr int kReduceBlock = 256;
// The reduction of one rigidity bin runs in one workgroup; a served request
// reduces its few bins alone, so each one takes a whole CU's worth of waves.
constexpr int kBinBlock = 1024;

template <typename T, int B = kReduceBlock>
__device__ __forceinline__ T block_sum(T v, T* sh)
{
    // fixed-order tree: wave shuffles, then the wave partials in LDS
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int wid = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[wid] = v;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < B / 64; ++i) t += sh[i];
        sh[0] = t;
    }
    __syncthreads();
    t = sh[0];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double lis_weight(const LisDev& L, double P)
{
    // f_LIS(P) = J_LIS(P) / P^2
    return L.norm * ::pow(P, -L.index) / (P * P);
}

// Energy form: U = 4 pi p^2 f / v is transported with the loss weight, so a
// particle contributes beta0 / beta_ex J_LIS(P_ex) exp(-loss) to J_mod(P0).
__device__ __forceinline__ double beta_of(const LisDev& L, double P)
{
    const double pc = L.abs_z * P;
    return pc / ::sqrt(pc * pc + L.mass * L.mass);
}

__device__ __forceinline__ double energy_weight(const LisDev& L, double beta0, double P,
                                                double loss)
{
    return beta0 / beta_of(L, P) * (L.norm * ::pow(P, -L.index)) * ::exp(-loss);
}

__global__ void __launch_bounds__(kBinBlock) k_reduce(const ReduceArgs a)
{
    __shared__ uint32_t hist[kNHist];
    __shared__ double shd[kBinBlock / 64];
    __shared__ unsigned long long shu[kBinBlock / 64];
    const uint32_t sidx = a.seg_base + blockIdx.x;
    const SegmentDev sg = a.segs[sidx];
    const LisDev L = a.lis[sg.job];
    for (int i = threadIdx.x; i < kNHist; i += kBinBlock) hist[i] = 0u;
    __syncthreads();
    double sw = 0.0, st = 0.0;
    unsigned long long sn = 0, ncap = 0, nnan = 0, nused = 0;
    const double inv_p0 = 1.0 / sg.P0;
    const double beta0 = L.energy ? beta_of(L, sg.P0) : 0.0;
    for (uint32_t i = threadIdx.x; i < sg.count; i += kBinBlock) {
        const uint32_t o = sg.out_offset + i;
        const uint32_t nf = a.exNF[o];
        const uint32_t fl = nf >> kFlagShift;
        sn += nf & ((1u << kFlagShift) - 1u);
        if (fl & kFlagCapped) {
            ++ncap;
            continue;
        }
        if (fl & kFlagNaN) {
            ++nnan;
            continue;
        }
        const double P = a.exP[o];
        sw += L.energy ? energy_weight(L, beta0, P, a.exL[o]) : lis_weight(L, P);
        st += a.exT[o];
        ++nused;
        int j = (int)::floor(128.0 * ::log10(P * inv_p0) / 3.0);
        j = j < 0 ? 0 : (j > 128 ? 128 : j);
        atomicAdd(&hist[j], 1u);
    }
    const double SW = block_sum<double, kBinBlock>(sw, shd);
    const double ST = block_sum<double, kBinBlock>(st, shd);
    const unsigned long long SN = block_sum<unsigned long long, kBinBlock>(sn, shu);
    const unsigned long long NC = block_sum<unsigned long long, kBinBlock>(ncap, shu);
    const unsigned long long NN = block_sum<unsigned long long, kBinBlock>(nnan, shu);
    const unsigned long long NU = block_sum<unsigned long long, kBinBlock>(nused, shu);
    const double N = (double)NU;
    const double mean = NU > 0 ? SW / N : 0.0;
    double ss = 0.0;
    if (NU > 1) {
        for (uint32_t i = threadIdx.x; i < sg.count; i += kBinBlock) {
            const uint32_t o = sg.out_offset + i;
            if ((a.exNF[o] >> kFlagShift) != 0u) continue;
            const double w = L.energy ? energy_weight(L, beta0, a.exP[o], a.exL[o])
                                      : lis_weight(L, a.exP[o]);
            const double dw = w - mean;
            ss += dw * dw;
        }
    }
    const double SS = block_sum<double, kBinBlock>(ss, shd);
    __syncthreads();
    const uint32_t ob = a.out_base + blockIdx.x;
    if (a.hist != nullptr)
        for (int i = threadIdx.x; i < kNHist; i += kBinBlock)
            a.hist[(size_t)ob * kNHist + i] = hist[i];
    if (threadIdx.x == 0) {
        // momentum form: mean of f_LIS(P_ex) times P0^2; energy form: the mean
        // contribution itself
        const double p2 = L.energy ? 1.0 : sg.P0 * sg.P0;
        if (a.flux) a.flux[ob] = p2 * mean;
        if (a.flux_se) a.flux_se[ob] = NU > 1 ? p2 * ::sqrt(SS / (N - 1.0) / N) : 0.0;
        if (a.mean_t) a.mean_t[ob] = NU > 0 ? ST / N : 0.0;
        if (a.steps) a.steps[ob] = SN;
        if (a.n_capped) a.n_capped[ob] = (uint32_t)NC;
        if (a.n_nan) a.n_nan[ob] = (uint32_t)NN;
    }
}

hipError_t launch_reduce(const ReduceArgs& a, uint32_t n_segs, hipStream_t s)
{
    if (n_segs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n_segs), dim3(kBinBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Re-weighting of stored exit records with tabulated spectra (Eq.(4) with
// other J_LIS): one workgroup per (segment, group of kReweightGroup spectra).
// ln J is linear in ln P between knots ln P = lnP0 + k dlnP, with the end
// segments extended.  The group's tables sit in LDS; each particle's ln P and
// its form-dependent factor are computed once for the whole group.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kReduceBlock) k_reweight(const ReweightArgs a)
{
    __shared__ double tab[kReweightGroup * kMaxLisKnots];
    __shared__ double shd[kReduceBlock / 64];
    const uint32_t sidx = a.seg_base + blockIdx.x;
    const uint32_t l0 = blockIdx.y * kReweightGroup;
    const uint32_t nl = a.n_lis - l0 < (uint32_t)kReweightGroup ? a.n_lis - l0
                                                                 : (uint32_t)kReweightGroup;
    for (uint32_t i = threadIdx.x; i < nl * a.n_knots; i += kReduceBlock)
        tab[i] = a.lnJ[(size_t)l0 * a.n_knots + i];
    __syncthreads();
    const SegmentDev sg = a.segs[sidx];
    const LisDev L = a.lis[sg.job];
    const double beta0 = L.energy ? beta_of(L, sg.P0) : 0.0;
    const double p02 = sg.P0 * sg.P0;
    const double inv_d = 1.0 / a.dlnP;
    const int kmax = (int)a.n_knots - 2;
    // weight of particle o with table t (the factor is beta0/beta_ex exp(-loss)
    // in the energy form, P0^2/P_ex^2 in the momentum form)
    auto factor_and_pos = [&](uint32_t o, double* fac, int* k, double* f) {
        const double P = a.exP[o];
        *fac = L.energy ? beta0 / beta_of(L, P) * ::exp(-a.exL[o]) : p02 / (P * P);
        const double x = (::log(P) - a.lnP0) * inv_d;
        // clamp before the conversion; beyond the ends f extrapolates
        const double xc = x < 0.0 ? 0.0 : (x > (double)kmax ? (double)kmax : x);
        const int kk = (int)::floor(xc);
        *k = kk;
        *f = x - (double)kk;
    };
    double acc[kReweightGroup];
    for (int l = 0; l < kReweightGroup; ++l) acc[l] = 0.0;
    unsigned long long nused = 0;
    for (uint32_t i = threadIdx.x; i < sg.count; i += kReduceBlock) {
        const uint32_t o = sg.out_offset + i;
        if ((a.exNF[o] >> kFlagShift) != 0u) continue;  // capped or non-finite
        double fac, f;
        int k;
        factor_and_pos(o, &fac, &k, &f);
        ++nused;
#pragma unroll
        for (int l = 0; l < kReweightGroup; ++l) {
            if ((uint32_t)l < nl) {
                const double* t = tab + l * a.n_knots;
                acc[l] += fac * ::exp(t[k] + f * (t[k + 1] - t[k]));
            }
        }
    }
    __shared__ unsigned long long shu[kReduceBlock / 64];
    const double N = (double)block_sum<unsigned long long>(nused, shu);
    double mean[kReweightGroup];
    for (int l = 0; l < kReweightGroup; ++l) {
        const double S = block_sum<double>(acc[l], shd);
        mean[l] = N > 0.0 ? S / N : 0.0;
        acc[l] = 0.0;
    }
    if (N > 1.0) {
        for (uint32_t i = threadIdx.x; i < sg.count; i += kReduceBlock) {
            const uint32_t o = sg.out_offset + i;
            if ((a.exNF[o] >> kFlagShift) != 0u) continue;
            double fac, f;
            int k;
            factor_and_pos(o, &fac, &k, &f);
#pragma unroll
            for (int l = 0; l < kReweightGroup; ++l) {
                if ((uint32_t)l < nl) {
                    const double* t = tab + l * a.n_knots;
                    const double d = fac * ::exp(t[k] + f * (t[k + 1] - t[k])) - mean[l];
                    acc[l] += d * d;
                }
            }
        }
    }
    for (int l = 0; l < kReweightGroup; ++l) {
        const double SS = block_sum<double>(acc[l], shd);
        if (threadIdx.x == 0 && (uint32_t)l < nl) {
            const size_t ob = (size_t)(l0 + l) * a.total_bins + a.out_base + blockIdx.x;
            a.flux[ob] = mean[l];
            a.flux_se[ob] = N > 1.0 ? ::sqrt(SS / (N - 1.0) / N) : 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// Exit histogram over the reached range (Sec. IV.A: the largest exit energy of
// the sample sets the histogram's binning): one workgroup per bin takes the
// largest used exit rigidity P_max, then counts ln(P_ex / P0) in n_hist equal
// bins over [0, ln(P_max / P0)] (index floor(n_hist x / x_max), the record at
// P_max in the last bin) with LDS atomics.  Capped and non-finite records are
// left out.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_max(double v, double* sh)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    const int wid = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int i = 1; i < kReduceBlock / 64; ++i) t = fmax(t, sh[i]);
        sh[0] = t;
    }
    __syncthreads();
    const double t = sh[0];
    __syncthreads();
    return t;
}

__global__ void __launch_bounds__(kReduceBlock) k_exit_range(const RangeArgs a)
{
    __shared__ uint32_t h[kMaxRangeBins];
    __shared__ double shd[kReduceBlock / 64];
    const SegmentDev sg = a.segs[a.seg_base + blockIdx.x];
    double pm = 0.0;
    for (uint32_t i = threadIdx.x; i < sg.count; i += kReduceBlock) {
        const uint32_t o = sg.out_offset + i;
        if ((a.exNF[o] >> kFlagShift) == 0u) pm = fmax(pm, a.exP[o]);
    }
    pm = block_max(pm, shd);
    for (uint32_t k = threadIdx.x; k < a.n_hist; k += kReduceBlock) h[k] = 0u;
    __syncthreads();
    if (pm > 0.0) {
        const double xmax = ::log(pm / sg.P0);
        for (uint32_t i = threadIdx.x; i < sg.count; i += kReduceBlock) {
            const uint32_t o = sg.out_offset + i;
            if ((a.exNF[o] >> kFlagShift) != 0u) continue;
            uint32_t k = 0;
            if (xmax > 0.0) {
                const double x = ::log(a.exP[o] / sg.P0);
                const double f = ::floor((double)a.n_hist * x / xmax);
                k = f <= 0.0 ? 0u : (f >= (double)a.n_hist ? a.n_hist - 1u : (uint32_t)f);
            }
            atomicAdd(&h[k], 1u);
        }
    }
    __syncthreads();
    const size_t ob = (size_t)a.out_base + blockIdx.x;
    for (uint32_t k = threadIdx.x; k < a.n_hist; k += kReduceBlock)
        a.hist[ob * a.n_hist + k] = h[k];
    if (threadIdx.x == 0) a.p_max[ob] = pm;
}

hipError_t launch_exit_range(const RangeArgs& a, uint32_t n_segs, hipStream_t s)
{
    if (n_segs == 0 || a.n_hist == 0 || a.n_hist > (uint32_t)kMaxRangeBins)
        return n_segs == 0 ? hipSuccess : hipErrorInvalidValue;
    hipLaunchKernelGGL(k_exit_range, dim3(n_segs), dim3(kReduceBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reweight(const ReweightArgs& a, uint32_t n_segs, hipStream_t s)
{
    if (n_segs == 0 || a.n_lis == 0) return hipSuccess;
    const uint32_t groups = (a.n_lis + kReweightGroup - 1) / kReweightGroup;
    hipLaunchKernelGGL(k_reweight, dim3(n_segs, groups), dim3(kReduceBlock), 0, s, a);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint32_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

// One workgroup: the leftovers of a slice are few (none unless the slice ran a
// kernel variant with fewer lanes than the previous one).
__global__ void __launch_bounds__(256) k_slice_close(const CloseArgs a)
{
    const SliceDev& sl = a.sl;
    const uint32_t n_in = min(*sl.n_resume, sl.park_cap);
    const uint32_t in_head = *sl.resume_head;
    const uint32_t n_lin = min(*sl.n_left_in, sl.left_cap);
    const uint32_t lin_head = *sl.left_in_head;
    for (uint32_t i = (in_head < n_in ? in_head : n_in) + threadIdx.x; i < n_in; i += blockDim.x) {
        const uint32_t seg = sl.resume.seg[i];
        if (a.job_cancel != nullptr && a.job_cancel[a.segs[seg].job] != 0u) continue;
        const uint32_t o = atomicAdd(sl.suspend_count, 1u);
        if (o >= sl.park_cap) {
            *sl.overflow = 1u;
            continue;
        }
        const ParkDev& in = sl.resume;
        const ParkDev& out = sl.suspend;
        out.r[o] = in.r[i];
        out.P[o] = in.P[i];
        out.t[o] = in.t[i];
        out.th[o] = in.th[i];
        out.ph[o] = in.ph[i];
        out.T[o] = in.T[i];
        out.lam[o] = in.lam[i];
        out.n[o] = in.n[i];
        out.seg[o] = seg;
        out.pid[o] = in.pid[i];
    }
    for (uint32_t i = (lin_head < n_lin ? lin_head : n_lin) + threadIdx.x; i < n_lin;
         i += blockDim.x) {
        const ChunkDev ch = sl.left_in[i];
        if (a.job_cancel != nullptr && a.job_cancel[a.segs[ch.seg].job] != 0u) continue;
        const uint32_t o = atomicAdd(sl.leftover_count, 1u);
        if (o >= sl.left_cap) {
            *sl.overflow = 1u;
            continue;
        }
        sl.leftover[o] = ch;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (*a.head > a.q_tail) *a.head = a.q_tail;
        for (int k = 0; k < 4; ++k) a.next_counters[k] = 0u;
    }
}

hipError_t launch_slice_close(const CloseArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_slice_close, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void k_pack_exits(const double* P, const double* T, const uint32_t* NF,
                             const double* L, const double* R, const double* Th,
                             const double* Ph, uint32_t n, ExitRecDev* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ExitRecDev e;
    e.P = P[i];
    e.t = T[i];
    e.r = R ? R[i] : 0.0;
    e.th = Th ? Th[i] : 0.0;
    e.ph = Ph ? Ph[i] : 0.0;
    e.n = NF[i] & ((1u << kFlagShift) - 1u);
    e.flags = NF[i] >> kFlagShift;
    e.loss = L ? L[i] : 0.0;
    out[i] = e;
}

hipError_t launch_pack_exits(const double* P, const double* T, const uint32_t* NF,
                             const double* L, const double* R, const double* Th,
                             const double* Ph, uint32_t n, ExitRecDev* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_exits, dim3((n + 255) / 256), dim3(256), 0, s, P, T, NF, L, R, Th,
                       Ph, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagnostics.
// ---------------------------------------------------------------------------
__global__ void k_probe_rng(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                            uint32_t c3, uint32_t n, uint32_t* words, double* z64, float* z32)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 x = philox4x32_10(k0, k1, c0 + i, c1, c2, c3);
    if (words) {
        words[4 * (size_t)i + 0] = x.x;
        words[4 * (size_t)i + 1] = x.y;
        words[4 * (size_t)i + 2] = x.z;
        words[4 * (size_t)i + 3] = x.w;
    }
    if (z64) {
        double z[3];
        normals<double, 3>(k0, k1, c0 + i, c1, c2, c3, z);
        for (int j = 0; j < 3; ++j) z64[3 * (size_t)i + j] = z[j];
    }
    if (z32) {
        float z[3];
        normals<float, 3>(k0, k1, c0 + i, c1, c2, c3, z);
        for (int j = 0; j < 3; ++j) z32[3 * (size_t)i + j] = z[j];
    }
}

hipError_t launch_probe_rng(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                            uint32_t c3, uint32_t n, uint32_t* words, double* z64, float* z32,
                            hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_rng, dim3((n + 255) / 256), dim3(256), 0, s, k0, k1, c0, c1, c2,
                       c3, n, words, z64, z32);
    return hipGetLastError();
}

template <typename R>
__global__ void k_probe_coeffs(const JobDev<R>* job, const RegionDev<R>* reg, const double* pts,
                               uint32_t n, double* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const JobReg<R> J = load_job(*job);
    const double P = pts[4 * (size_t)i + 0], r = pts[4 * (size_t)i + 1];
    const R th = (R)pts[4 * (size_t)i + 2], ph = (R)pts[4 * (size_t)i + 3];
    Coef3<R> c;
    coeffs3d<R, true>(J, reg[region_at<R, true>(J, job, r, th, ph)], r, P, th, ph, c);
    double* o = out + (size_t)kProbeOut * i;
    o[0] = c.Ar;
    o[1] = c.At;
    o[2] = c.Ap;
    o[3] = c.AP;
    o[4] = c.Brr;
    o[5] = c.Bpr;
    o[6] = c.Bpp;
    o[7] = c.Btt;
    o[8] = c.dt;
    o[9] = c.Hw;
    o[10] = c.vdr;
    o[11] = c.vdt;
    o[12] = c.vdp;
    o[13] = c.Krr;
    o[14] = c.Krp;
    o[15] = c.kpar;
}

hipError_t launch_probe_coeffs_fp64(const JobDev<double>* job, const RegionDev<double>* reg,
                                    const double* pts, uint32_t n, double* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_coeffs<double>, dim3((n + 63) / 64), dim3(64), 0, s, job, reg,
                       pts, n, out);
    return hipGetLastError();
}

hipError_t launch_probe_coeffs_mixed(const JobDev<float>* job, const RegionDev<float>* reg,
                                     const double* pts, uint32_t n, double* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_coeffs<float>, dim3((n + 63) / 64), dim3(64), 0, s, job, reg, pts,
                       n, out);
    return hipGetLastError();
}

// Region and exit decision at points (r, theta, phi), with the integrator's
// own device functions.
template <typename R>
__global__ void k_probe_locate(const JobDev<R>* job, const double* pts, uint32_t n,
                               int32_t* region, int32_t* outside)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const JobReg<R> J = load_job(*job);
    const double r = pts[3 * (size_t)i + 0];
    const R th = (R)pts[3 * (size_t)i + 1], ph = (R)pts[3 * (size_t)i + 2];
    region[i] = region_at<R, true>(J, job, r, th, ph);
    outside[i] = outside_boundary<R, true>(J, job, r, th, ph) ? 1 : 0;
}

hipError_t launch_probe_locate_fp64(const JobDev<double>* job, const RegionDev<double>*,
                                    const double* pts, uint32_t n, int32_t* region,
                                    int32_t* outside, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_locate<double>, dim3((n + 63) / 64), dim3(64), 0, s, job, pts, n,
                       region, outside);
    return hipGetLastError();
}

hipError_t launch_probe_locate_mixed(const JobDev<float>* job, const RegionDev<float>*,
                                     const double* pts, uint32_t n, int32_t* region,
                                     int32_t* outside, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_locate<float>, dim3((n + 63) / 64), dim3(64), 0, s, job, pts, n,
                       region, outside);
    return hipGetLastError();
}

}  // namespace cosmica
