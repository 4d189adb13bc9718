// Device functions shared by the step kernels and the adjoint kernels, so
// that a recomputed step performs exactly the arithmetic of the forward step.
#pragma once

#include "snn_internal.h"

namespace snn {

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the key bumped by the Weyl constants between
// rounds.  Only the first output word is needed for a Bernoulli draw.
__device__ __forceinline__ uint32_t philox_first_word(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                                      uint32_t key0, uint32_t key1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a_lo = 0xD2511F53u * x0, a_hi = __umulhi(0xD2511F53u, x0);
        const uint32_t b_lo = 0xCD9E8D57u * x2, b_hi = __umulhi(0xCD9E8D57u, x2);
        x0 = b_hi ^ x1 ^ key0;
        x1 = b_lo;
        x2 = a_hi ^ x3 ^ key1;
        x3 = a_lo;
        key0 += 0x9E3779B9u;
        key1 += 0xBB67AE85u;
    }
    return x0;
}

// Wave-wide inclusive sum (64 lanes).
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Lane `l` (uniform) of a 64-bit value.
__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, uint32_t l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (int)l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), (int)l);
    return ((uint64_t)hi << 32) | lo;
}

// A 64-bit value known to be the same in every lane, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Fixed-point increment of one delivered synapse: g_scale * g on the
// 2^-40 uS grid (s_fix = g_scale * 2^40; the product of two fp32 values is
// exact in double, so the only rounding is the final one).  The library
// keeps every increment below 2^51 in magnitude, so it is rounded to an
// integer by the classic addition of 1.5 * 2^52: the sum lies in
// [2^52, 2^53), where the spacing of doubles is 1, so the addition rounds x to
// the nearest integer (ties to even) and that integer is the difference of the
// sum's bit pattern and the constant's.
__device__ __forceinline__ long long fix_increment(double s_fix, float w)
{
    const double kMagic = 6755399441055744.0;   // 1.5 * 2^52
    const double y = s_fix * (double)w + kMagic;
    return (long long)(__double_as_longlong(y) - __double_as_longlong(kMagic));
}

__device__ __forceinline__ int64_t fix_decay(int64_t g, double d)
{
    return __double2ll_rn((double)g * d);
}

// Synaptic + external current of a neuron with start-of-step voltage v0 and
// delivered conductances g[0..n_in).
__device__ __forceinline__ double syn_current(const Seg &S, const int64_t *g, double v0)
{
    double iin = S.i_ext;
#pragma unroll
    for (int q = 0; q < kMaxIn; ++q)
        if (q < S.n_in) iin += (double)g[q] * kFixInv * (S.in_erev[q] - v0);
    return iin;
}

// Traub-Miles right-hand side at (v, m, h, n): rates and the four
// derivatives; iin is the injected current held over the step.
struct HHRates {
    double am, bm, ah, bh, an, bn;
};

// The rates from five device-library exponentials (any V, NaN included).
// am, bm and an are c x / (e^x - 1) (limit c at x = 0; expm1 keeps the
// quotient accurate near 0).  bm and bh share one exponential: with
// x2 = (v + 25) / 5 and E = e^x2 - 1, e^(-x2) = 1 / (1 + E), so
// bh = 4 / (e^(-x2) + 1) = 4 (1 + E) / (2 + E) (E overflowing means e^(-x2) = 0,
// where bh is 4).  The four quotients take one division: the reciprocal of
// the product of the denominators, then products of the others.  A zero
// denominator (x = 0 only) enters the product as 1; where the product is not
// a finite nonzero number (V far outside the physiological range, or NaN)
// the lane divides four times instead (the choice is the lane's own, so a
// neuron's rates do not depend on the other neurons of its wavefront).  A
// NaN voltage gives NaN rates.
__device__ __noinline__ HHRates hh_rates_lib(double v)
{
    HHRates r;
    const double x1 = (-52.0 - v) * 0.25, x2 = (v + 25.0) * 0.2, x3 = (-50.0 - v) * 0.2;
    const double e1 = expm1(x1), e2 = expm1(x2), e3 = expm1(x3);
    const double f1 = x1 == 0.0 ? 1.0 : e1, f2 = x2 == 0.0 ? 1.0 : e2, f3 = x3 == 0.0 ? 1.0 : e3;
    const double f4 = 2.0 + e2;
    const double p12 = f1 * f2, p123 = p12 * f3, prod = p123 * f4;
    double i1, i2, i3, i4;
    if (isfinite(prod) && prod != 0.0) {
        const double q = 1.0 / prod;
        i4 = q * p123;
        const double q123 = q * f4;
        i3 = q123 * p12;
        const double q12 = q123 * f3;
        i2 = q12 * f1;
        i1 = q12 * f2;
    } else {
        i1 = 1.0 / f1;
        i2 = 1.0 / f2;
        i3 = 1.0 / f3;
        i4 = 1.0 / f4;
    }
    r.am = 1.28 * (x1 == 0.0 ? 1.0 : x1 * i1);
    r.bm = 1.4 * (x2 == 0.0 ? 1.0 : x2 * i2);
    r.an = 0.16 * (x3 == 0.0 ? 1.0 : x3 * i3);
    r.bh = e2 < 1e300 ? 4.0 * (1.0 + e2) * i4 : 4.0;
    r.ah = 0.128 * exp((-48.0 - v) * (1.0 / 18.0));
    r.bn = 0.5 * exp((-55.0 - v) * 0.025);
    return r;
}

// x / (e^x - 1) near x = 0 by its series 1 - x/2 + x^2/12 - x^4/720 (the
// next term, x^6/30240, is below 5e-16 for |x| < 1/64).
__device__ __forceinline__ double xexpm1_series(double x)
{
    const double x2 = x * x;
    return 1.0 - 0.5 * x + x2 * (1.0 / 12.0) - x2 * x2 * (1.0 / 720.0);
}

// The rates from one exponential.  The five exponents are linear in v with
// slopes -1/4, 1/5, -1/5, -1/18 and -1/40, all integer multiples of 1/360, so
// with u = e^(-v/360):
//   e^((-52 - v)/4)  = e^-13 u^90      e^(-(v + 25)/5) = e^-5 u^72
//   e^((-50 - v)/5)  = e^-10 u^72      e^((-48 - v)/18) = e^(-8/3) u^20
//   e^((-55 - v)/40) = e^(-11/8) u^9
// u's powers come from repeated products (relative error about 90 times
// u's, near 1e-14).  am = 1.28 x1/(e^x1 - 1), an = 0.16 x3/(e^x3 - 1), and
// bm = 1.4 x2/(e^x2 - 1) = 1.4 x2 e^-x2/(1 - e^-x2); where |x| < 1/64 the
// quotient is its series instead (the difference would cancel).  bh =
// 4/(e^-x2 + 1).  The four denominators share one division as in
// hh_rates_lib.  For |v| <= 1000 mV the powers stay far from overflow;
// beyond (a neuron running away, or NaN) the library path is used.
__device__ __forceinline__ HHRates hh_rates(double v)
{
    if (!(fabs(v) <= 1000.0)) return hh_rates_lib(v);
    constexpr double kE13 = 0x1.2f6053b981d98p-19;   // e^-13
    constexpr double kEm5 = 0x1.b993fe00d5376p-8;    // e^-5
    constexpr double kE10 = 0x1.7cd79b5647c9bp-15;   // e^-10
    constexpr double kAh = 0x1.236f49a3adb34p-7;     // 0.128 e^(-8/3)
    constexpr double kBn = 0x1.02e8620c7602cp-3;     // 0.5 e^(-11/8)
    constexpr double kSmall = 1.0 / 64.0;
    HHRates r;
    const double u = exp(v * (-1.0 / 360.0));
    const double u2 = u * u, u4 = u2 * u2, u8 = u4 * u4, u16 = u8 * u8;
    const double u9 = u8 * u, u18 = u16 * u2, u20 = u16 * u4, u36 = u18 * u18, u72 = u36 * u36, u90 = u72 * u18;
    const double x1 = (-52.0 - v) * 0.25, x2 = (v + 25.0) * 0.2, x3 = (-50.0 - v) * 0.2;
    const double e1 = kE13 * u90, em2 = kEm5 * u72, e3 = kE10 * u72;
    const bool s1 = fabs(x1) < kSmall, s2 = fabs(x2) < kSmall, s3 = fabs(x3) < kSmall;
    const double f1 = s1 ? 1.0 : e1 - 1.0, f2 = s2 ? 1.0 : 1.0 - em2, f3 = s3 ? 1.0 : e3 - 1.0;
    const double f4 = em2 + 1.0;
    const double p12 = f1 * f2, p123 = p12 * f3, prod = p123 * f4;
    double i1, i2, i3, i4;
    if (isfinite(prod) && prod != 0.0) {
        const double q = 1.0 / prod;
        i4 = q * p123;
        const double q123 = q * f4;
        i3 = q123 * p12;
        const double q12 = q123 * f3;
        i2 = q12 * f1;
        i1 = q12 * f2;
    } else {
        i1 = 1.0 / f1;
        i2 = 1.0 / f2;
        i3 = 1.0 / f3;
        i4 = 1.0 / f4;
    }
    r.am = 1.28 * (s1 ? xexpm1_series(x1) : x1 * i1);
    r.bm = 1.4 * (s2 ? xexpm1_series(x2) : x2 * em2 * i2);
    r.an = 0.16 * (s3 ? xexpm1_series(x3) : x3 * i3);
    r.bh = 4.0 * i4;
    r.ah = kAh * u20;
    r.bn = kBn * u9;
    return r;
}

// One forward-Euler substep, every right-hand side from the substep-start state.
__device__ __forceinline__ void hh_substep(const Seg &S, double hs, double hc, double iin, double &v, double &m,
                                           double &h, double &n)
{
    const HHRates r = hh_rates(v);
    const double n2 = n * n;
    const double iion = S.gna * (m * m * m * h) * (v - S.ena) + S.gk * (n2 * n2) * (v - S.ek) + S.gl * (v - S.el);
    const double vn = v + hc * (iin - iion);
    const double mn = m + hs * (r.am * (1.0 - m) - r.bm * m);
    const double hn = h + hs * (r.ah * (1.0 - h) - r.bh * h);
    const double nn = n + hs * (r.an * (1.0 - n) - r.bn * n);
    v = vn;
    m = mn;
    h = hn;
    n = nn;
}

// Whether x stays finite once held in the fp32 state arrays: |x| below
// FLT_MAX plus half its ulp (anything larger rounds to infinity; NaN fails).
// The NaN count of the conductance sweep (Fig. 1) counts a neuron once, at
// the step its V leaves this range.
__device__ __forceinline__ bool fits_fp32(double x)
{
    return fabs(x) < 0x1.ffffffp127;
}

// Izhikevich (2003) neuron, the model of the 4:1 network of Section 5.1
// (its reference [9]): v' = 0.04 v^2 + 5 v + 140 - u + I, u' = a (b v - u).
// One forward-Euler substep, both right-hand sides from the substep-start
// state, iin (synaptic + external) held over the step.  A step whose end
// value reaches kIzhPeak is a spike: v <- c, u <- u + d.
constexpr double kIzhPeak = 30.0;   // mV

__device__ __forceinline__ void izh_substep(double ia, double ib, double hs, double iin, double &v, double &u)
{
    const double dv = 0.04 * v * v + 5.0 * v + 140.0 - u + iin;
    const double du = ia * (ib * v - u);
    v = v + hs * dv;
    u = u + hs * du;
}

// A double held as an fp32 pair (hi = fl32(x), lo = fl32(x - hi)).
__device__ __forceinline__ double pair_load(const float *hi, const float *lo, int64_t i)
{
    return (double)hi[i] + (double)lo[i];
}

__device__ __forceinline__ void pair_split(double x, float &hi, float &lo)
{
    hi = (float)x;
    lo = (float)(x - (double)hi);
}

}  // namespace snn
