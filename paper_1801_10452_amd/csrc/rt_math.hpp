// rt_math.hpp -- scalar primitives used by the device math, overloadable per number type.
//
// Device code instantiates the templates with double (geodesic, fluid frame) and float or
// double (transfer).  The host instantiates them once with OpCounted to count the
// algorithmic work of a step: +, -, * count one flop each (a fused multiply-add is written
// as a product and a sum, so it counts two); divisions, square roots and transcendental
// calls count as "special" operations and not as flops.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace rt {

// ---------------------------------------------------------------- double / float (device and host)
__host__ __device__ inline double rcp(double x) { return 1.0 / x; }
__host__ __device__ inline float rcp(float x) { return 1.0f / x; }
__host__ __device__ inline double sqrt_(double x) { return ::sqrt(x); }
__host__ __device__ inline float sqrt_(float x) { return ::sqrtf(x); }
__host__ __device__ inline double cbrt_(double x) { return ::cbrt(x); }
__host__ __device__ inline float cbrt_(float x) { return ::cbrtf(x); }
__host__ __device__ inline double exp_(double x) { return ::exp(x); }
__host__ __device__ inline float exp_(float x) { return ::expf(x); }
__host__ __device__ inline double expm1_(double x) { return ::expm1(x); }
__host__ __device__ inline float expm1_(float x) { return ::expm1f(x); }
__host__ __device__ inline double log_(double x) { return ::log(x); }
__host__ __device__ inline float log_(float x) { return ::logf(x); }
__host__ __device__ inline double fabs_(double x) { return ::fabs(x); }
__host__ __device__ inline float fabs_(float x) { return ::fabsf(x); }
__host__ __device__ inline double fmin_(double a, double b) { return ::fmin(a, b); }
__host__ __device__ inline double fmax_(double a, double b) { return ::fmax(a, b); }
__host__ __device__ inline void sincos_(double x, double* s, double* c) { ::sincos(x, s, c); }
__host__ __device__ inline void sincospi_(double x, double* s, double* c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    ::sincospi(x, s, c);
#else
    *s = std::sin(M_PI * x);
    *c = std::cos(M_PI * x);
#endif
}
__host__ __device__ inline bool finite_(double x) { return ::isfinite(x); }
__host__ __device__ inline double val(double x) { return x; }

// sin and cos for moderate arguments (|x| < 1e3 keeps the reduction exact): x = k pi/2 + r with
// k = rint(2x/pi) and r from a three-term Cody-Waite subtraction (pi/2 split into a 40-bit head,
// so k times the head is exact, and two tails), then Taylor polynomials of sin r through r^17
// and cos r through r^18 on |r| <= pi/4 (truncation below 1e-19) and the quadrant identities.
__host__ __device__ inline void sincos_small(double x, double* s, double* c)
{
    const double k = __builtin_rint(x * 0.6366197723675814);
    double r = __builtin_fma(-k, 1.5707963267941523, x);
    r = __builtin_fma(-k, 7.443547480486623e-13, r);
    r = __builtin_fma(-k, -1.2536990206932499e-29, r);
    // power sums in y = r^2, smallest terms first (each coefficient a multiplicand, so that it is
    // read from scalar registers instead of being copied into vector registers as an FMA addend)
    const double y = r * r, y2 = y * y, y3 = y2 * y, y4 = y2 * y2;
    const double y5 = y4 * y, y6 = y4 * y2, y7 = y4 * y3, y8 = y4 * y4;
    double ps = (1.0 / 355687428096000.0) * y7;
    ps = ps + (-1.0 / 1307674368000.0) * y6;
    ps = ps + (1.0 / 6227020800.0) * y5;
    ps = ps + (-1.0 / 39916800.0) * y4;
    ps = ps + (1.0 / 362880.0) * y3;
    ps = ps + (-1.0 / 5040.0) * y2;
    ps = ps + (1.0 / 120.0) * y;
    ps = ps + (-1.0 / 6.0);
    double pc = (-1.0 / 6402373705728000.0) * y8;
    pc = pc + (1.0 / 20922789888000.0) * y7;
    pc = pc + (-1.0 / 87178291200.0) * y6;
    pc = pc + (1.0 / 479001600.0) * y5;
    pc = pc + (-1.0 / 3628800.0) * y4;
    pc = pc + (1.0 / 40320.0) * y3;
    pc = pc + (-1.0 / 720.0) * y2;
    pc = pc + (1.0 / 24.0) * y;
    pc = pc + (-0.5);
    const double r2 = y;
    const double sn = r + r * r2 * ps;
    const double cs = 1.0 + r2 * pc;
    const int q = (int)k & 3;
    const double a = (q & 1) ? cs : sn;   // |sin x|
    const double b = (q & 1) ? sn : cs;   // |cos x|
    *s = (q & 2) ? -a : a;
    *c = ((q + 1) & 2) ? -b : b;
}

// Reciprocal without the IEEE division sequence: the hardware estimate (about 2^-26 relative
// error) refined by two Newton-Raphson steps r <- r (2 - x r), which square the error each
// time (full double precision; not correctly rounded in every case).
__host__ __device__ inline double rcp_nr(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

// Float reciprocal: the hardware estimate (about 1 ulp) refined by one Newton-Raphson step.
__host__ __device__ inline float rcpf_nr(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
#else
    return 1.0f / x;
#endif
}

// 1/sqrt(x): hardware estimate refined by two Newton-Raphson steps r <- r (3 - x r^2) / 2.
__host__ __device__ inline double rsqrt_nr(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    r = r * __builtin_fma(-h * r, r, 1.5);
    return r * __builtin_fma(-h * r, r, 1.5);
#else
    return 1.0 / std::sqrt(x);
#endif
}

// e^x as a float for an argument held in double: x log2(e) = n + f with n = rint and |f| <= 1/2
// formed in double, then 2^f from the hardware exp2 (about 1 ulp on [-1/2, 1/2]) scaled by 2^n.
// The relative error stays near one float ulp for any x, where expf((float)x) would lose
// |x| ulps to the rounding of its argument.  Results below the float range flush to zero.
__host__ __device__ inline float exp_mixed(double x)
{
    const double z = x * 1.4426950408889634;
    // below 2^-160 the result is 0 (selected, not branched on, so that independent calls can
    // be interleaved); the clamp keeps the power of two in range there
    const double n = __builtin_rint(z < 160.0 ? (z > -200.0 ? z : -200.0) : 160.0);
    const float f = (float)(z - n);
#if defined(__HIP_DEVICE_COMPILE__)
    const float r = __builtin_ldexpf(__builtin_amdgcn_exp2f(f), (int)n);
#else
    const float r = std::ldexp(std::exp2(f), (int)n);
#endif
    return z < -160.0 ? 0.0f : r;
}

// e^y - 1 in float: for |y| < 1 the Taylor series through y^11 (truncation below 2e-9 relative),
// otherwise the hardware exp2 of y log2(e) less one, which loses at most a factor e/(e - 1) to
// cancellation there; both are formed and one selected (no branch).  About half the
// instructions of the library expm1f, within a few float ulps of it.
__host__ __device__ inline float expm1_f(float y)
{
#if defined(__HIP_DEVICE_COMPILE__)
    float q = 1.0f / 39916800.0f;
    q = __builtin_fmaf(q, y, 1.0f / 3628800.0f);
    q = __builtin_fmaf(q, y, 1.0f / 362880.0f);
    q = __builtin_fmaf(q, y, 1.0f / 40320.0f);
    q = __builtin_fmaf(q, y, 1.0f / 5040.0f);
    q = __builtin_fmaf(q, y, 1.0f / 720.0f);
    q = __builtin_fmaf(q, y, 1.0f / 120.0f);
    q = __builtin_fmaf(q, y, 1.0f / 24.0f);
    q = __builtin_fmaf(q, y, 1.0f / 6.0f);
    q = __builtin_fmaf(q, y, 0.5f);
    const float series = __builtin_fmaf(y * y, q, y);
    const float direct = __builtin_amdgcn_exp2f(y * 1.4426950408889634f) - 1.0f;
    return __builtin_fabsf(y) < 1.0f ? series : direct;
#else
    return std::expm1(y);
#endif
}

// Natural logarithm of a positive, normal double: x = m 2^e with m in [1/sqrt2, sqrt2),
// ln m = 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.1716, from the series
// 2 (s + s^3/3 + ... + s^17/17) (next term below 2e-16 relative), and e ln2 added with ln2
// split into a 32-bit head (exact products) and a tail.  About a third of the instructions of
// the library log, relative error a few 1e-16.
__host__ __device__ inline double log_pos(double x)
{
    int e;
    double m = __builtin_frexp(x, &e);   // m in [1/2, 1)
    if (m < 0.70710678118654752) {
        m = m + m;
        e -= 1;
    }
    const double s = (m - 1.0) * rcp_nr(m + 1.0);
    const double s2 = s * s;
    const double s4 = s2 * s2, s6 = s4 * s2, s8 = s4 * s4, s10 = s8 * s2, s12 = s8 * s4, s14 = s8 * s6;
    double p = (1.0 / 17.0) * s14;
    p = p + (1.0 / 15.0) * s12;
    p = p + (1.0 / 13.0) * s10;
    p = p + (1.0 / 11.0) * s8;
    p = p + (1.0 / 9.0) * s6;
    p = p + (1.0 / 7.0) * s4;
    p = p + (1.0 / 5.0) * s2;
    p = p + 1.0 / 3.0;
    const double lm = 2.0 * s + 2.0 * s * s2 * p;
    const double de = (double)e;
    return de * 0.6931471805599453094 + (de * 2.319046813846299558e-17 + lm);
}

// Cube root of a positive double in the float range: 2^(log2(x)/3) from the hardware float
// log2 and exp2 (relative error a few 1e-6 for |log2 x| up to ~128), refined by one Newton step
// in double, t <- t + (x - t^3) / (3 t^2), which squares the error (the quotient's float
// precision only scales the already small correction): relative error near 1e-11.
__host__ __device__ inline double cbrt_refined(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float xf = (float)x;
    const float tf = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(xf) * (1.0f / 3.0f));
    const double td = (double)tf;
    return td + (x - td * td * td) * (double)__builtin_amdgcn_rcpf(3.0f * tf * tf);
#else
    const float tf = ::cbrtf((float)x);
    const double td = (double)tf;
    return td + (x - td * td * td) * (double)(1.0f / (3.0f * tf * tf));
#endif
}

// ---------------------------------------------------------------- operation counting (host only)
struct OpTally {
    double flops = 0.0, special = 0.0;
};
extern OpTally g_tally;

struct OpCounted {
    double v;
    OpCounted(double x = 0.0) : v(x) {}
};
inline OpCounted operator+(OpCounted a, OpCounted b) { g_tally.flops += 1; return a.v + b.v; }
inline OpCounted operator-(OpCounted a, OpCounted b) { g_tally.flops += 1; return a.v - b.v; }
inline OpCounted operator*(OpCounted a, OpCounted b) { g_tally.flops += 1; return a.v * b.v; }
inline OpCounted operator/(OpCounted a, OpCounted b) { g_tally.special += 1; return a.v / b.v; }
inline OpCounted operator-(OpCounted a) { return -a.v; }
inline OpCounted& operator+=(OpCounted& a, OpCounted b) { a = a + b; return a; }
inline OpCounted& operator-=(OpCounted& a, OpCounted b) { a = a - b; return a; }
inline OpCounted& operator*=(OpCounted& a, OpCounted b) { a = a * b; return a; }
inline bool operator<(OpCounted a, OpCounted b) { return a.v < b.v; }
inline bool operator>(OpCounted a, OpCounted b) { return a.v > b.v; }
inline bool operator<=(OpCounted a, OpCounted b) { return a.v <= b.v; }
inline bool operator>=(OpCounted a, OpCounted b) { return a.v >= b.v; }
inline OpCounted rcp(OpCounted x) { g_tally.special += 1; return 1.0 / x.v; }
inline OpCounted rcp_nr(OpCounted x) { g_tally.special += 1; return 1.0 / x.v; }
inline OpCounted rsqrt_nr(OpCounted x) { g_tally.special += 1; return 1.0 / std::sqrt(x.v); }
inline OpCounted sqrt_(OpCounted x) { g_tally.special += 1; return std::sqrt(x.v); }
inline OpCounted cbrt_(OpCounted x) { g_tally.special += 1; return std::cbrt(x.v); }
inline OpCounted exp_(OpCounted x) { g_tally.special += 1; return std::exp(x.v); }
inline OpCounted expm1_(OpCounted x) { g_tally.special += 1; return std::expm1(x.v); }
inline OpCounted log_(OpCounted x) { g_tally.special += 1; return std::log(x.v); }
inline OpCounted log_pos(OpCounted x) { g_tally.special += 1; return std::log(x.v); }
inline OpCounted fabs_(OpCounted x) { return std::fabs(x.v); }
inline OpCounted fmin_(OpCounted a, OpCounted b) { return std::fmin(a.v, b.v); }
inline OpCounted fmax_(OpCounted a, OpCounted b) { return std::fmax(a.v, b.v); }
inline void sincos_(OpCounted x, OpCounted* s, OpCounted* c)
{
    g_tally.special += 1;
    *s = std::sin(x.v);
    *c = std::cos(x.v);
}
inline void sincos_small(OpCounted x, OpCounted* s, OpCounted* c) { sincos_(x, s, c); }
inline void sincospi_(OpCounted x, OpCounted* s, OpCounted* c)
{
    g_tally.special += 1;
    *s = std::sin(M_PI * x.v);
    *c = std::cos(M_PI * x.v);
}
inline bool finite_(OpCounted x) { return std::isfinite(x.v); }
inline double val(OpCounted x) { return x.v; }

}  // namespace rt
