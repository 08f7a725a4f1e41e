// ks_geodesic.hpp -- null geodesics of the Kerr metric in Kerr-Schild coordinates.
//
// State y = (t~, r, theta, phi~, k^t, k^r, k^theta, k^phi), integrated with the
// classical fourth-order Runge-Kutta scheme (Sec. 2.2.1 of Bronzwaer et al. 2018) of
// dx/dlambda = k, dk/dlambda = -Gamma k k (Sec. 2.2) with the paper's adaptive step
// (Sec. 2.2) written in the logarithmic KS chart (x1 = ln r, x2 = theta/pi, x3 = phi).
//
// The connection term is evaluated in closed form in registers.  With the metric depending
// on (r, theta) only,
//     Gamma^a_{mn} k^m k^n = g^{ab} ( Gdot_{bn} k^n - 1/2 (d_b g_{mn}) k^m k^n ),
//     Gdot_{bn} = k^r d_r g_{bn} + k^theta d_theta g_{bn},
// which is the connection formula of Sec. 2.1 contracted with k twice.  The Kerr-Schild form
// of the metric (Sec. 2.1) is used to contract it: g = g0 + z l l with z = 2 M r / Sigma, the
// null covector l = (1, 1, 0, -a sin^2) and g0 flat space in oblate spheroidal coordinates, so
// that F_b splits into a short flat-space part and a z l l part built from z, its two
// derivatives and l.k; the inverse metric is used in its closed form.
#pragma once
#include "rt_math.hpp"

namespace rk {

// Per-ray constants of the spacetime.
template <class T>
struct Spin {
    T a, a2, M;
    T twoM, m2a, twoa2;   // 2 M, -2 a, 2 a^2
};

template <class T>
__host__ __device__ inline Spin<T> make_spin(T a, T M)
{
    Spin<T> s;
    s.a = a;
    s.a2 = a * a;
    s.M = M;
    s.twoM = T(2.0) * M;
    s.m2a = T(-2.0) * a;
    s.twoa2 = T(2.0) * s.a2;
    return s;
}

// dk/dlambda = -Gamma k k at state y, given s = sin(theta), c = cos(theta).
// F_b = Gdot_{bn} k^n - 1/2 (d_b g_mn) k^m k^n for g = g0 + z l l:
//   z l l part:  zd l_b L + z (k.d l_b) L + z l_b Ld - 1/2 (d_b z) L^2 - z L (d_b l_m) k^m,
//   with L = l.k, zd = k^r dz/dr + k^theta dz/dtheta, and d_theta l_phi = -2 a s c the only
//   derivative of l (Ld = k^theta (d_theta l_phi) k^phi);
//   flat part:   g0 = diag(-1, 1, Sigma) with g0_{r phi} = l_phi, g0_{phi phi} = (r^2 + a^2) sin^2;
// then raised with the closed-form inverse metric.
template <class T>
__host__ __device__ inline void ks_accel(const Spin<T>& sp, const T* y, T s, T c, T* dk)
{
    using namespace rt;
    const T a = sp.a, a2 = sp.a2;
    const T r = y[1];
    const T kt = y[4], kr = y[5], kh = y[6], kp = y[7];
    const T s2 = s * s, sc = s * c;
    const T r2 = r * r;
    const T a2c2 = a2 * (c * c);
    const T sig = r2 + a2c2;
    const T w = rcp_nr(sig * s2);                           // 1/(Sigma sin^2)
    const T isig = w * s2;                                  // 1/Sigma
    const T twoMr = sp.twoM * r;
    const T z = twoMr * isig;                               // 2 M r / Sigma
    const T zr = sp.twoM * (a2c2 - r2) * (isig * isig);     // dz/dr
    const T zt = z * (sp.twoa2 * sc) * isig;                // dz/dtheta
    const T lp = -a * s2;                                   // l_phi
    const T dl = sp.m2a * sc;                               // d l_phi / dtheta
    const T L = (kt + kr) + lp * kp;                        // l.k
    const T ld = kh * dl;                                   // k^c d_c l_phi
    const T Ld = ld * kp;
    const T zd = kr * zr + kh * zt;                         // k^c d_c z
    const T L2 = L * L;
    const T zL = z * L;
    const T khh = kh * kh, kpp = kp * kp;
    const T ra = r2 + a2;
    const T F1t = zd * L + z * Ld;                          // z l l part of F_t (the flat part is 0)
    const T F_t = F1t;
    const T F_r = F1t - T(0.5) * zr * L2 + (Ld - r * (khh + s2 * kpp));
    const T F_h = T(2.0) * r * kr * kh - T(0.5) * zt * L2 - dl * kp * (zL + kr) - sc * (a2 * khh + ra * kpp);
    const T F_p = lp * F1t + zL * ld + kr * (T(2.0) * r * s2 * kp + ld) + T(2.0) * ra * sc * kh * kp;
    // inverse metric: g^tt = -(1+z), g^tr = z, g^rr = Delta/Sigma, g^rp = a/Sigma,
    // g^hh = 1/Sigma, g^pp = 1/(Sigma sin^2)
    const T gi_rr = (ra - twoMr) * isig;
    const T ai = a * isig;
    dk[0] = F_t + z * (F_t - F_r);
    dk[1] = -(z * F_t + gi_rr * F_r + ai * F_p);
    dk[2] = -isig * F_h;
    dk[3] = -(ai * F_r + w * F_p);
}

// f = dy/dlambda (the full eight-component right-hand side).
template <class T>
__host__ __device__ inline void ks_rhs(const Spin<T>& sp, const T* y, T* f)
{
    T s, c;
    rt::sincos_(y[2], &s, &c);
    f[0] = y[4];
    f[1] = y[5];
    f[2] = y[6];
    f[3] = y[7];
    ks_accel(sp, y, s, c, f + 4);
}

// sin and cos of theta + d from s0 = sin(theta), c0 = cos(theta): Taylor polynomials of sin d
// (through d^9) and cos d (through d^10), whose truncation errors for |d| <= 0.1 are below
// 3e-18 relative and 3e-21 absolute, and the angle-addition formulas; larger |d| falls back to
// a full sincos.  With the step rule's eps = 0.05 a stage moves theta by at most about 0.08.
// The polynomials are summed as power sums, each coefficient a multiplicand: a coefficient that
// is an FMA addend must be copied into vector registers first, one multiplicand is read from
// scalar registers as it is.
template <class T>
__host__ __device__ inline void sincos_add(T th, T d, T s0, T c0, T* s, T* c);

template <class T>
__host__ __device__ inline void sincos_shift(T th0, T s0, T c0, T th, T* s, T* c)
{
    sincos_add(th, th - th0, s0, c0, s, c);
}

// The same with the angle th and its offset d from the angle of (s0, c0) given separately (d
// computed by the caller without cancellation); th is used only by the fallback.
template <class T>
__host__ __device__ inline void sincos_add(T th, T d, T s0, T c0, T* s, T* c)
{
    using namespace rt;
    if (fabs_(d) > T(0.1)) {
        sincos_small(th, s, c);
        return;
    }
    // smallest terms first
    const T d2 = d * d, d4 = d2 * d2, d6 = d4 * d2, d8 = d4 * d4;
    T ps = T(1.0 / 362880.0) * d8;
    ps = ps + T(-1.0 / 5040.0) * d6;
    ps = ps + T(1.0 / 120.0) * d4;
    ps = ps + T(-1.0 / 6.0) * d2;            // sin d / d - 1
    const T sd = d + d * ps;
    T cdm1 = T(-1.0 / 3628800.0) * (d8 * d2);
    cdm1 = cdm1 + T(1.0 / 40320.0) * d8;
    cdm1 = cdm1 + T(-1.0 / 720.0) * d6;
    cdm1 = cdm1 + T(1.0 / 24.0) * d4;
    cdm1 = cdm1 + T(-0.5) * d2;              // cos d - 1
    *s = s0 + (s0 * cdm1 + c0 * sd);
    *c = c0 + (c0 * cdm1 - s0 * sd);
}

// The same for a half step (|d| <= 0.05, about twice the largest half-step move of theta at
// eps = 0.05): sin d through d^7 and cos d through d^8, truncation below 2e-18 relative and
// 3e-20 absolute.
template <class T>
__host__ __device__ inline void sincos_shift_half(T th0, T s0, T c0, T th, T* s, T* c)
{
    using namespace rt;
    const T d = th - th0;
    if (fabs_(d) > T(0.05)) {
        sincos_small(th, s, c);
        return;
    }
    const T d2 = d * d, d4 = d2 * d2, d6 = d4 * d2;
    T ps = T(-1.0 / 5040.0) * d6;
    ps = ps + T(1.0 / 120.0) * d4;
    ps = ps + T(-1.0 / 6.0) * d2;            // sin d / d - 1
    const T sd = d + d * ps;
    T cdm1 = T(1.0 / 40320.0) * (d4 * d4);
    cdm1 = cdm1 + T(-1.0 / 720.0) * d6;
    cdm1 = cdm1 + T(1.0 / 24.0) * d4;
    cdm1 = cdm1 + T(-0.5) * d2;              // cos d - 1
    *s = s0 + (s0 * cdm1 + c0 * sd);
    *c = c0 + (c0 * cdm1 - s0 * sd);
}

// Positive step size of the adaptive rule (Sec. 2.2),
//   1/dl = (|k^x1| + d)/eps + (|k^x2| + d)/(eps min(x2, 1 - x2)) + (|k^x3| + d)/eps
// with k^x1 = k^r / r, k^x2 = k^theta / pi, x2 = theta / pi, k^x3 = k^phi, evaluated with a
// single division.  `edge` is floored at 1e-12.
template <class T>
__host__ __device__ inline T step_size(T eps, const T* y)
{
    using namespace rt;
    const T d = T(1e-40);
    const T r = y[1];
    const T x2 = y[2] * T(M_1_PI);
    const T edge = fmax_(fmin_(x2, T(1.0) - x2), T(1e-12));
    const T den = (fabs_(y[5]) + d * r) * edge + (fabs_(y[6]) * T(M_1_PI) + d) * r + (fabs_(y[7]) + d) * r * edge;
    return eps * r * edge * rcp_nr(den);
}

// The work count treats sincos_shift and sincos_shift_half as one sine-cosine evaluation.
inline void sincos_shift(rt::OpCounted th0, rt::OpCounted s0, rt::OpCounted c0, rt::OpCounted th,
                         rt::OpCounted* s, rt::OpCounted* c)
{
    (void)th0; (void)s0; (void)c0;
    rt::sincos_(th, s, c);
}
inline void sincos_shift_half(rt::OpCounted th0, rt::OpCounted s0, rt::OpCounted c0, rt::OpCounted th,
                              rt::OpCounted* s, rt::OpCounted* c)
{
    sincos_shift(th0, s0, c0, th, s, c);
}

// One classical RK4 step of size dl (negative: away from the camera) on y = (x, k).  s0, c0
// are sin and cos of y[2]; the three later stages get theirs with sincos_shift (the two
// half-step stages with its shorter half-step form).  The position
// derivative of a stage is that stage's wave vector, so only dk/dlambda is evaluated.
template <class T>
__host__ __device__ inline void rk4_step(const Spin<T>& sp, T* y, T dl, T s0, T c0)
{
    T t[8], acc[8], dk[4];
    T s, c;
    ks_accel(sp, y, s0, c0, dk);
    const T h2 = T(0.5) * dl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        acc[i] = y[4 + i];
        acc[4 + i] = dk[i];
        t[i] = y[i] + h2 * y[4 + i];
        t[4 + i] = y[4 + i] + h2 * dk[i];
    }
    sincos_shift_half(y[2], s0, c0, t[2], &s, &c);
    ks_accel(sp, t, s, c, dk);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        acc[i] = acc[i] + T(2.0) * t[4 + i];
        acc[4 + i] = acc[4 + i] + T(2.0) * dk[i];
        t[i] = y[i] + h2 * t[4 + i];
        t[4 + i] = y[4 + i] + h2 * dk[i];
    }
    sincos_shift_half(y[2], s0, c0, t[2], &s, &c);
    ks_accel(sp, t, s, c, dk);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        acc[i] = acc[i] + T(2.0) * t[4 + i];
        acc[4 + i] = acc[4 + i] + T(2.0) * dk[i];
        t[i] = y[i] + dl * t[4 + i];
        t[4 + i] = y[4 + i] + dl * dk[i];
    }
    sincos_shift(y[2], s0, c0, t[2], &s, &c);
    ks_accel(sp, t, s, c, dk);
    const T h6 = dl * T(1.0 / 6.0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        y[i] = y[i] + h6 * (acc[i] + t[4 + i]);
        y[4 + i] = y[4 + i] + h6 * (acc[4 + i] + dk[i]);
    }
}

// One second-order Runge-Kutta (midpoint) step: dk/dlambda at y and at y + (dl/2) f(y), then
// y + dl f(midpoint).  The paper names RK2 for its timing runs without spelling it out; the
// midpoint rule is the reading taken.
template <class T>
__host__ __device__ inline void rk2_step(const Spin<T>& sp, T* y, T dl, T s0, T c0)
{
    T t[8], dk[4];
    T s, c;
    ks_accel(sp, y, s0, c0, dk);
    const T h2 = T(0.5) * dl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        t[i] = y[i] + h2 * y[4 + i];
        t[4 + i] = y[4 + i] + h2 * dk[i];
    }
    sincos_shift_half(y[2], s0, c0, t[2], &s, &c);
    ks_accel(sp, t, s, c, dk);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        y[i] = y[i] + dl * t[4 + i];
        y[4 + i] = y[4 + i] + dl * dk[i];
    }
}

// One velocity-Verlet step (Sec. 2.2.2) with A = dk/dlambda at y carried in acc:
//   x' = x + k dl + A dl^2/2,  k_p = k + A dl,  A' = accel(x', k_p),  k' = k + (A + A') dl/2,
// with the corrector A' = accel(x', k') and k' recomputed once more.  acc returns the last
// evaluated derivative.  One connection evaluation per step (two with the corrector).
template <class T>
__host__ __device__ inline void verlet_step(const Spin<T>& sp, T* y, T* acc, T dl, bool corrector, T s0, T c0)
{
    T t[8], dk[4];
    T s, c;
    const T hh = T(0.5) * dl * dl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        t[i] = y[i] + y[4 + i] * dl + hh * acc[i];
        t[4 + i] = y[4 + i] + acc[i] * dl;
    }
    sincos_shift(y[2], s0, c0, t[2], &s, &c);
    ks_accel(sp, t, s, c, dk);
    const T h2 = T(0.5) * dl;
#pragma unroll
    for (int i = 0; i < 4; ++i) t[4 + i] = y[4 + i] + h2 * (acc[i] + dk[i]);
    if (corrector) {
        ks_accel(sp, t, s, c, dk);
#pragma unroll
        for (int i = 0; i < 4; ++i) t[4 + i] = y[4 + i] + h2 * (acc[i] + dk[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        y[i] = t[i];
        y[4 + i] = t[4 + i];
        acc[i] = dk[i];
    }
}

// Virtual camera (Sec. 2.3) at radius r_cam and polar angle incl, impact parameters
// (alpha, beta): E = 1, L = -alpha sin(i), Q = beta^2 + cos^2(i)(alpha^2 - a^2),
// k_theta = sign(beta) sqrt|Q - L^2 cot^2(i) + a^2 cos^2(i)|, k_r > 0 from the null
// condition with the Boyer-Lindquist inverse metric, raised and mapped to KS with the
// appendix matrix (k^t~ = k^t + 2 M r/Delta k^r, k^phi~ = k^phi + a/Delta k^r).
template <class T>
__host__ __device__ inline void camera_ray(const Spin<T>& sp, T r, T incl, T sin_i, T cos_i, T alpha,
                                           T beta, T t_init, T* y)
{
    using namespace rt;
    const T a = sp.a, a2 = sp.a2, M = sp.M;
    const T L = -alpha * sin_i;
    const T Q = beta * beta + cos_i * cos_i * (alpha * alpha - a2);
    const T cot = cos_i * rcp(sin_i);
    const T kth = (beta >= T(0.0) ? T(1.0) : T(-1.0)) * sqrt_(fabs_(Q - L * L * cot * cot + a2 * cos_i * cos_i));
    const T s2 = sin_i * sin_i, c2 = cos_i * cos_i;
    const T sig = r * r + a2 * c2;
    const T del = r * r - T(2.0) * M * r + a2;
    const T isd = rcp(sig * del);
    const T A = (r * r + a2) * (r * r + a2) - a2 * del * s2;
    const T gtt = -A * isd;
    const T gtp = -T(2.0) * M * a * r * isd;
    const T gpp = (del - a2 * s2) * isd * rcp(s2);
    const T grr = del * rcp(sig);
    const T ghh = rcp(sig);
    // g^tt k_t^2 + 2 g^tp k_t k_p + g^pp k_p^2 + g^hh k_h^2 + g^rr k_r^2 = 0, k_t = -1
    const T rest = gtt - T(2.0) * gtp * L + gpp * L * L + ghh * kth * kth;
    const T kr_cov = sqrt_(fmax_(-rest * rcp(grr), T(0.0)));
    const T kt_up = -gtt + gtp * L;
    const T kr_up = grr * kr_cov;
    const T kh_up = ghh * kth;
    const T kp_up = -gtp + gpp * L;
    const T idel = rcp(del);
    y[0] = t_init;
    y[1] = r;
    y[2] = incl;
    y[3] = T(0.0);
    y[4] = kt_up + T(2.0) * M * r * idel * kr_up;
    y[5] = kr_up;
    y[6] = kh_up;
    y[7] = kp_up + a * idel * kr_up;
}

// Pole crossing: (theta, phi) -> (-theta, phi + pi) or (2 pi - theta, phi + pi) is the same
// point and the polar velocity changes sign.  Returns 1 if the state was reflected.
template <class T>
__host__ __device__ inline int reflect_pole(T* y)
{
    if (y[2] < T(0.0)) {
        y[2] = -y[2];
    } else if (y[2] > T(M_PI)) {
        y[2] = T(2.0 * M_PI) - y[2];
    } else {
        return 0;
    }
    y[3] = y[3] + T(M_PI);
    y[6] = -y[6];
    return 1;
}

}  // namespace rk
