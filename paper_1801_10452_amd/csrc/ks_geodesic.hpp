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
// which is the connection formula of Sec. 2.1 contracted with k twice; only the seven
// non-zero KS metric components and their r and theta derivatives appear, and the inverse
// metric is used in its closed form.
#pragma once
#include "rt_math.hpp"

namespace rk {

// Per-ray constants of the spacetime.
template <class T>
struct Spin {
    T a, a2, M;
};

template <class T>
__host__ __device__ inline Spin<T> make_spin(T a, T M)
{
    Spin<T> s;
    s.a = a;
    s.a2 = a * a;
    s.M = M;
    return s;
}

// f = dy/dlambda.
template <class T>
__host__ __device__ inline void ks_rhs(const Spin<T>& sp, const T* y, T* f)
{
    using namespace rt;
    const T a = sp.a, a2 = sp.a2, M = sp.M;
    const T r = y[1], th = y[2];
    const T kt = y[4], kr = y[5], kh = y[6], kp = y[7];
    T s, c;
    sincos_(th, &s, &c);
    const T s2 = s * s, c2 = c * c, sc2 = T(2.0) * s * c;
    const T r2 = r * r;
    const T sig = r2 + a2 * c2;
    const T w = rcp(sig * s2);            // 1/(Sigma sin^2)
    const T isig = w * s2;                // 1/Sigma
    const T twoMr = T(2.0) * M * r;
    const T z = twoMr * isig;             // 2 M r / Sigma
    const T z1 = T(1.0) + z;
    const T isig2 = isig * isig;
    const T zr = T(2.0) * M * (a2 * c2 - r2) * isig2;   // dz/dr
    const T zt = z * a2 * sc2 * isig;                   // dz/dtheta
    // d/dr and d/dtheta of g_tt, g_tr, g_rr (all equal to dz), g_tp, g_rp, g_hh, g_pp
    const T dr_tp = -a * s2 * zr;
    const T dt_tp = -a * (sc2 * z + s2 * zt);
    const T dt_rp = -a * (sc2 * z1 + s2 * zt);
    const T dr_hh = T(2.0) * r;
    const T dt_hh = -a2 * sc2;
    const T s4 = s2 * s2;
    const T dr_pp = T(2.0) * r * s2 + a2 * s4 * zr;
    const T dt_pp = sc2 * (sig - a2 * s2) + T(2.0) * a2 * s2 * sc2 * z1 + a2 * s4 * zt;
    // Gdot = k^r d_r g + k^theta d_theta g
    const T gd_z = kr * zr + kh * zt;          // tt, tr, rr
    const T gd_tp = kr * dr_tp + kh * dt_tp;
    const T gd_rp = kr * dr_tp + kh * dt_rp;   // d_r g_rp = d_r g_tp
    const T gd_hh = kr * dr_hh + kh * dt_hh;
    const T gd_pp = kr * dr_pp + kh * dt_pp;
    // A_b = Gdot_{bn} k^n
    const T A_t = gd_z * (kt + kr) + gd_tp * kp;
    const T A_r = gd_z * (kt + kr) + gd_rp * kp;
    const T A_h = gd_hh * kh;
    const T A_p = gd_tp * kt + gd_rp * kr + gd_pp * kp;
    // 1/2 (d_b g_mn) k^m k^n for b = r, theta
    const T ktr = kt + kr;
    const T q_z = ktr * ktr;                   // k^t k^t + 2 k^t k^r + k^r k^r
    const T kpk = kp * ktr;                    // k^phi (k^t + k^r)
    const T khh = kh * kh, kpp = kp * kp;
    const T Q_r = T(0.5) * (zr * q_z + dr_hh * khh + dr_pp * kpp) + dr_tp * kpk;
    const T Q_h = T(0.5) * (zt * q_z + dt_hh * khh + dt_pp * kpp) + dt_tp * kp * kt + dt_rp * kp * kr;
    const T F_t = A_t;
    const T F_r = A_r - Q_r;
    const T F_h = A_h - Q_h;
    const T F_p = A_p;
    // inverse metric: g^tt = -(1+z), g^tr = z, g^rr = Delta/Sigma, g^rp = a/Sigma,
    // g^hh = 1/Sigma, g^pp = 1/(Sigma sin^2)
    const T gi_rr = (r2 - twoMr + a2) * isig;
    f[0] = kt;
    f[1] = kr;
    f[2] = kh;
    f[3] = kp;
    f[4] = z1 * F_t - z * F_r;
    f[5] = -(z * F_t + gi_rr * F_r + a * isig * F_p);
    f[6] = -isig * F_h;
    f[7] = -(a * isig * F_r + w * F_p);
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
    return eps * r * edge / den;
}

// One classical RK4 step of size dl (negative: away from the camera).
template <class T>
__host__ __device__ inline void rk4_step(const Spin<T>& sp, T* y, T dl)
{
    T k[8], acc[8], t[8];
    ks_rhs(sp, y, k);
    const T h2 = T(0.5) * dl;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        acc[i] = k[i];
        t[i] = y[i] + h2 * k[i];
    }
    ks_rhs(sp, t, k);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        acc[i] = acc[i] + T(2.0) * k[i];
        t[i] = y[i] + h2 * k[i];
    }
    ks_rhs(sp, t, k);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        acc[i] = acc[i] + T(2.0) * k[i];
        t[i] = y[i] + dl * k[i];
    }
    ks_rhs(sp, t, k);
    const T h6 = dl * T(1.0 / 6.0);
#pragma unroll
    for (int i = 0; i < 8; ++i) y[i] = y[i] + h6 * (acc[i] + k[i]);
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
