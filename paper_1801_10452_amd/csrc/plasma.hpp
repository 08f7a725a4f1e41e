// plasma.hpp -- fluid sampling, fluid frame, thermal-synchrotron closure, transfer update.
#pragma once
#include "device_types.hpp"
#include "ks_geodesic.hpp"
#include "rt_math.hpp"

namespace pl {

// CGS constants (CODATA 2018).
constexpr double C_LIGHT = 2.99792458e10;
constexpr double Q_E = 4.80320471e-10;
constexpr double ME_CGS = 9.1093837015e-28;
constexpr double H_PLANCK = 6.62607015e-27;
constexpr double MP_CGS = 1.67262192369e-24;
constexpr double PI_D = 3.14159265358979323846;
constexpr double NUC_PER_GAUSS = Q_E / (2.0 * PI_D * ME_CGS * C_LIGHT);      // e/(2 pi m_e c)
constexpr double J_PREF = 1.4142135623730951 * PI_D * Q_E * Q_E / (3.0 * C_LIGHT);  // sqrt2 pi e^2/(3c)
constexpr double TWO_11_12 = 1.8877486253633868;                          // 2^(11/12)
constexpr double PLANCK_PREF = 2.0 * H_PLANCK / (C_LIGHT * C_LIGHT);      // 2h/c^2
constexpr double H_OVER_MEC2 = H_PLANCK / (ME_CGS * C_LIGHT * C_LIGHT);      // h/(m_e c^2)

// theta -> x2 of the MKS polar map theta = pi x2 + (1-h)/2 sin(2 pi x2) (appendix KS-MKS).
// The paper inverts the map with Newton-Raphson; here Halley's iteration (same function, third
// order) is run from the warm start x0 with the paper's reset to 0.05 when an iterate leaves
// [0, 1] or the derivative vanishes.  It stops after the update that moved x2 by less than
// 1e-6: that update leaves an error of order (1e-6)^3, i.e. x2 is converged to rounding, the
// same root the paper's iteration converges to.
// One Halley update of x2 at x, given s = sin(2 pi x), c = cos(2 pi x).
template <class T>
__host__ __device__ inline T mks_halley(T h, T th, T x, T s, T c)
{
    using namespace rt;
    const T hh = T(0.5) * (T(1.0) - h);
    const T f = T(PI_D) * x + hh * s - th;
    const T fp = T(PI_D) * (T(1.0) + (T(1.0) - h) * c);
    const T fpp = T(-2.0 * PI_D * PI_D) * (T(1.0) - h) * s;
    T xn;
    if (fabs_(fp) < T(1e-300)) {
        xn = T(0.05);
    } else {
        const T den = T(2.0) * fp * fp - f * fpp;
        xn = (den > fp * fp * T(0.5)) ? x - T(2.0) * f * fp * rcp_nr(den) : x - f * rcp_nr(fp);
        if (xn < T(0.0) || xn > T(1.0)) xn = T(0.05);
    }
    return xn;
}

template <class T>
__host__ __device__ inline T mks_x2(T h, T th, T x0)
{
    using namespace rt;
    T x = x0;
    for (int n = 0; n < 50; ++n) {
        T s, c;
        sincos_small(T(2.0 * PI_D) * x, &s, &c);   // x in [0, 1]: argument in [0, 2 pi]
        const T xn = mks_halley(h, th, x, s, c);
        const T dx = fabs_(xn - x);
        x = xn;
        if (dx < T(1e-6)) break;
    }
    return x;
}

// Bilinear combination of the four corner values of each field (weights w1 along x1, w2
// along x2).
template <class T>
__host__ __device__ inline void bilerp4(const T* a, const T* b, const T* c, const T* d, T w1, T w2, T* out)
{
    const T u1 = T(1.0) - w1, u2 = T(1.0) - w2;
    for (int f = 0; f < 4; ++f) out[f] = u2 * (u1 * a[f] + w1 * b[f]) + w2 * (u1 * c[f] + w1 * d[f]);
}

template <class V>
__device__ inline void cell_values(const V& q, double v[4])
{
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}

// Bilinear interpolation between cell centres (clamped to the edge centres in the outer
// half cells) of snapshot s at fractional cell coordinates computed by the caller.  The four
// cells are (j0, i0), (j0, i0 + 1), (j0 + 1, i0), (j0 + 1, i0 + 1); a grid holds fewer than 2^31
// cells (checked at upload), so their index is 32-bit.
__device__ inline void bilinear(const DevGrid& g, int s, int i0, int j0, double w1, double w2, double out[4])
{
    const int idx = (s * g.n2 + j0) * g.n1 + i0;
    double a[4], b[4], c[4], d[4];
    if (g.is_f64) {
        const double4* p = reinterpret_cast<const double4*>(g.cells) + idx;
        cell_values(p[0], a);
        cell_values(p[1], b);
        cell_values(p[g.n1], c);
        cell_values(p[g.n1 + 1], d);
    } else {
        const float4* p = reinterpret_cast<const float4*>(g.cells) + idx;
        cell_values(p[0], a);
        cell_values(p[1], b);
        cell_values(p[g.n1], c);
        cell_values(p[g.n1 + 1], d);
    }
    bilerp4(a, b, c, d, w1, w2, out);
}

// Density modulation of the synthetic time series at snapshot time ts:
// 1 + A sum_{m=1..4} cos(m psi + phase_m), psi = phi - Omega_K ts, Omega_K = 1/(r^1.5 + a_gen),
// with cos(m psi), sin(m psi) from the Chebyshev recurrence of one sincos.
__device__ inline double modulation(const DevGrid& g, double r, double ph, double ts)
{
    if (g.mod_amp == 0.0) return 1.0;
    const double om = rt::rcp_nr(r * r * rt::rsqrt_nr(r) + g.a_gen);   // 1 / (r^1.5 + a_gen)
    // reduce the phase by whole turns (two-term 2 pi, exact head) before the small-argument sincos
    const double arg = ph - om * ts;
    const double turns = __builtin_rint(arg * 0.15915494309189535);
    double red = __builtin_fma(-turns, 6.2831853071795862, arg);
    red = __builtin_fma(-turns, 2.4492935982947064e-16, red);
    double s1, c1;
    rt::sincos_small(red, &s1, &c1);
    double cm = c1, sm = s1, acc = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        acc += cm * g.mod_cos[m] - sm * g.mod_sin[m];
        const double cn = cm * c1 - sm * s1;
        const double sn = sm * c1 + cm * s1;
        cm = cn;
        sm = sn;
    }
    return 1.0 + g.mod_amp * acc;
}

// x2(theta), the inverse of the MKS polar map: cubic Hermite interpolation between the grid's
// table nodes (x2 and dx2/dtheta solved by Newton's iteration on the host, uniform in theta), whose
// node count the upload chose so that the interpolation is within 1e-12 of the root; a grid whose
// table cannot reach that (x2_refine) takes Halley's iteration from the interpolated value to
// convergence, with the paper's reset rule (mks_x2).
__device__ inline double x2_of_theta(const DevGrid& g, double th)
{
    const double q = ::fmin(::fmax(th * g.x2_inv_dth, 0.0), (double)g.x2n - 1e-9);
    const int i = (int)q;
    const double s = q - i;
    const double2 A = g.x2tab[i], B = g.x2tab[i + 1];
    const double s2 = s * s, s3 = s2 * s;
    const double h00 = 2.0 * s3 - 3.0 * s2 + 1.0, h10 = s3 - 2.0 * s2 + s;
    const double h01 = -2.0 * s3 + 3.0 * s2, h11 = s3 - s2;
    const double x0 = h00 * A.x + h10 * A.y + h01 * B.x + h11 * B.y;
    if (!g.x2_refine) return x0;
    return mks_x2(g.hslope, th, x0);
}

__device__ inline bool in_plasma(const DevGrid& g, double r) { return r >= g.r_in && r <= g.r_out; }

// GRMHD primitives {rho, u, b, Omega} in code units -> {n_e, Theta_e, B, Omega} (Sec. 4.2.2:
// n_e = rho rho0 / (m_e + m_p), B = b B0 with B0 = c sqrt(4 pi rho0); Sec. 5: the proton-to-
// electron temperature ratio R = R_low / (1 + beta^2) + R_high beta^2 / (1 + beta^2) with
// beta = P_gas / P_mag, P_gas = (gamma - 1) u, P_mag = b^2 / 2; Theta_e = (m_p / m_e) P_gas /
// rho / (1 + R), the gas pressure shared by ions and electrons).  R is formed as
// (R_low P_mag^2 + R_high P_gas^2) / (P_mag^2 + P_gas^2), finite for b = 0; a cell without
// density or pressure has Theta_e = 0 (no emission).
__device__ inline void code_to_cgs(const DevGrid& g, double v[4])
{
    const double rho = v[0], pg = g.gam1 * v[1], pm = 0.5 * v[2] * v[2];
    const double pg2 = pg * pg, pm2 = pm * pm;
    const double den = pm2 + pg2;
    const double R = den > 0.0 ? (g.r_low * pm2 + g.r_high * pg2) * rt::rcp_nr(den) : g.r_high;
    const double the = (rho > 0.0 && v[1] > 0.0) ? g.thetae_fac * v[1] * rt::rcp_nr(rho * (1.0 + R)) : 0.0;
    v[0] = rho * g.ne_scale;
    v[1] = the;
    v[2] = v[2] * g.b_scale;
}

// Fluid quantities {n_e, Theta_e, B, Omega} at the ray point y = (t, r, theta, phi); the caller
// has checked that r lies in the grid's radial range.  A code-unit grid is interpolated in its
// primitives and converted at the sample point.
__device__ inline void sample_fluid(const DevGrid& g, int slow_light, int fast_snap, const double* y, double out[4])
{
    const double r = y[1];
    const double x1 = rt::log_pos(r);
    const double x2 = x2_of_theta(g, y[2]);
    double f1 = (x1 - g.lnr_in) * g.inv_d1 - 0.5;
    double f2 = x2 * g.n2 - 0.5;
    f1 = ::fmin(::fmax(f1, 0.0), (double)(g.n1 - 1));
    f2 = ::fmin(::fmax(f2, 0.0), (double)(g.n2 - 1));
    int i0 = (int)::floor(f1), j0 = (int)::floor(f2);
    i0 = i0 > g.n1 - 2 ? g.n1 - 2 : i0;
    j0 = j0 > g.n2 - 2 ? g.n2 - 2 : j0;
    const double w1 = f1 - i0, w2 = f2 - j0;
    int s0 = fast_snap;
    double w = 0.0;
    if (slow_light && g.n_snap > 1) {
        // clamp before the conversion so that any finite time maps to a valid snapshot pair
        const double q = ::fmin(::fmax((y[0] - g.t0) * g.inv_dt, -1.0), (double)g.n_snap);
        s0 = (int)::floor(q);
        s0 = s0 < 0 ? 0 : (s0 > g.n_snap - 2 ? g.n_snap - 2 : s0);
        w = ::fmin(::fmax(q - s0, 0.0), 1.0);
    }
    double v0[4];
    bilinear(g, s0, i0, j0, w1, w2, v0);
    v0[0] *= modulation(g, r, y[3], g.t0 + s0 * g.dt_snap);
    if (w > 0.0) {
        double v1[4];
        bilinear(g, s0 + 1, i0, j0, w1, w2, v1);
        v1[0] *= modulation(g, r, y[3], g.t0 + (s0 + 1) * g.dt_snap);
#pragma unroll
        for (int f = 0; f < 4; ++f) out[f] = (1.0 - w) * v0[f] + w * v1[f];
    } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) out[f] = v0[f];
    }
    if (g.units) code_to_cgs(g, out);
}

// Fluid frame of a circular flow u = u^t (1, 0, 0, Omega) in the KS metric, with the ZAMO
// angular velocity where Omega is not timelike.  Returns nu_r = -k.u and the cosine of the
// fluid-frame angle between k and the unit toroidal field b ~ (u_phi, 0, 0, -u_t).
template <class T>
__host__ __device__ inline bool fluid_frame(T a, T a2, T M, const T* y, T s, T c, T omega, T* nu_r, T* cos_b)
{
    using namespace rt;
    const T r = y[1];
    const T s2 = s * s;
    const T sig = r * r + a2 * c * c;
    const T z = T(2.0) * M * r * rcp_nr(sig);
    const T z1 = T(1.0) + z;
    const T gtt = z - T(1.0);
    const T gtp = -a * z * s2;
    const T grp = -a * s2 * z1;
    const T gpp = s2 * (sig + a2 * s2 * z1);
    bool zamo = false;
    T D = -(gtt + T(2.0) * gtp * omega + gpp * omega * omega);
    if (D <= T(1e-10)) {
        omega = -gtp / gpp;
        D = -(gtt + T(2.0) * gtp * omega + gpp * omega * omega);
        zamo = true;
    }
    const T ut = rsqrt_nr(D);
    const T up = omega * ut;
    const T u_t = gtt * ut + gtp * up;
    const T u_p = gtp * ut + gpp * up;
    const T kt = y[4], kr = y[5], kp = y[7];
    const T k_t = gtt * kt + z * kr + gtp * kp;
    const T k_p = gtp * kt + grp * kr + gpp * kp;
    const T nr = -(k_t * ut + k_p * up);
    const T bb = gtt * u_p * u_p - T(2.0) * gtp * u_p * u_t + gpp * u_t * u_t;
    const T kb = (k_t * u_p - k_p * u_t) * rsqrt_nr(bb);
    T cb = kb * rcp_nr(nr);
    cb = fmin_(fmax_(cb, T(-1.0)), T(1.0));
    *nu_r = nr;
    *cos_b = cb;
    return zamo;
}

// ln K2(1/Theta) from the octave table: the binary exponent and mantissa of Theta select the
// interval (no logarithm), cubic Hermite interpolation inside it.  Outside the table's range
// the large- and small-argument expansions of K2 are exact to rounding there:
//   x = 1/Theta > 128:   ln K2 = -x + 1/2 ln(pi / 2x) + ln(1 + sum_k a_k x^-k),
//                        a_k = prod_{i=1..k} (16 - (2i - 1)^2) / (k! 8^k) (Hankel's series,
//                        Abramowitz & Stegun 9.7.2; six terms leave < 1e-14 at x = 128);
//   x = 1/Theta < 2^-14: ln K2 = ln(2 / x^2) - x^2 / 4 (K2 = 2/x^2 - 1/2 + O(x^2 ln x)).
__host__ __device__ inline double ln_k2_theta(const K2Table& t, double the)
{
    if (the < t.th_lo) {
        const double x = 1.0 / the, u = the * 0.125;   // u = 1/(8x)
        // 1 + a_1/x + ... + a_6/x^6 with a_k/x^k = c_k u^k, c_k = prod (16 - (2i-1)^2) / k!
        double p = 1.0 + u * (15.0 + u * (52.5 + u * (-157.5 + u * (1299.375 + u * (-16891.875 + u * 295607.8125)))));
        return -x + 0.5 * rt::log_pos(0.5 * PI_D * the) + rt::log_pos(p);
    }
    if (the > t.th_hi) {
        const double x = 1.0 / the;
        return 0.6931471805599453 + 2.0 * rt::log_pos(the) - 0.25 * x * x;
    }
    int e;
    const double m = __builtin_frexp(the, &e);           // the = m 2^e, m in [1/2, 1)
    const double q = (m - 0.5) * (double)(2 * t.nsub);   // exact: a power-of-two scaling
    int j = (int)q;
    j = j < t.nsub - 1 ? j : t.nsub - 1;
    const double s = q - j;
    const double4 E = t.tab[(e - t.e_lo) * t.nsub + j];
    const double s2 = s * s, s3 = s2 * s;
    const double h00 = 2.0 * s3 - 3.0 * s2 + 1.0, h10 = s3 - 2.0 * s2 + s;
    const double h01 = -2.0 * s3 + 3.0 * s2, h11 = s3 - s2;
    return h00 * E.x + h10 * E.y + h01 * E.z + h11 * E.w;
}

// Emission j_nu and absorption alpha_nu in the fluid frame (Sec. 4.2.2): Leung et al. fit
// with nu_s = (2/9) nu_c Theta_e^2 sin(theta_B), X = nu/nu_s,
// (X^1/2 + 2^11/12 X^1/6)^2 = X^1/3 (X^1/3 + 2^11/12)^2, and alpha = j / B_nu.  *bnu gets
// B_nu (the source function j/alpha of thermal emission).  ln_k2 = ln K2(1/Theta_e): 1/K2 and
// the cut-off exp(-X^1/3) are applied as one exponential, since either alone leaves the double
// range for cold plasma (Theta_e below ~0.0014) where their product need not.
template <class T>
__host__ __device__ inline void closure_exact(T nu, T ne, T the, T bf, T sinb, T ln_k2, T* j, T* alpha, T* bnu)
{
    using namespace rt;
    const T nu_s = T(2.0 / 9.0 * NUC_PER_GAUSS) * bf * the * the * sinb;
    const T X = nu / nu_s;
    const T t = cbrt_(X);
    const T tc = t + T(TWO_11_12);
    const T jv = T(J_PREF) * ne * nu_s * t * tc * tc * exp_(-(t + ln_k2));
    const T B = T(PLANCK_PREF) * nu * nu * nu / expm1_(T(H_OVER_MEC2) * nu / the);
    *j = jv;
    *alpha = jv / B;
    *bnu = B;
}

// Contribution of one step to the observed intensity before attenuation by the optical depth
// already between the point and the camera, A = S (1 - exp(-dtau)) / nu_r^3 (j ds / nu_r^3
// when dtau = 0), and the step's optical depth dtau = alpha ds (Sec. 3.1, per-step formal
// solution in the backward scheme).
template <class T>
__host__ __device__ inline void step_source(T j, T al, T S, T ds, T inr3, T& A, T& dtau)
{
    using namespace rt;
    dtau = al * ds;
    A = (dtau > T(0.0)) ? S * (-expm1_(-dtau)) * inr3 : j * ds * inr3;
}

// Backward formal-solution update of one frequency (Sec. 3.1): the step's emission with
// source S = j/alpha over optical depth dtau = alpha ds, attenuated by the optical depth tau
// already between the point and the camera, in observed units (1/nu_r^3).
template <class T>
__host__ __device__ inline void transfer_update(T j, T al, T S, T ds, T inr3, T& I, T& tau)
{
    using namespace rt;
    const T dtau = al * ds;
    const T att = exp_(-tau);
    const T add = (dtau > T(0.0)) ? att * S * (-expm1_(-dtau)) * inr3 : att * j * ds * inr3;
    I = I + add;
    tau = tau + dtau;
}

}  // namespace pl
