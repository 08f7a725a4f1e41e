/* raptor_oracle.c -- plain, slow, obviously correct CPU FP64 oracle of the RAPTOR hot path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the benchmark's
 * CPU-baseline leg, never by the product path.  It shares no code with the GPU library.
 *
 * Every step follows Bronzwaer et al. 2018 (RAPTOR I, arXiv:1801.10452); each function
 * names the passage it implements.  Where the paper is silent the reading taken is stated
 * at the function.  Geometrized units (G = c = M = 1) for geometry, CGS for the plasma.
 *
 * Design rule: no blocking, fusion or reordering beyond what the definitions state.
 * The connection is built from the generic formula (Sec. 2.1, connection equation) with
 * metric derivatives from complex-step differentiation (Squire & Trapp 1998), which is
 * exact to rounding for the analytic Kerr metric functions; the metric inverse is a plain
 * Gauss-Jordan inversion; K2 is its integral representation evaluated by the trapezoid
 * rule (exponentially convergent for this integrand).
 */
#include "raptor_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CGS constants (CODATA 2018), held here as data. */
#define O_C     2.99792458e10
#define O_G     6.67430e-8
#define O_MSUN  1.98847e33
#define O_PC    3.085677581e18
#define O_E     4.80320471e-10
#define O_ME    9.1093837015e-28
#define O_H     6.62607015e-27
#define O_KB    1.380649e-16
#define O_MP    1.67262192369e-24

#define IDX(a, b) ((a) * 4 + (b))

/* ===================================================================================== */
/* Spacetime                                                                            */
/* ===================================================================================== */

/* Kerr metric, covariant, in ingoing Kerr-Schild coordinates (t~, r, theta, phi~) for
 * mass M and spin a.  The paper names this chart (Sec. 2.4) and gives its relation to
 * Boyer-Lindquist coordinates (appendix, BL-KS transformation); the component form is
 * the textbook one.  Written over complex arguments so that the complex-step method
 * yields exact derivatives. */
static void ks_metric_c(double a, double M, double complex r, double complex th,
                        double complex g[16])
{
    double complex s = csin(th), c = ccos(th);
    double complex s2 = s * s, c2 = c * c;
    double complex sig = r * r + a * a * c2;
    double complex z = 2.0 * M * r / sig;
    for (int i = 0; i < 16; ++i) g[i] = 0.0;
    g[IDX(0, 0)] = -(1.0 - z);
    g[IDX(0, 1)] = g[IDX(1, 0)] = z;
    g[IDX(0, 3)] = g[IDX(3, 0)] = -a * z * s2;
    g[IDX(1, 1)] = 1.0 + z;
    g[IDX(1, 3)] = g[IDX(3, 1)] = -a * s2 * (1.0 + z);
    g[IDX(2, 2)] = sig;
    g[IDX(3, 3)] = s2 * (sig + a * a * s2 * (1.0 + z));
}

void orc_ks_metric(double a, double M, double r, double th, double g[16])
{
    double complex gc[16];
    ks_metric_c(a, M, r, th, gc);
    for (int i = 0; i < 16; ++i) g[i] = creal(gc[i]);
}

/* g_{mu nu} and dg[rho*16 + mu*4 + nu] = d_rho g_{mu nu}.  The metric does not depend on
 * t~ or phi~ (stationary, axisymmetric), so only rho = r, theta are non-zero. */
void orc_ks_metric_derivs(double a, double M, double r, double th, double g[16], double dg[64])
{
    const double hstep = 1e-30;
    double complex gr[16], gt[16];
    ks_metric_c(a, M, r + I * hstep, th, gr);
    ks_metric_c(a, M, r, th + I * hstep, gt);
    memset(dg, 0, 64 * sizeof(double));
    for (int i = 0; i < 16; ++i) {
        g[i] = creal(gr[i]);
        dg[16 * 1 + i] = cimag(gr[i]) / hstep;
        dg[16 * 2 + i] = cimag(gt[i]) / hstep;
    }
}

/* Kerr metric in Boyer-Lindquist coordinates (used only at the camera, Sec. 2.3). */
void orc_bl_metric(double a, double M, double r, double th, double g[16])
{
    double s = sin(th), c = cos(th);
    double s2 = s * s, c2 = c * c;
    double sig = r * r + a * a * c2;
    double del = r * r - 2.0 * M * r + a * a;
    memset(g, 0, 16 * sizeof(double));
    g[IDX(0, 0)] = -(1.0 - 2.0 * M * r / sig);
    g[IDX(0, 3)] = g[IDX(3, 0)] = -2.0 * M * a * r * s2 / sig;
    g[IDX(1, 1)] = sig / del;
    g[IDX(2, 2)] = sig;
    g[IDX(3, 3)] = (r * r + a * a + 2.0 * M * r * a * a * s2 / sig) * s2;
}

/* Gauss-Jordan inversion with partial pivoting; returns 0 on success. */
int orc_invert4(const double m[16], double inv[16])
{
    double w[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            w[i][j] = m[IDX(i, j)];
            w[i][j + 4] = (i == j) ? 1.0 : 0.0;
        }
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int i = col + 1; i < 4; ++i)
            if (fabs(w[i][col]) > fabs(w[piv][col])) piv = i;
        if (w[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < 8; ++j) { double t = w[col][j]; w[col][j] = w[piv][j]; w[piv][j] = t; }
        double d = w[col][col];
        for (int j = 0; j < 8; ++j) w[col][j] /= d;
        for (int i = 0; i < 4; ++i) {
            if (i == col) continue;
            double f = w[i][col];
            for (int j = 0; j < 8; ++j) w[i][j] -= f * w[col][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) inv[IDX(i, j)] = w[i][j + 4];
    return 0;
}

/* Connection coefficients, Sec. 2.1 (connection equation):
 * Gamma^alpha_{mu nu} = 1/2 g^{alpha rho} (d_mu g_{nu rho} + d_nu g_{mu rho} - d_rho g_{mu nu}).
 * gam[alpha*16 + mu*4 + nu]. */
void orc_christoffel(double a, double M, const double x[4], double gam[64])
{
    double g[16], dg[64], gi[16];
    orc_ks_metric_derivs(a, M, x[1], x[2], g, dg);
    orc_invert4(g, gi);
    for (int al = 0; al < 4; ++al)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) {
                double s = 0.0;
                for (int rho = 0; rho < 4; ++rho)
                    s += gi[IDX(al, rho)] * (dg[16 * mu + IDX(nu, rho)] + dg[16 * nu + IDX(mu, rho)]
                                             - dg[16 * rho + IDX(mu, nu)]);
                gam[16 * al + IDX(mu, nu)] = 0.5 * s;
            }
}

/* Right-hand side of the first-order geodesic system, Sec. 2.2:
 * dx^alpha/dlambda = k^alpha, dk^alpha/dlambda = -Gamma^alpha_{mu nu} k^mu k^nu. */
void orc_geodesic_rhs(double a, double M, const double y[8], double f[8])
{
    double gam[64];
    orc_christoffel(a, M, y, gam);
    const double* k = y + 4;
    for (int al = 0; al < 4; ++al) {
        f[al] = k[al];
        double s = 0.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) s += gam[16 * al + IDX(mu, nu)] * k[mu] * k[nu];
        f[4 + al] = -s;
    }
}

/* Adaptive step, Sec. 2.2 (adaptive step-size equations), applied in the paper's
 * logarithmic KS chart: x1 = ln r, x2 = theta/pi in [0,1], x3 = phi.  Chart components of
 * k are k^r / r, k^theta / pi and k^phi; the returned size is positive (the caller sets the
 * direction).  delta protects against division by zero as in the paper. */
double orc_step_size(double eps, const double x[4], const double k[4])
{
    const double delta = 1e-40;
    double r = x[1], th = x[2];
    double x2 = th / M_PI;
    double edge = fmin(x2, 1.0 - x2);
    if (edge < 1e-12) edge = 1e-12;
    double d1 = eps / (fabs(k[1] / r) + delta);
    double d2 = eps * edge / (fabs(k[2] / M_PI) + delta);
    double d3 = eps / (fabs(k[3]) + delta);
    return 1.0 / (1.0 / d1 + 1.0 / d2 + 1.0 / d3);
}

/* Classical fourth-order Runge-Kutta step on y = (x, k), Sec. 2.2.1.  The printed second
 * position coefficient reads k + C1x/2; the standard scheme (which the wave-vector lines of
 * the same equation follow) uses the state at the midpoint, i.e. f evaluated at
 * y + C1/2 for all eight components -- this is what is done here. */
void orc_rk4_step(double a, double M, const double y[8], double dl, double yout[8])
{
    double c1[8], c2[8], c3[8], c4[8], t[8];
    orc_geodesic_rhs(a, M, y, c1);
    for (int i = 0; i < 8; ++i) { c1[i] *= dl; t[i] = y[i] + 0.5 * c1[i]; }
    orc_geodesic_rhs(a, M, t, c2);
    for (int i = 0; i < 8; ++i) { c2[i] *= dl; t[i] = y[i] + 0.5 * c2[i]; }
    orc_geodesic_rhs(a, M, t, c3);
    for (int i = 0; i < 8; ++i) { c3[i] *= dl; t[i] = y[i] + c3[i]; }
    orc_geodesic_rhs(a, M, t, c4);
    for (int i = 0; i < 8; ++i) {
        c4[i] *= dl;
        yout[i] = y[i] + (c1[i] + 2.0 * c2[i] + 2.0 * c3[i] + c4[i]) / 6.0;
    }
}

/* Second-order Runge-Kutta (midpoint) step.  The paper names RK2 only for its timing runs;
 * the midpoint rule is the reading taken here: C1 = dl f(y), y_new = y + dl f(y + C1/2). */
void orc_rk2_step(double a, double M, const double y[8], double dl, double yout[8])
{
    double c1[8], c2[8], t[8];
    orc_geodesic_rhs(a, M, y, c1);
    for (int i = 0; i < 8; ++i) t[i] = y[i] + 0.5 * dl * c1[i];
    orc_geodesic_rhs(a, M, t, c2);
    for (int i = 0; i < 8; ++i) yout[i] = y[i] + dl * c2[i];
}

/* Velocity Verlet step, Sec. 2.2.2: with A_n = (dk/dlambda)_n,
 *   x_{n+1} = x_n + k_n dl + A_n dl^2 / 2,   k_p = k_n + A_n dl,
 *   A_{n+1} = -Gamma(x_{n+1}) k_p k_p,       k_{n+1} = k_n + (A_n + A_{n+1}) dl / 2,
 * and with the corrector the derivative is evaluated once more with k_p = k_{n+1} and the last
 * line repeated.  acc holds A_n on entry and the last evaluated derivative on return. */
void orc_verlet_step(double a, double M, const double y[8], double acc[4], double dl, int corrector,
                     double yout[8])
{
    double t[8], f[8];
    for (int i = 0; i < 4; ++i) {
        t[i] = y[i] + y[4 + i] * dl + 0.5 * acc[i] * dl * dl;
        t[4 + i] = y[4 + i] + acc[i] * dl;
    }
    orc_geodesic_rhs(a, M, t, f);
    for (int i = 0; i < 4; ++i) t[4 + i] = y[4 + i] + 0.5 * (acc[i] + f[4 + i]) * dl;
    if (corrector) {
        orc_geodesic_rhs(a, M, t, f);
        for (int i = 0; i < 4; ++i) t[4 + i] = y[4 + i] + 0.5 * (acc[i] + f[4 + i]) * dl;
    }
    for (int i = 0; i < 4; ++i) acc[i] = f[4 + i];
    memcpy(yout, t, 8 * sizeof(double));
}

/* One step of the chosen integrator.  Verlet carries the derivative from step to step in
 * acc; *have_acc = 0 asks for it to be evaluated at y first (start of a ray, or after a pole
 * reflection changed the chart). */
static void geo_step(double a, double M, int integrator, const double y[8], double acc[4], int* have_acc,
                     double dl, double yout[8])
{
    if (integrator == ORC_RK2) {
        orc_rk2_step(a, M, y, dl, yout);
    } else if (integrator == ORC_VERLET || integrator == ORC_VERLET_CORR) {
        if (!*have_acc) {
            double f[8];
            orc_geodesic_rhs(a, M, y, f);
            for (int i = 0; i < 4; ++i) acc[i] = f[4 + i];
        }
        orc_verlet_step(a, M, y, acc, dl, integrator == ORC_VERLET_CORR, yout);
        *have_acc = 1;
    } else {
        orc_rk4_step(a, M, y, dl, yout);
    }
}

static int state_finite(const double y[8])
{
    for (int i = 0; i < 8; ++i)
        if (!isfinite(y[i])) return 0;
    return 1;
}

/* Crossing the polar axis: (theta, phi) -> (-theta, phi + pi) or (2 pi - theta, phi + pi)
 * names the same point, and the polar velocity changes sign.  (The paper does not discuss
 * pole crossings; this is the coordinate identity.) */
static int reflect_pole(double y[8])
{
    if (y[2] < 0.0) {
        y[2] = -y[2];
    } else if (y[2] > M_PI) {
        y[2] = 2.0 * M_PI - y[2];
    } else {
        return 0;
    }
    y[3] += M_PI;
    y[6] = -y[6];
    return 1;
}

/* Termination tests after a step (reading: the paper only fixes the horizon radius
 * r_+ = M + sqrt(M^2 - a^2), appendix BL-KS).  Returns a status, 0 if the ray goes on. */
static int termination(const double y[8], int steps, int max_steps, double r_stop, double r_escape)
{
    if (y[1] < r_stop) return ORC_HORIZON;
    if (y[1] > r_escape) return ORC_ESCAPED;
    if (steps >= max_steps) return ORC_MAXSTEP;
    return ORC_RUNNING;
}

int orc_integrate(double a, double M, const double y0[8], double eps, int max_steps,
                  double r_stop, double r_escape, int integrator, double* traj, double* dls, int cap,
                  orc_ray_info* info)
{
    double y[8], yn[8], acc[4];
    int have_acc = 0;
    memcpy(y, y0, sizeof y);
    int steps = 0, poles = 0, status = ORC_RUNNING;
    while (status == ORC_RUNNING) {
        double dl = -orc_step_size(eps, y, y + 4);
        geo_step(a, M, integrator, y, acc, &have_acc, dl, yn);
        memcpy(y, yn, sizeof y);
        ++steps;
        if (!state_finite(y)) { status = ORC_NUMERIC; break; }
        if (reflect_pole(y)) { ++poles; have_acc = 0; }
        if (traj && steps <= cap) {
            memcpy(traj + 8 * (steps - 1), y, sizeof y);
            if (dls) dls[steps - 1] = dl;
        }
        status = termination(y, steps, max_steps, r_stop, r_escape);
    }
    if (info) { info->status = status; info->steps = steps; info->samples = 0; info->poles = poles; }
    return steps;
}

/* ===================================================================================== */
/* Thin accretion disk (Sec. 4.2.1)                                                     */
/* ===================================================================================== */

/* Innermost stable circular orbit (Bardeen, Press & Teukolsky 1972):
 * r = 3 + Z2 - sign(a) sqrt((3 - Z1)(3 + Z1 + 2 Z2)),
 * Z1 = 1 + (1 - a^2)^(1/3) ((1 + a)^(1/3) + (1 - a)^(1/3)), Z2 = sqrt(3 a^2 + Z1^2). */
double orc_isco(double a)
{
    double z1 = 1.0 + cbrt(1.0 - a * a) * (cbrt(1.0 + a) + cbrt(1.0 - a));
    double z2 = sqrt(3.0 * a * a + z1 * z1);
    double s = a >= 0.0 ? 1.0 : -1.0;
    return 3.0 + z2 - s * sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

/* The crossing point (reading: the paper does not say how crossings are located): when a step
 * from y to y' brackets theta = pi/2, the affine parameter of the crossing is estimated by
 * linear interpolation of theta, then refined by two Newton iterations on theta(lambda), each
 * integrating one step of that length from y with the same integrator (dtheta/dlambda = k^theta).
 * The crossing state is thus an integrated state, on which k_t and k_phi keep their conserved
 * values.  The disk gas moves on prograde Keplerian circles, Omega = 1/(r^(3/2) + a). */
void orc_trace_disk_ray(const orc_camera* cam, const orc_opts* o, double r_disk_out, double alpha, double beta,
                        double* g, double* r_cross, double* Iv, orc_ray_info* info)
{
    double M = o->metric_mass, a = cam->spin;
    double rh = M + sqrt(M * M - a * a);
    double r_stop = o->r_stop_factor * rh;
    double r_in = orc_isco(a);
    double y[8], yn[8], acc[4], acc0[4];
    int have_acc = 0;
    orc_camera_ray(cam, M, alpha, beta, 0.0, y, NULL);
    int steps = 0, poles = 0, status = ORC_RUNNING;
    *g = 0.0; *r_cross = 0.0; *Iv = 0.0;
    while (status == ORC_RUNNING) {
        double dl = -orc_step_size(o->eps, y, y + 4);
        int had_acc = have_acc;
        memcpy(acc0, acc, sizeof acc);
        geo_step(a, M, o->integrator, y, acc, &have_acc, dl, yn);
        ++steps;
        if (!state_finite(yn)) { status = ORC_NUMERIC; break; }
        double h0 = y[2] - 0.5 * M_PI, h1 = yn[2] - 0.5 * M_PI;
        if (h0 * h1 < 0.0) {
            double lam = dl * h0 / (h0 - h1), yc[8], ac[4];
            for (int it = 0; it < 3; ++it) {
                int hc = had_acc;
                memcpy(ac, acc0, sizeof ac);
                geo_step(a, M, o->integrator, y, ac, &hc, lam, yc);
                if (it < 2) lam += (0.5 * M_PI - yc[2]) / yc[6];
            }
            *r_cross = yc[1];
            if (yc[1] >= r_in && yc[1] <= r_disk_out) {
                double u[4], b[4], nr, cb;
                double omega = 1.0 / (pow(yc[1], 1.5) + a);
                orc_fluid_frame(a, M, yc, yc + 4, omega, u, b, &nr, &cb);
                *g = 1.0 / nr;
                *Iv = (*g) * (*g) * (*g) / (yc[1] * yc[1]);
                status = ORC_DISK;
            } else {
                status = ORC_PLANE;
            }
            break;
        }
        memcpy(y, yn, sizeof y);
        if (reflect_pole(y)) { ++poles; have_acc = 0; }
        status = termination(y, steps, o->max_steps, r_stop, cam->r_cam);
    }
    if (info) { info->status = status; info->steps = steps; info->samples = 0; info->poles = poles; }
}

void orc_trace_disk_image(const orc_camera* cam, const orc_opts* o, double r_disk_out, double* g, double* Iv,
                          orc_ray_info* info, int n_threads)
{
    long n = (long)cam->nx * cam->ny;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
#endif
    for (long p = 0; p < n; ++p) {
        double al, be, rc;
        orc_pixel_alpha_beta(cam, (int)(p % cam->nx), (int)(p / cam->nx), &al, &be);
        orc_trace_disk_ray(cam, o, r_disk_out, al, be, &g[p], &rc, &Iv[p], info ? &info[p] : NULL);
    }
}

void orc_disk_profile(const orc_camera* cam, const double* g, const double* Iv, int n_bins, double g_lo,
                      double g_hi, double* profile)
{
    double dA = (2.0 * cam->fov_half / cam->nx) * (2.0 * cam->fov_half / cam->ny);
    for (int b = 0; b < n_bins; ++b) profile[b] = 0.0;
    for (long p = 0; p < (long)cam->nx * cam->ny; ++p) {
        if (!(Iv[p] > 0.0)) continue;
        double q = (g[p] - g_lo) / (g_hi - g_lo) * n_bins;
        if (q < 0.0 || q >= n_bins) continue;
        profile[(int)q] += Iv[p] * dA;
    }
}

/* ===================================================================================== */
/* Camera                                                                               */
/* ===================================================================================== */

/* Pixel centres (reading: the paper gives the alpha, beta ranges only).  alpha_i spans
 * [-F, F] left to right, beta_j spans [-F, F] with row j = 0 at beta = -F. */
void orc_pixel_alpha_beta(const orc_camera* cam, int i, int j, double* alpha, double* beta)
{
    double F = cam->fov_half;
    *alpha = -F + (i + 0.5) * (2.0 * F / cam->nx);
    *beta = -F + (j + 0.5) * (2.0 * F / cam->ny);
}

/* Virtual camera, Sec. 2.3 (Bardeen's construction) and appendix BL-KS.
 * E = 1, L = -alpha E sin i, Q = E^2 [beta^2 + cos^2 i (alpha^2 - a^2)].  The printed Q
 * has (alpha^2 - 1) and the printed k_theta lacks the a^2 of the Carter term; both are
 * read as the Bardeen / Carter forms (the two cancel at theta = i, giving k_theta = beta).
 * k_r follows from the null condition with k^r > 0 (photon moving toward the camera); the
 * vector is raised with the BL inverse metric and mapped to KS with the appendix matrix.
 * The BL->KS offsets of t and phi are dropped: constants along the camera sphere that do
 * not affect a stationary axisymmetric fluid; the ray starts at t~ = t_init, phi~ = 0. */
void orc_camera_ray(const orc_camera* cam, double M, double alpha, double beta,
                    double t_init, double y[8], double kcov_bl[4])
{
    double a = cam->spin;
    double inc = cam->incl_deg * M_PI / 180.0;
    double r = cam->r_cam, th = inc;
    double E = 1.0;
    double L = -alpha * E * sqrt(1.0 - cos(inc) * cos(inc));
    double Q = E * E * (beta * beta + cos(inc) * cos(inc) * (alpha * alpha - a * a));
    double cot = cos(th) / sin(th);
    double sgn = (beta >= 0.0) ? 1.0 : -1.0;
    double kth = sgn * sqrt(fabs(Q - L * L * cot * cot + a * a * E * E * cos(th) * cos(th)));

    double gbl[16], gi[16];
    orc_bl_metric(a, M, r, th, gbl);
    orc_invert4(gbl, gi);
    /* null condition g^{mu nu} k_mu k_nu = 0 as a quadratic in k_r */
    double kc[4] = {-E, 0.0, kth, L};
    double qa = gi[IDX(1, 1)];
    double qb = 0.0, qc = 0.0;
    for (int mu = 0; mu < 4; ++mu) {
        if (mu == 1) continue;
        qb += 2.0 * gi[IDX(1, mu)] * kc[mu];
        for (int nu = 0; nu < 4; ++nu)
            if (nu != 1) qc += gi[IDX(mu, nu)] * kc[mu] * kc[nu];
    }
    double disc = qb * qb - 4.0 * qa * qc;
    if (disc < 0.0) disc = 0.0;
    kc[1] = (-qb + sqrt(disc)) / (2.0 * qa);
    double kup[4];
    for (int mu = 0; mu < 4; ++mu) {
        kup[mu] = 0.0;
        for (int nu = 0; nu < 4; ++nu) kup[mu] += gi[IDX(mu, nu)] * kc[nu];
    }
    double del = r * r - 2.0 * M * r + a * a;
    y[0] = t_init;
    y[1] = r;
    y[2] = th;
    y[3] = 0.0;
    y[4] = kup[0] + 2.0 * M * r / del * kup[1];
    y[5] = kup[1];
    y[6] = kup[2];
    y[7] = kup[3] + a / del * kup[1];
    if (kcov_bl) memcpy(kcov_bl, kc, sizeof kc);
}

/* ===================================================================================== */
/* Fluid grid                                                                           */
/* ===================================================================================== */

/* theta -> x2 for MKS, appendix KS-MKS: Newton-Raphson on
 * f(x2) = pi x2 + (1-h)/2 sin(2 pi x2) - theta, f' = pi (1 + (1-h) cos(2 pi x2)), with the
 * paper's reset to 0.05 when the iterate leaves [0,1] or f' vanishes, stopping when
 * |x2_{n+1} - x2_n| < 1e-14.  Reading: the start value is theta/pi (exact for h = 1). */
double orc_mks_x2(double h, double th, int* iters)
{
    double x = th / M_PI;
    int n = 0;
    for (n = 1; n <= 50; ++n) {
        double f = M_PI * x + 0.5 * (1.0 - h) * sin(2.0 * M_PI * x) - th;
        double fp = M_PI * (1.0 + (1.0 - h) * cos(2.0 * M_PI * x));
        double xn;
        if (fabs(fp) < 1e-300) {
            xn = 0.05;
        } else {
            xn = x - f / fp;
            if (xn < 0.0 || xn > 1.0) xn = 0.05;
        }
        double dx = fabs(xn - x);
        x = xn;
        if (dx < 1e-14) break;
    }
    if (iters) *iters = n;
    return x;
}

static double cell(const orc_grid* g, int s, int j, int i, int f)
{
    size_t idx = (((size_t)s * g->n2 + j) * g->n1 + i) * 4 + f;
    return g->is_f64 ? ((const double*)g->cells)[idx] : (double)((const float*)g->cells)[idx];
}

/* Bilinear interpolation between cell centres in (x1, x2) (reading: the paper does not
 * state its interpolation); coordinates in the outer half cells clamp to the edge centre. */
static void bilinear(const orc_grid* g, int s, double x1, double x2, double v[4])
{
    double lo = log(g->r_in), d1 = (log(g->r_out) - lo) / g->n1;
    double f1 = (x1 - lo) / d1 - 0.5;
    double f2 = x2 * g->n2 - 0.5;
    if (f1 < 0.0) f1 = 0.0;
    if (f1 > g->n1 - 1) f1 = g->n1 - 1;
    if (f2 < 0.0) f2 = 0.0;
    if (f2 > g->n2 - 1) f2 = g->n2 - 1;
    int i0 = (int)floor(f1), j0 = (int)floor(f2);
    if (i0 > g->n1 - 2) i0 = g->n1 - 2;
    if (j0 > g->n2 - 2) j0 = g->n2 - 2;
    double w1 = f1 - i0, w2 = f2 - j0;
    for (int f = 0; f < 4; ++f)
        v[f] = (1.0 - w2) * ((1.0 - w1) * cell(g, s, j0, i0, f) + w1 * cell(g, s, j0, i0 + 1, f))
             + w2 * ((1.0 - w1) * cell(g, s, j0 + 1, i0, f) + w1 * cell(g, s, j0 + 1, i0 + 1, f));
}

/* Azimuthal modulation of the density of the synthetic time series at snapshot time ts. */
static double modulation(const orc_grid* g, double r, double ph, double ts)
{
    if (g->mod_amp == 0.0) return 1.0;
    double om = 1.0 / (pow(r, 1.5) + g->a_gen);
    double s = 0.0;
    for (int m = 1; m <= 4; ++m) s += cos(m * (ph - om * ts) + g->mod_phase[m - 1]);
    return 1.0 + g->mod_amp * s;
}

/* Fluid quantities {n_e, Theta_e, B, Omega} at (t, r, theta, phi).  Outside [r_in, r_out]
 * there is no plasma (returns 0).  Fast light (Sec. 5) reads the snapshot at the frame time;
 * slow light interpolates linearly in t between the two snapshots around the ray's own
 * coordinate time, clamped at the ends of the series. */
int orc_grid_sample(const orc_grid* g, int slow_light, double t_frame, double r, double th,
                    double ph, double t, double out[4])
{
    if (!(r >= g->r_in && r <= g->r_out)) return 0;
    double x1 = log(r);
    double x2 = orc_mks_x2(g->hslope, th, NULL);
    int s0 = 0;
    double w = 0.0;
    if (slow_light && g->n_snap > 1) {
        double q = (t - g->t0) / g->dt_snap;
        s0 = (int)floor(q);
        if (s0 < 0) s0 = 0;
        if (s0 > g->n_snap - 2) s0 = g->n_snap - 2;
        w = q - s0;
        if (w < 0.0) w = 0.0;
        if (w > 1.0) w = 1.0;
    } else {
        s0 = (int)floor((t_frame - g->t0) / g->dt_snap + 0.5);
        if (s0 < 0) s0 = 0;
        if (s0 > g->n_snap - 1) s0 = g->n_snap - 1;
    }
    double v0[4];
    bilinear(g, s0, x1, x2, v0);
    v0[0] *= modulation(g, r, ph, g->t0 + s0 * g->dt_snap);
    if (w > 0.0) {
        double v1[4];
        bilinear(g, s0 + 1, x1, x2, v1);
        v1[0] *= modulation(g, r, ph, g->t0 + (s0 + 1) * g->dt_snap);
        for (int f = 0; f < 4; ++f) out[f] = (1.0 - w) * v0[f] + w * v1[f];
    } else {
        for (int f = 0; f < 4; ++f) out[f] = v0[f];
    }
    return 1;
}

/* GRMHD code units (Sec. 4.2.2): the density scale rho0 = M / L^3 with L = G M_bh / c^2 and
 * the mass unit M (the model's free parameter), the field scale B0 = c sqrt(4 pi rho0), and
 * n_e = rho rho0 / (m_e + m_p).  Electron temperature (Sec. 5): the proton-to-electron
 * temperature ratio R = R_low / (1 + beta_p^2) + R_high beta_p^2 / (1 + beta_p^2) with the
 * plasma beta beta_p = P_gas / P_mag, P_mag = b^2 / 2 and, for an ideal gas of adiabatic
 * index gamma, P_gas = (gamma - 1) u.  Reading (the paper does not print it): the gas
 * pressure is shared by protons and electrons, P_gas = n k (T_p + T_e), so that
 * Theta_e = k T_e / (m_e c^2) = (m_p / m_e) (P_gas / rho) / (1 + R) in code units.  b = 0
 * means beta_p infinite (R = R_high); no density or no internal energy means Theta_e = 0. */
void orc_code_to_cgs(const orc_grid* g, double mass_msun, const double prim[4], double out[4])
{
    double L = orc_length_unit(mass_msun);
    double rho0 = g->mass_unit_g / (L * L * L);
    double B0 = O_C * sqrt(4.0 * M_PI * rho0);
    double rho = prim[0], u = prim[1], b = prim[2];
    double pgas = (g->gamma_ad - 1.0) * u;
    double pmag = 0.5 * b * b;
    double R;
    if (pmag > 0.0) {
        double beta = pgas / pmag;
        R = g->r_low / (1.0 + beta * beta) + g->r_high * beta * beta / (1.0 + beta * beta);
    } else {
        R = g->r_high;
    }
    out[0] = rho * rho0 / (O_ME + O_MP);
    out[1] = (rho > 0.0 && u > 0.0) ? (O_MP / O_ME) * (pgas / rho) / (1.0 + R) : 0.0;
    out[2] = b * B0;
    out[3] = prim[3];
}

/* ===================================================================================== */
/* Fluid frame and closure                                                              */
/* ===================================================================================== */

/* Fluid four-velocity of a circular flow u = u^t (1, 0, 0, Omega), normalised u.u = -1
 * (Sec. 2.1, timelike normalisation); when Omega is not timelike at this point the zero-
 * angular-momentum observer's Omega = -g_tphi / g_phiphi is used instead (reading).
 * nu_r = -k^mu u_mu is the fluid-frame frequency per unit observed frequency (Sec. 3.1).
 * b is the unit toroidal field orthogonal to u, b ~ (u_phi, 0, 0, -u_t); cos_b is the
 * fluid-frame cosine between the photon direction and b, (k.b)/nu_r (the pitch angle the
 * emissivity needs, Sec. 4.2.2).  Returns 1 if the ZAMO fallback was used. */
int orc_fluid_frame(double a, double M, const double x[4], const double k[4], double omega,
                    double u[4], double b[4], double* nu_r, double* cos_b)
{
    double g[16];
    orc_ks_metric(a, M, x[1], x[2], g);
    int zamo = 0;
    double D = -(g[IDX(0, 0)] + 2.0 * g[IDX(0, 3)] * omega + g[IDX(3, 3)] * omega * omega);
    if (D <= 1e-10) {
        omega = -g[IDX(0, 3)] / g[IDX(3, 3)];
        D = -(g[IDX(0, 0)] + 2.0 * g[IDX(0, 3)] * omega + g[IDX(3, 3)] * omega * omega);
        zamo = 1;
    }
    double ut = 1.0 / sqrt(D);
    u[0] = ut; u[1] = 0.0; u[2] = 0.0; u[3] = omega * ut;
    double ul[4];
    for (int m = 0; m < 4; ++m) {
        ul[m] = 0.0;
        for (int n = 0; n < 4; ++n) ul[m] += g[IDX(m, n)] * u[n];
    }
    double nr = 0.0;
    for (int m = 0; m < 4; ++m) nr -= k[m] * ul[m];
    b[0] = ul[3]; b[1] = 0.0; b[2] = 0.0; b[3] = -ul[0];
    double bb = 0.0;
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) bb += g[IDX(m, n)] * b[m] * b[n];
    double bn = sqrt(bb);
    for (int m = 0; m < 4; ++m) b[m] /= bn;
    double kb = 0.0;
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) kb += g[IDX(m, n)] * k[m] * b[n];
    double cb = kb / nr;
    if (cb > 1.0) cb = 1.0;
    if (cb < -1.0) cb = -1.0;
    *nu_r = nr;
    *cos_b = cb;
    return zamo;
}

/* Modified Bessel function K_2(x) from its integral representation
 * K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt, evaluated in the scaled form
 * e^x K_2(x) = int_0^inf exp(-x (cosh t - 1)) cosh(2 t) dt so that cold plasma (large x, where
 * K_2 itself leaves the double range near x = 700) keeps its value.  Trapezoid rule with step
 * h = 1/32, shrunk like x^-1/2 above x = 100 where the integrand's peak at t = 0 narrows like
 * x^-1/2: the error of the trapezoid rule for this entire, doubly-exponentially decaying
 * integrand, about exp(-2 pi^2 / (x h^2)), then stays below exp(-200) for every x. */
double orc_bessel_k2_scaled(double x)
{
    double h = 1.0 / 32.0;
    if (x > 100.0) h /= sqrt(x / 100.0);
    double sum = 0.5;
    for (int n = 1; n < 10000000; ++n) {
        double t = n * h;
        double term = exp(-x * (cosh(t) - 1.0)) * cosh(2.0 * t);
        sum += term;
        if (term < 1e-20 * sum) break;
    }
    return h * sum;
}

double orc_bessel_k2(double x) { return exp(-x) * orc_bessel_k2_scaled(x); }

/* ln K_2(x), finite wherever the scaled integral is. */
double orc_ln_bessel_k2(double x) { return log(orc_bessel_k2_scaled(x)) - x; }

/* Planck function, Sec. 4.2.2: B_nu = (2 h nu^3 / c^2) / (exp(h nu / (m_e c^2 Theta_e)) - 1). */
double orc_planck(double nu, double thetae)
{
    return 2.0 * O_H * nu * nu * nu / (O_C * O_C) / expm1(O_H * nu / (O_ME * O_C * O_C * thetae));
}

/* Thermal synchrotron closure, Sec. 4.2.2: the Leung et al. fit for j_nu with
 * nu_s = (2/9)(e B / 2 pi m_e c) Theta_e^2 sin(theta), X = nu / nu_s, and Kirchhoff's law
 * alpha_nu = j_nu / B_nu.  K2 is exact (mode EXACT) or the paper's 2 Theta_e^2 (K2_PAPER).
 * CONST returns the given constants (test closure).  Fluid-frame quantities, CGS. */
void orc_closure(int mode, double nu, double ne, double thetae, double bfield, double cos_b,
                 double const_j, double const_alpha, double* j, double* alpha)
{
    if (mode == ORC_CLOSURE_CONST) { *j = const_j; *alpha = const_alpha; return; }
    double s2 = 1.0 - cos_b * cos_b;
    double sinb = s2 > 0.0 ? sqrt(s2) : 0.0;
    if (!(ne > 0.0 && thetae > 0.0 && bfield > 0.0 && sinb > 0.0)) { *j = 0.0; *alpha = 0.0; return; }
    double nu_c = O_E * bfield / (2.0 * M_PI * O_ME * O_C);
    double nu_s = (2.0 / 9.0) * nu_c * thetae * thetae * sinb;
    double X = nu / nu_s;
    /* 1/K2 and the cut-off exp(-X^1/3) are applied as one exponential: each alone can leave the
     * double range for cold plasma (Theta_e below ~0.0014) where their product does not */
    double ln_k2 = (mode == ORC_CLOSURE_K2_PAPER) ? log(2.0 * thetae * thetae) : orc_ln_bessel_k2(1.0 / thetae);
    double shape = sqrt(X) + pow(2.0, 11.0 / 12.0) * pow(X, 1.0 / 6.0);
    double jv = sqrt(2.0) * M_PI * O_E * O_E * ne * nu_s / (3.0 * O_C) * shape * shape * exp(-cbrt(X) - ln_k2);
    *j = jv;
    *alpha = jv / orc_planck(nu, thetae);
}

/* ===================================================================================== */
/* Transfer                                                                              */
/* ===================================================================================== */

double orc_length_unit(double mass_msun) { return O_G * mass_msun * O_MSUN / (O_C * O_C); }

/* One ray, camera to plasma, Sec. 3 (backward scheme) with the geodesic of Sec. 2.
 * Reading of the discretisation (the paper does not print it): after each accepted step
 * that does not terminate the ray, the plasma is sampled at the new point and the step
 * contributes, for every frequency,
 *     ds = nu_r |dlambda| L,  dtau = alpha ds,
 *     I += exp(-tau) (j/alpha) (1 - exp(-dtau)) / nu_r^3   (j ds / nu_r^3 exp(-tau) if alpha = 0),
 *     tau += dtau,
 * i.e. the formal solution with coefficients constant over the step (Sec. 3.1, second
 * formal-solution equation), attenuated by the optical depth already between the point and
 * the camera (backward-transfer equation), and converted to observed intensity with the
 * invariant I/nu^3 (Sec. 3.1).
 *
 * Optical-depth-aware step (Sec. 3.1, backward scheme: a step for the geodesic and one for the
 * transfer, the smaller taken; the paper gives no rule for the transfer step).  Reading: with
 * tau_step > 0 the transfer step is the affine step over which the absorption of the last
 * sample, at the most absorbing traced frequency, gives an optical depth of tau_step,
 * tau_step / max_f(alpha_f nu_r L); before the first sample, and after a step that took no
 * sample or one without absorption, there is no transfer limit.  The optional cut-off
 * (tau_cutoff) is applied as described below. */
int orc_trace_ray(const orc_camera* cam, const orc_grid* grid, const orc_opts* o,
                  double alpha, double beta, const double* nu, int n_nu, double* Iout,
                  orc_ray_info* info, orc_step_rec* rec, int rec_cap)
{
    if (n_nu < 1 || n_nu > ORC_MAX_NU) return -1;
    double M = o->metric_mass, a = cam->spin;
    double rh = M + sqrt(M * M - a * a);
    double r_stop = o->r_stop_factor * rh;
    double Lu = orc_length_unit(o->mass_msun);
    double y[8], yn[8], acc[4];
    int have_acc = 0;
    orc_camera_ray(cam, M, alpha, beta, cam->t_frame + cam->r_cam, y, NULL);
    double tau[ORC_MAX_NU];
    for (int f = 0; f < n_nu; ++f) { Iout[f] = 0.0; tau[f] = 0.0; }
    int steps = 0, samples = 0, poles = 0, status = ORC_RUNNING;
    double rt_rate = 0.0;   /* d tau / d|lambda| at the last sample, most absorbing frequency */
    while (status == ORC_RUNNING) {
        double h = orc_step_size(o->eps, y, y + 4);
        if (o->tau_step > 0.0 && rt_rate > 0.0) h = fmin(h, o->tau_step / rt_rate);
        double dl = -h;
        rt_rate = 0.0;
        geo_step(a, M, o->integrator, y, acc, &have_acc, dl, yn);
        memcpy(y, yn, sizeof y);
        ++steps;
        if (!state_finite(y)) { status = ORC_NUMERIC; break; }
        if (reflect_pole(y)) { ++poles; have_acc = 0; }
        status = termination(y, steps, o->max_steps, r_stop, cam->r_cam);
        orc_step_rec* rr = (rec && steps <= rec_cap) ? &rec[steps - 1] : NULL;
        if (rr) {
            memcpy(rr->x, y, 4 * sizeof(double));
            memcpy(rr->k, y + 4, 4 * sizeof(double));
            rr->dl = dl; rr->sampled = 0; rr->nu_r = rr->j = rr->alpha = rr->ds = 0.0;
        }
        if (status != ORC_RUNNING) break;
        double fl[4];
        if (!orc_grid_sample(grid, o->slow_light, cam->t_frame, y[1], y[2], y[3], y[0], fl)) continue;
        if (grid->units == 1) {
            double prim[4] = {fl[0], fl[1], fl[2], fl[3]};
            orc_code_to_cgs(grid, o->mass_msun, prim, fl);
        }
        double u[4], b[4], nr, cb;
        orc_fluid_frame(a, M, y, y + 4, fl[3], u, b, &nr, &cb);
        ++samples;
        /* reading: a sample whose fluid-frame frequency is not positive -- possible only through
         * integration error, for the low-order integrators in the last step before the horizon --
         * has no defined emission or absorption and adds nothing */
        if (!(nr > 0.0)) continue;
        double ds = nr * fabs(dl) * Lu;
        for (int f = 0; f < n_nu; ++f) {
            double jv, av;
            orc_closure(o->closure, nu[f] * nr, fl[0], fl[1], fl[2], cb, o->const_j, o->const_alpha, &jv, &av);
            double dtau = av * ds;
            double add = (dtau > 0.0) ? exp(-tau[f]) * (jv / av) * (-expm1(-dtau)) / (nr * nr * nr)
                                      : exp(-tau[f]) * jv * ds / (nr * nr * nr);
            Iout[f] += add;
            tau[f] += dtau;
            rt_rate = fmax(rt_rate, av * nr * Lu);
            if (rr && f == 0) { rr->sampled = 1; rr->nu_r = nr; rr->j = jv; rr->alpha = av; rr->ds = ds; }
        }
        /* optical-depth cut-off (Sec. 3.1, backward scheme): once the material between the
         * point and the camera is opaque at every frequency, emission from further along the
         * ray reaches the camera attenuated by at least exp(-tau_cutoff) and the ray stops */
        if (o->tau_cutoff > 0.0) {
            double tmin = tau[0];
            for (int f = 1; f < n_nu; ++f) tmin = fmin(tmin, tau[f]);
            if (tmin >= o->tau_cutoff) { status = ORC_OPAQUE; break; }
        }
    }
    if (status == ORC_NUMERIC)
        for (int f = 0; f < n_nu; ++f) Iout[f] = 0.0;
    if (info) { info->status = status; info->steps = steps; info->samples = samples; info->poles = poles; }
    return 0;
}

int orc_trace_pixels(const orc_camera* cam, const orc_grid* grid, const orc_opts* o,
                      const double* nu, int n_nu, const int64_t* pix, int64_t n_pix,
                      double* Iout, orc_ray_info* info, int n_threads)
{
    if (n_nu < 1 || n_nu > ORC_MAX_NU) return -1;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(n_threads)
#endif
    for (int64_t p = 0; p < n_pix; ++p) {
        int i = (int)(pix[p] % cam->nx), j = (int)(pix[p] / cam->nx);
        double al, be;
        orc_pixel_alpha_beta(cam, i, j, &al, &be);
        orc_trace_ray(cam, grid, o, al, be, nu, n_nu, Iout + p * n_nu, info ? &info[p] : NULL, NULL, 0);
    }
    return 0;
}

/* Solid angle of one pixel seen from distance D: (2F/nx)(2F/ny) L^2 / D^2 (Sec. 4.2.2, flux
 * density as the sum of I over the image). */
double orc_pixel_solid_angle(const orc_camera* cam, const orc_opts* o)
{
    double Lu = orc_length_unit(o->mass_msun), D = o->dist_pc * O_PC;
    return (2.0 * cam->fov_half / cam->nx) * (2.0 * cam->fov_half / cam->ny) * Lu * Lu / (D * D);
}

/* Forward (plasma -> camera) recursion over a recorded path, Sec. 3.1: the formal solution
 * applied step by step from the far end, I_n = I_{n+1} exp(-dtau_n) + S_n (1 - exp(-dtau_n))
 * in observed units.  Used only to cross-check the backward sum. */
double orc_forward_transfer(const orc_step_rec* rec, int n)
{
    double Iv = 0.0;
    for (int m = n - 1; m >= 0; --m) {
        if (!rec[m].sampled) continue;
        double nr = rec[m].nu_r, dtau = rec[m].alpha * rec[m].ds;
        double src = (dtau > 0.0) ? (rec[m].j / rec[m].alpha) * (-expm1(-dtau)) / (nr * nr * nr)
                                  : rec[m].j * rec[m].ds / (nr * nr * nr);
        Iv = Iv * exp(-dtau) + src;
    }
    return Iv;
}

/* ===================================================================================== */
/* MLP surrogate of the closure: 3 -> 64 -> 64 -> 64 -> 64 -> 2, SiLU on hidden layers.    */
/* Parameter layout: for each layer l, W_l [out][in] row-major then b_l [out].            */
/* ===================================================================================== */

static const int mlp_dims[6] = {3, 64, 64, 64, 64, 2};

int orc_mlp_param_count(void)
{
    int n = 0;
    for (int l = 0; l < 5; ++l) n += mlp_dims[l + 1] * mlp_dims[l] + mlp_dims[l + 1];
    return n;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double silu_d(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* forward of one row, keeping pre-activations z[l][*] and activations h[l][*] */
static void mlp_row(const double* p, const double* x, double z[5][64], double h[6][64])
{
    for (int i = 0; i < 3; ++i) h[0][i] = x[i];
    const double* q = p;
    for (int l = 0; l < 5; ++l) {
        int ni = mlp_dims[l], no = mlp_dims[l + 1];
        const double* W = q;
        const double* b = q + no * ni;
        for (int o = 0; o < no; ++o) {
            double s = b[o];
            for (int i = 0; i < ni; ++i) s += W[o * ni + i] * h[l][i];
            z[l][o] = s;
            h[l + 1][o] = (l < 4) ? silu(s) : s;
        }
        q += no * ni + no;
    }
}

void orc_mlp_forward(const double* params, const double* x, int64_t n, double* y)
{
    for (int64_t r = 0; r < n; ++r) {
        double z[5][64], h[6][64];
        mlp_row(params, x + 3 * r, z, h);
        y[2 * r] = h[5][0];
        y[2 * r + 1] = h[5][1];
    }
}

/* Gradient of sum_r sum_o dy[r][o] * y[r][o] with respect to the parameters. */
void orc_mlp_backward(const double* params, const double* x, const double* dy, int64_t n,
                      double* dparams)
{
    int np = orc_mlp_param_count();
    int off[5], o = 0;
    for (int l = 0; l < 5; ++l) { off[l] = o; o += mlp_dims[l + 1] * mlp_dims[l] + mlp_dims[l + 1]; }
    memset(dparams, 0, (size_t)np * sizeof(double));
    for (int64_t r = 0; r < n; ++r) {
        double z[5][64], h[6][64], g[64], gp[64];
        mlp_row(params, x + 3 * r, z, h);
        g[0] = dy[2 * r];
        g[1] = dy[2 * r + 1];
        for (int l = 4; l >= 0; --l) {
            int ni = mlp_dims[l], no = mlp_dims[l + 1];
            const double* W = params + off[l];
            double* dW = dparams + off[l];
            double* db = dW + no * ni;
            /* g holds dL/dz_l (for l = 4, z = output) */
            for (int oo = 0; oo < no; ++oo) {
                db[oo] += g[oo];
                for (int i = 0; i < ni; ++i) dW[oo * ni + i] += g[oo] * h[l][i];
            }
            if (l == 0) break;
            for (int i = 0; i < ni; ++i) {
                double s = 0.0;
                for (int oo = 0; oo < no; ++oo) s += W[oo * ni + i] * g[oo];
                gp[i] = s * silu_d(z[l - 1][i]);
            }
            memcpy(g, gp, (size_t)ni * sizeof(double));
        }
    }
}
