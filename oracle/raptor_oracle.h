/* raptor_oracle.h -- plain CPU FP64 oracle of the RAPTOR hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or constant
 * with the GPU library; the two meet only in the seeded inputs handed to both.
 *
 * Geometrized units G = c = M = 1 for geometry, CGS for plasma quantities.
 * Status codes of a ray: 1 horizon, 2 escaped, 3 step limit, 4 non-finite state.
 */
#ifndef RAPTOR_ORACLE_H
#define RAPTOR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double spin, incl_deg, r_cam, fov_half;
    int32_t nx, ny;
    double t_frame;
} orc_camera;

typedef struct {
    int32_t n1, n2, n_snap, is_f64;
    double r_in, r_out, hslope, a_gen, t0, dt_snap;
    double mod_amp, mod_phase[4];
    const void* cells;               /* [n_snap][n2][n1][4] = {n_e, Theta_e, B, Omega} */
    /* units = 1: the cells hold GRMHD primitives {rho, u, b, Omega} in code units, converted at
     * each sample with the mass unit and the R_low / R_high electron model */
    int32_t units, reserved;
    double mass_unit_g, r_low, r_high, gamma_ad;
} orc_grid;

enum { ORC_CLOSURE_EXACT = 0, ORC_CLOSURE_K2_PAPER = 1, ORC_CLOSURE_CONST = 2 };
enum { ORC_RUNNING = 0, ORC_HORIZON = 1, ORC_ESCAPED = 2, ORC_MAXSTEP = 3, ORC_NUMERIC = 4, ORC_OPAQUE = 5,
       ORC_DISK = 6, ORC_PLANE = 7 };

/* integrators of the geodesic (Sec. 2.2): classical RK4, the second-order midpoint rule, and
 * velocity Verlet without and with the corrector pass */
enum { ORC_RK4 = 0, ORC_RK2 = 1, ORC_VERLET = 2, ORC_VERLET_CORR = 3 };

typedef struct {
    double eps, r_stop_factor;
    int32_t max_steps, closure, slow_light, integrator;
    double mass_msun, dist_pc, const_j, const_alpha, metric_mass;
    double tau_cutoff;               /* > 0: stop a ray once tau >= tau_cutoff at every frequency */
    double tau_step;                 /* > 0: optical-depth-aware step, at most tau_step of optical
                                        depth per step at the last sample's absorption */
} orc_opts;

typedef struct {
    int32_t status, steps, samples, poles;
} orc_ray_info;

/* one recorded step: state after the step, the step size and the sample (frequency 0) */
typedef struct {
    double x[4], k[4], dl;
    int32_t sampled, pad_;
    double nu_r, j, alpha, ds;       /* fluid-frame values of the sample */
} orc_step_rec;

/* spacetime ------------------------------------------------------------------------ */
void orc_ks_metric(double a, double M, double r, double th, double g[16]);
void orc_ks_metric_derivs(double a, double M, double r, double th, double g[16], double dg[64]);
void orc_bl_metric(double a, double M, double r, double th, double g[16]);
int  orc_invert4(const double m[16], double inv[16]);
void orc_christoffel(double a, double M, const double x[4], double gam[64]);
void orc_geodesic_rhs(double a, double M, const double y[8], double f[8]);
double orc_step_size(double eps, const double x[4], const double k[4]);
void orc_rk4_step(double a, double M, const double y[8], double dl, double yout[8]);
void orc_rk2_step(double a, double M, const double y[8], double dl, double yout[8]);
/* velocity Verlet; acc: dk/dlambda at y on entry, the last evaluated derivative on return */
void orc_verlet_step(double a, double M, const double y[8], double acc[4], double dl, int corrector,
                     double yout[8]);
/* integrate from y0 with the paper's step rule and the given integrator (ORC_RK4 ...); records
 * up to cap states (after each step) */
int  orc_integrate(double a, double M, const double y0[8], double eps, int max_steps,
                   double r_stop, double r_escape, int integrator, double* traj, double* dls, int cap,
                   orc_ray_info* info);

/* camera ----------------------------------------------------------------------------- */
void orc_pixel_alpha_beta(const orc_camera* cam, int i, int j, double* alpha, double* beta);
void orc_camera_ray(const orc_camera* cam, double M, double alpha, double beta,
                    double t_init, double y[8], double kcov_bl[4]);

/* grid --------------------------------------------------------------------------------- */
double orc_mks_x2(double hslope, double th, int* iters);
/* code-unit primitives {rho, u, b, Omega} -> {n_e, Theta_e, B, Omega} for a black hole of
 * mass_msun solar masses (Sec. 4.2.2 scaling, Sec. 5 temperature-ratio model) */
void orc_code_to_cgs(const orc_grid* g, double mass_msun, const double prim[4], double out[4]);
int  orc_grid_sample(const orc_grid* g, int slow_light, double t_frame, double r, double th,
                     double ph, double t, double out[4]);

/* fluid frame and closure -------------------------------------------------------------- */
int  orc_fluid_frame(double a, double M, const double x[4], const double k[4], double omega,
                     double u[4], double b[4], double* nu_r, double* cos_b);
double orc_bessel_k2(double x);
double orc_bessel_k2_scaled(double x);   /* e^x K_2(x) */
double orc_ln_bessel_k2(double x);      /* ln K_2(x) */
void orc_closure(int mode, double nu, double ne, double thetae, double bfield, double cos_b,
                 double const_j, double const_alpha, double* j, double* alpha);
double orc_planck(double nu, double thetae);

/* thin disk (Sec. 4.2.1) ------------------------------------------------------------------ */
/* radius of the innermost stable circular orbit for signed spin a (a < 0: retrograde disk) */
double orc_isco(double a);
/* One ray of the thin-disk test: integrate until the first crossing of the equatorial plane.
 * If it lands on the disk (r_isco <= r <= r_disk_out) the status is ORC_DISK, *g the ratio
 * E_obs/E_em against the Keplerian disk and *I = g^3 r^-2 (emission proportional to r^-2, no
 * absorption); a first crossing off the disk gives ORC_PLANE and I = 0 (higher-order images
 * are not counted), any other end the usual status and I = 0. */
void orc_trace_disk_ray(const orc_camera* cam, const orc_opts* o, double r_disk_out, double alpha, double beta,
                        double* g, double* r_cross, double* Iv, orc_ray_info* info);
/* every pixel of cam (OpenMP over pixels); g, I: [ny][nx]; info may be NULL */
void orc_trace_disk_image(const orc_camera* cam, const orc_opts* o, double r_disk_out, double* g, double* Iv,
                          orc_ray_info* info, int n_threads);
/* line profile: profile[b] = sum over pixels with g in bin b of I * dalpha dbeta (M^2) */
void orc_disk_profile(const orc_camera* cam, const double* g, const double* Iv, int n_bins, double g_lo,
                      double g_hi, double* profile);

/* transfer and products ---------------------------------------------------------------- */
/* Frequencies per ray: 1 <= n_nu <= ORC_MAX_NU; the tracing calls return -1 (and write
 * nothing) outside that range, 0 otherwise. */
enum { ORC_MAX_NU = 64 };
int  orc_trace_ray(const orc_camera* cam, const orc_grid* grid, const orc_opts* o,
                   double alpha, double beta, const double* nu, int n_nu, double* I,
                   orc_ray_info* info, orc_step_rec* rec, int rec_cap);
int  orc_trace_pixels(const orc_camera* cam, const orc_grid* grid, const orc_opts* o,
                      const double* nu, int n_nu, const int64_t* pix, int64_t n_pix,
                      double* I /* [n_pix][n_nu] */, orc_ray_info* info /* [n_pix] or NULL */,
                      int n_threads);
double orc_pixel_solid_angle(const orc_camera* cam, const orc_opts* o);
double orc_forward_transfer(const orc_step_rec* rec, int n);
double orc_length_unit(double mass_msun);

/* MLP closure (fp64 reference of the surrogate network) -------------------------------- */
int  orc_mlp_param_count(void);
void orc_mlp_forward(const double* params, const double* x /* [n][3] */, int64_t n,
                     double* y /* [n][2] */);
void orc_mlp_backward(const double* params, const double* x, const double* dy, int64_t n,
                      double* dparams);

#ifdef __cplusplus
}
#endif
#endif
