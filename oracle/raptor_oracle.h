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
} orc_grid;

enum { ORC_CLOSURE_EXACT = 0, ORC_CLOSURE_K2_PAPER = 1, ORC_CLOSURE_CONST = 2 };
enum { ORC_RUNNING = 0, ORC_HORIZON = 1, ORC_ESCAPED = 2, ORC_MAXSTEP = 3, ORC_NUMERIC = 4 };

typedef struct {
    double eps, r_stop_factor;
    int32_t max_steps, closure, slow_light, pad_;
    double mass_msun, dist_pc, const_j, const_alpha, metric_mass;
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
/* integrate from y0 with the paper's step rule; records up to cap states (after each step) */
int  orc_integrate(double a, double M, const double y0[8], double eps, int max_steps,
                   double r_stop, double r_escape, double* traj, double* dls, int cap,
                   orc_ray_info* info);

/* camera ----------------------------------------------------------------------------- */
void orc_pixel_alpha_beta(const orc_camera* cam, int i, int j, double* alpha, double* beta);
void orc_camera_ray(const orc_camera* cam, double M, double alpha, double beta,
                    double t_init, double y[8], double kcov_bl[4]);

/* grid --------------------------------------------------------------------------------- */
double orc_mks_x2(double hslope, double th, int* iters);
int  orc_grid_sample(const orc_grid* g, int slow_light, double t_frame, double r, double th,
                     double ph, double t, double out[4]);

/* fluid frame and closure -------------------------------------------------------------- */
int  orc_fluid_frame(double a, double M, const double x[4], const double k[4], double omega,
                     double u[4], double b[4], double* nu_r, double* cos_b);
double orc_bessel_k2(double x);
void orc_closure(int mode, double nu, double ne, double thetae, double bfield, double cos_b,
                 double const_j, double const_alpha, double* j, double* alpha);
double orc_planck(double nu, double thetae);

/* transfer and products ---------------------------------------------------------------- */
void orc_trace_ray(const orc_camera* cam, const orc_grid* grid, const orc_opts* o,
                   double alpha, double beta, const double* nu, int n_nu, double* I,
                   orc_ray_info* info, orc_step_rec* rec, int rec_cap);
void orc_trace_pixels(const orc_camera* cam, const orc_grid* grid, const orc_opts* o,
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
