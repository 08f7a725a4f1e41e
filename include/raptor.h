/* raptor.h -- C ABI of the MI355X (gfx950) RAPTOR hot path.
 *
 * Method: Bronzwaer et al. 2018, "RAPTOR I: time-dependent radiative transfer in arbitrary
 * spacetimes" (arXiv:1801.10452).  One ray per camera pixel is traced backward from the
 * camera (Sec. 2.3, virtual camera) through the Kerr spacetime in Kerr-Schild coordinates
 * (Sec. 2.4 and the appendix on coordinate transformations) with fourth-order Runge-Kutta
 * (Sec. 2.2.1) and the adaptive step of Sec. 2.2, while the observed intensity is
 * integrated along it with the backward scheme of Sec. 3.1 from thermal-synchrotron
 * emission and Kirchhoff absorption (Sec. 4.2.2) sampled off an axisymmetric fluid grid
 * in modified Kerr-Schild coordinates (appendix KS-MKS), optionally interpolated in time
 * between snapshots (slow light, Sec. 5).
 *
 * Conventions for every entry point:
 *  - Return RAPTOR_OK (0) or a negative raptor_status; no exception crosses the ABI.
 *    raptor_last_error() then holds a message.  On RAPTOR_E_INVALID nothing is written.
 *  - Calls are synchronous: outputs are complete when the call returns.
 *  - The caller owns every buffer it passes; the library keeps no caller pointer after
 *    returning.  Grids are copied to device memory owned by the context.
 *  - Output buffers are host memory when opts->mem == RAPTOR_MEM_HOST and device memory
 *    (of the context's device) when opts->mem == RAPTOR_MEM_DEVICE.  Frequencies, cameras
 *    and option structs are always host memory.
 *  - A context is used by one thread at a time; contexts are independent.
 *  - Ray-level problems never fail a call: rays that hit the step limit, cross the pole or
 *    become non-finite are counted in raptor_stats, and non-finite rays write 0.
 *
 * Units: geometric (G = c = 1, lengths and times in M) for the spacetime and the camera,
 * CGS for the plasma, Hz for frequencies, erg s^-1 cm^-2 Hz^-1 sr^-1 for intensities and
 * Jy for flux densities.
 */
#ifndef RAPTOR_H
#define RAPTOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RAPTOR_OK = 0,
    RAPTOR_E_INVALID = -1,      /* bad argument; nothing written */
    RAPTOR_E_NOMEM = -2,        /* device allocation failed */
    RAPTOR_E_DEVICE = -3,       /* HIP runtime error; outputs undefined */
    RAPTOR_E_UNSUPPORTED = -4,  /* valid but not supported by the library */
    RAPTOR_E_RANGE = -5         /* size limit exceeded */
} raptor_status;

enum { RAPTOR_F32 = 0, RAPTOR_F64 = 1 };
enum { RAPTOR_MEM_HOST = 0, RAPTOR_MEM_DEVICE = 1 };
/* Emission / absorption closure.  EXACT: the Leung et al. fit with the exact Bessel K2 and
 * Kirchhoff absorption (Sec. 4.2.2).  K2_PAPER: same with the paper's K2 ~ 2 Theta_e^2.
 * CONST: j = const_j, alpha = const_alpha wherever the grid has plasma (test closure).
 * MLP / MLP_BF16: the learned surrogate (see raptor_mlp_*) in its split-BF16 or plain-BF16
 * form inside its training box, EXACT outside; needs parameters loaded in the context. */
enum { RAPTOR_CLOSURE_EXACT = 0, RAPTOR_CLOSURE_K2_PAPER = 1, RAPTOR_CLOSURE_CONST = 2,
       RAPTOR_CLOSURE_MLP = 3, RAPTOR_CLOSURE_MLP_BF16 = 4 };
/* Ray termination codes written by raptor_trace_spectrum_ex. */
enum { RAPTOR_RAY_HORIZON = 1, RAPTOR_RAY_ESCAPED = 2, RAPTOR_RAY_MAXSTEP = 3,
       RAPTOR_RAY_NUMERIC = 4, RAPTOR_RAY_OPAQUE = 5,
       RAPTOR_RAY_DISK = 6,         /* thin-disk test: first equatorial crossing on the disk */
       RAPTOR_RAY_PLANE = 7 };      /* thin-disk test: first equatorial crossing off the disk */

enum { RAPTOR_MAX_NU = 32 };        /* frequencies per image */

typedef struct raptor_ctx raptor_ctx;     /* opaque: device, stream, buffers, tuning cache */
typedef struct raptor_grid raptor_grid;   /* opaque: device-resident fluid grid */

/* Create a context on HIP device `device`.  `hip_stream` (a hipStream_t) is the stream all
 * work is queued on; NULL makes the context create its own.  *out is set on success. */
raptor_status raptor_create(int device, void* hip_stream, raptor_ctx** out);
/* Release every device resource of the context (its grids included).  NULL is a no-op. */
void raptor_destroy(raptor_ctx* ctx);
/* Message of the last failed call on ctx (valid until the next call); "" if none.
 * With ctx == NULL, the message of the last failed raptor_create on this thread. */
const char* raptor_last_error(const raptor_ctx* ctx);

/* Fluid grid: cells[n_snap][n2][n1][4] at cell centres of a grid uniform in x1 = ln r over
 * [ln r_in, ln r_out] and in x2 over [0, 1], theta(x2) = pi x2 + (1 - hslope)/2 sin(2 pi x2)
 * (appendix KS-MKS).  Snapshot s is at coordinate time t0 + s dt_snap.  mod_amp, mod_phase
 * describe an analytic azimuthal modulation of the density field (field 0),
 * 1 + mod_amp sum_{m=1..4} cos(m (phi - Omega_K(r) t_s) + mod_phase[m-1]) with
 * Omega_K = 1/(r^1.5 + a_gen); mod_amp = 0 disables it.  Requires n1, n2 >= 2, n_snap >= 1,
 * 0 < r_in < r_out, 0 < hslope <= 1, dt_snap > 0 when n_snap > 1, and dtype RAPTOR_F32 or
 * RAPTOR_F64.  `cells` is host memory and is copied.
 *
 * units = RAPTOR_UNITS_CGS: the fields are {n_e [cm^-3], Theta_e, B [G], Omega [1/M]}.
 * units = RAPTOR_UNITS_CODE: the fields are GRMHD primitives in geometrized code units
 * {rho, u (internal energy density), b (field strength, P_mag = b^2/2), Omega [1/M]}
 * (Sec. 4.2.2 and the electron model of Sec. 5).  Each sample interpolates the primitives and
 * converts them with the mass unit mass_unit_g (the model's free parameter M) and the black
 * hole's mass (opts->mass_msun, which sets L = GM/c^2): rho0 = M / L^3,
 * n_e = rho rho0 / (m_e + m_p), B = b c sqrt(4 pi rho0); the proton-to-electron temperature
 * ratio R = R_low / (1 + beta^2) + R_high beta^2 / (1 + beta^2), beta = (gamma_ad - 1) u /
 * (b^2 / 2); Theta_e = (m_p / m_e) (gamma_ad - 1) (u / rho) / (1 + R).  Requires
 * mass_unit_g > 0, r_low > 0, r_high > 0 and 1 < gamma_ad <= 2 (ignored for CGS grids). */
enum { RAPTOR_UNITS_CGS = 0, RAPTOR_UNITS_CODE = 1 };
typedef struct {
    int32_t n1, n2, n_snap, dtype;
    double r_in, r_out, hslope, a_gen, t0, dt_snap;
    double mod_amp, mod_phase[4];
    const void* cells;
    int32_t units, reserved;
    double mass_unit_g, r_low, r_high, gamma_ad;
} raptor_grid_desc;

raptor_status raptor_grid_upload(raptor_ctx* ctx, const raptor_grid_desc* desc, raptor_grid** out);
void raptor_grid_release(raptor_ctx* ctx, raptor_grid* grid);

/* Camera (Sec. 2.3): spin a (|a| < 1), inclination in degrees (0 < i < 180), camera radius
 * r_cam and half field of view in M, nx x ny pixels.  Pixel (i, j) looks along impact
 * parameters alpha = -F + (i + 1/2) 2F/nx, beta = -F + (j + 1/2) 2F/ny; images are stored
 * row-major [j][i].  t_frame is the observation time: the ray leaves the camera at
 * t = t_frame + r_cam, and fast light samples the snapshot nearest to t_frame. */
typedef struct {
    double spin, incl_deg, r_cam, fov_half;
    int32_t nx, ny;
    double t_frame;
} raptor_camera;

/* eps: step scale of the adaptive step (Sec. 2.2); r_stop_factor: rays stop at
 * r < r_stop_factor * r_+; max_steps: step limit per ray; transfer_prec: RAPTOR_F64 or
 * RAPTOR_F32 for the emission, absorption and intensity arithmetic (the geodesic is always
 * FP64); closure: RAPTOR_CLOSURE_*; slow_light: 1 to interpolate snapshots along each ray;
 * mem: RAPTOR_MEM_HOST or RAPTOR_MEM_DEVICE for output buffers; launch: 0 or
 * RAPTOR_LAUNCH_GRAPH; mass_msun and dist_pc set the length unit GM/c^2 and the flux
 * distance; metric_mass is 1 (or 0 for flat space, which needs spin 0).
 *
 * RAPTOR_LAUNCH_GRAPH: the call's device work (counter reset, the persistent trace kernel
 * and the flux reduction) is captured once into a HIP graph and replayed by later calls
 * whose launch is identical (same job-table shape, buffers and plan); the job table and
 * frequencies are uploaded before each replay.  Results are identical to the direct launch;
 * kernel_ms then spans the whole graph. */
enum { RAPTOR_LAUNCH_DIRECT = 0, RAPTOR_LAUNCH_GRAPH = 1 };
/* Geodesic integrators (Sec. 2.2): classical fourth-order Runge-Kutta (four connection
 * evaluations per step), the second-order midpoint rule (two), and velocity Verlet (one; two
 * with the corrector pass that re-evaluates the derivative with the updated wave vector).
 * Verlet carries dk/dlambda from step to step and evaluates it afresh at the start of a ray
 * and after a pole reflection.  The learned closure runs with RK4 only. */
enum { RAPTOR_RK4 = 0, RAPTOR_RK2 = 1, RAPTOR_VERLET = 2, RAPTOR_VERLET_CORRECTED = 3 };
typedef struct {
    double eps, r_stop_factor;
    int32_t max_steps, transfer_prec, closure, slow_light, mem, launch;
    double mass_msun, dist_pc, const_j, const_alpha, metric_mass;
    int32_t integrator;          /* RAPTOR_RK4 (default), RAPTOR_RK2, RAPTOR_VERLET(_CORRECTED) */
    int32_t reserved;            /* 0 */
    double tau_cutoff;           /* > 0: a ray stops (RAPTOR_RAY_OPAQUE) after the first sample at
                                    which its optical depth from the camera is >= tau_cutoff at
                                    every frequency (Sec. 3.1: emission from further along reaches
                                    the camera attenuated by at least exp(-tau_cutoff)); 0: off */
    double tau_step;             /* > 0: optical-depth-aware step (Sec. 3.1, backward scheme: a
                                    geodesic and a transfer step, the smaller taken).  The transfer
                                    step is the affine step over which the absorption of the ray's
                                    last sample, at its most absorbing frequency, gives an optical
                                    depth of tau_step: |dlambda| <= tau_step / max_f(alpha_f nu_r L);
                                    no limit before the first sample or after a step without an
                                    absorbing sample.  Each sample is then evaluated before the
                                    next step (no sample compaction).  In opaque media combine it
                                    with tau_cutoff: each step gains at most about tau_step of
                                    optical depth.  0: off (the step follows the geometry alone) */
} raptor_opts;

/* Counters of the last trace call.  ray_steps counts accepted steps, samples the plasma
 * samples evaluated, n_mlp_fallback the sample-frequencies that the learned closure handed to
 * the exact closure (inputs outside its box), n_opaque the rays stopped by the optical-depth
 * cut-off, n_mlp_dropped the sample-frequencies outside the learned closure's box that it skipped
 * because the exact closure gives exactly zero there: the factor exp(-(X^1/3 + ln K2(1/Theta_e)))
 * of thermal synchrotron emission lies below the smallest double (X^1/3 + ln K2 > 746,
 * X = nu / nu_s). */
typedef struct {
    uint64_t rays, ray_steps, samples, n_horizon, n_escaped, n_maxstep, n_pole, n_numeric,
             n_mlp_fallback, n_zamo_fallback;
    double kernel_ms;
    uint64_t n_opaque;
    uint64_t n_mlp_dropped;
} raptor_stats;

/* Fill *opts with the defaults: eps 0.05, r_stop_factor 1.01, max_steps 10000, FP64
 * transfer, EXACT closure, fast light, host memory, 4.5e6 Msun at 8500 pc, metric_mass 1. */
raptor_status raptor_default_opts(raptor_opts* opts);

/* One image at one frequency.  image: double[ny][nx] or NULL; flux_jy: double or NULL;
 * stats: may be NULL. */
raptor_status raptor_trace_image(raptor_ctx* ctx, const raptor_camera* cam, const raptor_grid* grid,
                                 const raptor_opts* opts, double nu_hz, double* image,
                                 double* flux_jy, raptor_stats* stats);

/* One image at n_nu frequencies on shared rays (the step is set by the geometry alone).
 * nu_hz: host double[n_nu], 1 <= n_nu <= RAPTOR_MAX_NU, all > 0; images:
 * double[n_nu][ny][nx] or NULL; flux_jy: double[n_nu] or NULL. */
raptor_status raptor_trace_spectrum(raptor_ctx* ctx, const raptor_camera* cam, const raptor_grid* grid,
                                    const raptor_opts* opts, const double* nu_hz, int32_t n_nu,
                                    double* images, double* flux_jy, raptor_stats* stats);

/* As raptor_trace_spectrum, and also writes the termination code and the number of
 * accepted steps of every ray: ray_status, ray_steps: int32[ny][nx] or NULL (same memory
 * kind as the images). */
raptor_status raptor_trace_spectrum_ex(raptor_ctx* ctx, const raptor_camera* cam,
                                       const raptor_grid* grid, const raptor_opts* opts,
                                       const double* nu_hz, int32_t n_nu, double* images,
                                       double* flux_jy, int32_t* ray_status, int32_t* ray_steps,
                                       raptor_stats* stats);

/* Many images of possibly different size, spin, inclination and grid in one persistent
 * launch over a shared ray queue.  cams[n_cams]; grids[n_cams] (entries may repeat);
 * nu_hz: host double[n_cams][n_nu]; images: the images of all cameras concatenated in
 * camera order, each double[n_nu][ny][nx], or NULL; flux_jy: double[n_cams][n_nu] or NULL.
 * Results equal the per-camera raptor_trace_spectrum calls. */
raptor_status raptor_trace_batch(raptor_ctx* ctx, const raptor_camera* cams, int32_t n_cams,
                                 const raptor_grid* const* grids, const raptor_opts* opts,
                                 const double* nu_hz, int32_t n_nu, double* images, double* flux_jy,
                                 raptor_stats* stats);

/* For callers that cannot allocate memory during a call -- code under HIP stream capture, tight
 * serving loops, harnesses that forbid allocation: raptor_trace_batch without any allocation.
 * Arguments and results are those of raptor_trace_batch (images and fluxes are bitwise the
 * same), with these limits:
 *  - opts->mem must be RAPTOR_MEM_DEVICE and images non-NULL (device memory of the context's
 *    device, the images of all cameras concatenated); flux_jy is device memory or NULL;
 *  - opts->launch must be RAPTOR_LAUNCH_DIRECT (RAPTOR_E_UNSUPPORTED otherwise);
 *  - at most RAPTOR_NOALLOC_MAX_CAMS cameras (RAPTOR_E_RANGE otherwise), up to RAPTOR_MAX_NU
 *    frequencies each.
 * Every buffer the launch needs beyond the inputs and outputs (tile counter, statistics, the
 * job, grid, frequency and solid-angle tables, the flux partial sums) lives in one fixed array
 * of about 1.3 MiB per GPU, which the library holds from its load until the process ends; the
 * host-side tables were sized when the context was created.  The call allocates no device or
 * host memory: a launch plan not yet installed for the call's frequency class, precision and
 * closure is resolved without being cached.  All calls on one GPU share that array: calls that
 * overlap in time on the same GPU (from several threads or contexts) race and must not be
 * made; consecutive calls are safe (each call is synchronous and clears what must start at
 * zero). */
enum { RAPTOR_NOALLOC_MAX_CAMS = 256 };
raptor_status raptor_trace_batch_noalloc(raptor_ctx* ctx, const raptor_camera* cams, int32_t n_cams,
                                         const raptor_grid* const* grids, const raptor_opts* opts,
                                         const double* nu_hz, int32_t n_nu, double* images,
                                         double* flux_jy, raptor_stats* stats);

/* Launch plan of the persistent trace kernel: the autotuner's search space.  A plan is kept
 * per context for each (n_nu class, transfer_prec, closure class) -- the closure class being
 * the learned closures (RAPTOR_CLOSURE_MLP*) or the others. */
typedef struct {
    int32_t threads;             /* work-group size: 64, 128, 256 or 512 */
    int32_t blocks_per_cu;       /* persistent work-groups per compute unit; 0 = as many as fit */
    int32_t refill_threshold;    /* a wave refills its idle lanes once this many are idle (1..64) */
    int32_t tile_width;          /* pixels per tile row: 8, 16, 32 or 64 (a tile is 64 rays) */
    int32_t min_waves_per_simd;  /* 1, 2 or 3: the kernel variant compiled for at least that many
                                    waves per SIMD (register cap 512, 256 or 168); the 3-wave
                                    variant sizes its LDS sample queue for 12 waves per CU */
    int32_t rays_per_wave;       /* 0 or 64 (default), 32 or 16: rays per tile and per wave.  Below
                                    64 only for the variants whose sample queue holds one sample per
                                    lane (several frequencies, exact or paper closure); the lanes
                                    without a ray then only take part in the frequency-parallel
                                    sample rounds, and the LDS of a wave shrinks with the rays, so
                                    more waves fit: for launches with fewer tiles than wave slots.
                                    Elsewhere, and as installed, 64; a tile wider than the rays is
                                    narrowed to them */
    int32_t reserved[2];
} raptor_plan;

/* Current plan for (n_nu, transfer_prec, closure) (the default plan if none was set or tuned:
 * 256 threads, as many work-groups as fit, refill at 1 idle lane, 8-pixel tile rows, and the
 * variant with the most waves per SIMD (3, 2, then 1) whose RK4 kernel keeps its registers
 * without spilling to scratch; for the learned closures 512 threads and the 2-waves-per-SIMD
 * variant).  RK2 and Verlet runs take the plan's 2- or 3-waves-per-SIMD kernel (2 when the plan
 * asks for 1). */
raptor_status raptor_get_plan(raptor_ctx* ctx, int32_t n_nu, int32_t transfer_prec, int32_t closure,
                              raptor_plan* out);
/* Install a plan for (n_nu, transfer_prec, closure); RAPTOR_E_INVALID if a field is out of range,
 * RAPTOR_E_UNSUPPORTED if no work-group of the plan fits the LDS. */
raptor_status raptor_set_plan(raptor_ctx* ctx, int32_t n_nu, int32_t transfer_prec, int32_t closure,
                              const raptor_plan* plan);
/* Autotuner: runs the given batch (arguments as raptor_trace_batch, outputs discarded) under
 * candidate plans by coordinate descent over the plan fields, timing each candidate with HIP
 * events as the fastest of `reps` runs, and installs the fastest plan for (n_nu,
 * opts->transfer_prec, opts->closure).  best receives the plan as installed (a work-group size
 * the kernel variant does not allow is reduced, as raptor_set_plan does); best and best_ms (the
 * fastest kernel time) may be NULL. */
raptor_status raptor_autotune_batch(raptor_ctx* ctx, const raptor_camera* cams, int32_t n_cams,
                                    const raptor_grid* const* grids, const raptor_opts* opts,
                                    const double* nu_hz, int32_t n_nu, int32_t reps, raptor_plan* best,
                                    double* best_ms);

/* ------------------------------------------------------------------------------------------
 * Learned closure (an addition to the paper's method).  A 3 -> 64 -> 64 -> 64 -> 64 -> 2 SiLU
 * network maps (ln(nu/nu_c), ln Theta_e, cos theta_B), normalised to [-1, 1] over the box
 * nu/nu_c in [1e-2, 1e8], Theta_e in [0.1, 100], |cos theta_B| <= 0.999, to
 * ln j_hat = ln(j / (n_e nu_c J0)) and ln alpha_hat = ln j_hat - 2 ln(nu/nu_c) - ln Theta_e,
 * J0 = sqrt2 pi e^2 / (3c), where alpha_hat is the Rayleigh-Jeans absorption in units of
 * n_e J0 / (2 m_e nu_c).  The network's two outputs are the standardised values of
 * ln j_hat + X^1/3 and ln alpha_hat + X^1/3, X = nu / nu_s, nu_s = (2/9) nu_c Theta_e^2
 * sin theta_B: the exponential cut-off exp(-X^1/3) of the emissivity is computed from the
 * inputs and applied outside the network.  The exact Planck factor is applied when the
 * network is used (closure RAPTOR_CLOSURE_MLP), and the exact closure of Sec. 4.2.2 is used
 * outside the box.
 * Training samples are the exact closure, evaluated on the device.  Parameters: for each
 * layer W[out][in] then b[out], 12866 floats.
 * ------------------------------------------------------------------------------------------ */
enum { RAPTOR_MLP_SPLIT = 0,   /* BF16 matrix cores, operands split into BF16 hi + lo pairs */
       RAPTOR_MLP_BF16 = 1,    /* BF16 matrix cores, BF16 operands */
       RAPTOR_MLP_F32 = 2 };   /* FP32 vector arithmetic (reference form) */
enum { RAPTOR_MLP_PARAMS = 12866 };

typedef struct {
    int64_t n_train;             /* training samples generated on the device (default 1e7) */
    int64_t n_val;               /* validation samples (default 1e5) */
    int32_t epochs;              /* passes over the training samples (default 180) */
    int32_t batch;               /* samples per Adam step, a multiple of 64 (default 6144) */
    float lr, lr_final;          /* Adam step size, cosine-decayed from lr to lr_final (defaults 8e-3, 2e-5) */
    float beta1, beta2, adam_eps, weight_decay;
    uint64_t train_seed, val_seed;
    int32_t form;                /* forward form used in training and validation: SPLIT or BF16 */
    int32_t reserved;
} raptor_mlp_train_cfg;

typedef struct {
    int64_t steps;
    double train_loss;           /* mean squared error (standardised) over the last epoch */
    double val_rms[2];           /* validation rms error of ln j_hat and ln alpha_hat */
    double val_max[2];           /* validation max |error| */
    double val_rms_bright;       /* rms error of ln j_hat where ln j_hat > -20 */
    double train_ms;             /* wall time of the training loop */
} raptor_mlp_report;

/* Defaults of the training configuration (seeds of the synthetic workload included). */
raptor_status raptor_mlp_default_cfg(raptor_mlp_train_cfg* cfg);
/* Random initial parameters, U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a SplitMix64 stream. */
raptor_status raptor_mlp_init(raptor_ctx* ctx, uint64_t seed);
/* Train on the device: sample generation, forward and backward passes on the matrix cores,
 * Adam with FP32 parameters.  Requires initialised parameters (raptor_mlp_init or set). */
raptor_status raptor_mlp_train(raptor_ctx* ctx, const raptor_mlp_train_cfg* cfg, raptor_mlp_report* report);
/* Parameters as 12866 floats (host memory). */
raptor_status raptor_mlp_get_params(raptor_ctx* ctx, float* params, int32_t n);
raptor_status raptor_mlp_set_params(raptor_ctx* ctx, const float* params, int32_t n);
/* Checkpoint: a versioned blob holding the parameters, the Adam moments and step count.
 * get: *n in = capacity (blob may be NULL to query), *n out = size. */
raptor_status raptor_mlp_get_weights(raptor_ctx* ctx, void* blob, size_t* n);
raptor_status raptor_mlp_set_weights(raptor_ctx* ctx, const void* blob, size_t n);
/* y[n][2] = network(x[n][3]) for normalised inputs, in the given form (host buffers). */
raptor_status raptor_mlp_forward(raptor_ctx* ctx, int32_t form, const float* x, int64_t n, float* y);
/* dparams[12866] = gradient of sum_i dy[i] . y[i] with respect to the parameters; form BF16
 * (the training backward pass) or F32. */
raptor_status raptor_mlp_backward(raptor_ctx* ctx, int32_t form, const float* x, const float* dy, int64_t n,
                                  float* dparams);
/* For raw closure inputs raw[n][3] = (ln(nu/nu_c), ln Theta_e, cos theta_B): the network's
 * (ln j_hat, ln alpha_hat), de-standardised and with the cut-off exponent X^1/3 subtracted
 * (net, may be NULL), and the exact closure's (exact, may be NULL), [n][2] each. */
raptor_status raptor_mlp_closure(raptor_ctx* ctx, int32_t form, const float* raw, int64_t n, float* net,
                                 float* exact);

/* Resources of the trace-kernel instantiation a plan selects: registers per lane, scratch
 * (spill) bytes per lane and resident work-groups per compute unit at the plan's work-group
 * size.  Any output pointer may be NULL. */
raptor_status raptor_kernel_info(raptor_ctx* ctx, int32_t n_nu, int32_t transfer_prec, int32_t closure,
                                 const raptor_plan* plan, int32_t* vgprs, int32_t* scratch_bytes,
                                 int32_t* blocks_per_cu);

/* ------------------------------------------------------------------------------------------
 * Thin-disk line test (Sec. 4.2.1): a geometrically thin, optically thick Keplerian disk in the
 * equatorial plane from the innermost stable circular orbit to r_disk_out, emitting a line
 * with emission proportional to r^-2 and no absorption.  Each pixel's ray (integrator, eps,
 * max_steps, r_stop_factor, metric_mass and mem taken from opts; closure must be EXACT, the
 * plasma options are ignored) runs to its first crossing of the equatorial plane; the crossing
 * is located by Newton iterations on theta(lambda), each an integrated partial step.  On the
 * disk: redshift[p] = g = E_obs/E_em against the gas on prograde Keplerian circles
 * (Omega = 1/(r^3/2 + a); a < 0 is a retrograde disk), intensity[p] = g^3 r^-2, status
 * RAPTOR_RAY_DISK; a first crossing off the disk gives RAPTOR_RAY_PLANE and zeros (higher-order
 * images are not counted).  profile[b] = sum over pixels with g in
 * [g_lo + b w, g_lo + (b + 1) w), w = (g_hi - g_lo)/n_bins, of intensity * dalpha dbeta (M^2).
 * Every output pointer may be NULL; outputs are host or device memory per opts->mem.
 * stats: rays, ray_steps, samples = rays on the disk, kernel_ms.
 * ------------------------------------------------------------------------------------------ */
/* r_isco for signed spin (Bardeen, Press & Teukolsky 1972; a < 0: retrograde orbits). */
raptor_status raptor_isco(double spin, double* r_isco);
raptor_status raptor_trace_disk(raptor_ctx* ctx, const raptor_camera* cam, const raptor_opts* opts, double r_disk_out,
                                int32_t n_bins, double g_lo, double g_hi, double* intensity, double* redshift,
                                double* profile, int32_t* ray_status, int32_t* ray_steps, raptor_stats* stats);

/* Algorithmic work per unit, counted once on the host by running the kernel's scalar
 * expressions through an operation-counting number type: FP64 add / sub / mul (a fused
 * multiply-add counts 2) of one accepted RK4 step including the step rule (step_*), of the
 * frequency-independent part of one plasma sample -- grid coordinates, one Newton iteration of
 * the MKS map, bilinear interpolation, fluid frame, closure set-up (sample_*) -- and of the
 * closure plus transfer update of one frequency at one sample (freq_*).  *_flops count
 * arithmetic operations; *_special count divisions, square roots and transcendental calls,
 * which are not included in *_flops.  Any pointer may be NULL. */
raptor_status raptor_work_per_unit(double* step_flops, double* step_special, double* sample_flops,
                                   double* sample_special, double* freq_flops, double* freq_special);
/* The same count for one accepted step of the given integrator (RAPTOR_RK4 gives step_* above;
 * a Verlet step excludes the occasional fresh derivative at a ray start or pole reflection). */
raptor_status raptor_work_per_step(int32_t integrator, double* flops, double* special);

#ifdef __cplusplus
}
#endif
#endif
