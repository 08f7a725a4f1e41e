// device_types.hpp -- plain structs shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

// Fluid grid resident in device memory, cells[n_snap][n2][n1] of float4 or double4
// {n_e, Theta_e, B, Omega}.
struct DevGrid {
    const void* cells;
    const double2* x2tab;      // {x2, dx2/dtheta * dtheta} at the x2n + 1 nodes theta = i pi / x2n
    int x2n, x2_refine;        // x2_refine: the table misses 1e-12 somewhere, refine by Halley's iteration
    double x2_inv_dth;         // x2n / pi
    int n1, n2, n_snap, is_f64;
    double lnr_in, inv_d1, r_in, r_out, hslope, a_gen, t0, dt_snap, inv_dt, mod_amp;
    double mod_cos[4], mod_sin[4];   // cos / sin of the modulation phases
    // GRMHD code units (units = 1): per-call scales (they depend on the black hole's mass) and
    // the electron model
    int units, pad2;
    double ne_scale;                 // rho0 / (m_e + m_p): n_e per unit code density
    double b_scale;                  // c sqrt(4 pi rho0): gauss per unit code field
    double r_low, r_high, gam1;      // temperature-ratio model, gamma_ad - 1
    double thetae_fac;               // (m_p / m_e) (gamma_ad - 1)
};

// One image of a launch.  Rays are numbered tile by tile (64 rays per tile, 8 x 8 pixels by
// default; the tile width is a launch-plan parameter);
// the job owns the global tiles [tile_base, tile_base + tiles_x * tiles_y).
struct DevJob {
    double a, incl, sin_i, cos_i, r_cam, fov, dalpha, dbeta, r_stop, t_init;
    long long tile_base;
    long long out_base;    // offset of this job's first image in the intensity buffer (doubles)
    long long pix_base;    // offset of this job's pixels in the per-ray info buffers
    int nx, ny, tiles_x, n_nu;
    int grid, nu_base, fast_snap, pad;
};

// ln K2(1/Theta) on octaves of Theta: Theta = m 2^e with m in [1/2, 1) (frexp), octave
// e = e_lo + o (o < n_oct) split into nsub intervals uniform in m.  Entry o nsub + j holds
// {f0, d0, f1, d1}: ln K2 at the interval's two ends and its derivatives with respect to the
// interval's own coordinate s in [0, 1] (cubic Hermite).  Outside [th_lo, th_hi] the lookup
// takes K2's large- and small-argument expansions instead.
struct K2Table {
    const double4* tab;
    int e_lo, n_oct, nsub, pad;
    double th_lo, th_hi;
};

enum : int {
    ST_RAYS = 0, ST_STEPS, ST_SAMPLES, ST_HORIZON, ST_ESCAPED, ST_MAXSTEP, ST_POLE, ST_NUMERIC,
    ST_MLP_FALLBACK, ST_ZAMO, ST_OPAQUE, ST_MLP_DROPPED, ST_COUNT
};

struct TraceParams {
    const DevJob* jobs;
    const DevGrid* grids;
    const double* nu;          // frequencies, per job at nu_base
    double* out;               // intensities [job image][n_nu][ny][nx]
    int* ray_status;           // optional, per pixel at pix_base
    int* ray_steps;            // optional
    unsigned int* tile_counter;
    unsigned long long* stats; // ST_COUNT counters
    K2Table k2;
    long long n_tiles;
    int n_jobs, max_steps, closure, slow_light, integrator, pad;
    int refill_threshold, tile_shift;   // tile width = 1 << tile_shift pixels, height rays / width
    // rays per tile and per wave (64, or 32 / 16 for the kernels whose sample queue holds one
    // sample per lane: the other lanes then only take part in the frequency-parallel rounds)
    int rays_per_wave, rays_shift;
    double eps, M, length_unit, const_j, const_alpha, tau_cutoff;
    double tau_step;           // > 0: optical-depth-aware step (at most tau_step per step at the last sample)
    // learned closure (closure == CL_MLP): FP32 parameters and padded BF16 hi / lo weights
    const float* mlp_P;
    const unsigned short* mlp_W;
    const unsigned short* mlp_Wlo;
};

// CL_MLP evaluates the network in split BF16 form, CL_MLP_BF16 in plain BF16 form
enum : int { CL_EXACT = 0, CL_K2_PAPER = 1, CL_CONST = 2, CL_MLP = 3, CL_MLP_BF16 = 4 };
enum : int { RAY_RUNNING = 0, RAY_HORIZON = 1, RAY_ESCAPED = 2, RAY_MAXSTEP = 3, RAY_NUMERIC = 4, RAY_OPAQUE = 5,
             RAY_DISK = 6, RAY_PLANE = 7 };
// geodesic integrators (INTEG_VERLET_CORR runs the Verlet kernel with the corrector pass)
enum : int { INTEG_RK4 = 0, INTEG_RK2 = 1, INTEG_VERLET = 2, INTEG_VERLET_CORR = 3 };

// Thin-disk test: one camera, Keplerian disk between r_in (the ISCO) and r_out.
struct DiskParams {
    double a, incl, sin_i, cos_i, r_cam, fov, dalpha, dbeta, r_stop, r_in, r_out, eps, M;
    int nx, ny, max_steps, integrator;
    double* intensity;            // [ny][nx] or null
    double* redshift;             // [ny][nx] or null
    int* status;                  // [ny][nx] or null
    int* steps;                   // [ny][nx] or null
    unsigned long long* stats;    // [0] ray-steps, [1] rays on the disk
};
