// disk.hip -- the thin-disk line test (Sec. 4.2.1) on the GPU: one lane per pixel integrates
// its ray with the chosen integrator until the first crossing of the equatorial plane, locates
// the crossing by Newton iterations on theta(lambda) (each an integrated partial step from the
// state before the crossing), and, if the crossing lies on the Keplerian disk between the ISCO
// and the outer radius, records the ratio g = E_obs/E_em and the observed intensity g^3 r^-2
// (emission proportional to r^-2, no absorption; higher-order images are not counted).  A
// second kernel bins the pixel fluxes by g into the line profile, one block per bin summing
// the pixels in a fixed order.
#include "device_types.hpp"
#include "ks_geodesic.hpp"
#include "plasma.hpp"
#include "launch.hpp"

namespace {

constexpr double HALF_PI = 1.5707963267948966;

template <int INTEG>
__device__ inline void disk_step(const rk::Spin<double>& sp, double* y, double* acc, bool& have_acc, double dl,
                                 bool corrector, double s0, double c0)
{
    if (INTEG == INTEG_RK2) {
        rk::rk2_step(sp, y, dl, s0, c0);
    } else if (INTEG == INTEG_VERLET) {
        if (!have_acc) rk::ks_accel(sp, y, s0, c0, acc);
        rk::verlet_step(sp, y, acc, dl, corrector, s0, c0);
        have_acc = true;
    } else {
        rk::rk4_step(sp, y, dl, s0, c0);
    }
}

template <int INTEG>
__global__ void __launch_bounds__(256) disk_kernel(DiskParams p)
{
    const long long n = (long long)p.nx * p.ny;
    const rk::Spin<double> sp = rk::make_spin(p.a, p.M);
    const bool corrector = p.integrator == INTEG_VERLET_CORR;
    unsigned long long c_steps = 0, c_disk = 0;
    for (long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x; pix < n;
         pix += (long long)gridDim.x * blockDim.x) {
        const int px = (int)(pix % p.nx), py = (int)(pix / p.nx);
        const double alpha = -p.fov + (px + 0.5) * p.dalpha;
        const double beta = -p.fov + (py + 0.5) * p.dbeta;
        double y[8], acc[4] = {0.0, 0.0, 0.0, 0.0};
        bool have_acc = false;
        rk::camera_ray(sp, p.r_cam, p.incl, p.sin_i, p.cos_i, alpha, beta, 0.0, y);
        double s, c;
        rt::sincos_small(y[2], &s, &c);
        int steps = 0, status = RAY_RUNNING;
        double g = 0.0, I = 0.0;
        while (status == RAY_RUNNING) {
            const double dl = -rk::step_size(p.eps, y);
            double y0[8], acc0[4];
#pragma unroll
            for (int i = 0; i < 8; ++i) y0[i] = y[i];
#pragma unroll
            for (int i = 0; i < 4; ++i) acc0[i] = acc[i];
            const bool had_acc = have_acc;
            const double s0 = s, c0 = c;
            disk_step<INTEG>(sp, y, acc, have_acc, dl, corrector, s0, c0);
            ++steps;
            bool fin = true;
#pragma unroll
            for (int i = 0; i < 8; ++i) fin = fin && ::isfinite(y[i]);
            if (!fin) {
                status = RAY_NUMERIC;
                break;
            }
            const double h0 = y0[2] - HALF_PI, h1 = y[2] - HALF_PI;
            if (h0 * h1 < 0.0) {
                // crossing: linear estimate of its affine parameter, then two Newton iterations
                double lam = dl * h0 / (h0 - h1);
                double yc[8];
                for (int it = 0; it < 3; ++it) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) yc[i] = y0[i];
                    double ac[4] = {acc0[0], acc0[1], acc0[2], acc0[3]};
                    bool hc = had_acc;
                    disk_step<INTEG>(sp, yc, ac, hc, lam, corrector, s0, c0);
                    if (it < 2) lam += (HALF_PI - yc[2]) / yc[6];
                }
                const double rc = yc[1];
                if (rc >= p.r_in && rc <= p.r_out) {
                    const double omega = 1.0 / (rc * ::sqrt(rc) + p.a);
                    double sc, cc, nr, cb;
                    rt::sincos_small(yc[2], &sc, &cc);
                    pl::fluid_frame(p.a, p.a * p.a, p.M, yc, sc, cc, omega, &nr, &cb);
                    g = 1.0 / nr;
                    I = g * g * g / (rc * rc);
                    status = RAY_DISK;
                } else {
                    status = RAY_PLANE;
                }
                break;
            }
            if (rk::reflect_pole(y)) have_acc = false;
            rt::sincos_small(y[2], &s, &c);
            if (y[1] < p.r_stop)
                status = RAY_HORIZON;
            else if (y[1] > p.r_cam)
                status = RAY_ESCAPED;
            else if (steps >= p.max_steps)
                status = RAY_MAXSTEP;
        }
        if (p.intensity) p.intensity[pix] = I;
        if (p.redshift) p.redshift[pix] = g;
        if (p.status) p.status[pix] = status;
        if (p.steps) p.steps[pix] = steps;
        c_steps += steps;
        c_disk += status == RAY_DISK;
    }
    // one atomic per wave and counter
    for (int off = 32; off > 0; off >>= 1) {
        c_steps += __shfl_down(c_steps, off, 64);
        c_disk += __shfl_down(c_disk, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(p.stats + 0, c_steps);
        atomicAdd(p.stats + 1, c_disk);
    }
}

// profile[b] = sum of intensity * dA over the pixels whose g falls in bin b; block b scans all
// pixels in a fixed strided order and reduces in a fixed tree.
__global__ void __launch_bounds__(256) disk_profile_kernel(const double* intensity, const double* redshift,
                                                           long long n, int n_bins, double g_lo, double g_hi,
                                                           double dA, double* profile)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    double s = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) {
        const double I = intensity[i];
        if (!(I > 0.0)) continue;
        const double q = (redshift[i] - g_lo) / (g_hi - g_lo) * n_bins;
        if (q >= 0.0 && q < (double)n_bins && (int)q == b) s += I * dA;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) profile[b] = red[0];
}

}  // namespace

hipError_t launch_disk(const DiskParams& p, int blocks, hipStream_t st)
{
    if (p.integrator == INTEG_RK2)
        hipLaunchKernelGGL(disk_kernel<INTEG_RK2>, dim3(blocks), dim3(256), 0, st, p);
    else if (p.integrator == INTEG_VERLET || p.integrator == INTEG_VERLET_CORR)
        hipLaunchKernelGGL(disk_kernel<INTEG_VERLET>, dim3(blocks), dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL(disk_kernel<INTEG_RK4>, dim3(blocks), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_disk_profile(const double* intensity, const double* redshift, long long n, int n_bins, double g_lo,
                               double g_hi, double dA, double* profile, hipStream_t st)
{
    hipLaunchKernelGGL(disk_profile_kernel, dim3(n_bins), dim3(256), 0, st, intensity, redshift, n, n_bins, g_lo,
                       g_hi, dA, profile);
    return hipGetLastError();
}
