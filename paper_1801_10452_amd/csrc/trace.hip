// trace.hip -- the fused geodesic + radiative-transfer kernel and the flux reduction.
//
// One lane traces one ray (one camera pixel) backward from the camera: RK4 step of the null
// geodesic in Kerr-Schild coordinates (FP64, Sec. 2.2), termination tests, and at every
// accepted step inside the plasma the fluid sample, the fluid frame, the closure and the
// backward formal-solution update of every frequency (Sec. 3.1).  Waves are persistent: a
// wave takes 64-ray tiles (8 x 8 pixels) from a global counter shared by every image of the
// launch and hands their rays to its idle lanes as earlier rays finish, so lanes stay busy
// when rays end after very different numbers of steps.
#include "device_types.hpp"
#include "ks_geodesic.hpp"
#include "plasma.hpp"
#include "launch.hpp"

namespace {

__device__ inline int find_job(const DevJob* jobs, int n_jobs, long long tile)
{
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_base <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ inline unsigned lane_rank(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ inline unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Transfer arithmetic in precision TT (double or float); the closure inputs come in FP64.
template <class TT>
struct Transfer;

template <>
struct Transfer<double> {
    // per-sample, frequency-independent part
    double ne, the, bf, sinb, k2_inv, ds, inr3, nr;
    bool emits;
    __device__ inline void setup(const TraceParams& p, const double fl[4], double nr_, double cosb, double dsv)
    {
        ne = fl[0]; the = fl[1]; bf = fl[2];
        nr = nr_;
        ds = dsv;
        inr3 = 1.0 / (nr * nr * nr);
        const double s2 = 1.0 - cosb * cosb;
        sinb = s2 > 0.0 ? ::sqrt(s2) : 0.0;
        emits = (ne > 0.0 && the > 0.0 && bf > 0.0 && sinb > 0.0);
        k2_inv = 0.0;
        if (emits && p.closure != CL_CONST)
            k2_inv = (p.closure == CL_K2_PAPER) ? 1.0 / (2.0 * the * the) : ::exp(-pl::ln_k2(p.k2, ::log(the)));
    }
    __device__ inline void update(const TraceParams& p, double nu_obs, double& I, double& tau) const
    {
        double j, al, S;
        if (p.closure == CL_CONST) {
            j = p.const_j;
            al = p.const_alpha;
            S = al > 0.0 ? j / al : 0.0;
        } else if (emits) {
            pl::closure_exact(nu_obs * nr, ne, the, bf, sinb, k2_inv, &j, &al, &S);
        } else {
            return;
        }
        pl::transfer_update(j, al, S, ds, inr3, I, tau);
    }
};

template <>
struct Transfer<float> {
    float ne, the, nu_s, k2_inv, ds, inr3;
    double nr;
    bool emits;
    __device__ inline void setup(const TraceParams& p, const double fl[4], double nr_, double cosb, double dsv)
    {
        ne = (float)fl[0];
        the = (float)fl[1];
        nr = nr_;
        ds = (float)dsv;
        inr3 = (float)(1.0 / (nr_ * nr_ * nr_));
        const double s2 = 1.0 - cosb * cosb;
        const double sb = s2 > 0.0 ? ::sqrt(s2) : 0.0;
        emits = (fl[0] > 0.0 && fl[1] > 0.0 && fl[2] > 0.0 && sb > 0.0);
        nu_s = (float)((2.0 / 9.0) * pl::NUC_PER_GAUSS * fl[2] * fl[1] * fl[1] * sb);
        k2_inv = 0.0f;
        if (emits && p.closure != CL_CONST)
            k2_inv = (p.closure == CL_K2_PAPER) ? 1.0f / (2.0f * the * the)
                                               : ::expf(-(float)pl::ln_k2(p.k2, ::log(fl[1])));
    }
    __device__ inline void update(const TraceParams& p, double nu_obs, float& I, float& tau) const
    {
        float j, al, S;
        if (p.closure == CL_CONST) {
            j = (float)p.const_j;
            al = (float)p.const_alpha;
            S = al > 0.0f ? j / al : 0.0f;
        } else if (emits) {
            const float nuf = (float)(nu_obs * nr);
            const float X = nuf / nu_s;
            const float t = ::cbrtf(X);
            const float tc = t + 1.8877486253633868f;                 // 2^(11/12)
            j = 1.1396857174835936e-29f * ne * nu_s * k2_inv * t * tc * tc * ::expf(-t);
            const float q = nuf * 2.45215662654257e-16f;              // nu (2h/c^2)^(1/3)
            S = q * q * q / ::expm1f((float)pl::H_OVER_MEC2 * nuf / the);
            al = j / S;
        } else {
            return;
        }
        pl::transfer_update(j, al, S, ds, inr3, I, tau);
    }
};

template <int NNU, class TT>
__global__ void __launch_bounds__(256) trace_kernel(TraceParams p)
{
    const int lane = threadIdx.x & 63;
    const double M = p.M;

    double y[8];
    double a = 0.0, r_stop = 0.0, r_esc = 0.0, x2w = 0.5;
    int job = 0, steps = 0, pix = 0, n_nu = 0, nu_base = 0, grid = 0, fast_snap = 0;
    bool active = false;
    TT I[NNU], tau[NNU];
#pragma unroll
    for (int f = 0; f < NNU; ++f) { I[f] = TT(0); tau[f] = TT(0); }
#pragma unroll
    for (int i = 0; i < 8; ++i) y[i] = 0.0;

    unsigned long long c_rays = 0, c_steps = 0, c_samples = 0, c_hor = 0, c_esc = 0, c_max = 0, c_pole = 0,
                       c_num = 0, c_zamo = 0;

    long long next = 0, end = 0;   // rays of the current tile not yet handed out (wave-uniform)
    bool drained = false;

    while (true) {
        // ------------------------------------------------------------ refill idle lanes
        unsigned long long idle = __ballot(!active);
        int n_idle = __popcll(idle);
        if (n_idle >= p.refill_threshold || n_idle == 64) {
            while (n_idle > 0) {
                if (next == end) {
                    if (drained) break;
                    unsigned t = 0;
                    if (lane == 0) t = atomicAdd(p.tile_counter, 1u);
                    t = __shfl(t, 0, 64);
                    if ((long long)t >= p.n_tiles) {
                        drained = true;
                        break;
                    }
                    next = (long long)t * 64;
                    end = next + 64;
                }
                const long long avail = end - next;
                const unsigned rank = lane_rank(idle);
                if (!active && (long long)rank < avail) {
                    const long long ray = next + rank;
                    const long long tile = ray >> 6;
                    const int slot = (int)(ray & 63);
                    job = find_job(p.jobs, p.n_jobs, tile);
                    const DevJob& J = p.jobs[job];
                    const long long lt = tile - J.tile_base;
                    const int px = (int)(lt % J.tiles_x) * 8 + (slot & 7);
                    const int py = (int)(lt / J.tiles_x) * 8 + (slot >> 3);
                    if (px < J.nx && py < J.ny) {
                        const double alpha = -J.fov + (px + 0.5) * J.dalpha;
                        const double beta = -J.fov + (py + 0.5) * J.dbeta;
                        a = J.a;
                        const rk::Spin<double> sp = rk::make_spin(a, M);
                        rk::camera_ray(sp, J.r_cam, J.incl, J.sin_i, J.cos_i, alpha, beta, J.t_init, y);
                        r_stop = J.r_stop;
                        r_esc = J.r_cam;
                        x2w = y[2] * M_1_PI;
                        pix = py * J.nx + px;
                        n_nu = J.n_nu;
                        nu_base = J.nu_base;
                        grid = J.grid;
                        fast_snap = J.fast_snap;
                        steps = 0;
#pragma unroll
                        for (int f = 0; f < NNU; ++f) { I[f] = TT(0); tau[f] = TT(0); }
                        active = true;
                    }
                }
                next += (avail < n_idle) ? avail : n_idle;
                idle = __ballot(!active);
                n_idle = __popcll(idle);
            }
        }
        if (__ballot(active) == 0ull) break;   // every lane idle: the queue is drained

        // ------------------------------------------------------------ one step of every active ray
        if (active) {
            const rk::Spin<double> sp = rk::make_spin(a, M);
            const double dl = -rk::step_size(p.eps, y);
            rk::rk4_step(sp, y, dl);
            ++steps;
            int status = RAY_RUNNING;
            bool fin = true;
#pragma unroll
            for (int i = 0; i < 8; ++i) fin = fin && ::isfinite(y[i]);
            if (!fin) {
                status = RAY_NUMERIC;
            } else {
                c_pole += rk::reflect_pole(y);
                if (y[1] < r_stop)
                    status = RAY_HORIZON;
                else if (y[1] > r_esc)
                    status = RAY_ESCAPED;
                else if (steps >= p.max_steps)
                    status = RAY_MAXSTEP;
            }
            if (status == RAY_RUNNING) {
                const DevGrid& G = p.grids[grid];
                double fl[4];
                if (pl::sample_fluid(G, p.slow_light, fast_snap, y, &x2w, fl)) {
                    ++c_samples;
                    double nr, cb;
                    c_zamo += pl::fluid_frame(a, a * a, M, y, fl[3], &nr, &cb);
                    Transfer<TT> tr;
                    tr.setup(p, fl, nr, cb, nr * ::fabs(dl) * p.length_unit);
#pragma unroll
                    for (int f = 0; f < NNU; ++f)
                        if (f < n_nu) tr.update(p, p.nu[nu_base + f], I[f], tau[f]);
                }
            } else {
                const DevJob& J = p.jobs[job];
                const long long npix = (long long)J.nx * J.ny;
                double* o = p.out + J.out_base + pix;
#pragma unroll
                for (int f = 0; f < NNU; ++f)
                    if (f < n_nu) o[f * npix] = (status == RAY_NUMERIC) ? 0.0 : (double)I[f];
                if (p.ray_status) p.ray_status[J.pix_base + pix] = status;
                if (p.ray_steps) p.ray_steps[J.pix_base + pix] = steps;
                c_rays += 1;
                c_steps += steps;
                c_hor += status == RAY_HORIZON;
                c_esc += status == RAY_ESCAPED;
                c_max += status == RAY_MAXSTEP;
                c_num += status == RAY_NUMERIC;
                active = false;
            }
        }
    }

    // ------------------------------------------------------------ statistics, one atomic per counter per wave
    const unsigned long long s[ST_COUNT] = {wave_sum(c_rays), wave_sum(c_steps), wave_sum(c_samples), wave_sum(c_hor),
                                            wave_sum(c_esc), wave_sum(c_max), wave_sum(c_pole), wave_sum(c_num),
                                            0ull, wave_sum(c_zamo)};
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < ST_COUNT; ++i)
            if (s[i]) atomicAdd(p.stats + i, s[i]);
    }
}

// Flux density per (job, frequency): sum of the job's image times the pixel solid angle and
// 1e23 (erg/s/cm^2/Hz -> Jy).  One block per (job, frequency); every thread sums a fixed
// strided subset in order and the block combines the partial sums in a fixed tree, so the
// result does not depend on scheduling.
__global__ void __launch_bounds__(256) flux_kernel(const DevJob* jobs, const double* out, const double* pix_sr,
                                                   double* flux, int max_nu)
{
    const int job = blockIdx.x / max_nu, f = blockIdx.x % max_nu;
    const DevJob& J = jobs[job];
    __shared__ double part[256];
    double s = 0.0;
    if (f < J.n_nu) {
        const long long npix = (long long)J.nx * J.ny;
        const double* img = out + J.out_base + f * npix;
        for (long long i = threadIdx.x; i < npix; i += blockDim.x) s += img[i];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && f < J.n_nu) flux[job * max_nu + f] = part[0] * pix_sr[job] * 1e23;
}

__global__ void reset_kernel(unsigned int* tile_counter, unsigned long long* stats)
{
    if (threadIdx.x == 0) *tile_counter = 0u;
    if (threadIdx.x < ST_COUNT) stats[threadIdx.x] = 0ull;
}

template <int NNU, class TT>
hipError_t launch_nnu(const TraceParams& p, int blocks, int threads, hipStream_t st)
{
    hipLaunchKernelGGL((trace_kernel<NNU, TT>), dim3(blocks), dim3(threads), 0, st, p);
    return hipGetLastError();
}

template <class TT>
hipError_t launch_tt(const TraceParams& p, int max_nu, int blocks, int threads, hipStream_t st)
{
    if (max_nu <= 1) return launch_nnu<1, TT>(p, blocks, threads, st);
    if (max_nu <= 4) return launch_nnu<4, TT>(p, blocks, threads, st);
    if (max_nu <= 8) return launch_nnu<8, TT>(p, blocks, threads, st);
    if (max_nu <= 16) return launch_nnu<16, TT>(p, blocks, threads, st);
    return launch_nnu<32, TT>(p, blocks, threads, st);
}

}  // namespace

hipError_t launch_reset(unsigned int* tile_counter, unsigned long long* stats, hipStream_t st)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, st, tile_counter, stats);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceParams& p, int max_nu, bool fp32, int blocks, int threads, hipStream_t st)
{
    return fp32 ? launch_tt<float>(p, max_nu, blocks, threads, st) : launch_tt<double>(p, max_nu, blocks, threads, st);
}

hipError_t launch_flux(const DevJob* jobs, int n_jobs, const double* out, const double* pix_sr, double* flux,
                       int max_nu, hipStream_t st)
{
    hipLaunchKernelGGL(flux_kernel, dim3(n_jobs * max_nu), dim3(256), 0, st, jobs, out, pix_sr, flux, max_nu);
    return hipGetLastError();
}

const void* trace_kernel_symbol(int max_nu, bool fp32)
{
    if (fp32)
        return max_nu <= 1 ? (const void*)trace_kernel<1, float> : max_nu <= 4 ? (const void*)trace_kernel<4, float>
             : max_nu <= 8 ? (const void*)trace_kernel<8, float> : max_nu <= 16 ? (const void*)trace_kernel<16, float>
             : (const void*)trace_kernel<32, float>;
    return max_nu <= 1 ? (const void*)trace_kernel<1, double> : max_nu <= 4 ? (const void*)trace_kernel<4, double>
         : max_nu <= 8 ? (const void*)trace_kernel<8, double> : max_nu <= 16 ? (const void*)trace_kernel<16, double>
         : (const void*)trace_kernel<32, double>;
}

hipError_t trace_kernel_attributes(int max_nu, bool fp32, int* vgprs, int* spill_bytes, int* max_threads)
{
    hipFuncAttributes at;
    const hipError_t e = hipFuncGetAttributes(&at, trace_kernel_symbol(max_nu, fp32));
    if (e != hipSuccess) return e;
    if (vgprs) *vgprs = at.numRegs;
    if (spill_bytes) *spill_bytes = (int)at.localSizeBytes;
    if (max_threads) *max_threads = at.maxThreadsPerBlock;
    return hipSuccess;
}
