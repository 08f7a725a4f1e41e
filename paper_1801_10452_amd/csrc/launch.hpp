// launch.hpp -- host-callable launchers of the kernels in trace.hip.
#pragma once
#include "device_types.hpp"

hipError_t launch_reset(unsigned int* tile_counter, unsigned long long* stats, hipStream_t st);
// max_nu: largest frequency count of any job (selects the register-array size)
// wpe: the instantiation compiled for at least wpe waves per SIMD (1, 2 or 3: register caps
// 512, 256, 168)
hipError_t launch_trace(const TraceParams& p, int max_nu, bool fp32, int wpe, int blocks, int threads,
                        hipStream_t st);
// flux in two deterministic passes through flux_partials(n_jobs, max_nu) partial sums
// (FLUX_SPLIT per job and frequency)
constexpr int FLUX_SPLIT = 16;
size_t flux_partials(int n_jobs, int max_nu);
hipError_t launch_flux(const DevJob* jobs, int n_jobs, const double* out, const double* pix_sr, double* part,
                       double* flux, int max_nu, hipStream_t st);
hipError_t trace_kernel_attributes(int max_nu, bool fp32, int wpe, bool mlpc, int integ, int* vgprs,
                                   int* spill_bytes, int* max_threads);
// mlpc: the variant with the learned closure; integ: INTEG_* (the second-order integrators have
// the 2- and 3-waves-per-SIMD variants; a request for 1 takes 2)
const void* trace_kernel_symbol(int max_nu, bool fp32, int wpe, bool mlpc = false, int integ = INTEG_RK4);
// dynamic LDS bytes of a trace-kernel work-group of `threads` lanes (mlpc: plus the staged network)
// Dynamic LDS bytes of a trace launch; the same (wpe, mlpc, integ) select the instantiation in
// trace_kernel_symbol, whose sample queue this sizes.
size_t trace_kernel_lds(int max_nu, bool fp32, int wpe, int threads, bool mlpc, int integ, int rays = 64);
// whether the instantiation keeps one queued sample per lane with the intensity in LDS (the
// variants that may run fewer than 64 rays per wave)
bool trace_kernel_one_slot(int max_nu, bool fp32, int wpe, bool mlpc, int integ);
// Waves-per-SIMD variant actually instantiated for a requested one.
int kernel_wpe(int wpe, bool mlpc, int integ);

// ---- thin disk (disk.hip)
hipError_t launch_disk(const DiskParams& p, int blocks, hipStream_t st);
hipError_t launch_disk_profile(const double* intensity, const double* redshift, long long n, int n_bins, double g_lo,
                               double g_hi, double dA, double* profile, hipStream_t st);

// ---- learned closure (mlp.hip)
namespace mlp {
struct Net;
}
hipError_t mlp_launch_gen(const K2Table& k2, unsigned long long seed, long long n, float* X, float* T, float* raw,
                          hipStream_t st);
hipError_t mlp_launch_exact(const K2Table& k2, long long n, const float* raw, float* out, hipStream_t st);
// mode 0: MSE gradient against T; mode 1: gradient of sum DY . y
hipError_t mlp_launch_train(const mlp::Net& net, const float* X, const float* T, const float* DY, long long base,
                            long long n, int mode, float inv_batch, float* partial, float* loss, int waves,
                            hipStream_t st);
// mode 0: Adam + repack; mode 1: summed gradient to grad_out; mode 2: repack only
hipError_t mlp_launch_reduce(const float* partial, int n_waves, int mode, float* P, float* m, float* v, float lr,
                             float b1, float b2, float eps, float wd, float bc1, float bc2, float* grad_out,
                             unsigned short* W, unsigned short* Wlo, unsigned short* WT, hipStream_t st);
hipError_t mlp_launch_forward(const mlp::Net& net, bool split, const float* X, long long n, float* Y, hipStream_t st);
hipError_t mlp_launch_forward_f32(const float* P, const float* X, long long n, float* Y, hipStream_t st);
hipError_t mlp_launch_backward_f32(const float* P, const float* X, const float* DY, long long n, float* G,
                                   hipStream_t st);

// ---- the no-allocation batch entry point (noalloc.hip)
// Device scratch of raptor_trace_batch_noalloc: a fixed array per GPU holding the tile counter,
// the statistics, the job, grid, frequency and solid-angle tables, the fluxes when the caller
// passes none, and the flux partial sums, each region aligned to 256 bytes, for at most
// NOALLOC_MAX_JOBS images of up to RAPTOR_MAX_NU frequencies.
constexpr int NOALLOC_MAX_JOBS = 256;
constexpr size_t noalloc_round(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t NOALLOC_SCRATCH_BYTES =
    noalloc_round(sizeof(unsigned int)) + noalloc_round(ST_COUNT * sizeof(unsigned long long)) +
    noalloc_round(NOALLOC_MAX_JOBS * sizeof(DevJob)) + noalloc_round(NOALLOC_MAX_JOBS * sizeof(DevGrid)) +
    2 * noalloc_round((size_t)NOALLOC_MAX_JOBS * 32 * sizeof(double)) + noalloc_round(NOALLOC_MAX_JOBS * sizeof(double)) +
    noalloc_round((size_t)NOALLOC_MAX_JOBS * 32 * FLUX_SPLIT * sizeof(double));
// Device address of this process's scratch array on `device` (which must be current): looked
// up once per device with hipGetSymbolAddress and kept.
hipError_t noalloc_scratch_address(int device, void** ptr);
