// launch.hpp -- host-callable launchers of the kernels in trace.hip.
#pragma once
#include "device_types.hpp"

hipError_t launch_reset(unsigned int* tile_counter, unsigned long long* stats, hipStream_t st);
// max_nu: largest frequency count of any job (selects the register-array size)
// wpe: the instantiation compiled for at least wpe waves per SIMD (1, 2 or 3: register caps
// 512, 256, 168)
hipError_t launch_trace(const TraceParams& p, int max_nu, bool fp32, int wpe, int blocks, int threads,
                        hipStream_t st);
hipError_t launch_flux(const DevJob* jobs, int n_jobs, const double* out, const double* pix_sr, double* flux,
                       int max_nu, hipStream_t st);
hipError_t trace_kernel_attributes(int max_nu, bool fp32, int wpe, int* vgprs, int* spill_bytes, int* max_threads);
const void* trace_kernel_symbol(int max_nu, bool fp32, int wpe);
// dynamic LDS bytes of a trace-kernel work-group of `threads` lanes
size_t trace_kernel_lds(int max_nu, bool fp32, int threads);
