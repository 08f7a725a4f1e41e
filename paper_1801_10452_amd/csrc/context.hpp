// context.hpp -- internal state of a raptor context (shared by the host translation units).
#pragma once
#include "raptor.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "device_types.hpp"

namespace rctx {

constexpr double kG = 6.67430e-8;
constexpr double kMsun = 1.98847e33;
constexpr double kPc = 3.085677581e18;
constexpr double kC = 2.99792458e10;
constexpr double kPi = 3.14159265358979323846;

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    hipError_t reserve(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(n, 1);
        hipError_t e = hipMalloc(&p, want * sizeof(T));
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// One image of a trace call as the caller gave it.
struct JobIn {
    const raptor_camera* cam;
    const raptor_grid* grid;
    const double* nu;
};

// Host tables of the no-allocation batch entry point, sized once for its largest batch when
// the context is created.
constexpr int NOALLOC_JOBS = 256;
struct NoAllocHost {
    JobIn in[NOALLOC_JOBS];
    DevJob jobs[NOALLOC_JOBS];
    DevGrid grids[NOALLOC_JOBS];
    const raptor_grid* gl[NOALLOC_JOBS];
    double nus[NOALLOC_JOBS * RAPTOR_MAX_NU];
    double pixsr[NOALLOC_JOBS];
};

struct LaunchPlan {
    raptor_plan p{256, 0, 1, 8, 2, 64, {0, 0}};
    int blocks = 0;   // resolved work-group count
};

// Learned closure: FP32 parameters with Adam moments, padded BF16 copies, training samples.
struct MlpState {
    bool ready = false;
    long long adam_step = 0;
    DevBuf<float> P, m, v;
    DevBuf<unsigned short> W, Wlo, WT;
    DevBuf<float> partial, loss;
    DevBuf<float> Xtr, Ttr, Xva, Tva, RAWva;
    long long n_train = 0, n_val = 0;
    unsigned long long train_seed = 0, val_seed = 0;
    void release()
    {
        P.release(); m.release(); v.release(); W.release(); Wlo.release(); WT.release();
        partial.release(); loss.release(); Xtr.release(); Ttr.release(); Xva.release(); Tva.release(); RAWva.release();
    }
};

}  // namespace rctx

struct raptor_grid {
    DevGrid d{};
    double mass_unit_g = 0.0;   // code-unit grids: the model's mass unit
    void* cells = nullptr;
    double2* x2tab = nullptr;
    raptor_ctx* owner = nullptr;
};

struct raptor_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cu_count = 0;
    size_t lds_per_block = 65536;
    std::string err;
    rctx::DevBuf<DevJob> jobs;
    rctx::DevBuf<DevGrid> grids;
    rctx::DevBuf<double> nu, out, pixsr, flux, flux_part;
    rctx::DevBuf<int> status, steps;
    rctx::DevBuf<unsigned int> counter;
    rctx::DevBuf<unsigned long long> stats;
    rctx::DevBuf<double4> k2;
    K2Table k2t{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // graph replay of the batch launch: a capture-only stream, the instantiated graph and the
    // launch it was captured for (compared bytewise)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    std::vector<unsigned char> graph_key;
    std::vector<raptor_grid*> live;
    std::map<int, rctx::LaunchPlan> plans;   // key: frequency-count class * 2 + fp32
    rctx::MlpState mlp;
    // no-allocation entry point: this device's scratch array (device address) and host tables
    void* noalloc_scratch = nullptr;
    rctx::NoAllocHost* noalloc_host = nullptr;
};

namespace rctx {
raptor_status fail(raptor_ctx* ctx, raptor_status s, const std::string& msg);
raptor_status dev_fail(raptor_ctx* ctx, hipError_t e, const char* what);
}  // namespace rctx

#define RAPTOR_CK(call, what)                                              \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return rctx::dev_fail(ctx, e_, what);        \
    } while (0)
