// mlp_host.cpp -- C ABI of the learned closure: parameters, checkpoints, training loop,
// evaluation entry points.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "context.hpp"
#include "launch.hpp"
#include "mlp_device.hpp"

using namespace rctx;

namespace {

constexpr int NP = mlp::N_PARAMS;

struct BlobHeader {
    char magic[8];          // "RAPTMLP"
    uint32_t version;       // 1
    uint32_t n_params;
    int64_t adam_step;
    float lx_lo, lx_hi, lt_lo, lt_hi, cb_lo, cb_hi, mu_j, sigma_j, mu_a, sigma_a;
};

unsigned long long splitmix_host(unsigned long long seed, unsigned long long n)
{
    unsigned long long z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

raptor_status alloc_params(raptor_ctx* ctx)
{
    MlpState& S = ctx->mlp;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    RAPTOR_CK(S.P.reserve(NP), "allocating MLP parameters");
    RAPTOR_CK(S.m.reserve(NP), "allocating MLP parameters");
    RAPTOR_CK(S.v.reserve(NP), "allocating MLP parameters");
    RAPTOR_CK(S.W.reserve(mlp::PW_TOTAL), "allocating MLP weights");
    RAPTOR_CK(S.Wlo.reserve(mlp::PW_TOTAL), "allocating MLP weights");
    RAPTOR_CK(S.WT.reserve(mlp::PW_TOTAL), "allocating MLP weights");
    RAPTOR_CK(hipMemsetAsync(S.W.p, 0, mlp::PW_TOTAL * 2, ctx->stream), "clearing MLP weights");
    RAPTOR_CK(hipMemsetAsync(S.Wlo.p, 0, mlp::PW_TOTAL * 2, ctx->stream), "clearing MLP weights");
    RAPTOR_CK(hipMemsetAsync(S.WT.p, 0, mlp::PW_TOTAL * 2, ctx->stream), "clearing MLP weights");
    return RAPTOR_OK;
}

// upload parameters (and optionally moments), rebuild the BF16 copies
raptor_status install(raptor_ctx* ctx, const float* P, const float* m, const float* v, long long step)
{
    raptor_status s = alloc_params(ctx);
    if (s != RAPTOR_OK) return s;
    MlpState& S = ctx->mlp;
    std::vector<float> zero(NP, 0.0f);
    RAPTOR_CK(hipMemcpyAsync(S.P.p, P, NP * 4, hipMemcpyHostToDevice, ctx->stream), "uploading parameters");
    RAPTOR_CK(hipMemcpyAsync(S.m.p, m ? m : zero.data(), NP * 4, hipMemcpyHostToDevice, ctx->stream), "uploading moments");
    RAPTOR_CK(hipMemcpyAsync(S.v.p, v ? v : zero.data(), NP * 4, hipMemcpyHostToDevice, ctx->stream), "uploading moments");
    RAPTOR_CK(mlp_launch_reduce(nullptr, 0, 2, S.P.p, S.m.p, S.v.p, 0, 0, 0, 0, 0, 1, 1, nullptr, S.W.p, S.Wlo.p,
                                S.WT.p, ctx->stream),
              "packing weights");
    RAPTOR_CK(hipStreamSynchronize(ctx->stream), "packing weights");
    S.adam_step = step;
    S.ready = true;
    return RAPTOR_OK;
}

mlp::Net net_of(const MlpState& S)
{
    mlp::Net n;
    n.P = S.P.p;
    n.W = S.W.p;
    n.Wlo = S.Wlo.p;
    n.WT = S.WT.p;
    return n;
}

raptor_status need_ready(raptor_ctx* ctx)
{
    if (!ctx->mlp.ready) return fail(ctx, RAPTOR_E_INVALID, "the MLP has no parameters (init, set or train first)");
    return RAPTOR_OK;
}

raptor_status ensure_samples(raptor_ctx* ctx, DevBuf<float>& X, DevBuf<float>& T, DevBuf<float>* RAW, long long n,
                             unsigned long long seed, long long* have_n, unsigned long long* have_seed)
{
    if (*have_n == n && *have_seed == seed && X.p) return RAPTOR_OK;
    RAPTOR_CK(X.reserve((size_t)3 * n), "allocating training samples");
    RAPTOR_CK(T.reserve((size_t)2 * n), "allocating training samples");
    float* raw = nullptr;
    if (RAW) {
        RAPTOR_CK(RAW->reserve((size_t)3 * n), "allocating validation samples");
        raw = RAW->p;
    }
    RAPTOR_CK(mlp_launch_gen(ctx->k2t, seed, n, X.p, T.p, raw, ctx->stream), "generating samples");
    *have_n = n;
    *have_seed = seed;
    return RAPTOR_OK;
}

bool form_ok(int f) { return f == RAPTOR_MLP_SPLIT || f == RAPTOR_MLP_BF16 || f == RAPTOR_MLP_F32; }

}  // namespace

extern "C" {

raptor_status raptor_mlp_default_cfg(raptor_mlp_train_cfg* c)
{
    if (!c) return RAPTOR_E_INVALID;
    std::memset(c, 0, sizeof *c);
    c->n_train = 10000000;
    c->n_val = 100000;
    c->epochs = 180;
    c->batch = 6144;
    c->lr = 8e-3f;
    c->lr_final = 2e-5f;
    c->beta1 = 0.9f;
    c->beta2 = 0.999f;
    c->adam_eps = 1e-8f;
    c->weight_decay = 0.0f;
    c->train_seed = 1801104520ull + 100ull;
    c->val_seed = 1801104520ull + 101ull;
    c->form = RAPTOR_MLP_SPLIT;
    return RAPTOR_OK;
}

raptor_status raptor_mlp_init(raptor_ctx* ctx, uint64_t seed)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    std::vector<float> P(NP);
    const int dims[6] = {3, 64, 64, 64, 64, 2};
    int off = 0;
    unsigned long long k = 0;
    for (int L = 0; L < 5; ++L) {
        const int ni = dims[L], no = dims[L + 1];
        const double bound = 1.0 / std::sqrt((double)ni);
        for (int i = 0; i < no * ni + no; ++i) {
            const double u = (double)(splitmix_host(seed, k++) >> 11) * (1.0 / 9007199254740992.0);
            P[off + i] = (float)((2.0 * u - 1.0) * bound);
        }
        off += no * ni + no;
    }
    return install(ctx, P.data(), nullptr, nullptr, 0);
}

raptor_status raptor_mlp_set_params(raptor_ctx* ctx, const float* params, int32_t n)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!params || n != NP) return fail(ctx, RAPTOR_E_INVALID, "params must hold RAPTOR_MLP_PARAMS floats");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return fail(ctx, RAPTOR_E_INVALID, "parameters must be finite");
    return install(ctx, params, nullptr, nullptr, 0);
}

raptor_status raptor_mlp_get_params(raptor_ctx* ctx, float* params, int32_t n)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!params || n != NP) return fail(ctx, RAPTOR_E_INVALID, "params must hold RAPTOR_MLP_PARAMS floats");
    raptor_status s = need_ready(ctx);
    if (s != RAPTOR_OK) return s;
    RAPTOR_CK(hipMemcpyAsync(params, ctx->mlp.P.p, NP * 4, hipMemcpyDeviceToHost, ctx->stream), "reading parameters");
    RAPTOR_CK(hipStreamSynchronize(ctx->stream), "reading parameters");
    return RAPTOR_OK;
}

raptor_status raptor_mlp_get_weights(raptor_ctx* ctx, void* blob, size_t* n)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!n) return fail(ctx, RAPTOR_E_INVALID, "n is NULL");
    const size_t need = sizeof(BlobHeader) + (size_t)3 * NP * sizeof(float);
    if (!blob) {
        *n = need;
        return RAPTOR_OK;
    }
    if (*n < need) return fail(ctx, RAPTOR_E_RANGE, "blob too small");
    raptor_status s = need_ready(ctx);
    if (s != RAPTOR_OK) return s;
    BlobHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "RAPTMLP", 8);
    h.version = 1;
    h.n_params = NP;
    h.adam_step = ctx->mlp.adam_step;
    h.lx_lo = mlp::LX_LO; h.lx_hi = mlp::LX_HI; h.lt_lo = mlp::LT_LO; h.lt_hi = mlp::LT_HI;
    h.cb_lo = mlp::CB_LO; h.cb_hi = mlp::CB_HI;
    h.mu_j = mlp::MU_J; h.sigma_j = mlp::SIGMA_J; h.mu_a = mlp::MU_A; h.sigma_a = mlp::SIGMA_A;
    unsigned char* b = (unsigned char*)blob;
    std::memcpy(b, &h, sizeof h);
    float* f = (float*)(b + sizeof h);
    RAPTOR_CK(hipMemcpyAsync(f, ctx->mlp.P.p, NP * 4, hipMemcpyDeviceToHost, ctx->stream), "reading parameters");
    RAPTOR_CK(hipMemcpyAsync(f + NP, ctx->mlp.m.p, NP * 4, hipMemcpyDeviceToHost, ctx->stream), "reading moments");
    RAPTOR_CK(hipMemcpyAsync(f + 2 * NP, ctx->mlp.v.p, NP * 4, hipMemcpyDeviceToHost, ctx->stream), "reading moments");
    RAPTOR_CK(hipStreamSynchronize(ctx->stream), "reading the checkpoint");
    *n = need;
    return RAPTOR_OK;
}

raptor_status raptor_mlp_set_weights(raptor_ctx* ctx, const void* blob, size_t n)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    const size_t need = sizeof(BlobHeader) + (size_t)3 * NP * sizeof(float);
    if (!blob || n != need) return fail(ctx, RAPTOR_E_INVALID, "blob size does not match the library's network");
    BlobHeader h;
    std::memcpy(&h, blob, sizeof h);
    if (std::memcmp(h.magic, "RAPTMLP", 8) != 0 || h.version != 1 || h.n_params != (uint32_t)NP)
        return fail(ctx, RAPTOR_E_INVALID, "not a version-1 checkpoint of this network");
    if (h.lx_lo != mlp::LX_LO || h.lx_hi != mlp::LX_HI || h.lt_lo != mlp::LT_LO || h.lt_hi != mlp::LT_HI ||
        h.mu_j != mlp::MU_J || h.sigma_j != mlp::SIGMA_J || h.mu_a != mlp::MU_A || h.sigma_a != mlp::SIGMA_A)
        return fail(ctx, RAPTOR_E_INVALID, "checkpoint normalisation differs from the library's");
    const float* f = (const float*)((const unsigned char*)blob + sizeof h);
    for (int i = 0; i < NP; ++i)
        if (!std::isfinite(f[i])) return fail(ctx, RAPTOR_E_INVALID, "checkpoint holds non-finite parameters");
    return install(ctx, f, f + NP, f + 2 * NP, h.adam_step);
}

raptor_status raptor_mlp_train(raptor_ctx* ctx, const raptor_mlp_train_cfg* c, raptor_mlp_report* rep)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!c) return fail(ctx, RAPTOR_E_INVALID, "cfg is NULL");
    if (c->n_train < 64 || c->n_val < 1 || c->epochs < 1 || c->batch < 64 || c->batch % 64 || c->batch > c->n_train ||
        !(c->lr > 0) || !(c->lr_final >= 0) || !(c->beta1 >= 0 && c->beta1 < 1) || !(c->beta2 >= 0 && c->beta2 < 1) ||
        !(c->adam_eps > 0) || !(c->weight_decay >= 0) || (c->form != RAPTOR_MLP_SPLIT && c->form != RAPTOR_MLP_BF16))
        return fail(ctx, RAPTOR_E_INVALID, "bad training configuration");
    raptor_status s = need_ready(ctx);
    if (s != RAPTOR_OK) return s;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    MlpState& S = ctx->mlp;
    hipStream_t st = ctx->stream;
    if ((s = ensure_samples(ctx, S.Xtr, S.Ttr, nullptr, c->n_train, c->train_seed, &S.n_train, &S.train_seed)) !=
        RAPTOR_OK)
        return s;
    if ((s = ensure_samples(ctx, S.Xva, S.Tva, &S.RAWva, c->n_val, c->val_seed, &S.n_val, &S.val_seed)) != RAPTOR_OK)
        return s;
    const int waves = c->batch / 64;
    RAPTOR_CK(S.partial.reserve((size_t)waves * NP), "allocating gradient partials");
    const long long steps_per_epoch = c->n_train / c->batch;
    const long long total = steps_per_epoch * c->epochs;
    RAPTOR_CK(S.loss.reserve((size_t)2 * waves * steps_per_epoch), "allocating loss partials");
    const mlp::Net net = net_of(S);
    (void)c->form;   // training forward uses the split form (the backward pass is plain BF16)
    RAPTOR_CK(hipStreamSynchronize(st), "generating samples");
    const auto t0 = std::chrono::steady_clock::now();
    double last_loss = 0.0;
    for (long long step = 0; step < total; ++step) {
        const long long b = step % steps_per_epoch;
        RAPTOR_CK(mlp_launch_train(net, S.Xtr.p, S.Ttr.p, nullptr, b * c->batch, c->n_train, 0, 1.0f / c->batch,
                                   S.partial.p, S.loss.p + (size_t)2 * waves * b, waves, st),
                  "launching the training step");
        const double prog = (double)step / (double)total;
        const float lr = (float)(c->lr_final + 0.5 * (c->lr - c->lr_final) * (1.0 + std::cos(kPi * prog)));
        S.adam_step += 1;
        const float bc1 = (float)(1.0 - std::pow((double)c->beta1, (double)S.adam_step));
        const float bc2 = (float)(1.0 - std::pow((double)c->beta2, (double)S.adam_step));
        RAPTOR_CK(mlp_launch_reduce(S.partial.p, waves, 0, S.P.p, S.m.p, S.v.p, lr, c->beta1, c->beta2, c->adam_eps,
                                    c->weight_decay, bc1, bc2, nullptr, S.W.p, S.Wlo.p, S.WT.p, st),
                  "launching the Adam step");
        if (b == steps_per_epoch - 1) {
            std::vector<float> lh((size_t)2 * waves * steps_per_epoch);
            RAPTOR_CK(hipMemcpyAsync(lh.data(), S.loss.p, lh.size() * 4, hipMemcpyDeviceToHost, st), "reading losses");
            RAPTOR_CK(hipStreamSynchronize(st), "training");
            double sum = 0.0;
            for (float x : lh) sum += x;
            last_loss = sum / (2.0 * (double)steps_per_epoch * c->batch);
        }
    }
    RAPTOR_CK(hipStreamSynchronize(st), "training");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) {
        std::memset(rep, 0, sizeof *rep);
        rep->steps = total;
        rep->train_loss = last_loss;
        rep->train_ms = ms;
        // validation in the configured form
        DevBuf<float> Y;
        RAPTOR_CK(Y.reserve((size_t)2 * c->n_val), "allocating validation outputs");
        RAPTOR_CK(mlp_launch_forward(net, c->form == RAPTOR_MLP_SPLIT, S.Xva.p, c->n_val, Y.p, st), "validating");
        std::vector<float> y((size_t)2 * c->n_val), t((size_t)2 * c->n_val), raw((size_t)3 * c->n_val);
        RAPTOR_CK(hipMemcpyAsync(y.data(), Y.p, y.size() * 4, hipMemcpyDeviceToHost, st), "reading validation");
        RAPTOR_CK(hipMemcpyAsync(t.data(), S.Tva.p, t.size() * 4, hipMemcpyDeviceToHost, st), "reading validation");
        RAPTOR_CK(hipMemcpyAsync(raw.data(), S.RAWva.p, raw.size() * 4, hipMemcpyDeviceToHost, st),
                  "reading validation");
        RAPTOR_CK(hipStreamSynchronize(st), "validating");
        Y.release();
        double ss[2] = {0, 0}, mx[2] = {0, 0}, sb = 0.0;
        long long nb = 0;
        const float sig[2] = {mlp::SIGMA_J, mlp::SIGMA_A}, mu[2] = {mlp::MU_J, mlp::MU_A};
        for (long long i = 0; i < c->n_val; ++i) {
            for (int o = 0; o < 2; ++o) {
                const double e = (double)(y[2 * i + o] - t[2 * i + o]) * sig[o];
                ss[o] += e * e;
                mx[o] = std::max(mx[o], std::fabs(e));
                // bright: ln j_hat > -20 (the target is ln j_hat plus the cut-off exponent)
                if (o == 0 && t[2 * i] * sig[0] + mu[0] -
                                      mlp::cutoff_exponent(raw[3 * i], raw[3 * i + 1], raw[3 * i + 2]) > -20.0) {
                    sb += e * e;
                    ++nb;
                }
            }
        }
        for (int o = 0; o < 2; ++o) {
            rep->val_rms[o] = std::sqrt(ss[o] / c->n_val);
            rep->val_max[o] = mx[o];
        }
        rep->val_rms_bright = nb ? std::sqrt(sb / nb) : 0.0;
    }
    return RAPTOR_OK;
}

raptor_status raptor_mlp_forward(raptor_ctx* ctx, int32_t form, const float* x, int64_t n, float* y)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!x || !y || n < 1 || !form_ok(form)) return fail(ctx, RAPTOR_E_INVALID, "bad arguments to raptor_mlp_forward");
    raptor_status s = need_ready(ctx);
    if (s != RAPTOR_OK) return s;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    DevBuf<float> X, Y;
    RAPTOR_CK(X.reserve((size_t)3 * n), "allocating inputs");
    RAPTOR_CK(Y.reserve((size_t)2 * n), "allocating outputs");
    RAPTOR_CK(hipMemcpyAsync(X.p, x, (size_t)12 * n, hipMemcpyHostToDevice, ctx->stream), "uploading inputs");
    if (form == RAPTOR_MLP_F32)
        RAPTOR_CK(mlp_launch_forward_f32(ctx->mlp.P.p, X.p, n, Y.p, ctx->stream), "launching the forward pass");
    else
        RAPTOR_CK(mlp_launch_forward(net_of(ctx->mlp), form == RAPTOR_MLP_SPLIT, X.p, n, Y.p, ctx->stream),
                  "launching the forward pass");
    RAPTOR_CK(hipMemcpyAsync(y, Y.p, (size_t)8 * n, hipMemcpyDeviceToHost, ctx->stream), "reading outputs");
    RAPTOR_CK(hipStreamSynchronize(ctx->stream), "running the forward pass");
    X.release();
    Y.release();
    return RAPTOR_OK;
}

raptor_status raptor_mlp_backward(raptor_ctx* ctx, int32_t form, const float* x, const float* dy, int64_t n,
                                  float* dparams)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!x || !dy || !dparams || n < 1 || (form != RAPTOR_MLP_BF16 && form != RAPTOR_MLP_F32))
        return fail(ctx, RAPTOR_E_INVALID, "bad arguments to raptor_mlp_backward");
    raptor_status s = need_ready(ctx);
    if (s != RAPTOR_OK) return s;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    MlpState& S = ctx->mlp;
    DevBuf<float> X, D, G;
    RAPTOR_CK(X.reserve((size_t)3 * n), "allocating inputs");
    RAPTOR_CK(D.reserve((size_t)2 * n), "allocating inputs");
    RAPTOR_CK(G.reserve(NP), "allocating gradients");
    RAPTOR_CK(hipMemcpyAsync(X.p, x, (size_t)12 * n, hipMemcpyHostToDevice, ctx->stream), "uploading inputs");
    RAPTOR_CK(hipMemcpyAsync(D.p, dy, (size_t)8 * n, hipMemcpyHostToDevice, ctx->stream), "uploading inputs");
    if (form == RAPTOR_MLP_F32) {
        RAPTOR_CK(hipMemsetAsync(G.p, 0, NP * 4, ctx->stream), "clearing gradients");
        RAPTOR_CK(mlp_launch_backward_f32(S.P.p, X.p, D.p, n, G.p, ctx->stream), "launching the backward pass");
    } else {
        const int waves = (int)((n + 63) / 64);
        DevBuf<float> part;
        RAPTOR_CK(part.reserve((size_t)waves * NP), "allocating gradient partials");
        RAPTOR_CK(mlp_launch_train(net_of(S), X.p, nullptr, D.p, 0, n, 1, 1.0f, part.p, nullptr, waves, ctx->stream),
                  "launching the backward pass");
        RAPTOR_CK(mlp_launch_reduce(part.p, waves, 1, nullptr, nullptr, nullptr, 0, 0, 0, 0, 0, 1, 1, G.p, nullptr,
                                    nullptr, nullptr, ctx->stream),
                  "reducing gradients");
        RAPTOR_CK(hipStreamSynchronize(ctx->stream), "running the backward pass");
        part.release();
    }
    RAPTOR_CK(hipMemcpyAsync(dparams, G.p, NP * 4, hipMemcpyDeviceToHost, ctx->stream), "reading gradients");
    RAPTOR_CK(hipStreamSynchronize(ctx->stream), "running the backward pass");
    X.release();
    D.release();
    G.release();
    return RAPTOR_OK;
}

raptor_status raptor_mlp_closure(raptor_ctx* ctx, int32_t form, const float* raw, int64_t n, float* net, float* exact)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!raw || n < 1 || !form_ok(form) || (!net && !exact))
        return fail(ctx, RAPTOR_E_INVALID, "bad arguments to raptor_mlp_closure");
    if (net) {
        raptor_status s = need_ready(ctx);
        if (s != RAPTOR_OK) return s;
    }
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    if (exact) {
        DevBuf<float> R, E;
        RAPTOR_CK(R.reserve((size_t)3 * n), "allocating inputs");
        RAPTOR_CK(E.reserve((size_t)2 * n), "allocating outputs");
        RAPTOR_CK(hipMemcpyAsync(R.p, raw, (size_t)12 * n, hipMemcpyHostToDevice, ctx->stream), "uploading inputs");
        RAPTOR_CK(mlp_launch_exact(ctx->k2t, n, R.p, E.p, ctx->stream), "launching the exact closure");
        RAPTOR_CK(hipMemcpyAsync(exact, E.p, (size_t)8 * n, hipMemcpyDeviceToHost, ctx->stream), "reading outputs");
        RAPTOR_CK(hipStreamSynchronize(ctx->stream), "running the exact closure");
        R.release();
        E.release();
    }
    if (net) {
        std::vector<float> x((size_t)3 * n), y((size_t)2 * n);
        for (int64_t i = 0; i < n; ++i) {
            x[3 * i] = mlp::norm_lx(raw[3 * i]);
            x[3 * i + 1] = mlp::norm_lt(raw[3 * i + 1]);
            x[3 * i + 2] = mlp::norm_cb(raw[3 * i + 2]);
        }
        raptor_status s = raptor_mlp_forward(ctx, form, x.data(), n, y.data());
        if (s != RAPTOR_OK) return s;
        for (int64_t i = 0; i < n; ++i) {
            const double tc = mlp::cutoff_exponent(raw[3 * i], raw[3 * i + 1], raw[3 * i + 2]);
            net[2 * i] = (float)(y[2 * i] * mlp::SIGMA_J + mlp::MU_J - tc);
            net[2 * i + 1] = (float)(y[2 * i + 1] * mlp::SIGMA_A + mlp::MU_A - tc);
        }
    }
    return RAPTOR_OK;
}

}  // extern "C"
