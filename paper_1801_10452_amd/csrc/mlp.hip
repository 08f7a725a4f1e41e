// mlp.hip -- training and evaluation kernels of the learned closure (see mlp_device.hpp).
//
//  gen_kernel        training / validation samples: counter-based SplitMix64 inputs over the
//                    box and targets from the exact closure (Leung fit, tabulated K2) in the
//                    log domain, FP64
//  train_kernel      one wave per 64 samples: forward (split BF16 MFMA), MSE gradient,
//                    backward (BF16 MFMA) and the wave's partial parameter gradient
//  reduce_kernel     fixed-order sum of the wave partials; Adam step on the FP32 parameters
//                    and re-packing of the BF16 hi / lo copies -- or the plain gradient
//  forward_kernel    batched inference from an LDS copy of the network (16x16x32 MFMA)
//  forward_f32 / backward_f32   FP32 reference path (one thread per sample, no matrix cores)
#include "launch.hpp"
#include "mlp_device.hpp"
#include "plasma.hpp"

namespace mlp {
namespace {

__device__ inline unsigned long long splitmix(unsigned long long seed, unsigned long long n)
{
    unsigned long long z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ inline double uniform01(unsigned long long seed, unsigned long long n)
{
    return (double)(splitmix(seed, n) >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

// Exact closure for raw inputs (ln x, ln Theta, cos), x = nu/nu_c, in the log domain:
// j / (n_e nu_c J0) = (nu_s/nu_c) / K2(1/Theta) t (t + 2^11/12)^2 exp(-t), t = (x nu_c/nu_s)^1/3,
// nu_s/nu_c = (2/9) Theta^2 sin(theta_B); alpha_hat = j_hat / (x^2 Theta).  Returns the network
// targets y0 = ln j_hat + t, y1 = ln alpha_hat + t, and t.
__device__ inline void exact_targets(const K2Table& k2, double lx, double lth, double cb, double* y0, double* y1,
                                     double* tc)
{
    const double th = ::exp(lth);
    const double sb = ::sqrt(::fmax(1.0 - cb * cb, 0.0));
    const double ns = (2.0 / 9.0) * th * th * sb;
    const double t = ::cbrt(::exp(lx) / ns);
    const double y = ::log(ns) - pl::ln_k2_theta(k2, th) + ::log(t) + 2.0 * ::log(t + pl::TWO_11_12);
    *y0 = y;
    *y1 = y - 2.0 * lx - lth;
    *tc = t;
}

__global__ void gen_kernel(K2Table k2, unsigned long long seed, long long n, float* X, float* T, float* raw)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u0 = uniform01(seed, 3ull * i), u1 = uniform01(seed, 3ull * i + 1), u2 = uniform01(seed, 3ull * i + 2);
    const double lx = (double)LX_LO + u0 * ((double)LX_HI - (double)LX_LO);
    const double lth = (double)LT_LO + u1 * ((double)LT_HI - (double)LT_LO);
    const double cb = -0.999 + 1.998 * u2;
    double t0, t1, tc;
    exact_targets(k2, lx, lth, cb, &t0, &t1, &tc);
    X[3 * i] = norm_lx((float)lx);
    X[3 * i + 1] = norm_lt((float)lth);
    X[3 * i + 2] = norm_cb((float)cb);
    T[2 * i] = (float)((t0 - MU_J) / SIGMA_J);
    T[2 * i + 1] = (float)((t1 - MU_A) / SIGMA_A);
    if (raw) {
        raw[3 * i] = (float)lx;
        raw[3 * i + 1] = (float)lth;
        raw[3 * i + 2] = (float)cb;
    }
}

// exact ln j_hat and ln alpha_hat for given raw inputs (accuracy checks)
__global__ void exact_kernel(K2Table k2, long long n, const float* raw, float* out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t0, t1, tc;
    exact_targets(k2, raw[3 * i], raw[3 * i + 1], raw[3 * i + 2], &t0, &t1, &tc);
    out[2 * i] = (float)(t0 - tc);
    out[2 * i + 1] = (float)(t1 - tc);
}

// ------------------------------------------------------------------------------------------
// Training: one work-group of four waves per 64 samples.
// LDS: Z[4][64][ZS] pre-activations (BF16, [sample][feature]), two dZ buffers [64][ZS] (BF16),
// X[64][XS] inputs (BF16), 8 loss floats.  Rows are padded by four BF16 (8 bytes): a fragment
// read or store touches 16 rows, or 4 rows four samples apart, and with the padding those start
// in different banks.
// ------------------------------------------------------------------------------------------
constexpr int ZS = 68, XS = 20, ZL = 64 * ZS;   // row strides and the size of one [64][ZS] array
constexpr int TR_LDS = (4 * ZL + 2 * ZL + 64 * XS) * 2 + 8 * 4;

// Work-group barrier that orders LDS accesses only.  The fences are limited to the local address
// space: a plain work-group fence would also wait for every global store in flight (the partial
// gradients), which the other waves never read.
__device__ inline void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ inline void store4(unsigned short* p, float a, float b, float c, float d)
{
    *reinterpret_cast<bf16x4*>(p) = pack4(a, b, c, d);
}
__device__ inline f32x4 load4(const unsigned short* p)
{
    const bf16x4 v = *reinterpret_cast<const bf16x4*>(p);
    return f32x4{bf2f((unsigned short)v.x), bf2f((unsigned short)v.y), bf2f((unsigned short)v.z),
                 bf2f((unsigned short)v.w)};
}

// K = samples fragment of a [sample][feature] BF16 array (row stride rs): lane holds the four
// samples 16 kt + 4 g + j of feature f0 + n, optionally through the SiLU.
template <bool ACT>
__device__ inline bf16x4 frag_samples(const unsigned short* M, int rs, int f0, int kt, int lane)
{
    const int n = lane & 15, s0 = 16 * kt + 4 * (lane >> 4);
    float v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float z = bf2f(M[(s0 + j) * rs + f0 + n]);
        v[j] = ACT ? silu(z) : z;
    }
    return pack4(v[0], v[1], v[2], v[3]);
}

// dW[out][in] = sum_s dZ[s][out] H[s][in] over the work-group's 64 samples; writes the partial.
// dZ: [64][ZS] BF16 (first out_tiles*16 features used); H: [64][rs] BF16 (pre-activations if
// ACT, raw inputs otherwise); db[out] = sum_s dZ[s][out].
// in_tiles is 4 or 1.  With four input tiles, wave w takes input tile w against every output
// tile, so that it reads (and activates) its H fragments once; with one, wave w takes output
// tile w.  The bias of output tile t is summed by wave t from the dZ fragments it already holds:
// each lane adds its sixteen samples, then the four lane groups are combined in a fixed tree.
// Every entry is computed by one wave, with the same instruction sequence whichever wave it is.
// The partials are written with non-temporal stores: only the reduction reads them, once.
template <bool ACT>
__device__ inline void weight_grad(const unsigned short* dZ, const unsigned short* H, int rs, int out_tiles,
                                   int in_tiles, int out_dim, int in_dim, float* gW, float* gb, int wave, int lane)
{
    const int g4 = 4 * (lane >> 4), n = lane & 15;
    const int nt = in_tiles == 4 ? wave : 0;
    const int mt0 = in_tiles == 4 ? 0 : wave, mt1 = in_tiles == 4 ? out_tiles : wave + 1;
    bf16x4 hf[4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) hf[kt] = frag_samples<ACT>(H, rs, 16 * nt, kt, lane);
    const int in = 16 * nt + n;
    for (int mt = mt0; mt < mt1; ++mt) {
        f32x4 acc = f32x4{0, 0, 0, 0};
        float bs = 0.0f;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const bf16x4 d = frag_samples<false>(dZ, ZS, 16 * mt, kt, lane);
            acc = mfma(d, hf[kt], acc);
            bs += (bf2f((unsigned short)d.x) + bf2f((unsigned short)d.y)) +
                  (bf2f((unsigned short)d.z) + bf2f((unsigned short)d.w));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int out = 16 * mt + g4 + j;
            if (out < out_dim && in < in_dim) __builtin_nontemporal_store(acc[j], gW + out * in_dim + in);
        }
        if (mt == wave) {
            bs += __shfl_xor(bs, 16, 64);
            bs += __shfl_xor(bs, 32, 64);
            if (lane < 16 && 16 * mt + n < out_dim) __builtin_nontemporal_store(bs, gb + 16 * mt + n);
        }
    }
}

// dZ_prev[s][in] = (W^T dZ)[in][s] * silu'(Z_prev[s][in]) for the 16 samples of block cb.
__device__ inline void backprop_block(const unsigned short* WT, int out_pad, int k_tiles, const unsigned short* dZ,
                                      const unsigned short* Zp, unsigned short* dZp, int cb, int lane)
{
    const int g4 = 4 * (lane >> 4), s = 16 * cb + (lane & 15);
    bf16x4 b[4];
    for (int kt = 0; kt < k_tiles; ++kt) b[kt] = *reinterpret_cast<const bf16x4*>(dZ + s * ZS + 16 * kt + g4);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = f32x4{0, 0, 0, 0};
        for (int kt = 0; kt < k_tiles; ++kt) acc = mfma(frag_a(WT, out_pad, 16 * mt, 16 * kt, lane), b[kt], acc);
        const f32x4 z = load4(Zp + s * ZS + 16 * mt + g4);
        store4(dZp + s * ZS + 16 * mt + g4, acc.x * silu_grad(z.x), acc.y * silu_grad(z.y), acc.z * silu_grad(z.z),
               acc.w * silu_grad(z.w));
    }
}

// The work-group's copy of the BF16 weights in LDS: W hi and lo [out_pad][in_pad] and WT
// [in_pad][out_pad] of the five layers, each row padded by four BF16 so that the sixteen rows a
// fragment read touches start in different banks.  Offsets and strides in BF16 units.
namespace tw {
constexpr int out_pad(int L) { return L == 4 ? 16 : 64; }
constexpr int in_pad(int L) { return L == 0 ? 16 : 64; }
constexpr int w_stride(int L) { return in_pad(L) + 4; }
constexpr int t_stride(int L) { return out_pad(L) + 4; }
constexpr int w_size(int L) { return out_pad(L) * w_stride(L); }
constexpr int t_size(int L) { return in_pad(L) * t_stride(L); }
constexpr int w_off(int L) { return L == 0 ? 0 : w_off(L - 1) + w_size(L - 1); }
constexpr int t_off(int L) { return L == 0 ? 0 : t_off(L - 1) + t_size(L - 1); }
constexpr int COPY = w_off(5);   // BF16 per copy (W, W lo and WT have the same size)
constexpr int BYTES = 3 * COPY * 2;   // the biases follow at this byte offset
constexpr int BIAS_BYTES = 260 * 4;
static_assert(COPY == t_off(5), "W and WT copies of the same size");
}  // namespace tw
constexpr int PW_OF[5] = {PW1, PW2, PW3, PW4, PW5};

// Copy the padded global layouts into the LDS layout.  The three arrays are read in 16-byte
// chunks, chunk c of each array by thread c mod 256, all loads issued before the first LDS store
// so that their latencies overlap; each chunk lies in one row of one layer (rows are 16 or 64
// BF16 long) and goes to LDS as two 8-byte stores.  The FP32 biases follow as float [4][64]
// (hidden layers) and [2] (output) at byte offset tw::BYTES.  Requires 256 threads.
__device__ inline void stage_train_weights(const Net& net, unsigned short* dst)
{
    const int t = threadIdx.x;
    const float hb = net.P[hidden_bias_off(t >> 6) + (t & 63)];
    const float ob = t < 2 ? net.P[OFF_B5 + t] : 0.0f;
    constexpr int CH = PW_TOTAL / (8 * 256);   // chunks per thread and array
    static_assert(PW_TOTAL % (8 * 256) == 0, "whole chunks per thread");
    static_assert(tw::in_pad(0) == 16 && tw::in_pad(1) == 64 && tw::out_pad(4) == 16 && tw::out_pad(3) == 64,
                  "row lengths taken as 2^4 and 2^6 below");
    uint4 w[CH], wl[CH], wt[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int e = 8 * ((int)threadIdx.x + 256 * k);
        w[k] = *reinterpret_cast<const uint4*>(net.W + e);
        wl[k] = *reinterpret_cast<const uint4*>(net.Wlo + e);
        wt[k] = *reinterpret_cast<const uint4*>(net.WT + e);
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int e = 8 * ((int)threadIdx.x + 256 * k);
        const int L = (e >= PW2) + (e >= PW3) + (e >= PW4) + (e >= PW5);
        const int pw = L == 0 ? PW1 : L == 1 ? PW2 : L == 2 ? PW3 : L == 3 ? PW4 : PW5;
        const int wof = L == 0 ? tw::w_off(0) : L == 1 ? tw::w_off(1) : L == 2 ? tw::w_off(2)
                      : L == 3 ? tw::w_off(3) : tw::w_off(4);
        const int tof = L == 0 ? tw::t_off(0) : L == 1 ? tw::t_off(1) : L == 2 ? tw::t_off(2)
                      : L == 3 ? tw::t_off(3) : tw::t_off(4);
        const int lin = L == 0 ? 4 : 6, lout = L == 4 ? 4 : 6;   // log2 of in_pad, out_pad
        const int q = e - pw;
        const int dw = wof + (q >> lin) * ((1 << lin) + 4) + (q & ((1 << lin) - 1));
        const int dt = 2 * tw::COPY + tof + (q >> lout) * ((1 << lout) + 4) + (q & ((1 << lout) - 1));
        uint2* pw0 = reinterpret_cast<uint2*>(dst + dw);
        uint2* pw1 = reinterpret_cast<uint2*>(dst + tw::COPY + dw);
        uint2* pt = reinterpret_cast<uint2*>(dst + dt);
        pw0[0] = uint2{w[k].x, w[k].y};
        pw0[1] = uint2{w[k].z, w[k].w};
        pw1[0] = uint2{wl[k].x, wl[k].y};
        pw1[1] = uint2{wl[k].z, wl[k].w};
        pt[0] = uint2{wt[k].x, wt[k].y};
        pt[1] = uint2{wt[k].z, wt[k].w};
    }
    float* bias = reinterpret_cast<float*>(dst + 3 * tw::COPY);
    bias[t] = hb;
    if (t < 2) bias[256 + t] = ob;
}

// Weight source of forward_block reading that LDS copy.
template <bool SPLIT>
struct LdsTrainWeights {
    const unsigned short* lw;
    const float* lb;   // staged biases
    __device__ inline Split w(int layer, int mt, int kt, int lane) const
    {
        return frag_w<SPLIT>(lw + tw::w_off(layer), lw + tw::COPY + tw::w_off(layer),
                             tw::w_stride(layer), 16 * mt, 16 * kt, lane);
    }
    __device__ inline const float* bias(int layer) const { return lb + 64 * layer; }
    __device__ inline float out_bias(int o) const { return lb[256 + o]; }
};

// mode 0: gradient of the mean squared error against T (standardised targets), loss sums to
// loss[2 block], loss[2 block + 1]; mode 1: gradient of sum dY . y for given dY.
// A work-group of four waves takes 64 samples: in the forward pass and in every backward step
// (dZ through the transposed weights) wave w handles the 16 samples of column block w; the
// weight gradients, which sum over all 64 samples, are shared out by output tiles (see
// weight_grad).  Every result is computed by one wave with the instruction sequence a single
// wave would use for it, so the partial gradient does not depend on the wave count.
__global__ void __launch_bounds__(256) train_kernel(Net net, const float* X, const float* T, const float* DY, long long base,
                                                    long long n, int mode, float inv_batch, float* partial, float* loss)
{
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned short* Z = reinterpret_cast<unsigned short*>(lds);   // [4][64][ZS]
    unsigned short* dA = Z + 4 * ZL;                               // [64][ZS]
    unsigned short* dB = dA + ZL;                                  // [64][ZS]
    unsigned short* Xs = dB + ZL;                                  // [64][XS]
    float* lred = reinterpret_cast<float*>(Xs + 64 * XS);          // [4][2] per-wave loss sums
    unsigned short* lw = reinterpret_cast<unsigned short*>(lds + TR_LDS);   // tw layout
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g4 = 4 * (lane >> 4), nl = lane & 15;
    const long long s0 = base + 64ll * blockIdx.x;
    float* gw = partial + (size_t)blockIdx.x * N_PARAMS;
    float l0 = 0.0f, l1 = 0.0f;
    // this lane's sample of the wave's column block; its input and target are read before the
    // weights are staged so that the two latencies overlap
    const int s = 16 * wave + nl;
    const long long gs = s0 + s;
    const bool valid = gs < n;
    float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f, y0 = 0.0f, y1 = 0.0f;
    if (valid && lane < 16) {
        x0 = X[3 * gs];
        x1 = X[3 * gs + 1];
        x2 = X[3 * gs + 2];
        const float* Y = mode == 0 ? T : DY;
        y0 = Y[2 * gs];
        y1 = Y[2 * gs + 1];
    }
    stage_train_weights(net, lw);
    lds_sync();

    // ---- forward of this wave's column block; keep pre-activations, form dY = dZ5
    {
        Split bx;
        bx.hi = (lane < 16) ? pack4(x0, x1, x2, 0.0f) : bf16x4{0, 0, 0, 0};
        bx.lo = (lane < 16) ? split4(x0, x1, x2, 0.0f).lo : bf16x4{0, 0, 0, 0};
        store4(Xs + s * XS + g4, lane < 16 ? x0 : 0.0f, lane < 16 ? x1 : 0.0f, lane < 16 ? x2 : 0.0f, 0.0f);
        f32x4 z[16];
        const f32x4 o = forward_block<true>(LdsTrainWeights<true>{lw, reinterpret_cast<const float*>(lw + 3 * tw::COPY)}, bx, lane, z);
#pragma unroll
        for (int L = 0; L < 4; ++L)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const f32x4 v = z[4 * L + mt];
                store4(Z + L * ZL + s * ZS + 16 * mt + g4, v.x, v.y, v.z, v.w);
            }
        float d0 = 0.0f, d1 = 0.0f;
        if (lane < 16 && valid) {
            if (mode == 0) {
                const float e0 = o.x - y0, e1 = o.y - y1;
                l0 = e0 * e0;
                l1 = e1 * e1;
                d0 = e0 * inv_batch;
                d1 = e1 * inv_batch;
            } else {
                d0 = y0;
                d1 = y1;
            }
        }
        store4(dA + s * ZS + g4, d0, d1, 0.0f, 0.0f);   // dZ5 in features 0..15 (lanes >= 16 write zeros)
    }
    lds_sync();
    // ---- layer 5 (64 -> 2)
    weight_grad<true>(dA, Z + 3 * ZL, ZS, 1, 4, 2, 64, gw + OFF_W5, gw + OFF_B5, wave, lane);
    const unsigned short* lwt = lw + 2 * tw::COPY;
    backprop_block(lwt + tw::t_off(4), tw::t_stride(4), 1, dA, Z + 3 * ZL, dB, wave, lane);
    lds_sync();
    // ---- layers 4, 3, 2
    unsigned short* cur = dB;
    unsigned short* nxt = dA;
    const int offw[3] = {OFF_W4, OFF_W3, OFF_W2}, offb[3] = {OFF_B4, OFF_B3, OFF_B2};
    for (int i = 0; i < 3; ++i) {
        const int L = 3 - i;   // pre-activation index of this layer's input: Z[L - 1]
        weight_grad<true>(cur, Z + (L - 1) * ZL, ZS, 4, 4, 64, 64, gw + offw[i], gw + offb[i], wave, lane);
        backprop_block(lwt + tw::t_off(3 - i), tw::t_stride(3 - i), 4, cur, Z + (L - 1) * ZL, nxt,
                       wave, lane);
        lds_sync();
        unsigned short* t = cur;
        cur = nxt;
        nxt = t;
    }
    // ---- layer 1 (3 -> 64)
    weight_grad<false>(cur, Xs, XS, 4, 1, 64, 3, gw + OFF_W1, gw + OFF_B1, wave, lane);
    if (mode == 0) {
        // per-wave sums in a fixed tree, then the four waves in order
        for (int o = 32; o > 0; o >>= 1) {
            l0 += __shfl_xor(l0, o, 64);
            l1 += __shfl_xor(l1, o, 64);
        }
        if (lane == 0) {
            lred[2 * wave] = l0;
            lred[2 * wave + 1] = l1;
        }
        lds_sync();
        if (threadIdx.x == 0) {
            loss[2 * blockIdx.x] = ((lred[0] + lred[2]) + lred[4]) + lred[6];
            loss[2 * blockIdx.x + 1] = ((lred[1] + lred[3]) + lred[5]) + lred[7];
        }
    }
}

// Index of parameter p in the padded BF16 layouts (-1 for biases).
__device__ inline void padded_index(int p, int* iw, int* iwt)
{
    int off, in_dim, in_pad, out_pad, pw;
    if (p < OFF_B1) { off = OFF_W1; in_dim = 3; in_pad = 16; out_pad = 64; pw = PW1; }
    else if (p >= OFF_W2 && p < OFF_B2) { off = OFF_W2; in_dim = 64; in_pad = 64; out_pad = 64; pw = PW2; }
    else if (p >= OFF_W3 && p < OFF_B3) { off = OFF_W3; in_dim = 64; in_pad = 64; out_pad = 64; pw = PW3; }
    else if (p >= OFF_W4 && p < OFF_B4) { off = OFF_W4; in_dim = 64; in_pad = 64; out_pad = 64; pw = PW4; }
    else if (p >= OFF_W5 && p < OFF_B5) { off = OFF_W5; in_dim = 64; in_pad = 64; out_pad = 16; pw = PW5; }
    else { *iw = *iwt = -1; return; }
    const int out = (p - off) / in_dim, in = (p - off) % in_dim;
    *iw = pw + out * in_pad + in;
    *iwt = pw + in * out_pad + out;
}

// mode 0: Adam on P (with moments m, v, step t) then repack; mode 1: grad_out = summed gradient;
// mode 2: repack only.  A block of 256 threads takes 32 parameters: thread group g (threads
// 32 g .. 32 g + 31) sums the partials of the work-groups w = g mod 8 in order, and the eight
// group sums are added in a fixed tree, so the result does not depend on scheduling.
__global__ void __launch_bounds__(256) reduce_kernel(const float* partial, int n_waves, int mode, float* P, float* m,
                                                     float* v, float lr, float b1, float b2, float eps, float wd,
                                                     float bc1, float bc2, float* grad_out, unsigned short* W,
                                                     unsigned short* Wlo, unsigned short* WT)
{
    __shared__ float part8[8][32];
    const int grp = threadIdx.x >> 5;
    const int p = blockIdx.x * 32 + (threadIdx.x & 31);
    const bool owner = grp == 0 && p < N_PARAMS;
    // parameters and moments (mode 0) or parameters (mode 2) are read before the partials, so
    // that the latencies overlap; mode 1 has neither (P, m, v may be null)
    float p0 = 0.0f, m0 = 0.0f, v0 = 0.0f;
    if (owner && mode != 1) {
        p0 = P[p];
        if (mode == 0) {
            m0 = m[p];
            v0 = v[p];
        }
    }
    if (mode != 2) {
        // work-groups w + 8 j (j < R) of the group go to accumulator j: R loads in flight
        constexpr int R = 12;
        float a[R];
#pragma unroll
        for (int j = 0; j < R; ++j) a[j] = 0.0f;
        if (p < N_PARAMS) {
            for (int w = grp; w < n_waves; w += 8 * R) {
                float x[R];
#pragma unroll
                for (int j = 0; j < R; ++j) x[j] = w + 8 * j < n_waves ? partial[(size_t)(w + 8 * j) * N_PARAMS + p] : 0.0f;
#pragma unroll
                for (int j = 0; j < R; ++j) a[j] += x[j];
            }
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) a[j] += a[j + 6];   // fixed tree: 12 -> 6 -> 3 -> 1
#pragma unroll
        for (int j = 0; j < 3; ++j) a[j] += a[j + 3];
        part8[grp][threadIdx.x & 31] = (a[0] + a[1]) + a[2];
        __syncthreads();
    }
    if (!owner) return;
    float w = p0;
    if (mode != 2) {
        const int q = threadIdx.x;
        const float g = ((part8[0][q] + part8[1][q]) + (part8[2][q] + part8[3][q])) +
                        ((part8[4][q] + part8[5][q]) + (part8[6][q] + part8[7][q]));
        if (mode == 1) {
            grad_out[p] = g;
            return;
        }
        const float mm = b1 * m0 + (1.0f - b1) * g;
        const float vv = b2 * v0 + (1.0f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        w = p0 - lr * ((mm / bc1) / (sqrtf(vv / bc2) + eps) + wd * p0);
        P[p] = w;
    }
    int iw, iwt;
    padded_index(p, &iw, &iwt);
    if (iw >= 0) {
        const unsigned short hi = f2bf(w);
        W[iw] = hi;
        Wlo[iw] = f2bf(w - bf2f(hi));
        WT[iwt] = hi;
    }
}

// Batched inference through the same LDS-staged path as the trace kernel: 256 samples per
// work-group of four waves, one sample per lane.
template <bool SPLIT>
__global__ void __launch_bounds__(256) forward_kernel(Net net, const float* X, long long n, float* Y)
{
    extern __shared__ __align__(16) unsigned char lds[];
    stage_weights(net, lds, threadIdx.x, blockDim.x);
    __syncthreads();
    const long long i = 256ll * blockIdx.x + threadIdx.x;
    const bool active = i < n;
    float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
    if (active) {
        x0 = X[3 * i];
        x1 = X[3 * i + 1];
        x2 = X[3 * i + 2];
    }
    float y0, y1;
    forward_wave_lds<SPLIT>(lds, active, x0, x1, x2, &y0, &y1);
    if (active) {
        Y[2 * i] = y0;
        Y[2 * i + 1] = y1;
    }
}

// ---- FP32 reference path (no matrix cores) ------------------------------------------------
__device__ inline void f32_forward(const float* P, const float* x, float z[4][64], float h[5][64], float y[2])
{
    const int dims[6] = {3, 64, 64, 64, 64, 2};
    const int offs[5] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4, OFF_W5};
    for (int i = 0; i < 3; ++i) h[0][i] = x[i];
    for (int L = 0; L < 5; ++L) {
        const int ni = dims[L], no = dims[L + 1];
        const float* W = P + offs[L];
        const float* b = W + no * ni;
        for (int o = 0; o < no; ++o) {
            float s = b[o];
            for (int i = 0; i < ni; ++i) s += W[o * ni + i] * h[L][i];
            if (L < 4) {
                z[L][o] = s;
                h[L + 1][o] = silu(s);
            } else {
                y[o] = s;
            }
        }
    }
}

__global__ void forward_f32_kernel(const float* P, const float* X, long long n, float* Y)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float z[4][64], h[5][64], y[2];
    f32_forward(P, X + 3 * i, z, h, y);
    Y[2 * i] = y[0];
    Y[2 * i + 1] = y[1];
}

__global__ void backward_f32_kernel(const float* P, const float* X, const float* DY, long long n, float* G)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float z[4][64], h[5][64], y[2];
    f32_forward(P, X + 3 * i, z, h, y);
    const int dims[6] = {3, 64, 64, 64, 64, 2};
    const int offs[5] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4, OFF_W5};
    float g[64], gp[64];
    g[0] = DY[2 * i];
    g[1] = DY[2 * i + 1];
    for (int L = 4; L >= 0; --L) {
        const int ni = dims[L], no = dims[L + 1];
        const float* W = P + offs[L];
        float* gW = G + offs[L];
        float* gb = gW + no * ni;
        for (int o = 0; o < no; ++o) {
            atomicAdd(&gb[o], g[o]);
            for (int k = 0; k < ni; ++k) atomicAdd(&gW[o * ni + k], g[o] * h[L][k]);
        }
        if (L == 0) break;
        for (int k = 0; k < ni; ++k) {
            float s = 0.0f;
            for (int o = 0; o < no; ++o) s += W[o * ni + k] * g[o];
            gp[k] = s * silu_grad(z[L - 1][k]);
        }
        for (int k = 0; k < ni; ++k) g[k] = gp[k];
    }
}

}  // namespace mlp

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
hipError_t mlp_launch_gen(const K2Table& k2, unsigned long long seed, long long n, float* X, float* T, float* raw,
                          hipStream_t st)
{
    const int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(mlp::gen_kernel, dim3(blocks), dim3(256), 0, st, k2, seed, n, X, T, raw);
    return hipGetLastError();
}

hipError_t mlp_launch_exact(const K2Table& k2, long long n, const float* raw, float* out, hipStream_t st)
{
    hipLaunchKernelGGL(mlp::exact_kernel, dim3((int)((n + 255) / 256)), dim3(256), 0, st, k2, n, raw, out);
    return hipGetLastError();
}

hipError_t mlp_launch_train(const mlp::Net& net, const float* X, const float* T, const float* DY, long long base,
                            long long n, int mode, float inv_batch, float* partial, float* loss, int waves,
                            hipStream_t st)
{
    hipLaunchKernelGGL(mlp::train_kernel, dim3(waves), dim3(256), mlp::TR_LDS + mlp::tw::BYTES + mlp::tw::BIAS_BYTES, st, net, X, T,
                       DY, base, n, mode, inv_batch, partial, loss);
    return hipGetLastError();
}

hipError_t mlp_launch_reduce(const float* partial, int n_waves, int mode, float* P, float* m, float* v, float lr,
                             float b1, float b2, float eps, float wd, float bc1, float bc2, float* grad_out,
                             unsigned short* W, unsigned short* Wlo, unsigned short* WT, hipStream_t st)
{
    hipLaunchKernelGGL(mlp::reduce_kernel, dim3((mlp::N_PARAMS + 31) / 32), dim3(256), 0, st, partial, n_waves, mode,
                       P, m, v, lr, b1, b2, eps, wd, bc1, bc2, grad_out, W, Wlo, WT);
    return hipGetLastError();
}

hipError_t mlp_launch_forward(const mlp::Net& net, bool split, const float* X, long long n, float* Y, hipStream_t st)
{
    const int blocks = (int)((n + 255) / 256);
    if (split)
        hipLaunchKernelGGL(mlp::forward_kernel<true>, dim3(blocks), dim3(256), mlp::LDS_NET_BYTES, st, net, X, n, Y);
    else
        hipLaunchKernelGGL(mlp::forward_kernel<false>, dim3(blocks), dim3(256), mlp::LDS_NET_BYTES, st, net, X, n, Y);
    return hipGetLastError();
}

hipError_t mlp_launch_forward_f32(const float* P, const float* X, long long n, float* Y, hipStream_t st)
{
    hipLaunchKernelGGL(mlp::forward_f32_kernel, dim3((int)((n + 63) / 64)), dim3(64), 0, st, P, X, n, Y);
    return hipGetLastError();
}

hipError_t mlp_launch_backward_f32(const float* P, const float* X, const float* DY, long long n, float* G,
                                   hipStream_t st)
{
    hipLaunchKernelGGL(mlp::backward_f32_kernel, dim3((int)((n + 63) / 64)), dim3(64), 0, st, P, X, DY, n, G);
    return hipGetLastError();
}
