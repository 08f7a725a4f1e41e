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
#include "mlp_device.hpp"

#include <type_traits>

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

// Transfer arithmetic in precision TT (double or float); the closure inputs come in FP64.
template <class TT>
struct Transfer;

template <>
struct Transfer<double> {
    // per-sample, frequency-independent part
    double ne, the, bf, sinb, ln_k2, ds, inr3, nr;
    bool emits;
    bool live;   // the sample contributes (a positive fluid-frame frequency)
    // the state as doubles (kept in LDS between the phases of a frequency-parallel round)
    static constexpr int WORDS = 9;
    __device__ inline void to_words(double* w) const
    {
        w[0] = ne; w[1] = the; w[2] = bf; w[3] = sinb; w[4] = ln_k2; w[5] = ds; w[6] = inr3; w[7] = nr;
        w[8] = __hiloint2double((int)live, (int)emits);
    }
    __device__ inline void from_words(const double* w)
    {
        ne = w[0]; the = w[1]; bf = w[2]; sinb = w[3]; ln_k2 = w[4]; ds = w[5]; inr3 = w[6]; nr = w[7];
        emits = __double2loint(w[8]) != 0;
        live = __double2hiint(w[8]) != 0;
    }
    __device__ inline void setup(const TraceParams& p, const double fl[4], double nr_, double cosb, double dsv)
    {
        ne = fl[0]; the = fl[1]; bf = fl[2];
        nr = nr_;
        ds = dsv;
        inr3 = rt::rcp_nr(nr * nr * nr);
        const double s2 = 1.0 - cosb * cosb;
        sinb = s2 > 0.0 ? s2 * rt::rsqrt_nr(s2) : 0.0;
        emits = (ne > 0.0 && the > 0.0 && bf > 0.0 && sinb > 0.0);
        ln_k2 = 0.0;
        if (emits && p.closure != CL_CONST)
            ln_k2 = (p.closure == CL_K2_PAPER) ? ::log(2.0 * the * the) : pl::ln_k2_theta(p.k2, the);
    }
    __device__ inline void contribution(const TraceParams& p, double nu_obs, double& A, double& dtau) const
    {
        double j, al, S;
        if (p.closure == CL_CONST) {
            j = p.const_j;
            al = p.const_alpha;
            S = al > 0.0 ? j / al : 0.0;
        } else if (emits) {
            pl::closure_exact(nu_obs * nr, ne, the, bf, sinb, ln_k2, &j, &al, &S);
        } else {
            return;
        }
        pl::step_source(j, al, S, ds, inr3, A, dtau);
    }
    // frequencies nu_obs[0 .. cnt) of up to G (entries g >= cnt are left untouched)
    // (nothing for a sample that does not contribute, see `live`)
    template <int G, bool BRANCHES = (G == 1)>
    __device__ inline void contributions(const TraceParams& p, const double* nu_obs, int cnt, double* A,
                                         double* dtau) const
    {
        if (!live) return;
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (g < cnt) contribution(p, nu_obs[g], A[g], dtau[g]);
    }
};

// FP32 transfer.  The coefficients j, alpha, S and the step's contribution are float
// mantissas; the arguments of the exponentials whose size amplifies rounding -- X^1/3 in the
// emissivity (up to ~40 where the flux matters) and ln K2 -- are formed in double.  The
// factor 1/K2 exp(-X^1/3) = exp(-(ln K2 + X^1/3)) is split exactly into 2^-n 2^-f: the float
// arithmetic carries the mantissa 2^-f and the power of two 2^-n is applied in double at the
// end, so emission far below the float range (X^1/3 > 87, common at high frequencies) keeps its
// value instead of flushing to zero, and so does the large 1/K2 of cold plasma (Theta_e below
// ~0.01, where 1/K2 alone exceeds the float range).  The results (contribution and optical
// depth of the step) are doubles.
template <>
struct Transfer<float> {
    float ne, the, inv_the, nu_s, ds, inr3;
    double ln_k2;        // ln K2(1/Theta_e) (ln 2 Theta_e^2 for the paper's closure)
    double nr_inv_nus;   // nu_r / nu_s: X = nu_obs nu_r / nu_s in double
    double nr;
    bool emits;
    bool live;   // the sample contributes (a positive fluid-frame frequency)
    // the state as doubles, floats in pairs (kept in LDS between the phases of a
    // frequency-parallel round)
    static constexpr int WORDS = 7;
    __device__ static inline double pack(float a, float b)
    {
        return __hiloint2double((int)__float_as_uint(b), (int)__float_as_uint(a));
    }
    __device__ inline void to_words(double* w) const
    {
        w[0] = pack(ne, the); w[1] = pack(inv_the, nu_s); w[2] = pack(ds, inr3);
        w[3] = ln_k2; w[4] = nr_inv_nus; w[5] = nr;
        w[6] = __hiloint2double((int)live, (int)emits);
    }
    __device__ inline void from_words(const double* w)
    {
        ne = __uint_as_float((unsigned)__double2loint(w[0])); the = __uint_as_float((unsigned)__double2hiint(w[0]));
        inv_the = __uint_as_float((unsigned)__double2loint(w[1])); nu_s = __uint_as_float((unsigned)__double2hiint(w[1]));
        ds = __uint_as_float((unsigned)__double2loint(w[2])); inr3 = __uint_as_float((unsigned)__double2hiint(w[2]));
        ln_k2 = w[3]; nr_inv_nus = w[4]; nr = w[5];
        emits = __double2loint(w[6]) != 0;
        live = __double2hiint(w[6]) != 0;
    }
    __device__ inline void setup(const TraceParams& p, const double fl[4], double nr_, double cosb, double dsv)
    {
        ne = (float)fl[0];
        the = (float)fl[1];
        inv_the = rt::rcpf_nr(the);
        nr = nr_;
        ds = (float)dsv;
        inr3 = rt::rcpf_nr((float)(nr_ * nr_ * nr_));
        const double s2 = 1.0 - cosb * cosb;
        const double sb = s2 > 0.0 ? s2 * rt::rsqrt_nr(s2) : 0.0;
        emits = (fl[0] > 0.0 && fl[1] > 0.0 && fl[2] > 0.0 && sb > 0.0);
        const double nus = (2.0 / 9.0) * pl::NUC_PER_GAUSS * fl[2] * fl[1] * fl[1] * sb;
        nu_s = (float)nus;
        nr_inv_nus = emits ? nr_ * rt::rcp_nr(nus) : 0.0;
        ln_k2 = 0.0;
        if (emits && p.closure != CL_CONST)
            ln_k2 = (p.closure == CL_K2_PAPER) ? rt::log_pos(2.0 * fl[1] * fl[1]) : pl::ln_k2_theta(p.k2, fl[1]);
    }
    // One frequency's coefficients from tt = X^1/3 (X = nu_obs nu_r / nu_s): the power of two
    // 2^-n of exp(-(ln K2 + tt)) = 2^-n 2^-f, the float mantissas of j (jm, j = jm 2^-n) and of
    // the source S = B_nu, and the step's optical depth dt in double.
    struct Terms {
        double scale, dt;
        float jm, S;
    };
    __device__ inline Terms terms(double tt, double nu_obs) const
    {
        // exp(-(ln K2 + tt)) = 2^-n 2^-f, |f| <= 1/2; beyond 2^-1100 the emission is zero in
        // double too, and the exponent is kept above -1000 so that the scale stays finite
        const double z = ::fmax(::fmin((tt + ln_k2) * 1.4426950408889634, 1100.0), -1000.0);
        const double n = __builtin_rint(z);
        const float em = __builtin_amdgcn_exp2f(-(float)(z - n));
        Terms T;
        T.scale = __builtin_ldexp(1.0, -(int)n);
        const float t = (float)tt;
        const float tc = t + 1.8877486253633868f;                 // 2^(11/12)
        T.jm = 1.1396857174835936e-29f * ne * nu_s * t * tc * tc * em;   // j = jm 2^-n
        const float nuf = (float)(nu_obs * nr);
        const float q = nuf * 2.45215662654257e-16f;              // nu (2h/c^2)^(1/3)
        const float q3 = q * q * q;                               // 2 h nu^3 / c^2
        const float em1 = rt::expm1_f((float)pl::H_OVER_MEC2 * nuf * inv_the);
        T.S = q3 * rt::rcpf_nr(em1);                              // B_nu
        const float dtm = T.jm * em1 * rt::rcpf_nr(q3) * ds;      // dtau = dtm 2^-n
        T.dt = (double)dtm * T.scale;
        return T;
    }
    __device__ inline void contribution(const TraceParams& p, double nu_obs, double& A, double& dtau) const
    {
        contributions<1>(p, &nu_obs, 1, &A, &dtau);
    }
    // Frequencies nu_obs[0 .. cnt) of up to G at once, written without branches (unless G = 1
    // and BRANCHES) so that the G dependency chains interleave, and so that consecutive calls in
    // a loop stay free of branches; entries g >= cnt, frequencies whose emission is below
    // exp(-1e8), and every entry of a sample that does not emit or contribute (`live`), are
    // left untouched.
    template <int G, bool BRANCHES = (G == 1)>
    __device__ inline void contributions(const TraceParams& p, const double* nu_obs, int cnt, double* A,
                                         double* dtau) const
    {
        if (p.closure == CL_CONST) {
            if (!live) return;
            const float j = (float)p.const_j, al = (float)p.const_alpha;
            float Af, dtf;
            pl::step_source(j, al, al > 0.0f ? j / al : 0.0f, ds, inr3, Af, dtf);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (g < cnt) {
                    A[g] = Af;
                    dtau[g] = dtf;
                }
            }
            return;
        }
        if constexpr (G == 1 && BRANCHES) {
            // one frequency: branches skip the work that the selects below would only discard
            if (!(emits && live) || cnt < 1) return;
            const double X = nu_obs[0] * nr_inv_nus;
            if (!(X < 1e24)) return;   // exp(-X^1/3) < exp(-1e8): no emission, no absorption
            const Terms T = terms(rt::cbrt_refined(X), nu_obs[0]);
            dtau[0] = T.dt;
            if (T.dt > 1e-8)
                A[0] = (double)(T.S * -rt::expm1_f(-(float)T.dt) * inr3);
            else
                A[0] = (double)(T.jm * ds * inr3) * T.scale;   // S dtau = j ds to float precision
            return;
        }
        // a sample that does not emit goes through the same instructions, its results discarded
        const bool on = emits && live;
        bool ok[G];
        double tt[G], An[G], Dt[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double X = nu_obs[g] * nr_inv_nus;
            ok[g] = on && g < cnt && X < 1e24;   // beyond, exp(-X^1/3) < exp(-1e8): no emission, no absorption
            tt[g] = rt::cbrt_refined(ok[g] ? X : 1.0);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const Terms T = terms(tt[g], nu_obs[g]);
            // 1 - exp(-dtau) = dtau (1 - dtau/2 + ...): below 1e-8, S dtau = j ds to float precision
            const double a_thick = (double)(T.S * -rt::expm1_f(-(float)T.dt) * inr3);
            const double a_thin = (double)(T.jm * ds * inr3) * T.scale;
            An[g] = T.dt > 1e-8 ? a_thick : a_thin;
            Dt[g] = T.dt;
        }
        // The G results are consumed here, unconditionally, by empty asm statements: without
        // that the compiler sinks each chain into a branch on ok[g], one after another, and the
        // chains no longer interleave.
#pragma unroll
        for (int g = 0; g < G; ++g) asm volatile("" ::"v"(An[g]), "v"(Dt[g]));
#pragma unroll
        for (int g = 0; g < G; ++g) {
            A[g] = ok[g] ? An[g] : A[g];
            dtau[g] = ok[g] ? Dt[g] : dtau[g];
        }
    }
};

// Attenuation e^-tau of the accumulated optical depth (held in double in both precisions).
template <class TT>
__device__ inline TT attenuation(double tau);
template <>
__device__ inline double attenuation<double>(double tau) { return ::exp(-tau); }
template <>
__device__ inline float attenuation<float>(double tau) { return rt::exp_mixed(-tau); }

// ---------------------------------------------------------------------------------------
// Sample compaction.  A lane whose ray takes a step inside the plasma does not evaluate the
// sample at once: it queues the point (ten doubles) in its wave's LDS area, up to K per lane,
// its k-th in slot k * 64 + lane (consecutive lanes in consecutive slots of a queue layer).
// The wave evaluates queued samples together -- sample i of the selected list on lane i mod 64
// -- so the expensive part (MKS map, gather, fluid frame, closure) runs on full waves: once 64
// samples are queued (or a lane's queue is full) it evaluates the largest multiple of 64 of
// them, oldest first across the lanes, and leaves the rest queued; when a ray with queued
// samples terminates, or a full queue meets fewer than 64 samples, it evaluates everything.  Each owner folds its evaluated samples into (I, tau) in
// the order they were taken and moves the rest to the front of its queue, which keeps the
// backward transfer identical to evaluating every sample right after its step.
// ---------------------------------------------------------------------------------------
constexpr int N_FIELDS = 10;   // t, r, theta, phi, k^t, k^r, k^phi, |dlambda|, sin, cos

// What the evaluation of a queued sample needs from its ray's job.
struct LaneInfo {
    double a;
    int grid, fast_snap, nu_base, n_nu;
};

__device__ inline LaneInfo lane_info(const TraceParams& p, int job)
{
    const DevJob& J = p.jobs[job];
    return LaneInfo{J.a, J.grid, J.fast_snap, J.nu_base, J.n_nu};
}

template <int NNU, class TT, bool MLPC, int WPE>
struct Queue {
    // pending samples per lane: the most (up to three) for which the waves of the variant's
    // occupancy (two per SIMD, or three for the 3-waves-per-SIMD variant) fit a compute unit's
    // 160 KiB of LDS -- beside one copy of the network for the learned closure.  Results are
    // doubles in both precisions (an FP32 contribution carries its power-of-two scale, see
    // Transfer<float>).
    static constexpr int bytes_for(int k) { return 64 * k * (N_FIELDS * 8 + 2 * NNU * 8 + 4) + 64 * 4; }
    static constexpr int WAVES_PER_CU = 4 * (WPE >= 3 ? 3 : 2);
    static constexpr int BUDGET = (163840 - (MLPC ? mlp::LDS_NET_BYTES : 0)) / WAVES_PER_CU;
    static constexpr int K = bytes_for(3) <= BUDGET ? 3 : bytes_for(2) <= BUDGET ? 2 : 1;
    // a wave's area for `rays` rays per wave (64, or fewer with a one-sample queue): fields
    // [N_FIELDS][slots], results [slots][2 NNU], slot map [slots], job index of each lane [64]
    static constexpr size_t field_bytes(int rays) { return (size_t)N_FIELDS * rays * K * sizeof(double); }
    static constexpr size_t res_bytes(int rays) { return (size_t)2 * NNU * rays * K * sizeof(double); }
    static constexpr size_t map_bytes(int rays) { return (size_t)rays * K * sizeof(int); }
    static constexpr size_t INFO_BYTES = 64 * sizeof(int);
    // Several frequencies with one queued sample per lane (the kernel's FUSED form): the job
    // indices [64] and the slot map [64] first, then one record per ray of REC doubles -- its ten
    // queue fields, then its intensity and optical depth per frequency -- so that every address
    // is a compile-time offset from the record of a slot whatever the rays per wave.
    static constexpr bool ONE_SLOT = !MLPC && K == 1 && NNU > 1;
    static constexpr int REC = N_FIELDS + 2 * NNU;
    static constexpr size_t per_wave(int rays)
    {
        return ONE_SLOT ? (size_t)512 + (size_t)rays * REC * sizeof(double)
                        : (field_bytes(rays) + res_bytes(rays) + map_bytes(rays) + INFO_BYTES + 15) / 16 * 16;
    }
    static constexpr size_t PER_WAVE = per_wave(64);
};

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The frequency-independent part of a queued sample's evaluation: fluid state, fluid frame and
// the transfer set-up.  A sample whose fluid-frame frequency is not positive (integration error
// of a low-order integrator in the last step before the horizon) has no defined emission: its
// transfer stays non-emitting and it adds nothing.  Returns whether the fluid frame fell back to
// the ZAMO.
// Frequencies evaluated together (independent dependency chains) by one lane.
constexpr int FREQ_GROUP = 4;

template <class TT>
__device__ inline bool setup_sample(const TraceParams& p, const double* q, const LaneInfo& li, Transfer<TT>& tr)
{
    const DevGrid& G = p.grids[li.grid];
    const double y[8] = {q[0], q[1], q[2], q[3], q[4], q[5], 0.0, q[6]};
    double fl[4];
    pl::sample_fluid(G, p.slow_light, li.fast_snap, y, fl);
    double nr, cb;
    const bool zamo = pl::fluid_frame(li.a, li.a * li.a, p.M, y, q[8], q[9], fl[3], &nr, &cb);
    tr.emits = false;
    tr.live = nr > 0.0;
    if (tr.live) tr.setup(p, fl, nr, cb, nr * q[7] * p.length_unit);
    return zamo;
}

// Evaluate one queued sample: fluid state, fluid frame, closure, and per frequency the
// attenuation-free contribution A (observed units) and the optical depth dtau of the step.
template <int NNU, class TT>
__device__ inline bool eval_sample(const TraceParams& p, const double* q, const LaneInfo& li, double* A,
                                   double* dtau)
{
    Transfer<TT> tr;
    const bool zamo = setup_sample<TT>(p, q, li, tr);
#pragma unroll
    for (int f = 0; f < NNU; ++f) {
        A[f] = 0.0;
        dtau[f] = 0.0;
    }
    if (!tr.live) return zamo;
    constexpr int G = NNU < FREQ_GROUP ? NNU : FREQ_GROUP;
#pragma unroll
    for (int f = 0; f < NNU; f += G) {
        if (f < li.n_nu) {
            double nu[G];
#pragma unroll
            for (int g = 0; g < G; ++g) nu[g] = (f + g < li.n_nu) ? p.nu[li.nu_base + f + g] : 1.0;
            tr.template contributions<G>(p, nu, li.n_nu - f, A + f, dtau + f);
        }
    }
    return zamo;
}

// A sample's transfer set-up kept in LDS between the two phases of a frequency-parallel round:
// Transfer<TT>'s words in the sample's queue slot, in the fields the evaluation no longer needs
// (every field but the step length, which the fold still reads).
constexpr int SETUP_FIELDS[9] = {0, 1, 2, 3, 4, 5, 6, 8, 9};
template <class TT, int FS, int SS>
__device__ inline void store_setup(double* fields, int s, const Transfer<TT>& tr)
{
    static_assert(Transfer<TT>::WORDS <= 9, "the transfer set-up fits the sample's free queue fields");
    double w[Transfer<TT>::WORDS];
    tr.to_words(w);
#pragma unroll
    for (int k = 0; k < Transfer<TT>::WORDS; ++k) fields[SETUP_FIELDS[k] * FS + s * SS] = w[k];
}
template <class TT, int FS, int SS>
__device__ inline void load_setup(const double* fields, int s, Transfer<TT>& tr)
{
    double w[Transfer<TT>::WORDS];
#pragma unroll
    for (int k = 0; k < Transfer<TT>::WORDS; ++k) w[k] = fields[SETUP_FIELDS[k] * FS + s * SS];
    tr.from_words(w);
}

// The learned closure's step contribution in FP32 transfer, by the scheme of Transfer<float>: the
// network gives ln j_hat + X^1/3 and ln alpha_hat + X^1/3 (standardised); the cut-off factor
// exp(-X^1/3), common to j and alpha, is split exactly into 2^-n 2^-f, the float arithmetic
// carries 2^-f and the power of two is applied in double to the step's optical depth and
// contribution.  j = n_e nu_c J0 e^(ln j_hat), alpha = n_e J0 / (2 m_e nu_c) e^(ln alpha_hat)
// B_RJ/B_nu, and the source is their ratio.
__device__ inline void mlp_contribution_f32(const Transfer<float>& tr, float y0, float y1, double nu_obs, double nuc,
                                            double& A, double& dtau)
{
    const double X = nu_obs * tr.nr_inv_nus;
    if (!(X < 1e24)) return;   // exp(-X^1/3) < exp(-1e8): no emission, no absorption
    const double tt = rt::cbrt_refined(X);
    const double z = ::fmin(tt * 1.4426950408889634, 1100.0);
    const double n = __builtin_rint(z);
    const float em = __builtin_amdgcn_exp2f(-(float)(z - n));
    const double scale = __builtin_ldexp(1.0, -(int)n);
    const float ej = __expf(y0 * mlp::SIGMA_J + mlp::MU_J), ea = __expf(y1 * mlp::SIGMA_A + mlp::MU_A);
    const float nucf = (float)nuc;
    const float yy = (float)pl::H_OVER_MEC2 * (float)(nu_obs * tr.nr) * tr.inv_the;
    const float planck = (yy > 1e-4f) ? rt::expm1_f(yy) * rt::rcpf_nr(yy) : 1.0f + 0.5f * yy;   // B_RJ / B_nu
    const float jm = tr.ne * nucf * (float)pl::J_PREF * ej * em;                                 // j = jm 2^-n
    const float am = tr.ne * (float)(pl::J_PREF / (2.0 * pl::ME_CGS)) * rt::rcpf_nr(nucf) * ea * em * planck;
    const float dtm = am * tr.ds;                                                                // dtau = dtm 2^-n
    dtau = (double)dtm * scale;
    if (dtau > 1e-8) {
        A = (double)(jm * rt::rcpf_nr(am) * -rt::expm1_f(-(float)dtau) * tr.inr3);
    } else {
        // 1 - exp(-dtau) = dtau (1 - dtau/2 + ...): S dtau = j ds to float precision
        A = (double)(jm * tr.ds * tr.inr3) * scale;
    }
}

// Learned-closure variant of eval_sample for one round: every lane of the wave takes part in the
// network evaluations (one per frequency); lanes without a sample feed zeros.  Samples whose
// closure inputs leave the training box use the exact closure, except where the exact closure
// itself gives exactly zero: where X^1/3 + ln K2(1/Theta_e) exceeds MLP_ZERO_EXP, the factor
// exp(-(X^1/3 + ln K2)) lies below the smallest double, so j and alpha vanish in both transfer
// precisions (the FP32 transfer's power of two 2^-n has n >= 1076 there).  Those samples are
// skipped (counted as dropped) at no change to any result.
constexpr double MLP_ZERO_EXP = 746.0;

template <int NNU, class TT>
__device__ inline void eval_round_mlp(const TraceParams& p, const unsigned char* lds_net, bool has, const double* q,
                                      const LaneInfo& li, double* A, double* dtau, unsigned long long& c_zamo,
                                      unsigned long long& c_fallback, unsigned long long& c_dropped)
{
    double fl[4] = {0.0, 1.0, 1.0, 0.0};
    double nr = 1.0, cb = 0.0;
    bool zamo = false;
    Transfer<TT> tr;
    tr.emits = false;
    tr.live = false;
    if (has) {
        const DevGrid& G = p.grids[li.grid];
        const double y[8] = {q[0], q[1], q[2], q[3], q[4], q[5], 0.0, q[6]};
        pl::sample_fluid(G, p.slow_light, li.fast_snap, y, fl);
        zamo = pl::fluid_frame(li.a, li.a * li.a, p.M, y, q[8], q[9], fl[3], &nr, &cb);
        // a non-positive fluid-frame frequency has no defined emission (see eval_sample): the
        // transfer stays non-emitting and the sample adds nothing
        tr.live = nr > 0.0;
        if (tr.live) tr.setup(p, fl, nr, cb, nr * q[7] * p.length_unit);
    }
    c_zamo += __popcll(__ballot(zamo));
    const double nuc = pl::NUC_PER_GAUSS * fl[2];
    const float lth = (float)rt::log_pos(fl[1] > 0.0 ? fl[1] : 1.0);
    const double ds = nr * q[7] * p.length_unit;
    const double inr3 = has ? rt::rcp_nr(nr * nr * nr) : 0.0;
    // nu_s / nu: X = nu / nu_s, nu_s = (2/9) nu_c Theta_e^2 sin(theta_B)
    const double nus = (2.0 / 9.0) * nuc * fl[1] * fl[1] * ::sqrt(::fmax(1.0 - cb * cb, 0.0));
#pragma unroll 1
    for (int f = 0; f < NNU; ++f) {
        const bool act = has && f < li.n_nu;
        const double nu = act ? p.nu[li.nu_base + f] * nr : nuc;
        const float lx = (float)rt::log_pos(nu / nuc);
        const bool inb = act && tr.emits && mlp::in_box(lx, lth, (float)cb);
        // X^1/3 + ln K2 > MLP_ZERO_EXP  <=>  X > t_lim^3, t_lim = MLP_ZERO_EXP - ln K2 (X^1/3 >= 0)
        const double t_lim = MLP_ZERO_EXP - tr.ln_k2;
        const bool drop = act && tr.emits && !inb && (t_lim <= 0.0 || nu > t_lim * t_lim * t_lim * nus);
        c_fallback += __popcll(__ballot(act && tr.emits && !inb && !drop));
        c_dropped += __popcll(__ballot(drop));
        const float x0 = inb ? mlp::norm_lx(lx) : 0.0f, x1 = inb ? mlp::norm_lt(lth) : 0.0f,
                    x2 = inb ? mlp::norm_cb((float)cb) : 0.0f;
        float y0, y1;
        if (p.closure == CL_MLP_BF16)
            mlp::forward_wave_lds<false>(lds_net, inb, x0, x1, x2, &y0, &y1);
        else
            mlp::forward_wave_lds<true>(lds_net, inb, x0, x1, x2, &y0, &y1);
        if (!act) continue;
        A[f] = 0.0;
        dtau[f] = 0.0;
        if (inb) {
            if constexpr (std::is_same<TT, float>::value) {
                mlp_contribution_f32(tr, y0, y1, p.nu[li.nu_base + f], nuc, A[f], dtau[f]);
            } else {
                // the network gives ln j_hat + X^1/3 and ln alpha_hat + X^1/3 (standardised); the
                // coefficients are formed in double from them (their logs span hundreds)
                const double sb2 = 1.0 - cb * cb;
                const double tc = rt::cbrt_refined(nu / ((2.0 / 9.0) * nuc * fl[1] * fl[1] * ::sqrt(sb2)));
                const double lnj = y0 * mlp::SIGMA_J + mlp::MU_J - tc, lna = y1 * mlp::SIGMA_A + mlp::MU_A - tc;
                const double ne = fl[0];
                const double j = ne * nuc * pl::J_PREF * ::exp(lnj);
                const double yy = pl::H_OVER_MEC2 * nu / fl[1];
                const double planck = (yy > 1e-4) ? ::expm1(yy) / yy : 1.0 + 0.5 * yy;   // B_RJ / B_nu
                const double al = ne * pl::J_PREF / (2.0 * pl::ME_CGS * nuc) * ::exp(lna) * planck;
                pl::step_source(j, al, j / al, ds, inr3, A[f], dtau[f]);
            }
        } else if (tr.emits && !drop) {
            tr.contribution(p, p.nu[li.nu_base + f], A[f], dtau[f]);
        }
    }
}

// Work-groups of up to 256 lanes; up to 512 for the learned closure's 2-waves-per-SIMD variant,
// whose eight waves share one LDS copy of the network (a 512-lane group caps a kernel at 256
// registers per lane, which that variant fits anyway).
template <int NNU, class TT, int WPE, bool MLPC, int INTEG>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, (MLPC && WPE >= 2) ? 512 : 256),
                               amdgpu_waves_per_eu(WPE, 8)))
trace_kernel(TraceParams p)
{
    using Q = Queue<NNU, TT, MLPC, WPE>;
    constexpr int K = Q::K;
    // Several frequencies and a one-sample queue: the ray's intensity and optical depth per
    // frequency live in its row of the result area (I then tau, 2 NNU doubles) instead of
    // registers, and every round is evaluated frequency-parallel, each (sample, frequency) pair
    // folded into that row by the lane that computes it.
    constexpr bool FUSED = Q::ONE_SLOT;
    // rays per wave: lanes [0, RAYS) trace rays (the plan may give a one-sample-queue kernel
    // fewer than 64, the other lanes then only work in the sample rounds); RAYS * K queue slots
    const int RAYS = FUSED ? p.rays_per_wave : 64;
    // field f of queue slot s is fields[f * FS + s * SS]: field-major for the multi-slot queues,
    // slot-major (each sample's ten fields together) for the one-slot queues, whose slot count
    // varies with the rays per wave -- the strides stay compile-time constants either way
    constexpr int FS = FUSED ? 1 : 64 * K;
    constexpr int SS = FUSED ? Q::REC : 1;
    constexpr int RS = FUSED ? Q::REC : 2 * NNU;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    unsigned char* wbase = smem + (size_t)(threadIdx.x >> 6) * Q::per_wave(RAYS);
    double* fields;    // see FS, SS
    double* res;       // row of slot s at res + s * RS: [NNU] intensities or contributions, then [NNU] depths
    int* slot_map;     // [slots]
    int* lane_job;     // [64]
    if constexpr (FUSED) {
        lane_job = reinterpret_cast<int*>(wbase);
        slot_map = reinterpret_cast<int*>(wbase + 256);
        fields = reinterpret_cast<double*>(wbase + 512);
        res = fields + N_FIELDS;
    } else {
        fields = reinterpret_cast<double*>(wbase);
        res = reinterpret_cast<double*>(wbase + Q::field_bytes(64));
        slot_map = reinterpret_cast<int*>(wbase + Q::field_bytes(64) + Q::res_bytes(64));
        lane_job = reinterpret_cast<int*>(wbase + Q::field_bytes(64) + Q::res_bytes(64) + Q::map_bytes(64));
    }
    const double M = p.M;
    // learned closure: the work-group's copy of the network, after the queues of its waves
    unsigned char* lds_net = smem + (size_t)(blockDim.x >> 6) * Q::PER_WAVE;
    if (MLPC) {
        const mlp::Net net{p.mlp_P, p.mlp_W, p.mlp_Wlo, nullptr};
        mlp::stage_weights(net, lds_net, threadIdx.x, blockDim.x);
        __syncthreads();
    }

    // ray state of this lane (Verlet also carries dk/dlambda at y, valid when have_acc)
    double y[8];
    double vacc[4] = {0.0, 0.0, 0.0, 0.0};
    bool have_acc = false;
    double a = 0.0, r_stop = 0.0, r_esc = 0.0, sth = 0.0, cth = 1.0;
    // optical-depth-aware step: d tau / d|lambda| of the last sample at its most absorbing
    // frequency (0: no transfer limit on the next step)
    double rt_rate = 0.0;
    int job = 0, steps = 0, pix = 0, n_nu = 0, grid = 0, pending = 0;
    int qstep[K];   // step number of each queued sample (the optical-depth cut-off ends the ray there)
    bool active = false;
    // accumulated intensity and optical depth in double (the per-sample terms are TT)
    double I[NNU], tau[NNU];
#pragma unroll
    for (int f = 0; f < NNU; ++f) { I[f] = 0.0; tau[f] = 0.0; }
#pragma unroll
    for (int i = 0; i < 8; ++i) y[i] = 0.0;

    // wave-level statistics (ballot counts: scalar registers)
    unsigned long long c_rays = 0, c_steps = 0, c_samples = 0, c_hor = 0, c_esc = 0, c_max = 0, c_pole = 0,
                       c_num = 0, c_zamo = 0, c_fallback = 0, c_opq = 0, c_dropped = 0;

    long long next = 0, end = 0;   // rays of the current tile not yet handed out (wave-uniform)
    bool drained = false;

    while (true) {
        // ------------------------------------------------------------ refill idle lanes
        const bool ray_lane = lane < RAYS;
        unsigned long long idle = __ballot(!active && ray_lane);
        int n_idle = __popcll(idle);
        if (n_idle >= p.refill_threshold || n_idle == RAYS) {
            while (n_idle > 0) {
                if (next == end) {
                    if (drained) break;
                    unsigned t = 0;
                    if (lane == 0) t = atomicAdd(p.tile_counter, 1u);
                    t = __builtin_amdgcn_readfirstlane(t);
                    if ((long long)t >= p.n_tiles) {
                        drained = true;
                        break;
                    }
                    next = (long long)t * RAYS;
                    end = next + RAYS;
                }
                const long long avail = end - next;
                const unsigned rank = lane_rank(idle);
                if (!active && ray_lane && (long long)rank < avail) {
                    const long long ray = next + rank;
                    const long long tile = FUSED ? ray >> p.rays_shift : ray >> 6;
                    const int slot = (int)(ray & (RAYS - 1));
                    job = find_job(p.jobs, p.n_jobs, tile);
                    const DevJob& J = p.jobs[job];
                    const long long lt = tile - J.tile_base;
                    const int tw = 1 << p.tile_shift;
                    const int px = (int)(lt % J.tiles_x) * tw + (slot & (tw - 1));
                    const int py = (int)(lt / J.tiles_x) * (RAYS >> p.tile_shift) + (slot >> p.tile_shift);
                    if (px < J.nx && py < J.ny) {
                        const double alpha = -J.fov + (px + 0.5) * J.dalpha;
                        const double beta = -J.fov + (py + 0.5) * J.dbeta;
                        a = J.a;
                        const rk::Spin<double> sp = rk::make_spin(a, M);
                        rk::camera_ray(sp, J.r_cam, J.incl, J.sin_i, J.cos_i, alpha, beta, J.t_init, y);
                        rt::sincos_small(y[2], &sth, &cth);
                        r_stop = J.r_stop;
                        r_esc = J.r_cam;
                        pix = py * J.nx + px;
                        n_nu = J.n_nu;
                        grid = J.grid;
                        lane_job[lane] = job;
                        steps = 0;
                        rt_rate = 0.0;
                        have_acc = false;
#pragma unroll
                        for (int f = 0; f < NNU; ++f) { I[f] = 0.0; tau[f] = 0.0; }
                        if (FUSED) {
#pragma unroll
                            for (int f = 0; f < 2 * NNU; ++f) res[lane * RS + f] = 0.0;
                        }
                        active = true;
                    }
                }
                next += (avail < n_idle) ? avail : n_idle;
                idle = __ballot(!active && ray_lane);
                n_idle = __popcll(idle);
            }
        }
        const unsigned long long act = __ballot(active);
        if (act == 0ull) break;   // every lane idle (queues are empty): the tile queue is drained
        c_steps += __popcll(act);

        // ------------------------------------------------------------ one step of every active ray
        bool reflected = false;
        int status = RAY_RUNNING;
        if (active) {
            const rk::Spin<double> sp = rk::make_spin(a, M);
            double h = rk::step_size(p.eps, y);
            if (p.tau_step > 0.0 && rt_rate > 0.0) h = ::fmin(h, p.tau_step / rt_rate);
            rt_rate = 0.0;
            const double dl = -h;
            const double th0 = y[2], s0 = sth, c0 = cth;
            if (INTEG == INTEG_RK2) {
                rk::rk2_step(sp, y, dl, sth, cth);
            } else if (INTEG == INTEG_VERLET) {
                if (!have_acc) rk::ks_accel(sp, y, sth, cth, vacc);
                rk::verlet_step(sp, y, vacc, dl, p.integrator == INTEG_VERLET_CORR, sth, cth);
                have_acc = true;
            } else {
                rk::rk4_step(sp, y, dl, sth, cth);
            }
            ++steps;
            bool fin = true;
#pragma unroll
            for (int i = 0; i < 8; ++i) fin = fin && ::isfinite(y[i]);
            if (!fin) {
                status = RAY_NUMERIC;
            } else {
                reflected = rk::reflect_pole(y);
                if (reflected) have_acc = false;   // the carried derivative belongs to the old chart
                // sin and cos of the new theta from those of the old one (the step moves theta
                // little); after a reflection from scratch
                if (reflected)
                    rt::sincos_small(y[2], &sth, &cth);
                else
                    rk::sincos_shift(th0, s0, c0, y[2], &sth, &cth);
                if (y[1] < r_stop)
                    status = RAY_HORIZON;
                else if (y[1] > r_esc)
                    status = RAY_ESCAPED;
                else if (steps >= p.max_steps)
                    status = RAY_MAXSTEP;
            }
            if (status == RAY_RUNNING && pl::in_plasma(p.grids[grid], y[1])) {
                // queue the sample point
                const int s = pending * 64 + lane;   // queue layer `pending` of this lane
                fields[0 * FS + s * SS] = y[0];
                fields[1 * FS + s * SS] = y[1];
                fields[2 * FS + s * SS] = y[2];
                fields[3 * FS + s * SS] = y[3];
                fields[4 * FS + s * SS] = y[4];
                fields[5 * FS + s * SS] = y[5];
                fields[6 * FS + s * SS] = y[7];
                fields[7 * FS + s * SS] = -dl;
                fields[8 * FS + s * SS] = sth;
                fields[9 * FS + s * SS] = cth;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k == pending) qstep[k] = steps;
                ++pending;
            }
        }
        c_pole += __popcll(__ballot(reflected));

        // ------------------------------------------------------------ evaluate queued samples
        unsigned total = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) total += __popcll(__ballot(pending > k));
        // a ray that ends with queued samples needs all of them now; a full queue needs one slot;
        // with the optical-depth-aware step every sample is needed before its ray's next step
        const bool ending = __ballot(status != RAY_RUNNING && pending > 0) != 0ull || (p.tau_step > 0.0 && total > 0);
        const bool full = __ballot(pending == K) != 0ull;
        if (ending || full || total >= 64) {
            // whole rounds when there are 64 or more (the oldest samples, so a full queue always
            // gets its first one evaluated), everything when a ray ends or fewer are queued
            const unsigned n_eval = (ending || total < 64) ? total : (total & ~63u);
            // select the oldest samples: queue layer k (each lane's k-th sample) before layer k + 1,
            // within a layer by lane; `take` of this lane's samples are evaluated
            int take = 0;
            unsigned listed = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const unsigned long long b = __ballot(pending > k);
                const unsigned rank = lane_rank(b);
                if (pending > k && listed + rank < n_eval) {
                    slot_map[listed + rank] = k * 64 + lane;
                    take = k + 1;
                }
                const unsigned c = __popcll(b);
                listed += (c < n_eval - listed) ? c : (n_eval - listed);
            }
            wave_lds_sync();
            if (FUSED) {
                // phase 1: lane i sets up sample i (fluid, frame, transfer) and leaves the set-up
                // in the sample's queue slot (K = 1: slot = owner lane, n_eval <= 64)
                bool zamo = false;
                if (lane < n_eval) {
                    const int s = slot_map[lane];
                    double q[N_FIELDS];
#pragma unroll
                    for (int f = 0; f < N_FIELDS; ++f) q[f] = fields[f * FS + s * SS];
                    Transfer<TT> tr;
                    zamo = setup_sample<TT>(p, q, lane_info(p, lane_job[s]), tr);
                    store_setup<TT, FS, SS>(fields, s, tr);
                }
                c_zamo += __popcll(__ballot(zamo));
                wave_lds_sync();
                // phase 2: `per` consecutive lanes share a sample, lane c of them taking its
                // frequencies [c n, (c + 1) n), n = ceil(n_nu / per): contribution, then the fold
                // I += exp(-tau) A, tau += dtau into the owner's row
                const unsigned per = n_eval >= 64 ? 1u : (64u / n_eval < (unsigned)NNU ? 64u / n_eval : (unsigned)NNU);
                const unsigned mul = (65535u + per) / per;   // x / per = (x mul) >> 16 for x < 1024
                const unsigned is = ((unsigned)lane * mul) >> 16;
                const unsigned chunk = (unsigned)lane - is * per;
                double tmin = 1e300, dtmax = 0.0;
                if (is < n_eval) {
                    const int s = slot_map[is];
                    const LaneInfo li = lane_info(p, lane_job[s]);
                    const int c = (int)(((unsigned)(li.n_nu + per - 1) * mul) >> 16);
                    const int f0 = (int)chunk * c;
                    const int f1 = (f0 + c < li.n_nu) ? f0 + c : li.n_nu;
                    Transfer<TT> tr;
                    load_setup<TT, FS, SS>(fields, s, tr);
                    double* Ir = res + s * RS;
                    double* Tr = Ir + NNU;
                    constexpr int G = NNU < FREQ_GROUP ? NNU : FREQ_GROUP;
                    int f = f0;
                    for (; f + G <= f1; f += G) {
                        double nu[G], A[G], dt[G], t0[G];
                        TT att[G];   // formed before the contributions, so that the chains overlap
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            nu[g] = p.nu[li.nu_base + f + g];
                            A[g] = 0.0;
                            dt[g] = 0.0;
                            t0[g] = Tr[f + g];
                            att[g] = attenuation<TT>(t0[g]);
                        }
                        tr.template contributions<G>(p, nu, G, A, dt);
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            Ir[f + g] = Ir[f + g] + (double)att[g] * A[g];
                            const double t1 = t0[g] + dt[g];
                            Tr[f + g] = t1;
                            tmin = ::fmin(tmin, t1);
                            dtmax = ::fmax(dtmax, dt[g]);
                        }
                    }
                    for (; f < f1; ++f) {   // the rest one at a time, in the branch-free form
                        double A = 0.0, dt = 0.0;
                        const double nu1 = p.nu[li.nu_base + f];
                        tr.template contributions<1, false>(p, &nu1, 1, &A, &dt);
                        const double t0 = Tr[f];
                        Ir[f] = Ir[f] + (double)attenuation<TT>(t0) * A;
                        const double t1 = t0 + dt;
                        Tr[f] = t1;
                        tmin = ::fmin(tmin, t1);
                        dtmax = ::fmax(dtmax, dt);
                    }
                }
                // the sample's smallest optical depth and largest step depth over its frequencies:
                // reduced over its `per` lanes onto the first, which leaves them in the slot's
                // queue fields 8 and 9 (the set-up is no longer read)
                for (unsigned off = 1; off < per; off <<= 1) {
                    const double tm = __shfl_down(tmin, off, 64), dm = __shfl_down(dtmax, off, 64);
                    if (chunk + off < per) {
                        tmin = ::fmin(tmin, tm);
                        dtmax = ::fmax(dtmax, dm);
                    }
                }
                if (is < n_eval && chunk == 0) {
                    const int s = slot_map[is];
                    fields[8 * FS + s * SS] = tmin;
                    fields[9 * FS + s * SS] = dtmax;
                }
            } else if (!MLPC && NNU > 1 && n_eval < 64) {
                // fewer samples than lanes: the (sample, frequency) pairs are spread over the
                // wave.  Lane i sets up sample i (fluid, frame, transfer) and leaves the set-up
                // in the sample's queue slot; then `per` lanes share each sample, lane c of them
                // taking its frequencies [c n, (c + 1) n), n = ceil(n_nu / per).
                bool zamo = false;
                if (lane < n_eval) {
                    const int s = slot_map[lane];
                    double q[N_FIELDS];
#pragma unroll
                    for (int f = 0; f < N_FIELDS; ++f) q[f] = fields[f * FS + s * SS];
                    Transfer<TT> tr;
                    zamo = setup_sample<TT>(p, q, lane_info(p, lane_job[s & 63]), tr);
                    store_setup<TT, FS, SS>(fields, s, tr);
                }
                c_zamo += __popcll(__ballot(zamo));
                wave_lds_sync();
                const unsigned per = (64u / n_eval < (unsigned)NNU) ? 64u / n_eval : (unsigned)NNU;
                const unsigned mul = (65535u + per) / per;   // x / per = (x mul) >> 16 for x < 1024
                const unsigned is = ((unsigned)lane * mul) >> 16;
                if (is < n_eval) {
                    const int s = slot_map[is];
                    const LaneInfo li = lane_info(p, lane_job[s & 63]);
                    const int c = (int)(((unsigned)(li.n_nu + per - 1) * mul) >> 16);
                    const int f0 = (int)((unsigned)lane - is * per) * c;
                    const int f1 = (f0 + c < li.n_nu) ? f0 + c : li.n_nu;
                    Transfer<TT> tr;
                    load_setup<TT, FS, SS>(fields, s, tr);
                    constexpr int G = NNU < FREQ_GROUP ? NNU : FREQ_GROUP;
                    for (int f = f0; f < f1; f += G) {
                        const int cnt = f1 - f;
                        double nu[G], A[G], dt[G];
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            nu[g] = g < cnt ? p.nu[li.nu_base + f + g] : 1.0;
                            A[g] = 0.0;
                            dt[g] = 0.0;
                        }
                        tr.template contributions<G>(p, nu, cnt, A, dt);
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            if (g < cnt) {
                                res[s * RS + f + g] = A[g];
                                res[s * RS + NNU + f + g] = dt[g];
                            }
                        }
                    }
                }
            } else
            for (unsigned r0 = 0; r0 < n_eval; r0 += 64) {
                const unsigned i = r0 + lane;
                if (MLPC) {
                    // every lane takes part in the network evaluations of the round
                    const bool has = i < n_eval;
                    const int s = has ? slot_map[i] : 0;
                    double q[N_FIELDS];
#pragma unroll
                    for (int f = 0; f < N_FIELDS; ++f) q[f] = has ? fields[f * FS + s * SS] : 1.0;
                    double A[NNU], dt[NNU];
                    eval_round_mlp<NNU, TT>(p, lds_net, has, q, lane_info(p, lane_job[s & 63]), A, dt, c_zamo,
                                            c_fallback, c_dropped);
                    if (has) {
#pragma unroll
                        for (int f = 0; f < NNU; ++f) {
                            res[s * RS + f] = A[f];
                            res[s * RS + NNU + f] = dt[f];
                        }
                    }
                } else {
                    bool zamo = false;
                    if (i < n_eval) {
                        const int s = slot_map[i];
                        double q[N_FIELDS];
#pragma unroll
                        for (int f = 0; f < N_FIELDS; ++f) q[f] = fields[f * FS + s * SS];
                        double A[NNU], dt[NNU];
                        zamo = eval_sample<NNU, TT>(p, q, lane_info(p, lane_job[s & 63]), A, dt);
#pragma unroll
                        for (int f = 0; f < NNU; ++f) {
                            res[s * RS + f] = A[f];
                            res[s * RS + NNU + f] = dt[f];
                        }
                    }
                    c_zamo += __popcll(__ballot(zamo));
                }
            }
            c_samples += n_eval;
            wave_lds_sync();
            // each owner folds its evaluated samples in order: I += exp(-tau) A, tau += dtau; with
            // the optical-depth cut-off the ray ends after the first sample that makes it opaque
            // at every frequency, and its later queued samples are dropped
            bool cut = false;
            if (FUSED && take > 0) {
                const int s = lane;   // K = 1
                if (p.tau_step > 0.0) rt_rate = fields[9 * FS + s * SS] / fields[7 * FS + s * SS];
                if (p.tau_cutoff > 0.0 && fields[8 * FS + s * SS] >= p.tau_cutoff) {
                    cut = true;
                    status = RAY_OPAQUE;
                    steps = qstep[0];
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!FUSED && k < take && !cut) {
                    const int s = k * 64 + lane;
                    double tmin = 1e300, dtmax = 0.0;
#pragma unroll
                    for (int f = 0; f < NNU; ++f) {
                        if (f < n_nu) {
                            I[f] = I[f] + (double)attenuation<TT>(tau[f]) * res[s * RS + f];
                            tau[f] = tau[f] + res[s * RS + NNU + f];
                            tmin = ::fmin(tmin, tau[f]);
                            dtmax = ::fmax(dtmax, res[s * RS + NNU + f]);
                        }
                    }
                    // d tau / d|lambda| of this sample (the last one folded sets the next step)
                    if (p.tau_step > 0.0) rt_rate = dtmax / fields[7 * FS + s * SS];
                    if (p.tau_cutoff > 0.0 && tmin >= p.tau_cutoff) {
                        cut = true;
                        status = RAY_OPAQUE;
                        steps = qstep[k];
                    }
                }
            }
            // move the samples left queued to the front of this lane's queue
            const int left = cut ? 0 : pending - take;
            if (K > 1 && take > 0) {
#pragma unroll
                for (int j = 0; j + 1 < K; ++j) {
                    if (j < left) {
#pragma unroll
                        for (int f = 0; f < N_FIELDS; ++f)
                            fields[f * FS + (j * 64 + lane) * SS] = fields[f * FS + ((j + take) * 64 + lane) * SS];
                    }
                }
#pragma unroll
                for (int j = 0; j + 1 < K; ++j) {
                    int v = qstep[j];
#pragma unroll
                    for (int m = 1; m < K; ++m)
                        if (m == take && j + m < K) v = qstep[j + m];
                    qstep[j] = v;
                }
            }
            pending = left;
            wave_lds_sync();
        }

        // ------------------------------------------------------------ finished rays
        if (status != RAY_RUNNING) {
            const DevJob& J = p.jobs[job];
            const long long npix = (long long)J.nx * J.ny;
            double* o = p.out + J.out_base + pix;
#pragma unroll
            for (int f = 0; f < NNU; ++f)
                if (f < n_nu) o[f * npix] = (status == RAY_NUMERIC) ? 0.0 : (FUSED ? res[lane * RS + f] : I[f]);
            if (p.ray_status) p.ray_status[J.pix_base + pix] = status;
            if (p.ray_steps) p.ray_steps[J.pix_base + pix] = steps;
            active = false;
        }
        const unsigned long long done = __ballot(status != RAY_RUNNING);
        if (done) {
            c_rays += __popcll(done);
            c_hor += __popcll(__ballot(status == RAY_HORIZON));
            c_esc += __popcll(__ballot(status == RAY_ESCAPED));
            c_max += __popcll(__ballot(status == RAY_MAXSTEP));
            c_num += __popcll(__ballot(status == RAY_NUMERIC));
            c_opq += __popcll(__ballot(status == RAY_OPAQUE));
        }
    }

    // ------------------------------------------------------------ statistics, one atomic per counter per wave
    if (lane == 0) {
        const unsigned long long st[ST_COUNT] = {c_rays, c_steps, c_samples, c_hor, c_esc, c_max, c_pole, c_num,
                                                 c_fallback, c_zamo, c_opq, c_dropped};
#pragma unroll
        for (int i = 0; i < ST_COUNT; ++i)
            if (st[i]) atomicAdd(p.stats + i, st[i]);
    }
}

// Flux density per (job, frequency): the sum of the job's image times the pixel solid angle
// and 1e23 (erg/s/cm^2/Hz -> Jy).  Pass 1: FLUX_SPLIT blocks per (job, frequency), block b
// summing the pixels b * 256 + t + k * 256 * FLUX_SPLIT of every thread t in order and
// combining its threads in a fixed tree.  Pass 2: one thread per (job, frequency) adds the
// FLUX_SPLIT partial sums in order.  The result does not depend on scheduling.

__global__ void __launch_bounds__(256) flux_partial_kernel(const DevJob* jobs, const double* out, double* part,
                                                           int max_nu)
{
    const int b = blockIdx.x % FLUX_SPLIT;
    const int jf = blockIdx.x / FLUX_SPLIT;
    const int job = jf / max_nu, f = jf % max_nu;
    const DevJob& J = jobs[job];
    __shared__ double red[256];
    double s = 0.0;
    if (f < J.n_nu) {
        const long long npix = (long long)J.nx * J.ny;
        const double* img = out + J.out_base + f * npix;
        for (long long i = (long long)b * 256 + threadIdx.x; i < npix; i += 256ll * FLUX_SPLIT) s += img[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void flux_final_kernel(const DevJob* jobs, const double* part, const double* pix_sr, double* flux,
                                  int n_jobs, int max_nu)
{
    const int jf = blockIdx.x * blockDim.x + threadIdx.x;
    if (jf >= n_jobs * max_nu) return;
    const int job = jf / max_nu, f = jf % max_nu;
    if (f >= jobs[job].n_nu) return;
    double s = 0.0;
    for (int b = 0; b < FLUX_SPLIT; ++b) s += part[(size_t)jf * FLUX_SPLIT + b];
    flux[jf] = s * pix_sr[job] * 1e23;
}

__global__ void reset_kernel(unsigned int* tile_counter, unsigned long long* stats)
{
    if (threadIdx.x == 0) *tile_counter = 0u;
    if (threadIdx.x < ST_COUNT) stats[threadIdx.x] = 0ull;
}

// Instantiations: RK4 with every register budget (1, 2 or 3 waves per SIMD), the learned
// closure with 1 or 2, the second-order integrators with 2 or 3.
}  // namespace

int kernel_wpe(int wpe, bool mlpc, int integ)
{
    if (integ != INTEG_RK4) return wpe >= 3 ? 3 : 2;   // RK2 and Verlet: two or three waves per SIMD
    if (mlpc) return wpe >= 2 ? 2 : 1;
    return wpe >= 3 ? 3 : wpe == 2 ? 2 : 1;
}

namespace {

template <int NNU, class TT>
const void* symbol_of(int wpe, bool mlpc, int integ)
{
    const int w = kernel_wpe(wpe, mlpc, integ);
    if (integ == INTEG_RK2)
        return w == 3 ? (const void*)trace_kernel<NNU, TT, 3, false, INTEG_RK2>
                      : (const void*)trace_kernel<NNU, TT, 2, false, INTEG_RK2>;
    if (integ == INTEG_VERLET || integ == INTEG_VERLET_CORR)
        return w == 3 ? (const void*)trace_kernel<NNU, TT, 3, false, INTEG_VERLET>
                      : (const void*)trace_kernel<NNU, TT, 2, false, INTEG_VERLET>;
    if (mlpc)
        return w == 2 ? (const void*)trace_kernel<NNU, TT, 2, true, INTEG_RK4>
                      : (const void*)trace_kernel<NNU, TT, 1, true, INTEG_RK4>;
    return w == 3 ? (const void*)trace_kernel<NNU, TT, 3, false, INTEG_RK4>
         : w == 2 ? (const void*)trace_kernel<NNU, TT, 2, false, INTEG_RK4>
                  : (const void*)trace_kernel<NNU, TT, 1, false, INTEG_RK4>;
}

template <class TT>
const void* symbol_tt(int max_nu, int wpe, bool mlpc, int integ)
{
    if (max_nu <= 1) return symbol_of<1, TT>(wpe, mlpc, integ);
    if (max_nu <= 4) return symbol_of<4, TT>(wpe, mlpc, integ);
    if (max_nu <= 8) return symbol_of<8, TT>(wpe, mlpc, integ);
    if (max_nu <= 16) return symbol_of<16, TT>(wpe, mlpc, integ);
    return symbol_of<32, TT>(wpe, mlpc, integ);
}

}  // namespace

hipError_t launch_reset(unsigned int* tile_counter, unsigned long long* stats, hipStream_t st)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, st, tile_counter, stats);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceParams& p, int max_nu, bool fp32, int wpe, int blocks, int threads, hipStream_t st)
{
    const void* fn = trace_kernel_symbol(max_nu, fp32, wpe, p.closure >= CL_MLP, p.integrator);
    void* args[] = {const_cast<TraceParams*>(&p)};
    return hipLaunchKernel(fn, dim3(blocks), dim3(threads), args,
                           trace_kernel_lds(max_nu, fp32, wpe, threads, p.closure >= CL_MLP, p.integrator,
                                            p.rays_per_wave),
                           st);
}

size_t flux_partials(int n_jobs, int max_nu) { return (size_t)n_jobs * max_nu * FLUX_SPLIT; }

hipError_t launch_flux(const DevJob* jobs, int n_jobs, const double* out, const double* pix_sr, double* part,
                       double* flux, int max_nu, hipStream_t st)
{
    hipLaunchKernelGGL(flux_partial_kernel, dim3(n_jobs * max_nu * FLUX_SPLIT), dim3(256), 0, st, jobs, out, part,
                       max_nu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = n_jobs * max_nu;
    hipLaunchKernelGGL(flux_final_kernel, dim3((n + 255) / 256), dim3(256), 0, st, jobs, part, pix_sr, flux, n_jobs,
                       max_nu);
    return hipGetLastError();
}

// Visit the queue type of the instantiation that trace_kernel_symbol picks for the same arguments.
template <class F>
auto with_queue(int max_nu, bool fp32, int wpe, bool mlpc, int integ, F f)
{
    const int w = kernel_wpe(wpe, mlpc, integ);
    auto per_w = [&](auto tt, auto m, auto w) {
        using TT = decltype(tt);
        constexpr bool M = decltype(m)::value;
        constexpr int W = decltype(w)::value;
        if (max_nu <= 1) return f(Queue<1, TT, M, W>{});
        if (max_nu <= 4) return f(Queue<4, TT, M, W>{});
        if (max_nu <= 8) return f(Queue<8, TT, M, W>{});
        if (max_nu <= 16) return f(Queue<16, TT, M, W>{});
        return f(Queue<32, TT, M, W>{});
    };
    auto per_q = [&](auto tt, auto m) {
        return w == 3 ? per_w(tt, m, std::integral_constant<int, 3>{}) : per_w(tt, m, std::integral_constant<int, 2>{});
    };
    auto per = [&](auto tt) { return mlpc ? per_q(tt, std::true_type{}) : per_q(tt, std::false_type{}); };
    return fp32 ? per(0.0f) : per(0.0);
}

bool trace_kernel_one_slot(int max_nu, bool fp32, int wpe, bool mlpc, int integ)
{
    return !mlpc && max_nu > 1 && with_queue(max_nu, fp32, wpe, mlpc, integ, [](auto q) { return decltype(q)::K == 1; });
}

size_t trace_kernel_lds(int max_nu, bool fp32, int wpe, int threads, bool mlpc, int integ, int rays)
{
    const size_t per_wave =
        with_queue(max_nu, fp32, wpe, mlpc, integ, [&](auto q) { return decltype(q)::per_wave(rays); });
    return (size_t)(threads / 64) * per_wave + (mlpc ? (size_t)mlp::LDS_NET_BYTES : 0);
}

const void* trace_kernel_symbol(int max_nu, bool fp32, int wpe, bool mlpc, int integ)
{
    return fp32 ? symbol_tt<float>(max_nu, wpe, mlpc, integ) : symbol_tt<double>(max_nu, wpe, mlpc, integ);
}

hipError_t trace_kernel_attributes(int max_nu, bool fp32, int wpe, bool mlpc, int integ, int* vgprs,
                                   int* spill_bytes, int* max_threads)
{
    hipFuncAttributes at;
    const hipError_t e = hipFuncGetAttributes(&at, trace_kernel_symbol(max_nu, fp32, wpe, mlpc, integ));
    if (e != hipSuccess) return e;
    if (vgprs) *vgprs = at.numRegs;
    if (spill_bytes) *spill_bytes = (int)at.localSizeBytes;
    if (max_threads) *max_threads = at.maxThreadsPerBlock;
    return hipSuccess;
}
