// host.cpp -- the C ABI (include/raptor.h): context, validation, grid upload, job tables,
// kernel launches, deterministic flux reduction, statistics and the work-per-unit count.
#include "raptor.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "context.hpp"
#include "device_types.hpp"
#include "ks_geodesic.hpp"
#include "launch.hpp"
#include "plasma.hpp"

namespace rt {
OpTally g_tally;
}

namespace rctx {

raptor_status fail(raptor_ctx* ctx, raptor_status s, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    return s;
}

raptor_status dev_fail(raptor_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? RAPTOR_E_NOMEM : RAPTOR_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace rctx

namespace {

using namespace rctx;
thread_local std::string t_create_error;

// Octave table of ln K2(1/Theta) (see K2Table) from the C++17 library Bessel functions:
// Theta in [2^-7, 2^14] (21 octaves of 256 intervals, 168 KiB, L2-resident).  The derivative
// with respect to u = ln Theta is x K1/K2 + 2 (x = 1/Theta); on the interval [m_j, m_j+1] of
// an octave, du/ds = 1/(nsub + j + s).  Cubic Hermite error in ln K2 (host check against the
// library function): 9e-10 for Theta in [0.01, 0.1], 1.2e-10 in [0.1, 1], 2e-11 above 1.
void k2_entry(int e, int nsub, int j, double4* out)
{
    auto at = [&](int jj, double* f, double* g) {
        const double th = std::ldexp(0.5 + jj / (2.0 * nsub), e);
        const double x = 1.0 / th;
        const double k1 = std::cyl_bessel_k(1.0, x), k2 = std::cyl_bessel_k(2.0, x);
        *f = std::log(k2);
        *g = (x * k1 / k2 + 2.0) / (nsub + jj);
    };
    at(j, &out->x, &out->y);
    at(j + 1, &out->z, &out->w);
}

raptor_status build_k2_table(raptor_ctx* ctx)
{
    const int e_lo = -6, n_oct = 21, nsub = 256;
    const int n = n_oct * nsub;
    std::vector<double4> h(n);
    for (int o = 0; o < n_oct; ++o)
        for (int j = 0; j < nsub; ++j) k2_entry(e_lo + o, nsub, j, &h[o * nsub + j]);
    RAPTOR_CK(ctx->k2.reserve(n), "allocating the K2 table");
    RAPTOR_CK(hipMemcpy(ctx->k2.p, h.data(), n * sizeof(double4), hipMemcpyHostToDevice), "uploading the K2 table");
    ctx->k2t.tab = ctx->k2.p;
    ctx->k2t.e_lo = e_lo;
    ctx->k2t.n_oct = n_oct;
    ctx->k2t.nsub = nsub;
    ctx->k2t.th_lo = std::ldexp(0.5, e_lo);
    ctx->k2t.th_hi = std::nextafter(std::ldexp(0.5, e_lo + n_oct), 0.0);
    return RAPTOR_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

raptor_status check_opts(raptor_ctx* ctx, const raptor_opts* o)
{
    if (!o) return fail(ctx, RAPTOR_E_INVALID, "opts is NULL");
    if (!finite_pos(o->eps) || o->eps > 1.0) return fail(ctx, RAPTOR_E_INVALID, "eps must be in (0, 1]");
    if (!(std::isfinite(o->r_stop_factor) && o->r_stop_factor >= 1.0))
        return fail(ctx, RAPTOR_E_INVALID, "r_stop_factor must be >= 1");
    if (o->max_steps < 1) return fail(ctx, RAPTOR_E_INVALID, "max_steps must be >= 1");
    if (o->transfer_prec != RAPTOR_F32 && o->transfer_prec != RAPTOR_F64)
        return fail(ctx, RAPTOR_E_INVALID, "transfer_prec must be RAPTOR_F32 or RAPTOR_F64");
    if (o->closure < RAPTOR_CLOSURE_EXACT || o->closure > RAPTOR_CLOSURE_MLP_BF16)
        return fail(ctx, RAPTOR_E_INVALID, "unknown closure");
    if (o->closure >= RAPTOR_CLOSURE_MLP && !ctx->mlp.ready)
        return fail(ctx, RAPTOR_E_INVALID, "the MLP closure needs parameters (raptor_mlp_init / set / train)");
    if (o->slow_light != 0 && o->slow_light != 1) return fail(ctx, RAPTOR_E_INVALID, "slow_light must be 0 or 1");
    if (o->mem != RAPTOR_MEM_HOST && o->mem != RAPTOR_MEM_DEVICE) return fail(ctx, RAPTOR_E_INVALID, "unknown mem");
    if (o->launch != RAPTOR_LAUNCH_DIRECT && o->launch != RAPTOR_LAUNCH_GRAPH)
        return fail(ctx, RAPTOR_E_INVALID, "unknown launch mode");
    if (o->integrator < RAPTOR_RK4 || o->integrator > RAPTOR_VERLET_CORRECTED)
        return fail(ctx, RAPTOR_E_INVALID, "unknown integrator");
    if (!(std::isfinite(o->tau_cutoff) && o->tau_cutoff >= 0.0))
        return fail(ctx, RAPTOR_E_INVALID, "tau_cutoff must be finite and >= 0");
    if (!(std::isfinite(o->tau_step) && o->tau_step >= 0.0))
        return fail(ctx, RAPTOR_E_INVALID, "tau_step must be finite and >= 0");
    if (o->integrator != RAPTOR_RK4 && o->closure >= RAPTOR_CLOSURE_MLP)
        return fail(ctx, RAPTOR_E_UNSUPPORTED, "the learned closure runs with the RK4 integrator only");
    if (!finite_pos(o->mass_msun) || !finite_pos(o->dist_pc))
        return fail(ctx, RAPTOR_E_INVALID, "mass_msun and dist_pc must be positive");
    if (o->metric_mass != 0.0 && o->metric_mass != 1.0) return fail(ctx, RAPTOR_E_INVALID, "metric_mass must be 0 or 1");
    if (o->closure == RAPTOR_CLOSURE_CONST && !(std::isfinite(o->const_j) && std::isfinite(o->const_alpha) &&
                                                o->const_j >= 0.0 && o->const_alpha >= 0.0))
        return fail(ctx, RAPTOR_E_INVALID, "const_j and const_alpha must be finite and >= 0");
    return RAPTOR_OK;
}

raptor_status check_camera(raptor_ctx* ctx, const raptor_camera* c, const raptor_grid* g, const raptor_opts* o, int k)
{
    char buf[160];
    if (!c) return fail(ctx, RAPTOR_E_INVALID, "camera is NULL");
    if (!g) return fail(ctx, RAPTOR_E_INVALID, "grid is NULL");
    if (g->owner != ctx) return fail(ctx, RAPTOR_E_INVALID, "grid belongs to another context");
    const double M = o->metric_mass;
    if (!(std::isfinite(c->spin) && std::fabs(c->spin) < 1.0) || (M == 0.0 && c->spin != 0.0)) {
        std::snprintf(buf, sizeof buf, "camera %d: spin must satisfy |a| < 1 (and a = 0 in flat space)", k);
        return fail(ctx, RAPTOR_E_INVALID, buf);
    }
    if (!(c->incl_deg > 0.0 && c->incl_deg < 180.0)) {
        std::snprintf(buf, sizeof buf, "camera %d: inclination must be in (0, 180) degrees", k);
        return fail(ctx, RAPTOR_E_INVALID, buf);
    }
    const double rh = M + std::sqrt(std::max(M * M - c->spin * c->spin, 0.0));
    if (!(std::isfinite(c->r_cam) && c->r_cam > g->d.r_out && c->r_cam > o->r_stop_factor * rh)) {
        std::snprintf(buf, sizeof buf, "camera %d: r_cam must exceed the grid's r_out and the stop radius", k);
        return fail(ctx, RAPTOR_E_INVALID, buf);
    }
    if (!finite_pos(c->fov_half)) return fail(ctx, RAPTOR_E_INVALID, "fov_half must be positive");
    if (c->nx < 1 || c->ny < 1 || c->nx > 65536 || c->ny > 65536) {
        std::snprintf(buf, sizeof buf, "camera %d: nx, ny must be in [1, 65536]", k);
        return fail(ctx, RAPTOR_E_INVALID, buf);
    }
    if (!std::isfinite(c->t_frame)) return fail(ctx, RAPTOR_E_INVALID, "t_frame must be finite");
    return RAPTOR_OK;
}

bool plan_valid(const raptor_plan& p)
{
    const bool tw = p.tile_width == 8 || p.tile_width == 16 || p.tile_width == 32 || p.tile_width == 64;
    const bool rw = p.rays_per_wave == 0 || p.rays_per_wave == 16 || p.rays_per_wave == 32 || p.rays_per_wave == 64;
    return (p.threads == 64 || p.threads == 128 || p.threads == 256 || p.threads == 512) && p.blocks_per_cu >= 0 &&
           p.blocks_per_cu <= 64 && p.refill_threshold >= 1 && p.refill_threshold <= 64 && tw && rw &&
           (p.min_waves_per_simd >= 1 && p.min_waves_per_simd <= 3);
}

// Rays per wave and tile width a launch of this plan uses: fewer than 64 rays only where the
// instantiation that runs (frequency class, precision, closure class, integrator) keeps one
// sample per lane, and a tile no wider than the rays.
struct Geometry {
    int rays, tile_w;
};
Geometry launch_geometry(const raptor_plan& p, int n_nu, bool fp32, bool mlpc, int integ)
{
    Geometry g{64, p.tile_width};
    if ((p.rays_per_wave == 16 || p.rays_per_wave == 32) &&
        trace_kernel_one_slot(n_nu, fp32, p.min_waves_per_simd, mlpc, integ))
        g.rays = p.rays_per_wave;
    if (g.tile_w > g.rays) g.tile_w = g.rays;
    return g;
}

int plan_key(int n_nu, bool fp32, bool mlpc)
{
    const int nnu = n_nu <= 1 ? 1 : n_nu <= 4 ? 4 : n_nu <= 8 ? 8 : n_nu <= 16 ? 16 : 32;
    return (nnu * 2 + (fp32 ? 1 : 0)) * 2 + (mlpc ? 1 : 0);
}

// Resolve the work-group count of a plan: blocks_per_cu per compute unit, or as many as are
// resident at once when 0.
raptor_status resolve_plan(raptor_ctx* ctx, int max_nu, bool fp32, LaunchPlan* pl, bool mlpc = false)
{
    // the work-group size the instantiation allows (512 lanes only for the learned closure's
    // 2-waves-per-SIMD variant)
    int regs = 0, spill = 0, max_threads = 0;
    RAPTOR_CK(trace_kernel_attributes(max_nu, fp32, pl->p.min_waves_per_simd, mlpc, INTEG_RK4, &regs, &spill,
                                      &max_threads),
              "reading kernel attributes");
    while (pl->p.threads > 64 && pl->p.threads > max_threads) pl->p.threads /= 2;
    // rays per wave and tile width as the RK4 instantiation runs them (64 rays where it keeps
    // more than one sample per lane)
    const Geometry g = launch_geometry(pl->p, max_nu, fp32, mlpc, INTEG_RK4);
    pl->p.rays_per_wave = g.rays;
    pl->p.tile_width = g.tile_w;
    auto lds = [&]() {
        return trace_kernel_lds(max_nu, fp32, pl->p.min_waves_per_simd, pl->p.threads, mlpc, INTEG_RK4, g.rays);
    };
    // the per-wave sample queue lives in LDS: shrink the work-group until it fits
    while (pl->p.threads > 64 && lds() > ctx->lds_per_block) pl->p.threads /= 2;
    if (lds() > ctx->lds_per_block)
        return fail(ctx, RAPTOR_E_UNSUPPORTED, "the sample queue of one wave exceeds the LDS of a work-group");
    int per_cu = pl->p.blocks_per_cu;
    if (per_cu == 0) {
        RAPTOR_CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, trace_kernel_symbol(max_nu, fp32, pl->p.min_waves_per_simd, mlpc), pl->p.threads,
                      lds()),
                  "querying occupancy");
        per_cu = std::max(per_cu, 1);
    }
    pl->blocks = ctx->cu_count * per_cu;
    return RAPTOR_OK;
}

// The plan of (frequency class, precision, closure class): the installed one, else the default,
// which is then installed unless `install` is false (the no-allocation entry point resolves the
// default without adding it to the context's plan map).
raptor_status plan_for(raptor_ctx* ctx, int max_nu, bool fp32, LaunchPlan* out, bool mlpc = false, bool install = true)
{
    const int key = plan_key(max_nu, fp32, mlpc);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
        *out = it->second;
        return RAPTOR_OK;
    }
    LaunchPlan pl;
    if (mlpc) {
        pl.p.threads = 512;   // eight waves share one LDS copy of the network
    } else {
        // the most waves per SIMD whose instantiation holds its registers without scratch
        for (int w = 3; w >= 1; --w) {
            int regs = 0, spill = 0, maxt = 0;
            RAPTOR_CK(trace_kernel_attributes(max_nu, fp32, w, false, INTEG_RK4, &regs, &spill, &maxt),
                      "reading kernel attributes");
            pl.p.min_waves_per_simd = w;
            if (spill == 0) break;
        }
    }
    raptor_status s = resolve_plan(ctx, max_nu, fp32, &pl, mlpc);
    if (s != RAPTOR_OK) return s;
    if (install) ctx->plans[key] = pl;
    *out = pl;
    return RAPTOR_OK;
}

// The device work of a call as a HIP graph: reset, trace and flux kernels captured on the
// capture-only stream (nothing runs during capture) and replayed on the context's stream.  The
// graph is kept while later calls make the identical launch -- same kernel arguments (every
// buffer pointer and the job count included), frequency class, precision and plan -- and
// captured again otherwise.  It holds kernel nodes only; the uploads before it are ordinary
// stream-ordered copies.
raptor_status launch_graph(raptor_ctx* ctx, const TraceParams& p, int n_nu, bool fp32, const LaunchPlan& plan, int nj,
                           double* out)
{
    struct Key {
        TraceParams p;
        int n_nu, fp32, wpe, blocks, threads, nj;
        const double* out;
        const double* pixsr;
        double* flux;
        double* flux_part;
    } k;
    std::memset(&k, 0, sizeof k);
    k.p = p;
    k.n_nu = n_nu;
    k.fp32 = fp32;
    k.wpe = plan.p.min_waves_per_simd;
    k.blocks = plan.blocks;
    k.threads = plan.p.threads;
    k.nj = nj;
    k.out = out;
    k.pixsr = ctx->pixsr.p;
    k.flux = ctx->flux.p;
    k.flux_part = ctx->flux_part.p;
    const unsigned char* kb = reinterpret_cast<const unsigned char*>(&k);
    const bool same = ctx->graph && ctx->graph_key.size() == sizeof k &&
                      std::memcmp(ctx->graph_key.data(), kb, sizeof k) == 0;
    if (!same) {
        if (ctx->graph) {
            RAPTOR_CK(hipGraphExecDestroy(ctx->graph), "releasing the previous graph");
            ctx->graph = nullptr;
        }
        ctx->graph_key.clear();
        hipStream_t cs = ctx->cap_stream;
        RAPTOR_CK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "starting graph capture");
        hipError_t e = launch_reset(ctx->counter.p, ctx->stats.p, cs);
        if (e == hipSuccess) e = launch_trace(p, n_nu, fp32, plan.p.min_waves_per_simd, plan.blocks, plan.p.threads, cs);
        if (e == hipSuccess) e = launch_flux(ctx->jobs.p, nj, out, ctx->pixsr.p, ctx->flux_part.p, ctx->flux.p, n_nu, cs);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);   // always end the capture
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return dev_fail(ctx, e, "capturing the launch");
        }
        RAPTOR_CK(e2, "ending graph capture");
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        RAPTOR_CK(e, "instantiating the graph");
        ctx->graph = ge;
        ctx->graph_key.assign(kb, kb + sizeof k);
    }
    hipStream_t s = ctx->stream;
    RAPTOR_CK(hipEventRecord(ctx->ev0, s), "recording an event");
    RAPTOR_CK(hipGraphLaunch(ctx->graph, s), "launching the graph");
    RAPTOR_CK(hipEventRecord(ctx->ev1, s), "recording an event");
    return RAPTOR_OK;
}

// Host-side tables of a launch: one DevJob per image, the distinct grids (with this call's
// code-unit scales), the frequencies and the pixel solid angles.  The arrays belong to the
// caller (capacities: nj, nj, nj, nj * n_nu, nj).
struct HostTables {
    DevJob* jobs;
    DevGrid* grids;
    const raptor_grid** gl;
    double* nus;
    double* pixsr;
    int n_grids = 0;
    long long tiles = 0, outn = 0, pixn = 0;
};

raptor_status fill_tables(raptor_ctx* ctx, const JobIn* in, int nj, int n_nu, const raptor_opts* o, int tile_w,
                          int rays, HostTables* t)
{
    const int tile_h = rays / tile_w;
    const double M = o->metric_mass;
    const double Lu = kG * o->mass_msun * kMsun / (kC * kC);
    const double D = o->dist_pc * kPc;
    t->n_grids = 0;
    t->tiles = t->outn = t->pixn = 0;
    for (int k = 0; k < nj; ++k) {
        const raptor_camera& c = *in[k].cam;
        DevJob& J = t->jobs[k];
        std::memset(&J, 0, sizeof J);
        J.a = c.spin;
        J.incl = c.incl_deg * kPi / 180.0;
        J.sin_i = std::sqrt(1.0 - std::cos(J.incl) * std::cos(J.incl));
        J.cos_i = std::cos(J.incl);
        J.r_cam = c.r_cam;
        J.fov = c.fov_half;
        J.dalpha = 2.0 * c.fov_half / c.nx;
        J.dbeta = 2.0 * c.fov_half / c.ny;
        J.r_stop = o->r_stop_factor * (M + std::sqrt(std::max(M * M - c.spin * c.spin, 0.0)));
        J.t_init = c.t_frame + c.r_cam;
        J.nx = c.nx;
        J.ny = c.ny;
        J.tiles_x = (c.nx + tile_w - 1) / tile_w;
        J.n_nu = n_nu;
        J.tile_base = t->tiles;
        J.out_base = t->outn;
        J.pix_base = t->pixn;
        t->tiles += (long long)J.tiles_x * ((c.ny + tile_h - 1) / tile_h);
        t->outn += (long long)n_nu * c.nx * c.ny;
        t->pixn += (long long)c.nx * c.ny;
        int gi = 0;
        while (gi < t->n_grids && t->gl[gi] != in[k].grid) ++gi;
        if (gi == t->n_grids) t->gl[t->n_grids++] = in[k].grid;
        J.grid = gi;
        const DevGrid& G = in[k].grid->d;
        int fs = 0;
        if (G.n_snap > 1) {
            fs = (int)std::floor((c.t_frame - G.t0) / G.dt_snap + 0.5);
            fs = std::min(std::max(fs, 0), G.n_snap - 1);
        }
        J.fast_snap = fs;
        J.nu_base = k * n_nu;
        for (int f = 0; f < n_nu; ++f) t->nus[k * n_nu + f] = in[k].nu[f];
        t->pixsr[k] = J.dalpha * J.dbeta * Lu * Lu / (D * D);
    }
    if (t->tiles >= (1ll << 31) - 1) return fail(ctx, RAPTOR_E_RANGE, "too many pixels in one call");
    for (int i = 0; i < t->n_grids; ++i) {
        t->grids[i] = t->gl[i]->d;
        if (t->grids[i].units) {
            // code-unit scales of this call's black-hole mass: rho0 = M / L^3
            const double rho0 = t->gl[i]->mass_unit_g / (Lu * Lu * Lu);
            t->grids[i].ne_scale = rho0 / (pl::ME_CGS + pl::MP_CGS);
            t->grids[i].b_scale = kC * std::sqrt(4.0 * kPi * rho0);
        }
    }
    return RAPTOR_OK;
}

// Device buffers of a launch: the tables, the outputs the kernels write, the tile counter and
// the statistics.
struct DevTables {
    DevJob* jobs;
    DevGrid* grids;
    double* nu;
    double* pixsr;
    double* flux;
    double* flux_part;
    unsigned int* counter;
    unsigned long long* stats;
    double* out;
    int* rs;
    int* rn;
};

// Upload the tables, launch (reset, trace, flux; direct or as a replayed graph), copy the
// outputs the caller wants where it wants them, wait, and fill the statistics.
raptor_status launch_tables(raptor_ctx* ctx, const HostTables& h, const DevTables& d, int nj, int n_nu,
                            const raptor_opts* o, const LaunchPlan& plan, double* images, double* flux_jy,
                            int32_t* ray_status, int32_t* ray_steps, raptor_stats* st)
{
    const bool dev = o->mem == RAPTOR_MEM_DEVICE;
    const bool fp32 = o->transfer_prec == RAPTOR_F32;
    const Geometry geo = launch_geometry(plan.p, n_nu, fp32, o->closure >= RAPTOR_CLOSURE_MLP, o->integrator);
    const int tile_w = geo.tile_w;
    hipStream_t s = ctx->stream;
    RAPTOR_CK(hipMemcpyAsync(d.jobs, h.jobs, nj * sizeof(DevJob), hipMemcpyHostToDevice, s), "uploading jobs");
    RAPTOR_CK(hipMemcpyAsync(d.grids, h.grids, h.n_grids * sizeof(DevGrid), hipMemcpyHostToDevice, s),
              "uploading the grid table");
    RAPTOR_CK(hipMemcpyAsync(d.nu, h.nus, (size_t)nj * n_nu * sizeof(double), hipMemcpyHostToDevice, s),
              "uploading frequencies");
    RAPTOR_CK(hipMemcpyAsync(d.pixsr, h.pixsr, nj * sizeof(double), hipMemcpyHostToDevice, s),
              "uploading solid angles");

    TraceParams p;
    std::memset(&p, 0, sizeof p);   // padding included: the graph key compares the bytes
    p.jobs = d.jobs;
    p.grids = d.grids;
    p.nu = d.nu;
    p.out = d.out;
    p.ray_status = d.rs;
    p.ray_steps = d.rn;
    p.tile_counter = d.counter;
    p.stats = d.stats;
    p.k2 = ctx->k2t;
    p.n_tiles = h.tiles;
    p.n_jobs = nj;
    p.max_steps = o->max_steps;
    p.closure = o->closure;
    p.slow_light = o->slow_light;
    p.integrator = o->integrator;
    p.eps = o->eps;
    p.M = o->metric_mass;
    p.length_unit = kG * o->mass_msun * kMsun / (kC * kC);
    p.const_j = o->const_j;
    p.const_alpha = o->const_alpha;
    p.tau_cutoff = o->tau_cutoff;
    p.tau_step = o->tau_step;
    p.mlp_P = ctx->mlp.P.p;
    p.mlp_W = ctx->mlp.W.p;
    p.mlp_Wlo = ctx->mlp.Wlo.p;
    p.refill_threshold = plan.p.refill_threshold;
    p.tile_shift = tile_w == 8 ? 3 : tile_w == 16 ? 4 : tile_w == 32 ? 5 : 6;
    p.rays_per_wave = geo.rays;
    p.rays_shift = geo.rays == 16 ? 4 : geo.rays == 32 ? 5 : 6;

    if (o->launch == RAPTOR_LAUNCH_GRAPH) {
        raptor_status gs = launch_graph(ctx, p, n_nu, fp32, plan, nj, d.out);
        if (gs != RAPTOR_OK) return gs;
    } else {
        RAPTOR_CK(launch_reset(d.counter, d.stats, s), "launching reset");
        RAPTOR_CK(hipEventRecord(ctx->ev0, s), "recording an event");
        RAPTOR_CK(launch_trace(p, n_nu, fp32, plan.p.min_waves_per_simd, plan.blocks, plan.p.threads, s),
                  "launching the trace kernel");
        RAPTOR_CK(hipEventRecord(ctx->ev1, s), "recording an event");
        RAPTOR_CK(launch_flux(d.jobs, nj, d.out, d.pixsr, d.flux_part, d.flux, n_nu, s), "launching the flux reduction");
    }

    const hipMemcpyKind d2x = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (images && d.out != images)
        RAPTOR_CK(hipMemcpyAsync(images, d.out, h.outn * sizeof(double), d2x, s), "copying images");
    if (flux_jy && d.flux != flux_jy)
        RAPTOR_CK(hipMemcpyAsync(flux_jy, d.flux, (size_t)nj * n_nu * sizeof(double), d2x, s), "copying fluxes");
    if (ray_status && d.rs != ray_status)
        RAPTOR_CK(hipMemcpyAsync(ray_status, d.rs, h.pixn * sizeof(int), d2x, s), "copying ray status");
    if (ray_steps && d.rn != ray_steps)
        RAPTOR_CK(hipMemcpyAsync(ray_steps, d.rn, h.pixn * sizeof(int), d2x, s), "copying ray steps");
    unsigned long long hs[ST_COUNT];
    RAPTOR_CK(hipMemcpyAsync(hs, d.stats, sizeof hs, hipMemcpyDeviceToHost, s), "copying statistics");
    RAPTOR_CK(hipStreamSynchronize(s), "running the trace");
    if (st) {
        st->rays = hs[ST_RAYS];
        st->ray_steps = hs[ST_STEPS];
        st->samples = hs[ST_SAMPLES];
        st->n_horizon = hs[ST_HORIZON];
        st->n_escaped = hs[ST_ESCAPED];
        st->n_maxstep = hs[ST_MAXSTEP];
        st->n_pole = hs[ST_POLE];
        st->n_numeric = hs[ST_NUMERIC];
        st->n_mlp_fallback = hs[ST_MLP_FALLBACK];
        st->n_zamo_fallback = hs[ST_ZAMO];
        st->n_opaque = hs[ST_OPAQUE];
        st->n_mlp_dropped = hs[ST_MLP_DROPPED];
        float ms = 0.0f;
        RAPTOR_CK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "reading the kernel time");
        st->kernel_ms = ms;
    }
    return RAPTOR_OK;
}

raptor_status run_jobs(raptor_ctx* ctx, const JobIn* in, int nj, int n_nu, const raptor_opts* o, double* images,
                       double* flux_jy, int32_t* ray_status, int32_t* ray_steps, raptor_stats* st,
                       const LaunchPlan* force_plan = nullptr)
{
    const bool dev = o->mem == RAPTOR_MEM_DEVICE;
    const bool fp32 = o->transfer_prec == RAPTOR_F32;
    const bool mlpc = o->closure >= RAPTOR_CLOSURE_MLP;
    LaunchPlan plan;
    if (force_plan) {
        plan = *force_plan;
    } else {
        raptor_status ps = plan_for(ctx, n_nu, fp32, &plan, mlpc);
        if (ps != RAPTOR_OK) return ps;
    }
    std::vector<DevJob> jobs(nj);
    std::vector<DevGrid> grids(nj);
    std::vector<const raptor_grid*> gl(nj);
    std::vector<double> nus((size_t)nj * n_nu), pixsr(nj);
    HostTables h{jobs.data(), grids.data(), gl.data(), nus.data(), pixsr.data()};
    const Geometry geo = launch_geometry(plan.p, n_nu, o->transfer_prec == RAPTOR_F32,
                                         o->closure >= RAPTOR_CLOSURE_MLP, o->integrator);
    raptor_status fs = fill_tables(ctx, in, nj, n_nu, o, geo.tile_w, geo.rays, &h);
    if (fs != RAPTOR_OK) return fs;

    // ---- device buffers of the context, grown on demand
    RAPTOR_CK(ctx->jobs.reserve(nj), "allocating the job table");
    RAPTOR_CK(ctx->grids.reserve(h.n_grids), "allocating the grid table");
    RAPTOR_CK(ctx->nu.reserve((size_t)nj * n_nu), "allocating frequencies");
    RAPTOR_CK(ctx->pixsr.reserve(nj), "allocating solid angles");
    RAPTOR_CK(ctx->flux.reserve((size_t)nj * n_nu), "allocating fluxes");
    RAPTOR_CK(ctx->flux_part.reserve(flux_partials(nj, n_nu)), "allocating flux partial sums");
    DevTables d{ctx->jobs.p, ctx->grids.p, ctx->nu.p, ctx->pixsr.p, ctx->flux.p, ctx->flux_part.p,
                ctx->counter.p, ctx->stats.p, nullptr, nullptr, nullptr};
    if (dev && images) {
        d.out = images;
    } else {
        RAPTOR_CK(ctx->out.reserve(h.outn), "allocating intensities");
        d.out = ctx->out.p;
    }
    if (ray_status || ray_steps) {
        if (dev) {
            d.rs = ray_status;
            d.rn = ray_steps;
        } else {
            RAPTOR_CK(ctx->status.reserve(h.pixn), "allocating ray info");
            RAPTOR_CK(ctx->steps.reserve(h.pixn), "allocating ray info");
            d.rs = ray_status ? ctx->status.p : nullptr;
            d.rn = ray_steps ? ctx->steps.p : nullptr;
        }
    }
    return launch_tables(ctx, h, d, nj, n_nu, o, plan, images, flux_jy, ray_status, ray_steps, st);
}

raptor_status check_nu(raptor_ctx* ctx, const double* nu, int n_nu)
{
    if (!nu) return fail(ctx, RAPTOR_E_INVALID, "nu_hz is NULL");
    if (n_nu < 1 || n_nu > RAPTOR_MAX_NU) return fail(ctx, RAPTOR_E_INVALID, "n_nu must be in [1, RAPTOR_MAX_NU]");
    for (int f = 0; f < n_nu; ++f)
        if (!finite_pos(nu[f])) return fail(ctx, RAPTOR_E_INVALID, "frequencies must be finite and > 0");
    return RAPTOR_OK;
}

}  // namespace

extern "C" {

raptor_status raptor_create(int device, void* hip_stream, raptor_ctx** out)
{
    t_create_error.clear();
    if (!out) {
        t_create_error = "out is NULL";
        return RAPTOR_E_INVALID;
    }
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
        t_create_error = "no HIP device";
        return RAPTOR_E_DEVICE;
    }
    if (device < 0 || device >= n) {
        t_create_error = "device index out of range";
        return RAPTOR_E_INVALID;
    }
    raptor_ctx* ctx = new raptor_ctx();
    ctx->device = device;
    auto bail = [&](raptor_status s) {
        t_create_error = ctx->err;
        raptor_destroy(ctx);
        return s;
    };
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return bail(dev_fail(ctx, e, "selecting the device"));
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(dev_fail(ctx, e, "creating a stream"));
        ctx->own_stream = true;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return bail(dev_fail(ctx, e, "reading device properties"));
    ctx->cu_count = prop.multiProcessorCount;
    ctx->lds_per_block = prop.sharedMemPerBlock;
    if ((e = hipEventCreate(&ctx->ev0)) != hipSuccess || (e = hipEventCreate(&ctx->ev1)) != hipSuccess)
        return bail(dev_fail(ctx, e, "creating events"));
    e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(dev_fail(ctx, e, "creating the capture stream"));
    if ((e = ctx->counter.reserve(1)) != hipSuccess || (e = ctx->stats.reserve(ST_COUNT)) != hipSuccess)
        return bail(dev_fail(ctx, e, "allocating counters"));
    raptor_status s = build_k2_table(ctx);
    if (s != RAPTOR_OK) return bail(s);
    // the no-allocation entry point's device scratch on this device (current) and its host tables
    e = noalloc_scratch_address(device, &ctx->noalloc_scratch);
    if (e != hipSuccess) return bail(dev_fail(ctx, e, "looking up the no-allocation scratch"));
    ctx->noalloc_host = new rctx::NoAllocHost();
    *out = ctx;
    return RAPTOR_OK;
}

void raptor_destroy(raptor_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (raptor_grid* g : ctx->live) {
        if (g->cells) (void)hipFree(g->cells);
        if (g->x2tab) (void)hipFree(g->x2tab);
        delete g;
    }
    ctx->jobs.release();
    ctx->grids.release();
    ctx->nu.release();
    ctx->flux_part.release();
    ctx->out.release();
    ctx->pixsr.release();
    ctx->flux.release();
    ctx->status.release();
    ctx->steps.release();
    ctx->counter.release();
    ctx->stats.release();
    ctx->k2.release();
    ctx->mlp.release();
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx->noalloc_host;
    delete ctx;
}

const char* raptor_last_error(const raptor_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : t_create_error.c_str();
}

raptor_status raptor_default_opts(raptor_opts* o)
{
    if (!o) return RAPTOR_E_INVALID;
    std::memset(o, 0, sizeof *o);
    o->eps = 0.05;
    o->r_stop_factor = 1.01;
    o->max_steps = 10000;
    o->transfer_prec = RAPTOR_F64;
    o->closure = RAPTOR_CLOSURE_EXACT;
    o->slow_light = 0;
    o->mem = RAPTOR_MEM_HOST;
    o->mass_msun = 4.5e6;
    o->dist_pc = 8500.0;
    o->metric_mass = 1.0;
    o->integrator = RAPTOR_RK4;
    return RAPTOR_OK;
}

raptor_status raptor_grid_upload(raptor_ctx* ctx, const raptor_grid_desc* d, raptor_grid** out)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!d || !out || !d->cells) return fail(ctx, RAPTOR_E_INVALID, "desc, desc->cells and out must be non-NULL");
    if (d->n1 < 2 || d->n2 < 2 || d->n_snap < 1) return fail(ctx, RAPTOR_E_INVALID, "need n1, n2 >= 2 and n_snap >= 1");
    if (d->dtype != RAPTOR_F32 && d->dtype != RAPTOR_F64) return fail(ctx, RAPTOR_E_INVALID, "unknown grid dtype");
    if ((double)d->n_snap * d->n2 * d->n1 >= 2147483647.0)
        return fail(ctx, RAPTOR_E_RANGE, "a grid holds fewer than 2^31 cells");
    if (!(finite_pos(d->r_in) && std::isfinite(d->r_out) && d->r_out > d->r_in))
        return fail(ctx, RAPTOR_E_INVALID, "need 0 < r_in < r_out");
    if (!(d->hslope > 0.0 && d->hslope <= 1.0)) return fail(ctx, RAPTOR_E_INVALID, "hslope must be in (0, 1]");
    if (d->n_snap > 1 && !finite_pos(d->dt_snap)) return fail(ctx, RAPTOR_E_INVALID, "dt_snap must be > 0");
    if (!std::isfinite(d->t0) || !std::isfinite(d->mod_amp) || !std::isfinite(d->a_gen))
        return fail(ctx, RAPTOR_E_INVALID, "t0, mod_amp and a_gen must be finite");
    if (d->units != RAPTOR_UNITS_CGS && d->units != RAPTOR_UNITS_CODE)
        return fail(ctx, RAPTOR_E_INVALID, "units must be RAPTOR_UNITS_CGS or RAPTOR_UNITS_CODE");
    if (d->units == RAPTOR_UNITS_CODE &&
        !(finite_pos(d->mass_unit_g) && finite_pos(d->r_low) && finite_pos(d->r_high) && d->gamma_ad > 1.0 &&
          d->gamma_ad <= 2.0))
        return fail(ctx, RAPTOR_E_INVALID, "code units need mass_unit_g, r_low, r_high > 0 and 1 < gamma_ad <= 2");
    *out = nullptr;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    const size_t cell = d->dtype == RAPTOR_F64 ? 4 * sizeof(double) : 4 * sizeof(float);
    const size_t bytes = (size_t)d->n_snap * d->n2 * d->n1 * cell;
    raptor_grid* g = new raptor_grid();
    hipError_t e = hipMalloc(&g->cells, bytes);
    if (e != hipSuccess) {
        delete g;
        return dev_fail(ctx, e, "allocating the grid");
    }
    e = hipMemcpy(g->cells, d->cells, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(g->cells);
        delete g;
        return dev_fail(ctx, e, "uploading the grid");
    }
    // The MKS inverse x2(theta) as a cubic Hermite table on uniform theta nodes (Newton on the
    // host), with the node count doubled from 4096 until the interpolation error, checked at three
    // points of every interval, is at most 1e-12; where 32768 nodes do not reach it (strongly
    // concentrated grids, hslope below ~0.2) the kernel refines the table value by Halley's
    // iteration.
    const double hh = 0.5 * (1.0 - d->hslope);
    auto solve = [&](double th) {
        double x = th / kPi;
        for (int it = 0; it < 100; ++it) {
            const double f = kPi * x + hh * std::sin(2.0 * kPi * x) - th;
            const double fp = kPi * (1.0 + 2.0 * hh * std::cos(2.0 * kPi * x));
            const double xn = std::min(std::max(x - f / fp, 0.0), 1.0);
            const bool done = std::fabs(xn - x) < 1e-16;
            x = xn;
            if (done) break;
        }
        return x;
    };
    std::vector<double2> x2h;
    int x2n = 4096, refine = 1;
    for (; x2n <= 32768; x2n *= 2) {
        const double dth = kPi / x2n;
        x2h.assign(x2n + 1, double2{0.0, 0.0});
        for (int i = 0; i <= x2n; ++i) {
            const double x = solve(dth * i);
            x2h[i].x = x;
            x2h[i].y = dth / (kPi * (1.0 + 2.0 * hh * std::cos(2.0 * kPi * x)));   // dx2/dtheta * dtheta
        }
        double worst = 0.0;
        for (int i = 0; i < x2n && worst <= 1e-12; ++i) {
            for (double s : {0.25, 0.5, 0.75}) {
                const double s2 = s * s, s3 = s2 * s;
                const double v = (2.0 * s3 - 3.0 * s2 + 1.0) * x2h[i].x + (s3 - 2.0 * s2 + s) * x2h[i].y +
                                 (-2.0 * s3 + 3.0 * s2) * x2h[i + 1].x + (s3 - s2) * x2h[i + 1].y;
                worst = std::max(worst, std::fabs(v - solve(dth * (i + s))));
            }
        }
        if (worst <= 1e-12) {
            refine = 0;
            break;
        }
        if (x2n == 32768) break;
    }
    e = hipMalloc(&g->x2tab, (x2n + 1) * sizeof(double2));
    if (e == hipSuccess)
        e = hipMemcpy(g->x2tab, x2h.data(), (x2n + 1) * sizeof(double2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (g->x2tab) (void)hipFree(g->x2tab);
        (void)hipFree(g->cells);
        delete g;
        return dev_fail(ctx, e, "uploading the MKS table");
    }
    DevGrid& G = g->d;
    G.cells = g->cells;
    G.x2tab = g->x2tab;
    G.x2n = x2n;
    G.x2_refine = refine;
    G.x2_inv_dth = x2n / kPi;
    G.n1 = d->n1;
    G.n2 = d->n2;
    G.n_snap = d->n_snap;
    G.is_f64 = d->dtype == RAPTOR_F64;
    G.lnr_in = std::log(d->r_in);
    G.inv_d1 = d->n1 / (std::log(d->r_out) - std::log(d->r_in));
    G.r_in = d->r_in;
    G.r_out = d->r_out;
    G.hslope = d->hslope;
    G.a_gen = d->a_gen;
    G.t0 = d->t0;
    G.dt_snap = d->n_snap > 1 ? d->dt_snap : 1.0;
    G.inv_dt = 1.0 / G.dt_snap;
    G.mod_amp = d->mod_amp;
    for (int m = 0; m < 4; ++m) {
        G.mod_cos[m] = std::cos(d->mod_phase[m]);
        G.mod_sin[m] = std::sin(d->mod_phase[m]);
    }
    G.units = d->units;
    if (d->units == RAPTOR_UNITS_CODE) {
        g->mass_unit_g = d->mass_unit_g;
        G.r_low = d->r_low;
        G.r_high = d->r_high;
        G.gam1 = d->gamma_ad - 1.0;
        G.thetae_fac = pl::MP_CGS / pl::ME_CGS * G.gam1;
    }
    g->owner = ctx;
    ctx->live.push_back(g);
    *out = g;
    return RAPTOR_OK;
}

void raptor_grid_release(raptor_ctx* ctx, raptor_grid* g)
{
    if (!ctx || !g) return;
    auto it = std::find(ctx->live.begin(), ctx->live.end(), g);
    if (it == ctx->live.end()) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (g->cells) (void)hipFree(g->cells);
    if (g->x2tab) (void)hipFree(g->x2tab);
    ctx->live.erase(it);
    delete g;
}

raptor_status raptor_trace_spectrum_ex(raptor_ctx* ctx, const raptor_camera* cam, const raptor_grid* grid,
                                       const raptor_opts* opts, const double* nu_hz, int32_t n_nu, double* images,
                                       double* flux_jy, int32_t* ray_status, int32_t* ray_steps, raptor_stats* stats)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    raptor_status s;
    if ((s = check_opts(ctx, opts)) != RAPTOR_OK) return s;
    if ((s = check_nu(ctx, nu_hz, n_nu)) != RAPTOR_OK) return s;
    if ((s = check_camera(ctx, cam, grid, opts, 0)) != RAPTOR_OK) return s;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    const JobIn in{cam, grid, nu_hz};
    return run_jobs(ctx, &in, 1, n_nu, opts, images, flux_jy, ray_status, ray_steps, stats);
}

raptor_status raptor_trace_spectrum(raptor_ctx* ctx, const raptor_camera* cam, const raptor_grid* grid,
                                    const raptor_opts* opts, const double* nu_hz, int32_t n_nu, double* images,
                                    double* flux_jy, raptor_stats* stats)
{
    return raptor_trace_spectrum_ex(ctx, cam, grid, opts, nu_hz, n_nu, images, flux_jy, nullptr, nullptr, stats);
}

raptor_status raptor_trace_image(raptor_ctx* ctx, const raptor_camera* cam, const raptor_grid* grid,
                                 const raptor_opts* opts, double nu_hz, double* image, double* flux_jy,
                                 raptor_stats* stats)
{
    return raptor_trace_spectrum_ex(ctx, cam, grid, opts, &nu_hz, 1, image, flux_jy, nullptr, nullptr, stats);
}

static raptor_status batch_inputs(raptor_ctx* ctx, const raptor_camera* cams, int32_t n_cams,
                                  const raptor_grid* const* grids, const raptor_opts* opts, const double* nu_hz,
                                  int32_t n_nu, JobIn* in)
{
    raptor_status s;
    for (int k = 0; k < n_cams; ++k) {
        if ((s = check_nu(ctx, nu_hz + (size_t)k * n_nu, n_nu)) != RAPTOR_OK) return s;
        if ((s = check_camera(ctx, &cams[k], grids[k], opts, k)) != RAPTOR_OK) return s;
        in[k] = {&cams[k], grids[k], nu_hz + (size_t)k * n_nu};
    }
    return RAPTOR_OK;
}

// The checks of a batch call before its inputs are read.
static raptor_status batch_precheck(raptor_ctx* ctx, const raptor_camera* cams, int32_t n_cams,
                                    const raptor_grid* const* grids, const raptor_opts* opts, const double* nu_hz)
{
    raptor_status s;
    if (!cams || !grids || n_cams < 1) return fail(ctx, RAPTOR_E_INVALID, "need n_cams >= 1 cameras and grids");
    if ((s = check_opts(ctx, opts)) != RAPTOR_OK) return s;
    if (!nu_hz) return fail(ctx, RAPTOR_E_INVALID, "nu_hz is NULL");
    return RAPTOR_OK;
}

raptor_status raptor_trace_batch(raptor_ctx* ctx, const raptor_camera* cams, int32_t n_cams,
                                 const raptor_grid* const* grids, const raptor_opts* opts, const double* nu_hz,
                                 int32_t n_nu, double* images, double* flux_jy, raptor_stats* stats)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    raptor_status s = batch_precheck(ctx, cams, n_cams, grids, opts, nu_hz);
    if (s != RAPTOR_OK) return s;
    std::vector<JobIn> in(n_cams);
    s = batch_inputs(ctx, cams, n_cams, grids, opts, nu_hz, n_nu, in.data());
    if (s != RAPTOR_OK) return s;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    return run_jobs(ctx, in.data(), n_cams, n_nu, opts, images, flux_jy, nullptr, nullptr, stats);
}

raptor_status raptor_trace_batch_noalloc(raptor_ctx* ctx, const raptor_camera* cams, int32_t n_cams,
                                         const raptor_grid* const* grids, const raptor_opts* opts, const double* nu_hz,
                                         int32_t n_nu, double* images, double* flux_jy, raptor_stats* stats)
{
    static_assert(rctx::NOALLOC_JOBS == NOALLOC_MAX_JOBS && RAPTOR_NOALLOC_MAX_CAMS == NOALLOC_MAX_JOBS,
                  "one limit for the host tables and the device scratch");
    static_assert(RAPTOR_MAX_NU <= 32, "the device scratch holds 32 frequencies per image");
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    raptor_status s = batch_precheck(ctx, cams, n_cams, grids, opts, nu_hz);
    if (s != RAPTOR_OK) return s;
    if (n_cams > NOALLOC_MAX_JOBS)
        return fail(ctx, RAPTOR_E_RANGE, "raptor_trace_batch_noalloc takes at most RAPTOR_NOALLOC_MAX_CAMS (256) cameras");
    if (opts->mem != RAPTOR_MEM_DEVICE || !images)
        return fail(ctx, RAPTOR_E_INVALID,
                    "raptor_trace_batch_noalloc writes device outputs: needs opts->mem = RAPTOR_MEM_DEVICE and images");
    if (opts->launch != RAPTOR_LAUNCH_DIRECT)
        return fail(ctx, RAPTOR_E_UNSUPPORTED, "raptor_trace_batch_noalloc launches directly (RAPTOR_LAUNCH_DIRECT)");
    if (!ctx->noalloc_scratch || !ctx->noalloc_host)
        return fail(ctx, RAPTOR_E_DEVICE, "the context has no no-allocation scratch");
    rctx::NoAllocHost& na = *ctx->noalloc_host;
    if ((s = batch_inputs(ctx, cams, n_cams, grids, opts, nu_hz, n_nu, na.in)) != RAPTOR_OK) return s;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    const bool fp32 = opts->transfer_prec == RAPTOR_F32;
    LaunchPlan plan;
    if ((s = plan_for(ctx, n_nu, fp32, &plan, opts->closure >= RAPTOR_CLOSURE_MLP, false)) != RAPTOR_OK) return s;
    HostTables h{na.jobs, na.grids, na.gl, na.nus, na.pixsr};
    const Geometry geo = launch_geometry(plan.p, n_nu, fp32, opts->closure >= RAPTOR_CLOSURE_MLP, opts->integrator);
    if ((s = fill_tables(ctx, na.in, n_cams, n_nu, opts, geo.tile_w, geo.rays, &h)) != RAPTOR_OK) return s;
    // the launch's buffers, carved from the scratch in 256-byte aligned regions
    unsigned char* base = static_cast<unsigned char*>(ctx->noalloc_scratch);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* q = base + off;
        off += noalloc_round(bytes);
        return q;
    };
    DevTables d;
    d.counter = reinterpret_cast<unsigned int*>(take(sizeof(unsigned int)));
    d.stats = reinterpret_cast<unsigned long long*>(take(ST_COUNT * sizeof(unsigned long long)));
    d.jobs = reinterpret_cast<DevJob*>(take(n_cams * sizeof(DevJob)));
    d.grids = reinterpret_cast<DevGrid*>(take(h.n_grids * sizeof(DevGrid)));
    d.nu = reinterpret_cast<double*>(take((size_t)n_cams * n_nu * sizeof(double)));
    d.pixsr = reinterpret_cast<double*>(take(n_cams * sizeof(double)));
    d.flux = flux_jy ? flux_jy : reinterpret_cast<double*>(take((size_t)n_cams * n_nu * sizeof(double)));
    d.flux_part = reinterpret_cast<double*>(take(flux_partials(n_cams, n_nu) * sizeof(double)));
    d.out = images;
    d.rs = nullptr;
    d.rn = nullptr;
    if (off > NOALLOC_SCRATCH_BYTES) return fail(ctx, RAPTOR_E_RANGE, "the batch exceeds the no-allocation scratch");
    return launch_tables(ctx, h, d, n_cams, n_nu, opts, plan, images, flux_jy, nullptr, nullptr, stats);
}

raptor_status raptor_get_plan(raptor_ctx* ctx, int32_t n_nu, int32_t transfer_prec, int32_t closure,
                              raptor_plan* out)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!out || n_nu < 1 || n_nu > RAPTOR_MAX_NU || (transfer_prec != RAPTOR_F32 && transfer_prec != RAPTOR_F64) ||
        closure < RAPTOR_CLOSURE_EXACT || closure > RAPTOR_CLOSURE_MLP_BF16)
        return fail(ctx, RAPTOR_E_INVALID, "bad arguments to raptor_get_plan");
    LaunchPlan pl;
    raptor_status s = plan_for(ctx, n_nu, transfer_prec == RAPTOR_F32, &pl, closure >= RAPTOR_CLOSURE_MLP);
    if (s != RAPTOR_OK) return s;
    *out = pl.p;
    return RAPTOR_OK;
}

raptor_status raptor_set_plan(raptor_ctx* ctx, int32_t n_nu, int32_t transfer_prec, int32_t closure,
                              const raptor_plan* plan)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!plan || n_nu < 1 || n_nu > RAPTOR_MAX_NU || (transfer_prec != RAPTOR_F32 && transfer_prec != RAPTOR_F64) ||
        closure < RAPTOR_CLOSURE_EXACT || closure > RAPTOR_CLOSURE_MLP_BF16)
        return fail(ctx, RAPTOR_E_INVALID, "bad arguments to raptor_set_plan");
    if (!plan_valid(*plan)) return fail(ctx, RAPTOR_E_INVALID, "plan field out of range");
    LaunchPlan pl;
    pl.p = *plan;
    const bool fp32 = transfer_prec == RAPTOR_F32;
    const bool mlpc = closure >= RAPTOR_CLOSURE_MLP;
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    raptor_status s = resolve_plan(ctx, n_nu, fp32, &pl, mlpc);
    if (s != RAPTOR_OK) return s;
    ctx->plans[plan_key(n_nu, fp32, mlpc)] = pl;
    return RAPTOR_OK;
}

raptor_status raptor_autotune_batch(raptor_ctx* ctx, const raptor_camera* cams, int32_t n_cams,
                                    const raptor_grid* const* grids, const raptor_opts* opts, const double* nu_hz,
                                    int32_t n_nu, int32_t reps, raptor_plan* best, double* best_ms)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    raptor_status s = batch_precheck(ctx, cams, n_cams, grids, opts, nu_hz);
    if (s != RAPTOR_OK) return s;
    std::vector<JobIn> in(n_cams);
    s = batch_inputs(ctx, cams, n_cams, grids, opts, nu_hz, n_nu, in.data());
    if (s != RAPTOR_OK) return s;
    if (reps < 1 || reps > 100) return fail(ctx, RAPTOR_E_INVALID, "reps must be in [1, 100]");
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    raptor_opts o = *opts;
    o.mem = RAPTOR_MEM_DEVICE;   // outputs stay in the context's buffers
    const bool fp32 = o.transfer_prec == RAPTOR_F32;
    auto time_plan = [&](const raptor_plan& cand, double* ms) -> raptor_status {
        LaunchPlan pl;
        pl.p = cand;
        raptor_status r = resolve_plan(ctx, n_nu, fp32, &pl, o.closure >= RAPTOR_CLOSURE_MLP);
        if (r != RAPTOR_OK) return r;
        double bestv = 1e300;
        for (int i = 0; i < reps; ++i) {
            raptor_stats st;
            r = run_jobs(ctx, in.data(), n_cams, n_nu, &o, nullptr, nullptr, nullptr, nullptr, &st, &pl);
            if (r != RAPTOR_OK) return r;
            bestv = std::min(bestv, st.kernel_ms);
        }
        *ms = bestv;
        return RAPTOR_OK;
    };
    LaunchPlan cur;
    s = plan_for(ctx, n_nu, fp32, &cur, o.closure >= RAPTOR_CLOSURE_MLP);
    if (s != RAPTOR_OK) return s;
    raptor_plan bp = cur.p;
    double bms;
    if ((s = time_plan(bp, &bms)) != RAPTOR_OK) return s;
    // coordinate descent over the plan fields
    // (rays per wave before the tile width, which it bounds)
    const std::vector<std::vector<int>> values = {{1, 2, 3}, {64, 256, 512}, {0, 2, 4}, {1, 8, 16, 32}, {64, 32, 16},
                                                  {8, 16, 64}};
    const bool mlpc_c = o.closure >= RAPTOR_CLOSURE_MLP;
    for (int field = 0; field < (int)values.size(); ++field) {
        for (int v : values[field]) {
            raptor_plan c = bp;
            int* slot = field == 0 ? &c.min_waves_per_simd : field == 1 ? &c.threads : field == 2 ? &c.blocks_per_cu
                      : field == 3 ? &c.refill_threshold : field == 4 ? &c.rays_per_wave : &c.tile_width;
            if (*slot == v) continue;
            *slot = v;
            // rays per wave below 64 only where the instantiation keeps one sample per lane, and
            // no tile wider than the rays (it would run as the narrower one already timed)
            const Geometry cg = launch_geometry(c, n_nu, fp32, mlpc_c, o.integrator);
            if (field == 4 && cg.rays != v) continue;
            if (field == 5 && cg.tile_w != v) continue;
            double ms;
            if ((s = time_plan(c, &ms)) != RAPTOR_OK) return s;
            if (ms < bms) {
                bms = ms;
                bp = c;
            }
        }
    }
    LaunchPlan fin;
    fin.p = bp;
    if ((s = resolve_plan(ctx, n_nu, fp32, &fin, o.closure >= RAPTOR_CLOSURE_MLP)) != RAPTOR_OK) return s;
    const bool mlpc_t = o.closure >= RAPTOR_CLOSURE_MLP;
    ctx->plans[plan_key(n_nu, fp32, mlpc_t)] = fin;
    if (best) *best = fin.p;   // as installed: resolved against the instantiation's limits
    if (best_ms) *best_ms = bms;
    return RAPTOR_OK;
}

raptor_status raptor_kernel_info(raptor_ctx* ctx, int32_t n_nu, int32_t transfer_prec, int32_t closure,
                                 const raptor_plan* plan, int32_t* vgprs, int32_t* scratch_bytes,
                                 int32_t* blocks_per_cu)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    if (!plan || !plan_valid(*plan) || n_nu < 1 || n_nu > RAPTOR_MAX_NU ||
        (transfer_prec != RAPTOR_F32 && transfer_prec != RAPTOR_F64) || closure < RAPTOR_CLOSURE_EXACT ||
        closure > RAPTOR_CLOSURE_MLP_BF16)
        return fail(ctx, RAPTOR_E_INVALID, "bad arguments to raptor_kernel_info");
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    const bool fp32 = transfer_prec == RAPTOR_F32;
    const bool mlpc = closure >= RAPTOR_CLOSURE_MLP;
    int regs = 0, spill = 0, maxt = 0, per_cu = 0;
    RAPTOR_CK(trace_kernel_attributes(n_nu, fp32, plan->min_waves_per_simd, mlpc, INTEG_RK4, &regs, &spill, &maxt),
              "reading kernel attributes");
    RAPTOR_CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &per_cu, trace_kernel_symbol(n_nu, fp32, plan->min_waves_per_simd, mlpc), plan->threads,
                  trace_kernel_lds(n_nu, fp32, plan->min_waves_per_simd, plan->threads, mlpc, INTEG_RK4,
                                   launch_geometry(*plan, n_nu, fp32, mlpc, INTEG_RK4).rays)),
              "querying occupancy");
    if (vgprs) *vgprs = regs;
    if (scratch_bytes) *scratch_bytes = spill;
    if (blocks_per_cu) *blocks_per_cu = per_cu;
    return RAPTOR_OK;
}

static double isco_radius(double a)
{
    // Bardeen, Press & Teukolsky: prograde for a >= 0, retrograde for a < 0
    const double z1 = 1.0 + std::cbrt(1.0 - a * a) * (std::cbrt(1.0 + a) + std::cbrt(1.0 - a));
    const double z2 = std::sqrt(3.0 * a * a + z1 * z1);
    return 3.0 + z2 - (a >= 0.0 ? 1.0 : -1.0) * std::sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

raptor_status raptor_isco(double spin, double* r_isco)
{
    if (!r_isco || !(std::fabs(spin) < 1.0)) return RAPTOR_E_INVALID;
    *r_isco = isco_radius(spin);
    return RAPTOR_OK;
}

raptor_status raptor_trace_disk(raptor_ctx* ctx, const raptor_camera* cam, const raptor_opts* opts, double r_disk_out,
                                int32_t n_bins, double g_lo, double g_hi, double* intensity, double* redshift,
                                double* profile, int32_t* ray_status, int32_t* ray_steps, raptor_stats* stats)
{
    if (!ctx) return RAPTOR_E_INVALID;
    ctx->err.clear();
    raptor_status s;
    if (!cam) return fail(ctx, RAPTOR_E_INVALID, "camera is NULL");
    if ((s = check_opts(ctx, opts)) != RAPTOR_OK) return s;
    if (opts->closure != RAPTOR_CLOSURE_EXACT)
        return fail(ctx, RAPTOR_E_INVALID, "the thin-disk test has its own emission (closure must be EXACT)");
    if (!(std::fabs(cam->spin) < 1.0) || !(cam->incl_deg > 0.0 && cam->incl_deg < 180.0) || cam->nx < 1 ||
        cam->ny < 1 || !finite_pos(cam->fov_half) || !std::isfinite(cam->r_cam))
        return fail(ctx, RAPTOR_E_INVALID, "bad camera");
    const double M = opts->metric_mass;
    const double rh = M + std::sqrt(std::max(M * M - cam->spin * cam->spin, 0.0));
    const double r_in = isco_radius(cam->spin);
    if (!(r_disk_out > r_in) || !(cam->r_cam > r_disk_out) || !(cam->r_cam > opts->r_stop_factor * rh))
        return fail(ctx, RAPTOR_E_INVALID, "need r_isco < r_disk_out < r_cam and r_cam outside the horizon");
    if (profile && (n_bins < 1 || n_bins > (1 << 20) || !(g_hi > g_lo) || !std::isfinite(g_lo) || !std::isfinite(g_hi)))
        return fail(ctx, RAPTOR_E_INVALID, "bad profile binning");
    const long long n = (long long)cam->nx * cam->ny;
    if (n > (1ll << 31)) return fail(ctx, RAPTOR_E_RANGE, "too many pixels");
    RAPTOR_CK(hipSetDevice(ctx->device), "selecting the device");
    const bool dev = opts->mem == RAPTOR_MEM_DEVICE;
    // device buffers: the caller's in device mode, the context's otherwise (the profile needs
    // both images)
    double *dI = intensity, *dG = redshift;
    int *dS = ray_status, *dN = ray_steps;
    if (!dev || !intensity || !redshift) {
        RAPTOR_CK(ctx->out.reserve(2 * n), "allocating images");
        if (!dev || !intensity) dI = ctx->out.p;
        if (!dev || !redshift) dG = ctx->out.p + n;
    }
    if (!dev && (ray_status || ray_steps)) {
        RAPTOR_CK(ctx->status.reserve(n), "allocating ray info");
        RAPTOR_CK(ctx->steps.reserve(n), "allocating ray info");
        dS = ray_status ? ctx->status.p : nullptr;
        dN = ray_steps ? ctx->steps.p : nullptr;
    }
    double* dP = nullptr;
    if (profile) {
        if (dev) {
            dP = profile;
        } else {
            RAPTOR_CK(ctx->flux_part.reserve((size_t)n_bins), "allocating the profile");
            dP = ctx->flux_part.p;
        }
    }
    DiskParams p;
    std::memset(&p, 0, sizeof p);
    p.a = cam->spin;
    p.incl = cam->incl_deg * kPi / 180.0;
    p.sin_i = std::sin(p.incl);
    p.cos_i = std::cos(p.incl);
    p.r_cam = cam->r_cam;
    p.fov = cam->fov_half;
    p.dalpha = 2.0 * cam->fov_half / cam->nx;
    p.dbeta = 2.0 * cam->fov_half / cam->ny;
    p.r_stop = opts->r_stop_factor * rh;
    p.r_in = r_in;
    p.r_out = r_disk_out;
    p.eps = opts->eps;
    p.M = M;
    p.nx = cam->nx;
    p.ny = cam->ny;
    p.max_steps = opts->max_steps;
    p.integrator = opts->integrator;
    p.intensity = dI;
    p.redshift = dG;
    p.status = dS;
    p.steps = dN;
    p.stats = ctx->stats.p;
    hipStream_t st = ctx->stream;
    RAPTOR_CK(launch_reset(ctx->counter.p, ctx->stats.p, st), "launching reset");
    const int blocks = (int)std::min<long long>((n + 255) / 256, (long long)ctx->cu_count * 8);
    RAPTOR_CK(hipEventRecord(ctx->ev0, st), "recording an event");
    RAPTOR_CK(launch_disk(p, blocks, st), "launching the disk kernel");
    RAPTOR_CK(hipEventRecord(ctx->ev1, st), "recording an event");
    if (profile)
        RAPTOR_CK(launch_disk_profile(dI, dG, n, n_bins, g_lo, g_hi, p.dalpha * p.dbeta, dP, st),
                  "launching the profile");
    const hipMemcpyKind d2x = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (intensity && dI != intensity) RAPTOR_CK(hipMemcpyAsync(intensity, dI, n * 8, d2x, st), "copying images");
    if (redshift && dG != redshift) RAPTOR_CK(hipMemcpyAsync(redshift, dG, n * 8, d2x, st), "copying images");
    if (ray_status && dS != ray_status) RAPTOR_CK(hipMemcpyAsync(ray_status, dS, n * 4, d2x, st), "copying status");
    if (ray_steps && dN != ray_steps) RAPTOR_CK(hipMemcpyAsync(ray_steps, dN, n * 4, d2x, st), "copying steps");
    if (profile && dP != profile)
        RAPTOR_CK(hipMemcpyAsync(profile, dP, (size_t)n_bins * 8, d2x, st), "copying the profile");
    unsigned long long hs[ST_COUNT];
    RAPTOR_CK(hipMemcpyAsync(hs, ctx->stats.p, sizeof hs, hipMemcpyDeviceToHost, st), "copying statistics");
    RAPTOR_CK(hipStreamSynchronize(st), "running the disk test");
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->rays = (uint64_t)n;
        stats->ray_steps = hs[0];
        stats->samples = hs[1];
        float ms = 0.0f;
        RAPTOR_CK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "reading the kernel time");
        stats->kernel_ms = ms;
    }
    return RAPTOR_OK;
}

raptor_status raptor_work_per_step(int32_t integrator, double* flops, double* special)
{
    if (integrator < RAPTOR_RK4 || integrator > RAPTOR_VERLET_CORRECTED) return RAPTOR_E_INVALID;
    using C = rt::OpCounted;
    C y[8] = {C(0.0), C(9.0), C(1.1), C(0.3), C(1.05), C(-0.9), C(0.02), C(0.01)};
    C acc[4] = {C(0.01), C(-0.02), C(0.001), C(0.0001)};
    rt::g_tally = rt::OpTally{};
    const rk::Spin<C> sp = rk::make_spin(C(0.9375), C(1.0));
    const C dl = -rk::step_size(C(0.05), y);
    C s0, c0;
    rt::sincos_(y[2], &s0, &c0);
    if (integrator == RAPTOR_RK2)
        rk::rk2_step(sp, y, dl, s0, c0);
    else if (integrator == RAPTOR_RK4)
        rk::rk4_step(sp, y, dl, s0, c0);
    else
        rk::verlet_step(sp, y, acc, dl, integrator == RAPTOR_VERLET_CORRECTED, s0, c0);
    if (flops) *flops = rt::g_tally.flops;
    if (special) *special = rt::g_tally.special;
    return RAPTOR_OK;
}

raptor_status raptor_work_per_unit(double* step_flops, double* step_special, double* sample_flops,
                                   double* sample_special, double* freq_flops, double* freq_special)
{
    using C = rt::OpCounted;
    // one accepted step at a representative state (the count does not depend on the values)
    C y[8] = {C(0.0), C(9.0), C(1.1), C(0.3), C(1.05), C(-0.9), C(0.02), C(0.01)};
    rt::g_tally = rt::OpTally{};
    const rk::Spin<C> sp = rk::make_spin(C(0.9375), C(1.0));
    const C dl = -rk::step_size(C(0.05), y);
    C s0, c0;
    rt::sincos_(y[2], &s0, &c0);
    rk::rk4_step(sp, y, dl, s0, c0);
    if (step_flops) *step_flops = rt::g_tally.flops;
    if (step_special) *step_special = rt::g_tally.special;

    // one sample, frequency-independent part: grid coordinates (7), the MKS map's x2 from its
    // cubic Hermite table (22: cell position 2, basis 12, combination 8; grids whose table is
    // refined by Halley's iteration do more), bilinear interpolation, fluid frame, path length
    // (2), 1/nu_r^3 (2), sin theta_B (2), K2 lookup (Hermite, 20)
    rt::g_tally = rt::OpTally{};
    (void)rt::log_(y[1]);
    rt::g_tally.flops += 7 + 22;
    C a[4] = {1, 2, 3, 4}, b[4] = {1, 2, 3, 4}, c[4] = {1, 2, 3, 4}, d[4] = {1, 2, 3, 4}, o4[4];
    pl::bilerp4(a, b, c, d, C(0.3), C(0.6), o4);
    C nr, cb;
    (void)pl::fluid_frame(C(0.9375), C(0.9375 * 0.9375), C(1.0), y, C(0.891), C(0.454), C(0.05), &nr, &cb);
    rt::g_tally.flops += 2 + 2 + 2 + 20;
    rt::g_tally.special += 1 + 1 + 1;   // 1/nu_r^3, sqrt, exp of the K2 lookup
    if (sample_flops) *sample_flops = rt::g_tally.flops;
    if (sample_special) *sample_special = rt::g_tally.special;

    // closure and transfer update of one frequency
    rt::g_tally = rt::OpTally{};
    C nu = C(230e9) * nr;
    C j, al, S, I = C(0.0), tau = C(0.0);
    pl::closure_exact(nu, C(1e5), C(3.0), C(5.0), C(0.5), C(0.01), &j, &al, &S);
    C A, dtau;
    pl::step_source(j, al, S, C(1e10), C(0.8), A, dtau);
    I = I + rt::exp_(-tau) * A;   // fold into (I, tau)
    tau = tau + dtau;
    if (freq_flops) *freq_flops = rt::g_tally.flops;
    if (freq_special) *freq_special = rt::g_tally.special;
    return RAPTOR_OK;
}

}  // extern "C"
