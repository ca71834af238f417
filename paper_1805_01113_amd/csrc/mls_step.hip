// One immersed-boundary time step over all bodies (jitter, build, interp,
// direct forcing, spread), its HIP-graph capture, and per-kernel timing.
#include <cstring>

#include "mls_device.h"

using namespace mls;

namespace mls {

namespace {

constexpr int kBlock = 256;

#pragma clang fp contract(off)
// x = x0 + (u - 1/2) (2 amp), u on the 2^-24 lattice of [0, 1); plain FP32
// operations (no fused multiply-add) so the result is reproducible anywhere.
__global__ void __launch_bounds__(kBlock)
k_jitter(int64_t n, const float *__restrict__ x0, const float *__restrict__ y0, const float *__restrict__ z0,
         float *__restrict__ x, float *__restrict__ y, float *__restrict__ z, float amp2, uint64_t seed,
         const unsigned long long *__restrict__ step_ctr)
{
    const uint64_t step = *step_ctr;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n; l += (int64_t)gridDim.x * blockDim.x)
        jitter_marker(seed, step, n, l, amp2, x0[l], y0[l], z0[l], x[l], y[l], z[l]);
}
#pragma clang fp contract(on)

// Direct forcing (Sec. 2): F = (V_b - U) / dt per component.
__global__ void __launch_bounds__(kBlock)
k_force(int64_t n3, const float *__restrict__ vb, const float *__restrict__ U, float inv_dt, float *__restrict__ F)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = vb ? vb[i] : 0.0f;
        F[i] = (v - U[i]) * inv_dt;
    }
}

__global__ void k_step_advance(unsigned long long *step_ctr) { *step_ctr += 1ull; }

__global__ void k_step_set(unsigned long long *step_ctr, unsigned long long v) { *step_ctr = v; }

int grid_for(int64_t work, int cu)
{
    int64_t b = (work + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cu * 32;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_jitter(const Ctx &c, int64_t n, const float *x0, const float *y0, const float *z0, float *x,
                         float *y, float *z, float amp, uint64_t seed, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jitter, dim3(grid_for(n, c.cu_count)), dim3(kBlock), 0, s, n, x0, y0, z0, x, y, z,
                       2.0f * amp, seed, c.step_ctr);
    return hipGetLastError();
}

hipError_t launch_force(const Ctx &c, int64_t n, const float *vb, const float *U, float dt, float *F, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_force, dim3(grid_for(3 * n, c.cu_count)), dim3(kBlock), 0, s, 3 * n, vb, U, 1.0f / dt, F);
    return hipGetLastError();
}

hipError_t launch_step_advance(const Ctx &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, s, c.step_ctr);
    return hipGetLastError();
}

TimedLaunch::TimedLaunch(Ctx &c_, int id_, hipStream_t s_) : c(c_), id(id_), s(s_)
{
    if (id < 0 || !c.timing || c.capturing) return;
    while (c.ev_used + 2 > c.ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c.ev_pool.push_back(e);
    }
    a = c.ev_pool[c.ev_used++];
    b = c.ev_pool[c.ev_used++];
    if (hipEventRecord(a, s) != hipSuccess) {   // no timing for this launch
        a = nullptr;
        c.ev_used -= 2;
    }
}

TimedLaunch::~TimedLaunch()
{
    if (!a) return;
    if (hipEventRecord(b, s) == hipSuccess) c.ev_marks.push_back({id, {a, b}});
}

}  // namespace mls


struct mls_graph {
    mls_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t scratch_gen = 0;   // the context's scratch generation the capture saw
};

extern "C" {

mls_status mls_step(mls_ctx *ctx, const mls_step_desc *desc, const mls_step_buffers *b, void *stream)
{
    if (!ctx || !desc || !b) return MLS_E_ARG;
    Ctx &c = ctx->c;
    const int64_t n = b->n;
    if (n < 0 || !(desc->dt > 0.0f) || !(desc->jitter >= 0.0f) || (desc->flags & ~MLS_STEP_COMPACT) != 0)
        return MLS_E_ARG;
    if (n == 0) return MLS_OK;
    if (!b->x0 || !b->y0 || !b->z0 || !b->area || !b->home || !b->phi || !b->u || !b->v || !b->w || !b->U ||
        !b->F || !b->fx || !b->fy || !b->fz)
        return MLS_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float *bx = b->x0, *by = b->y0, *bz = b->z0;
    const bool jitter = desc->jitter > 0.0f;
    if (jitter && (!b->x || !b->y || !b->z)) return MLS_E_ARG;
    mls_status st = MLS_OK;
    hipError_t e;
    const bool fast = desc->method == MLS_FAST || desc->method == MLS_FAST_LINEAR;
    if (fast) {
        // tables are built once per context (before any graph capture)
        st = mls_fast_tables(ctx, nullptr, nullptr, nullptr, nullptr, nullptr, stream);
        if (st != MLS_OK) return st;
    }
    const bool learned = desc->method == MLS_LEARNED;
    if (learned && !c.mlp.loaded) return MLS_E_ARG;
    const bool sorted = desc->method == MLS_EXACT || (fast && fast_fused_ok(c)) || learned;
    if (jitter) {
        // the sorted step jitters inside its binning pass; the others first
        if (!sorted) {
            TimedLaunch t(c, MLS_K_JITTER, s);
            e = launch_jitter(c, n, b->x0, b->y0, b->z0, b->x, b->y, b->z, desc->jitter, desc->seed, s);
            if (e != hipSuccess) return MLS_E_HIP;
        }
        bx = b->x; by = b->y; bz = b->z;
    }
    if (sorted) {
        // exact MLS, or fast-MLS on a uniform grid, in spreading-tile order:
        // bin the markers from their positions, build with interpolation and
        // forcing fused (phi is not read back), spread reading each tile's
        // rows contiguously
        st = mls_reserve(ctx, n);
        if (st != MLS_OK) return st;
        const bool compact = desc->method == MLS_EXACT && (desc->flags & MLS_STEP_COMPACT);
        if (compact) {
            st = reserve_compact(ctx, n);
            if (st != MLS_OK) return st;
        }
        // the row width applies to this step's launches only
        struct NfReset {
            Ctx &c;
            ~NfReset() { c.step_nf = 0; }
        } nf_reset{c};
        c.step_nf = compact ? compact_nf(c) : 0;
        e = jitter ? launch_sort_positions(c, n, b->x0, b->y0, b->z0, s, b->x, b->y, b->z, desc->jitter, desc->seed)
                   : launch_sort_positions(c, n, bx, by, bz, s);
        if (e != hipSuccess) return MLS_E_HIP;
        if (learned) {
            // the network (with its exact fallback) in tile order, fused with
            // the interpolation, forcing and c_l F_l of its rows
            TimedLaunch t(c, MLS_K_BUILD_LEARNED, s);
            const LearnedInterp li = learned_interp(c, b->u, b->v, b->w, b->vb, b->area, desc->dt, b->U, b->F);
            e = launch_build_learned(c, n, bx, by, bz, b->home, b->phi, b->route, s, c.entries, &li);
        } else if (fast) {
            TimedLaunch t(c, MLS_K_FAST_INTERP, s);
            e = launch_fast_interp(c, n, bx, by, bz, b->home, b->phi, b->route, b->u, b->v, b->w, b->vb, b->area,
                                   desc->dt, b->U, b->F, s, desc->method == MLS_FAST_LINEAR);
        } else {
            TimedLaunch t(c, MLS_K_BUILD_INTERP, s);
            e = launch_build_interp(c, n, bx, by, bz, b->home, b->phi, b->route, b->u, b->v, b->w, b->vb, b->area,
                                    desc->dt, b->U, b->F, s);
        }
        if (e != hipSuccess) return MLS_E_HIP;
        e = launch_spread_sorted(c, n, b->home, b->phi, b->fx, b->fy, b->fz, s);
        if (e != hipSuccess) return MLS_E_HIP;
        c.step_sorted_n = n;
        return launch_step_advance(c, s) == hipSuccess ? MLS_OK : MLS_E_HIP;
    }
    st = mls_build(ctx, n, bx, by, bz, desc->method, b->home, b->phi, b->route, stream);
    if (st != MLS_OK) return st;
    st = mls_interp(ctx, n, b->home, b->phi, b->u, b->v, b->w, b->U, b->U + n, b->U + 2 * n, stream);
    if (st != MLS_OK) return st;
    {
        TimedLaunch t(c, MLS_K_FORCE, s);
        e = launch_force(c, n, b->vb, b->U, desc->dt, b->F, s);
    }
    if (e != hipSuccess) return MLS_E_HIP;
    st = mls_spread(ctx, n, b->home, b->phi, b->area, b->F, b->F + n, b->F + 2 * n, b->fx, b->fy, b->fz, stream);
    if (st != MLS_OK) return st;
    return launch_step_advance(c, s) == hipSuccess ? MLS_OK : MLS_E_HIP;
}

mls_status mls_step_order(mls_ctx *ctx, uint32_t *order, int64_t n, void *stream)
{
    if (!ctx || !order || n < 0) return MLS_E_ARG;
    Ctx &c = ctx->c;
    if (n != c.step_sorted_n) return MLS_E_ARG;
    if (n == 0) return MLS_OK;
    return hipMemcpyAsync(order, c.entries, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(stream)) == hipSuccess ? MLS_OK : MLS_E_HIP;
}

mls_status mls_step_counter_set(mls_ctx *ctx, uint64_t step, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    hipLaunchKernelGGL(k_step_set, dim3(1), dim3(1), 0, static_cast<hipStream_t>(stream), ctx->c.step_ctr,
                       (unsigned long long)step);
    return hipGetLastError() == hipSuccess ? MLS_OK : MLS_E_HIP;
}

mls_status mls_graph_create(mls_ctx *ctx, const mls_step_desc *desc, const mls_step_buffers *b, mls_graph **out)
{
    if (!ctx || !desc || !b || !out || (desc->flags & ~MLS_STEP_COMPACT) != 0) return MLS_E_ARG;
    *out = nullptr;
    Ctx &c = ctx->c;
    // everything that allocates or synchronises happens before the capture
    mls_status st = mls_reserve(ctx, b->n);
    if (st != MLS_OK) return st;
    if (desc->method == MLS_EXACT && (desc->flags & MLS_STEP_COMPACT)) {
        st = reserve_compact(ctx, b->n);
        if (st != MLS_OK) return st;
    }
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return MLS_E_HIP;
    if (desc->method == MLS_FAST || desc->method == MLS_FAST_LINEAR) {
        st = mls_fast_tables(ctx, nullptr, nullptr, nullptr, nullptr, nullptr, cs);
        if (st != MLS_OK) { hipStreamDestroy(cs); return st; }
    }
    if (hipStreamSynchronize(cs) != hipSuccess) { hipStreamDestroy(cs); return MLS_E_HIP; }
    auto *g = new mls_graph();
    g->ctx = ctx;
    c.capturing = true;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = mls_step(ctx, desc, b, cs);
        e = hipStreamEndCapture(cs, &g->graph);
    }
    c.capturing = false;
    if (e == hipSuccess && st == MLS_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    g->scratch_gen = c.scratch_gen;
    hipStreamDestroy(cs);
    if (e != hipSuccess || st != MLS_OK) {
        mls_graph_destroy(g);
        return st != MLS_OK ? st : MLS_E_HIP;
    }
    *out = g;
    return MLS_OK;
}

mls_status mls_graph_launch(mls_graph *g, int32_t n_steps, void *stream)
{
    if (!g || !g->exec || n_steps < 0) return MLS_E_ARG;
    // the context's scratch moved or its tiling changed since the capture:
    // the graph would address freed memory
    if (g->scratch_gen != g->ctx->c.scratch_gen) {
        g->ctx->c.last_error = "step graph captured before the context's scratch or tiling changed; create it again";
        return MLS_E_ARG;
    }
    for (int32_t i = 0; i < n_steps; ++i)
        if (hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) != hipSuccess) return MLS_E_HIP;
    return MLS_OK;
}

void mls_graph_destroy(mls_graph *g)
{
    if (!g) return;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
}

mls_status mls_timing_enable(mls_ctx *ctx, int32_t on)
{
    if (!ctx) return MLS_E_ARG;
    ctx->c.timing = on != 0;
    return MLS_OK;
}

mls_status mls_timing_get(mls_ctx *ctx, mls_timing *out, int32_t reset)
{
    if (!ctx || !out) return MLS_E_ARG;
    Ctx &c = ctx->c;
    if (hipDeviceSynchronize() != hipSuccess) return MLS_E_HIP;
    memset(out, 0, sizeof(*out));
    for (auto &m : c.ev_marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, m.second.first, m.second.second) != hipSuccess) return MLS_E_HIP;
        if (m.first >= 0 && m.first < MLS_K_COUNT) {
            out->ms[m.first] += ms;
            out->launches[m.first] += 1;
        }
    }
    if (reset) {
        c.ev_marks.clear();
        c.ev_used = 0;
    }
    return MLS_OK;
}

}  // extern "C"
