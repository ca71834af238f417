// C ABI of the MLS transfer library: context, argument checks, scratch
// management and error reporting.  Kernels live in mls_build.hip and
// mls_transfer.hip.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>

#include "mls_internal.h"

using namespace mls;


namespace {

constexpr unsigned long long kNoError = ~0ull;

mls_status fail(mls_ctx *ctx, mls_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

mls_status fail(mls_ctx *ctx, mls_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->c.last_error = buf;
    }
    return st;
}

mls_status hip_fail(mls_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? MLS_E_NOMEM : MLS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Nodes of component c along axis d.
int32_t comp_nodes(const Axis &a, int c, int d)
{
    return (c == d && !a.periodic) ? a.n + 1 : a.n;
}

}  // namespace

// Spreading tiles for the requested edge: a periodic axis of at most kMaxTile
// cells is one tile; a longer one is cut into equal tiles (the requested edge
// if it divides the axis, else its largest divisor between 4 and
// kMaxBoxTile; none -> MLS_E_ARG); a wall axis uses the requested edge.
// Derives the LDS boxes and the tile colours, (re)allocates the per-tile
// scratch and uploads the grid.  On error the previous tiling is kept.
mls_status mls::setup_tiles(Ctx &c, int want)
{
    if (want < 4 || want > kMaxBoxTile) return MLS_E_ARG;
    Grid g = c.g;
    for (int d = 0; d < 3; ++d) {
        Axis &a = g.ax[d];
        const int n = a.n;
        if (a.periodic) {
            a.tile = 0;
            if (n <= kMaxTile) a.tile = n;
            else if (n % want == 0) a.tile = want;
            for (int t = kMaxBoxTile; t >= 4 && !a.tile; --t)
                if (n % t == 0) a.tile = t;
            if (!a.tile) return MLS_E_ARG;
        } else {
            a.tile = want;
        }
    }
    for (int d = 0; d < 3; ++d) g.ax[d].inv_tile = 1.0f / (float)g.ax[d].tile;
    int64_t nt = 1;
    for (int d = 0; d < 3; ++d) {
        const Axis &a = g.ax[d];
        const int nn = a.periodic ? a.n : a.n + 1;
        g.ntile[d] = (nn + a.tile - 1) / a.tile;
        g.box[d] = (a.periodic && g.ntile[d] == 1) ? a.n : a.tile + 3;
        nt *= g.ntile[d];
    }
    g.ntiles = nt;
    // the fixed-point box of one component must fit the LDS of a workgroup
    const int64_t lds = (int64_t)g.box[0] * g.box[1] * g.box[2] * 8;
    if (lds > 160 * 1024) return MLS_E_ARG;
    // tile colours: tiles whose boxes may overlap get different colours.  Along
    // an axis the colour is the parity of the tile index; an odd number of
    // periodic tiles gives the last tile a third colour.
    int64_t colour_tiles[27] = {};
    {
        int64_t cnt[3][3];
        for (int d = 0; d < 3; ++d) {
            const int m = g.ntile[d];
            const bool periodic = g.ax[d].periodic != 0;
            g.ncol[d] = m == 1 ? 1 : ((periodic && (m & 1)) ? 3 : 2);
            if (g.ncol[d] == 1) { cnt[0][d] = 1; cnt[1][d] = 0; cnt[2][d] = 0; }
            else if (g.ncol[d] == 2) { cnt[0][d] = (m + 1) / 2; cnt[1][d] = m / 2; cnt[2][d] = 0; }
            else { cnt[0][d] = (m - 1) / 2; cnt[1][d] = (m - 1) / 2; cnt[2][d] = 1; }
        }
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) g.ncol_tiles[k][d] = (int32_t)cnt[k][d];
        for (int k = 0; k < 27; ++k) g.colour_base[k] = 0;
        int64_t base = 0;
        for (int cz = 0; cz < g.ncol[2]; ++cz)
            for (int cy = 0; cy < g.ncol[1]; ++cy)
                for (int cx = 0; cx < g.ncol[0]; ++cx) {
                    const int col = cx + g.ncol[0] * (cy + g.ncol[1] * cz);
                    colour_tiles[col] = cnt[cx][0] * cnt[cy][1] * cnt[cz][2];
                    g.colour_base[col] = base;
                    base += colour_tiles[col];
                }
    }
    // device scratch for the new tiling; one extra bucket (index nt) collects
    // markers without a valid support when the step bins markers from their
    // positions
    const int64_t nb = (nt + 1 + 2047) / 2048;
    uint32_t *tcount = nullptr, *toff = nullptr, *tcur = nullptr, *tact = nullptr, *bsum = nullptr,
             *tmax = nullptr;
    bool ok = hipMalloc((void **)&tcount, (nt + 1) * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc((void **)&toff, (nt + 2) * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc((void **)&tcur, (nt + 1) * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc((void **)&tact, nt * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc((void **)&bsum, (nb + 1) * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc((void **)&tmax, 3 * (nt + 1) * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess &&
         hipMemcpy(c.d_grid, &g, sizeof(Grid), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        hipFree(tcount); hipFree(toff); hipFree(tcur); hipFree(tact); hipFree(bsum); hipFree(tmax);
        hipMemcpy(c.d_grid, &c.g, sizeof(Grid), hipMemcpyHostToDevice);
        return MLS_E_NOMEM;
    }
    hipFree(c.tile_count); hipFree(c.tile_off); hipFree(c.tile_cursor);
    hipFree(c.tile_active); hipFree(c.block_sums); hipFree(c.tile_fmax);
    c.tile_count = tcount; c.tile_off = toff; c.tile_cursor = tcur; c.tile_active = tact; c.block_sums = bsum;
    c.tile_fmax = tmax;
    c.g = g;
    ++c.scratch_gen;
    for (int k = 0; k < 27; ++k) c.colour_tiles[k] = colour_tiles[k];
    c.spread_blocks_per_cu = std::max(1, std::min(c.spread_blocks_per_cu_req, (int)((160 * 1024) / (lds + 512))));
    c.opts.spread_tile = want;
    return MLS_OK;
}

namespace mls {

// Row width of the compact transfer function on this grid: gamma and one
// offset per axis when every axis is uniform, else gamma and three offsets
// per axis.
int compact_nf(const Ctx &c)
{
    return (c.g.ax[0].uniform && c.g.ax[1].uniform && c.g.ax[2].uniform) ? 7 : 13;
}

// Scratch of a compact exact step for n markers: the coefficient rows and the
// queue of rows solved in FP64.
mls_status reserve_compact(mls_ctx *ctx, int64_t n)
{
    Ctx &c = ctx->c;
    if (n <= c.coef_cap) return MLS_OK;
    hipDeviceSynchronize();
    ++c.scratch_gen;
    hipFree(c.coef_rows);
    hipFree(c.route_queue);
    c.coef_rows = nullptr;
    c.route_queue = nullptr;
    c.coef_cap = 0;
    const int64_t npad = (n + 63) / 64 * 64;
    hipError_t e = hipMalloc((void **)&c.coef_rows, (size_t)3 * kCoefStride<13> * npad * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&c.route_queue, (size_t)(1 + 3 * n) * sizeof(uint32_t));
    if (e != hipSuccess) {
        hipFree(c.coef_rows);
        c.coef_rows = nullptr;
        return hip_fail(ctx, e, "compact step scratch");
    }
    c.coef_cap = n;
    return MLS_OK;
}

}  // namespace mls

extern "C" {

#ifndef MLS_SOURCE_SHA256
#define MLS_SOURCE_SHA256 "unstamped"
#endif
// The build stamps the SHA-256 of the sources it compiled (csrc/ and
// include/mls.h), so a loaded library names them.
const char *mls_version(void) { return "mls_hip 0.2.0 (gfx950) src " MLS_SOURCE_SHA256; }

mls_status mls_ctx_create(mls_ctx **out, const mls_grid *grid, const mls_weight *weight, const mls_opts *opts)
{
    if (!out || !grid) return MLS_E_ARG;
    *out = nullptr;
    auto *ctx = new (std::nothrow) mls_ctx();
    if (!ctx) return MLS_E_NOMEM;
    Ctx &c = ctx->c;
    hipError_t e = hipGetDevice(&c.device);
    if (e != hipSuccess) { delete ctx; return MLS_E_HIP; }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device) == hipSuccess && cus > 0)
        c.cu_count = cus;

    // ---- grid checks and host-side geometry ----
    double hmin = std::numeric_limits<double>::infinity();
    int nonuniform = 0;
    for (int d = 0; d < 3; ++d) {
        const int n = grid->n[d];
        const double *f = grid->faces[d];
        if (n < 3 || !f) { delete ctx; return MLS_E_ARG; }
        c.h_faces[d].assign(f, f + n + 1);
        for (int i = 0; i <= n; ++i)
            if (!std::isfinite(f[i]) || (i > 0 && !(f[i] > f[i - 1]))) { delete ctx; return MLS_E_ARG; }
        c.h_centres[d].resize(n);
        for (int i = 0; i < n; ++i) c.h_centres[d][i] = 0.5 * (f[i] + f[i + 1]);
        Axis &a = c.g.ax[d];
        a.n = n;
        a.periodic = grid->periodic[d] ? 1 : 0;
        a.f0 = f[0];
        a.L = f[n] - f[0];
        a.inv_h = (double)n / a.L;
        const double w0 = f[1] - f[0];
        double wmin = w0, wmax = w0;
        bool bitwise = true;   // widths equal: one fast-MLS table serves the axis
        for (int i = 1; i < n; ++i) {
            const double wi = f[i + 1] - f[i];
            bitwise = bitwise && (std::fabs(wi - w0) <= 1e-12 * w0);   // equal up to face rounding
            wmin = std::min(wmin, wi);
            wmax = std::max(wmax, wi);
        }
        a.uniform = (wmax <= wmin * (1.0 + 1e-9)) ? 1 : 0;
        // exactly uniform: the stored coordinates are reproduced bit for bit by
        // f0 + i h and f0 + (i + 1/2) h (the device then computes them)
        a.h = a.L / (double)n;
        a.exact = a.uniform;
        for (int i = 0; i <= n && a.exact; ++i) a.exact = (f[i] == a.f0 + (double)i * a.h);
        for (int i = 0; i < n && a.exact; ++i) a.exact = (c.h_centres[d][i] == a.f0 + ((double)i + 0.5) * a.h);
        if (!bitwise) { ++nonuniform; c.stretched_axis = d; }
    }
    if (nonuniform > 1) c.stretched_axis = -2;   // fast-MLS unavailable (more than one stretched axis)
    for (int cc = 0; cc < 3; ++cc)
        for (int d = 0; d < 3; ++d) c.g.dims[cc][d] = comp_nodes(c.g.ax[d], cc, d);
    for (int cc = 0; cc < 3; ++cc)
        if (c.g.dims[cc][0] > 2048 || c.g.dims[cc][1] > 2048 || c.g.dims[cc][2] > 1024) { delete ctx; return MLS_E_ARG; }

    // control-volume widths (centre nodes: cells; face nodes: between centres)
    std::vector<float> wc[3], wf[3];
    for (int d = 0; d < 3; ++d) {
        const Axis &a = c.g.ax[d];
        const auto &f = c.h_faces[d];
        const auto &ce = c.h_centres[d];
        const int n = a.n;
        wc[d].resize(n);
        for (int i = 0; i < n; ++i) {
            wc[d][i] = (float)(f[i + 1] - f[i]);
            hmin = std::min(hmin, f[i + 1] - f[i]);
        }
        const int nf = a.periodic ? n : n + 1;
        wf[d].resize(nf);
        for (int i = 0; i < nf; ++i) {
            double lo, hi;
            if (a.periodic) {
                lo = i == 0 ? ce[n - 1] - a.L : ce[i - 1];
                hi = ce[i];
            } else {
                lo = i == 0 ? f[0] : ce[i - 1];
                hi = i == n ? f[n] : ce[i];
            }
            wf[d][i] = (float)(hi - lo);
            hmin = std::min(hmin, hi - lo);
        }
    }
    c.g.h_min = hmin;
    c.g.const_width = wc[0][0];
    for (int d = 0; d < 3; ++d) {
        for (float v : wc[d]) if (v != c.g.const_width) c.g.const_width = 0.f;
        for (float v : wf[d]) if (v != c.g.const_width) c.g.const_width = 0.f;
    }
    c.g.inv_cw2 = c.g.const_width > 0.f ? (float)(1.0 / ((double)c.g.const_width * c.g.const_width)) : 0.f;
    for (int d = 0; d < 3; ++d) {
        c.h_wc[d] = wc[d];
        c.h_wf[d] = wf[d];
    }
    const int want_tile = (opts && opts->spread_tile) ? opts->spread_tile : 8;
    if (want_tile < 4 || want_tile > kMaxBoxTile) { delete ctx; return MLS_E_ARG; }

    // ---- weight and options ----
    mls_weight wdef = {MLS_W_GAUSS_SHIFTED, 1.0, 1.5};
    const mls_weight &W = weight ? *weight : wdef;
    if (W.kind < 0 || W.kind > 2 || !(W.eps > 0.0) || !(W.radius > 0.0)) { delete ctx; return MLS_E_ARG; }
    c.w.kind = W.kind;
    c.w.inv_eps = (float)(1.0 / W.eps);
    c.w.inv_eps_d = 1.0 / W.eps;
    c.w.cut_d = std::exp(-(W.radius / W.eps) * (W.radius / W.eps));
    // the FP32 weight has one select-free form for every kind (see weight1)
    c.w.cut = W.kind == MLS_W_GAUSS_SHIFTED ? (float)c.w.cut_d : 0.0f;
    c.w.e2 = W.kind == MLS_W_CONST ? 0.0f : (float)(-1.4426950408889634 / (W.eps * W.eps));
    c.opts.kappa_tau = 1e6;
    c.opts.n_sub = 9;
    c.opts.fallback_tol = 1e-4;
    if (opts) {
        if (!(opts->kappa_tau >= 0.0) || opts->n_sub < 2 || opts->n_sub > 65 || !(opts->fallback_tol >= 0.0) ||
            (opts->spread_tile != 0 && (opts->spread_tile < 4 || opts->spread_tile > kMaxBoxTile))) {
            delete ctx;
            return MLS_E_ARG;
        }
        c.opts = *opts;
    }

    // ---- device geometry block ----
    size_t bytes = 0;
    size_t off_f[3], off_c[3], off_wc[3], off_wf[3];
    auto take = [&](size_t nbytes) { size_t o = bytes; bytes += (nbytes + 255) & ~size_t(255); return o; };
    for (int d = 0; d < 3; ++d) {
        off_f[d] = take(c.h_faces[d].size() * sizeof(double));
        off_c[d] = take(c.h_centres[d].size() * sizeof(double));
        off_wc[d] = take(wc[d].size() * sizeof(float));
        off_wf[d] = take(wf[d].size() * sizeof(float));
    }
    std::vector<unsigned char> blob(bytes, 0);
    for (int d = 0; d < 3; ++d) {
        memcpy(&blob[off_f[d]], c.h_faces[d].data(), c.h_faces[d].size() * sizeof(double));
        memcpy(&blob[off_c[d]], c.h_centres[d].data(), c.h_centres[d].size() * sizeof(double));
        memcpy(&blob[off_wc[d]], wc[d].data(), wc[d].size() * sizeof(float));
        memcpy(&blob[off_wf[d]], wf[d].data(), wf[d].size() * sizeof(float));
    }
    e = hipMalloc(&c.geom_block, bytes);
    if (e != hipSuccess) { delete ctx; return MLS_E_NOMEM; }
    e = hipMemcpy(c.geom_block, blob.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) { hipFree(c.geom_block); delete ctx; return MLS_E_HIP; }
    auto *base = static_cast<unsigned char *>(c.geom_block);
    for (int d = 0; d < 3; ++d) {
        Axis &a = c.g.ax[d];
        a.faces = reinterpret_cast<const double *>(base + off_f[d]);
        a.centres = reinterpret_cast<const double *>(base + off_c[d]);
        a.width_c = reinterpret_cast<const float *>(base + off_wc[d]);
        a.width_f = reinterpret_cast<const float *>(base + off_wf[d]);
    }
    if (hipMalloc((void **)&c.d_grid, sizeof(Grid)) != hipSuccess ||
        hipMemcpy(c.d_grid, &c.g, sizeof(Grid), hipMemcpyHostToDevice) != hipSuccess) {
        mls_ctx_destroy(ctx);
        return MLS_E_NOMEM;
    }
    if (hipMalloc((void **)&c.err, sizeof(ErrWord)) != hipSuccess ||
        hipMalloc((void **)&c.stats, sizeof(DevStats)) != hipSuccess ||
        hipMalloc((void **)&c.work, 128 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c.step_ctr, sizeof(unsigned long long)) != hipSuccess) {
        mls_ctx_destroy(ctx);
        return MLS_E_NOMEM;
    }
    const unsigned long long none = kNoError;
    hipMemcpy(c.err, &none, sizeof(none), hipMemcpyHostToDevice);
    hipMemset(c.stats, 0, sizeof(DevStats));
    hipMemset(c.work, 0, 128 * sizeof(uint32_t));
    hipMemset(c.step_ctr, 0, sizeof(unsigned long long));
    const mls_status ts = setup_tiles(c, want_tile);
    if (ts != MLS_OK) { mls_ctx_destroy(ctx); return ts; }
    // the allocation-free spreading's scratch address on this device
    if (noalloc_setup(c.device) != hipSuccess) { mls_ctx_destroy(ctx); return MLS_E_HIP; }
    if (hipDeviceSynchronize() != hipSuccess) { mls_ctx_destroy(ctx); return MLS_E_HIP; }
    *out = ctx;
    return MLS_OK;
}

void mls_ctx_destroy(mls_ctx *ctx)
{
    if (!ctx) return;
    Ctx &c = ctx->c;
    hipDeviceSynchronize();
    hipFree(c.geom_block);
    hipFree(c.d_grid);
    hipFree(c.err);
    hipFree(c.stats);
    hipFree(c.tables);
    hipFree(c.table_geo);
    hipFree(c.tile_count);
    hipFree(c.tile_off);
    hipFree(c.tile_cursor);
    hipFree(c.tile_active);
    hipFree(c.block_sums);
    hipFree(c.tile_fmax);
    hipFree(c.entries);
    hipFree(c.cf_rows);
    hipFree(c.marker_tile);
    hipFree(c.coef_rows);
    hipFree(c.route_queue);
    hipFree(c.refine_scratch);
    hipFree(c.grad_queue);
    hipFree(c.work);
    hipFree(c.step_ctr);
    mlp_free(c);
    for (hipEvent_t ev : c.ev_pool) hipEventDestroy(ev);
    delete ctx;
}

mls_status mls_reserve(mls_ctx *ctx, int64_t n)
{
    if (!ctx || n < 0) return MLS_E_ARG;
    Ctx &c = ctx->c;
    if (n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "too many markers (%lld)", (long long)n);
    if (n <= c.cap_markers) return MLS_OK;
    hipDeviceSynchronize();
    ++c.scratch_gen;
    hipFree(c.entries);
    hipFree(c.cf_rows);
    hipFree(c.marker_tile);
    c.entries = nullptr;
    c.cf_rows = nullptr;
    c.marker_tile = nullptr;
    c.cap_markers = 0;
    c.cf_stride = 0;
    const int64_t stride = (n + 63) / 64 * 64;
    hipError_t e = hipMalloc((void **)&c.entries, (size_t)n * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&c.cf_rows, (size_t)3 * stride * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&c.marker_tile, (size_t)n * sizeof(uint32_t));
    if (e != hipSuccess) {
        hipFree(c.entries);
        hipFree(c.cf_rows);
        c.entries = nullptr;
        c.cf_rows = nullptr;
        return hip_fail(ctx, e, "spread scratch");
    }
    c.cap_markers = n;
    c.cf_stride = stride;
    return MLS_OK;
}

static mls_status ensure_tables(mls_ctx *ctx, hipStream_t s)
{
    Ctx &c = ctx->c;
    if (c.tables) return MLS_OK;
    if (c.stretched_axis == -2)
        return fail(ctx, MLS_E_ARG, "fast-MLS needs a grid stretched along at most one axis");
    const int64_t rows = (int64_t)c.opts.n_sub * c.opts.n_sub * c.opts.n_sub;
    if (c.stretched_axis < 0) {
        c.n_tables = 1;
        c.table_first[0] = c.table_first[1] = 0;
    } else {
        const Axis &a = c.g.ax[c.stretched_axis];
        const int n0 = a.n;
        const int n1 = a.periodic ? a.n : a.n + 1;
        c.table_first[0] = 0;
        c.table_first[1] = n0;
        c.n_tables = n0 + n1;
    }
    hipError_t e = hipMalloc((void **)&c.tables, (size_t)c.n_tables * rows * kTableStride * sizeof(float));
    if (e != hipSuccess) { c.tables = nullptr; return hip_fail(ctx, e, "fast-MLS tables"); }
    e = hipMalloc((void **)&c.table_geo, (size_t)c.n_tables * 6 * sizeof(float));
    if (e != hipSuccess) { hipFree(c.tables); c.tables = nullptr; return hip_fail(ctx, e, "fast-MLS tables"); }
    e = launch_table_build(c, s);
    if (e != hipSuccess) {
        hipFree(c.tables); hipFree(c.table_geo);
        c.tables = nullptr; c.table_geo = nullptr;
        return hip_fail(ctx, e, "fast-MLS table build");
    }
    return MLS_OK;
}

mls_status mls_build(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, int32_t method,
                     uint32_t *home, float *phi, uint8_t *route, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count %lld", (long long)n);
    if (n > 0 && (!x || !y || !z || !home || !phi)) return fail(ctx, MLS_E_ARG, "null array");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    hipError_t e;
    switch (method) {
    case MLS_EXACT: {
        TimedLaunch t(c, MLS_K_BUILD_EXACT, s);
        e = launch_build_exact(c, n, x, y, z, home, phi, route, s);
        break;
    }
    case MLS_FAST:
    case MLS_FAST_LINEAR: {
        mls_status st = ensure_tables(ctx, s);
        if (st != MLS_OK) return st;
        TimedLaunch t(c, MLS_K_BUILD_FAST, s);
        e = launch_build_fast(c, n, x, y, z, home, phi, route, s, method == MLS_FAST_LINEAR);
        break;
    }
    case MLS_LEARNED: {
        if (!c.mlp.loaded) return fail(ctx, MLS_E_ARG, "MLS_LEARNED needs a network (mls_mlp_load)");
        TimedLaunch t(c, MLS_K_BUILD_LEARNED, s);
        e = launch_build_learned(c, n, x, y, z, home, phi, route, s);
        break;
    }
    default:
        return fail(ctx, MLS_E_ARG, "unknown or unavailable method %d", method);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "build launch");
    return MLS_OK;
}

mls_status mls_interp(mls_ctx *ctx, int64_t n, const uint32_t *home, const float *phi, const float *u,
                      const float *v, const float *w, float *U, float *V, float *W, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count");
    if (n > 0 && (!home || !phi || !u || !v || !w || !U || !V || !W)) return fail(ctx, MLS_E_ARG, "null array");
    hipError_t e;
    {
        TimedLaunch t(ctx->c, MLS_K_INTERP, static_cast<hipStream_t>(stream));
        e = launch_interp(ctx->c, n, home, phi, u, v, w, U, V, W, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "interp launch");
    return MLS_OK;
}

mls_status mls_spread(mls_ctx *ctx, int64_t n, const uint32_t *home, const float *phi, const float *area,
                      const float *Fx, const float *Fy, const float *Fz, float *fx, float *fy, float *fz,
                      void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count");
    if (n > 0 && (!home || !phi || !area || !Fx || !Fy || !Fz || !fx || !fy || !fz))
        return fail(ctx, MLS_E_ARG, "null array");
    if (n == 0) return MLS_OK;
    mls_status st = mls_reserve(ctx, n);
    if (st != MLS_OK) return st;
    hipError_t e = launch_spread(ctx->c, n, home, phi, area, Fx, Fy, Fz, fx, fy, fz, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "spread launch");
    return MLS_OK;
}

mls_status mls_spread_noalloc(mls_ctx *ctx, int64_t n, const uint32_t *home, const float *phi, const float *area,
                              const float *Fx, const float *Fy, const float *Fz, float *fx, float *fy, float *fz,
                              void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count");
    if (n > 0 && (!home || !phi || !area || !Fx || !Fy || !Fz || !fx || !fy || !fz))
        return fail(ctx, MLS_E_ARG, "null array");
    if (n == 0) return MLS_OK;
    if (noalloc_bytes(ctx->c, n) > (size_t)MLS_SPREAD_NOALLOC_BYTES)
        return fail(ctx, MLS_E_ARG, "spread_noalloc: markers and grid tiles need more scratch than the fixed "
                                    "MLS_SPREAD_NOALLOC_BYTES array holds");
    hipError_t e = launch_spread_noalloc(ctx->c, n, home, phi, area, Fx, Fy, Fz, fx, fy, fz,
                                         static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "spread_noalloc launch");
    return MLS_OK;
}

mls_status mls_collide(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                       const int32_t *body, int32_t *coll, uint8_t *flags, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count");
    if (n > 0 && (!x || !y || !z || !body || !coll)) return fail(ctx, MLS_E_ARG, "null array");
    hipError_t e;
    {
        TimedLaunch t(ctx->c, MLS_K_COLLIDE, static_cast<hipStream_t>(stream));
        e = launch_collide(ctx->c, n, x, y, z, body, coll, flags, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "collide launch");
    return MLS_OK;
}

mls_status mls_collide_clear(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                             int32_t *coll, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count");
    if (n > 0 && (!x || !y || !z || !coll)) return fail(ctx, MLS_E_ARG, "null array");
    hipError_t e;
    {
        TimedLaunch t(ctx->c, MLS_K_COLLIDE_CLEAR, static_cast<hipStream_t>(stream));
        e = launch_collide_clear(ctx->c, n, x, y, z, coll, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "collide clear launch");
    return MLS_OK;
}

mls_status mls_refine(mls_ctx *ctx, int64_t ntri, const int32_t *tri, int64_t nvert, const float *xv,
                      const float *yv, const float *zv, double ratio, int32_t level, int64_t capacity, float *x,
                      float *y, float *z, float *area, float *normal, int32_t *parent, uint8_t *tri_level,
                      int64_t *count, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (ntri < 0 || ntri > (int64_t)1 << 28) return fail(ctx, MLS_E_ARG, "bad triangle count");
    if (nvert < 0 || nvert > (int64_t)0x7fffffff) return fail(ctx, MLS_E_ARG, "bad vertex count");
    if (level < -1 || level > 3) return fail(ctx, MLS_E_ARG, "refinement level must be -1 (adaptive) or 0..3");
    if (level < 0 && !(ratio > 0.0 && ratio < 1e30)) return fail(ctx, MLS_E_ARG, "bad refinement ratio");
    if (capacity < 4 * ntri) return fail(ctx, MLS_E_ARG, "capacity below 4 markers per triangle");
    if (!count) return fail(ctx, MLS_E_ARG, "null count");
    if (ntri > 0 && (!tri || !xv || !yv || !zv || !x || !y || !z || !area || !normal || !parent || !tri_level))
        return fail(ctx, MLS_E_ARG, "null array");
    hipError_t e;
    {
        TimedLaunch t(ctx->c, MLS_K_REFINE, static_cast<hipStream_t>(stream));
        e = launch_refine(ctx->c, ntri, tri, nvert, xv, yv, zv, ratio, level, capacity, x, y, z, area, normal,
                          parent, tri_level, count, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "refine launch");
    return MLS_OK;
}

mls_status mls_build_grad(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                          int32_t stagger, uint32_t *home, float *phi, float *dphi, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count");
    if (stagger < 0 || stagger > 3) return fail(ctx, MLS_E_ARG, "staggering must be 0, 1, 2 (u, v, w) or 3 (cells)");
    if (n > 0 && (!x || !y || !z || !home || !phi || !dphi)) return fail(ctx, MLS_E_ARG, "null array");
    hipError_t e;
    {
        TimedLaunch t(ctx->c, MLS_K_BUILD_GRAD, static_cast<hipStream_t>(stream));
        e = launch_build_grad(ctx->c, n, x, y, z, stagger, home, phi, dphi, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "build_grad launch");
    return MLS_OK;
}

mls_status mls_interp_grad(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                           const float *u, const float *v, const float *w, float *U, float *G, const float *p,
                           float *P, float *GP, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count");
    if (n > 0 && (!x || !y || !z || !u || !v || !w || !G)) return fail(ctx, MLS_E_ARG, "null array");
    if (n > 0 && p && !P && !GP) return fail(ctx, MLS_E_ARG, "pressure given without an output");
    hipError_t e;
    {
        TimedLaunch t(ctx->c, MLS_K_INTERP_GRAD, static_cast<hipStream_t>(stream));
        e = launch_interp_grad(ctx->c, n, x, y, z, u, v, w, p, U, G, P, GP, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "interp_grad launch");
    return MLS_OK;
}

mls_status mls_sync(mls_ctx *ctx, void *stream, int64_t *first_bad)
{
    if (first_bad) *first_bad = -1;
    if (!ctx) return MLS_E_ARG;
    Ctx &c = ctx->c;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronize");
    unsigned long long w = 0;
    e = hipMemcpy(&w, c.err, sizeof(w), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "error word read");
    if (w == kNoError) return MLS_OK;
    const unsigned long long none = kNoError;
    hipMemcpy(c.err, &none, sizeof(none), hipMemcpyHostToDevice);
    const int status = -(int)(w & 0xff);
    const int64_t marker = (int64_t)(w >> 8);
    if (first_bad) *first_bad = marker;
    static const char *names[] = {"ok", "argument", "support leaves a wall axis", "singular moment matrix",
                                  "non-finite coordinate", "hip", "no memory", "spread contribution out of range"};
    const int idx = -status;
    return fail(ctx, (mls_status)status, "device error at marker %lld: %s", (long long)marker,
                (idx >= 0 && idx < 8) ? names[idx] : "unknown");
}

const char *mls_last_error(const mls_ctx *ctx)
{
    return ctx ? ctx->c.last_error.c_str() : "null context";
}

mls_status mls_stats_get(mls_ctx *ctx, mls_stats *out)
{
    if (!ctx || !out) return MLS_E_ARG;
    Ctx &c = ctx->c;
    if (hipDeviceSynchronize() != hipSuccess) return MLS_E_HIP;
    DevStats d;
    if (hipMemcpy(&d, c.stats, sizeof(d), hipMemcpyDeviceToHost) != hipSuccess) return MLS_E_HIP;
    out->fp64_solves = (int64_t)d.fp64_solves;
    out->fallbacks = (int64_t)d.fallbacks;
    out->learned = (int64_t)d.learned;
    float km;
    memcpy(&km, &d.kappa_max_bits, sizeof(km));
    out->kappa_max = km;
    uint32_t total = 0;
    if (c.cap_markers > 0)
        hipMemcpy(&total, c.tile_off + c.g.ntiles, sizeof(total), hipMemcpyDeviceToHost);
    out->spread_entries = total;
    out->spread_tiles = c.g.ntiles;
    return MLS_OK;
}

mls_status mls_stats_reset(mls_ctx *ctx)
{
    if (!ctx) return MLS_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MLS_E_HIP;
    return hipMemset(ctx->c.stats, 0, sizeof(DevStats)) == hipSuccess ? MLS_OK : MLS_E_HIP;
}

mls_status mls_fast_tables(mls_ctx *ctx, float *dst, int64_t *count, int32_t *row_stride, int32_t first[2],
                           int32_t *stretched_axis, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    mls_status st = ensure_tables(ctx, s);
    if (st != MLS_OK) return st;
    Ctx &c = ctx->c;
    if (count) *count = c.n_tables;
    if (row_stride) *row_stride = kTableStride;
    if (first) { first[0] = c.table_first[0]; first[1] = c.table_first[1]; }
    if (stretched_axis) *stretched_axis = c.stretched_axis;
    if (dst) {
        const size_t bytes = (size_t)c.n_tables * c.opts.n_sub * c.opts.n_sub * c.opts.n_sub * kTableStride *
                             sizeof(float);
        hipError_t e = hipMemcpyAsync(dst, c.tables, bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "table copy");
    }
    return MLS_OK;
}

// ---- learned surrogate --------------------------------------------------------

mls_status mls_mlp_load(mls_ctx *ctx, const float *params, const float *norm)
{
    if (!ctx || !params || !norm) return MLS_E_ARG;
    Ctx &c = ctx->c;
    for (int i = 0; i < kMlpParams; ++i)
        if (!std::isfinite(params[i])) return fail(ctx, MLS_E_ARG, "non-finite network parameter %d", i);
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(norm[i])) return fail(ctx, MLS_E_ARG, "non-finite input normalisation %d", i);
    hipError_t e = mlp_alloc(c);
    if (e != hipSuccess) return hip_fail(ctx, e, "network allocation");
    if (hipDeviceSynchronize() != hipSuccess) return MLS_E_HIP;
    Mlp &net = c.mlp;
    e = hipMemcpy(net.params, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(net.norm, norm, 12 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(net.m1, 0, 2 * (size_t)kMlpParams * sizeof(float));
    if (e != hipSuccess) return hip_fail(ctx, e, "network upload");
    memcpy(net.h_norm, norm, sizeof(net.h_norm));
    net.adam_step = 0;
    net.version += 1;
    net.loaded = true;
    return MLS_OK;
}

mls_status mls_mlp_get(mls_ctx *ctx, float *params, float *norm)
{
    if (!ctx) return MLS_E_ARG;
    Ctx &c = ctx->c;
    if (!c.mlp.loaded) return fail(ctx, MLS_E_ARG, "no network loaded");
    if (hipDeviceSynchronize() != hipSuccess) return MLS_E_HIP;
    if (params && hipMemcpy(params, c.mlp.params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return MLS_E_HIP;
    if (norm) memcpy(norm, c.mlp.h_norm, sizeof(c.mlp.h_norm));
    return MLS_OK;
}

mls_status mls_features(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, float *feat,
                        void *stream)
{
    if (!ctx) return MLS_E_ARG;
    if (n < 0 || n > (int64_t)0x1fffffff) return fail(ctx, MLS_E_ARG, "bad marker count");
    if (n > 0 && (!x || !y || !z || !feat)) return fail(ctx, MLS_E_ARG, "null array");
    hipError_t e = launch_features(ctx->c, n, x, y, z, feat, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "features launch");
    return MLS_OK;
}

static mls_status mlp_batch_check(mls_ctx *ctx, int64_t m, const float *feat, int64_t rows, const int64_t *idx)
{
    Ctx &c = ctx->c;
    if (!c.mlp.loaded) return fail(ctx, MLS_E_ARG, "no network loaded");
    if (m < 0 || m > ((int64_t)1 << 26)) return fail(ctx, MLS_E_ARG, "bad batch size %lld", (long long)m);
    if (m > 0 && !feat) return fail(ctx, MLS_E_ARG, "null array");
    if (rows < 0 || (!idx && m > rows)) return fail(ctx, MLS_E_ARG, "batch of %lld rows from %lld", (long long)m,
                                                    (long long)rows);
    hipError_t e = mlp_reserve(c, m);
    if (e != hipSuccess) return hip_fail(ctx, e, "training scratch");
    return MLS_OK;
}

mls_status mls_mlp_forward(mls_ctx *ctx, int64_t m, const float *feat, int64_t rows, const int64_t *idx, float *out,
                           void *stream)
{
    if (!ctx) return MLS_E_ARG;
    mls_status st = mlp_batch_check(ctx, m, feat, rows, idx);
    if (st != MLS_OK) return st;
    if (m > 0 && !out) return fail(ctx, MLS_E_ARG, "null array");
    hipError_t e = mlp_forward_batch(ctx->c, m, feat, rows, idx, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "network forward");
    return MLS_OK;
}

mls_status mls_mlp_grad(mls_ctx *ctx, int64_t m, const float *feat, const float *target, int64_t rows,
                        const int64_t *idx, float mu, float *grad, float *loss, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    mls_status st = mlp_batch_check(ctx, m, feat, rows, idx);
    if (st != MLS_OK) return st;
    if (m < 1 || !target || !grad || !loss) return fail(ctx, MLS_E_ARG, "null array or empty batch");
    if (!(mu >= 0.0f) || !std::isfinite(mu)) return fail(ctx, MLS_E_ARG, "bad mu");
    hipError_t e = mlp_grad_batch(ctx->c, m, feat, target, rows, idx, mu, grad, loss, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "network gradient");
    return MLS_OK;
}

mls_status mls_mlp_train_step(mls_ctx *ctx, int64_t m, const float *feat, const float *target, int64_t rows,
                              const int64_t *idx, float mu, float lr, float *loss, void *stream)
{
    if (!ctx) return MLS_E_ARG;
    mls_status st = mlp_batch_check(ctx, m, feat, rows, idx);
    if (st != MLS_OK) return st;
    if (m < 1 || !target) return fail(ctx, MLS_E_ARG, "null array or empty batch");
    if (!(mu >= 0.0f) || !std::isfinite(mu) || !(lr >= 0.0f) || !std::isfinite(lr))
        return fail(ctx, MLS_E_ARG, "bad mu or learning rate");
    Ctx &c = ctx->c;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = mlp_grad_batch(c, m, feat, target, rows, idx, mu, c.mlp.grad, loss ? loss : c.mlp.loss, s);
    if (e == hipSuccess) e = mlp_adam(c, lr, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "training step");
    return MLS_OK;
}

}  // extern "C"
