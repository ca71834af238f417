// Launch-shape autotuner (an addition to the paper's method).
//
// The tunable shapes are the spreading tile edge (which sets the LDS box of a
// tile workgroup and so how many fit a compute unit) and the resident
// workgroups per compute unit of the build, interpolation and spreading
// launches.  mls_autotune times candidates of each phase on the caller's own
// step buffers with HIP events, keeps the fastest and remembers it in a
// JSON-lines cache keyed by device architecture, compute units, grid, method
// and marker-count octave, so that a later run on the same kind of device and
// problem applies the stored shapes without timing.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "mls_internal.h"

using namespace mls;

namespace {

// Milliseconds of one call of fn on stream s: the fastest of `reps` timed
// calls after one untimed call.
template <typename F>
double time_call(hipStream_t s, int reps, F fn, bool &ok)
{
    hipEvent_t a = nullptr, b = nullptr;
    ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
    double best = 1e30;
    if (ok) ok = fn() == MLS_OK;
    for (int r = 0; r < reps && ok; ++r) {
        ok = hipEventRecord(a, s) == hipSuccess;
        ok = ok && fn() == MLS_OK;
        ok = ok && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
        float ms = 0.0f;
        ok = ok && hipEventElapsedTime(&ms, a, b) == hipSuccess;
        if (ok) best = std::min(best, (double)ms);
    }
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    return best;
}

std::string tune_key(const Ctx &c, int method, int flags, int64_t n)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c.device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    const int oct = n > 0 ? (int)std::floor(std::log2((double)n)) : 0;
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|cu%d|%dx%dx%d|p%d%d%d|s%d|m%d|f%d|n%d", arch.c_str(), c.cu_count, c.g.ax[0].n,
             c.g.ax[1].n, c.g.ax[2].n, c.g.ax[0].periodic, c.g.ax[1].periodic, c.g.ax[2].periodic, c.stretched_axis,
             method, flags, oct);
    return buf;
}

bool json_int(const std::string &line, const char *name, int &out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    out = (int)strtol(line.c_str() + p + pat.size(), nullptr, 10);
    return true;
}

bool json_double(const std::string &line, const char *name, double &out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    out = strtod(line.c_str() + p + pat.size(), nullptr);
    return true;
}

bool cache_lookup(const char *path, const std::string &key, mls_tune_report &rep)
{
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    const std::string pat = "\"key\":\"" + key + "\"";
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {   // the last entry of a key wins
        if (line.find(pat) == std::string::npos) continue;
        mls_tune t;
        if (json_int(line, "spread_tile", t.spread_tile) &&
            json_int(line, "spread_blocks_per_cu", t.spread_blocks_per_cu) &&
            json_int(line, "build_blocks_per_cu", t.build_blocks_per_cu) &&
            json_int(line, "interp_blocks_per_cu", t.interp_blocks_per_cu) &&
            json_int(line, "spread_threads", t.spread_threads)) {
            rep.best = t;
            json_double(line, "ms_build", rep.ms_build);
            json_double(line, "ms_interp", rep.ms_interp);
            json_double(line, "ms_spread", rep.ms_spread);
            found = true;
        }
    }
    return found;
}

void cache_append(const char *path, const std::string &key, const mls_tune_report &rep)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f,
            "{\"key\":\"%s\",\"spread_tile\":%d,\"spread_blocks_per_cu\":%d,\"build_blocks_per_cu\":%d,"
            "\"interp_blocks_per_cu\":%d,\"spread_threads\":%d,\"ms_build\":%.4f,\"ms_interp\":%.4f,"
            "\"ms_spread\":%.4f,\"candidates\":%d}\n",
            key.c_str(), rep.best.spread_tile, rep.best.spread_blocks_per_cu, rep.best.build_blocks_per_cu,
            rep.best.interp_blocks_per_cu, rep.best.spread_threads, rep.ms_build, rep.ms_interp, rep.ms_spread,
            rep.candidates);
    fclose(f);
}

bool bpc_ok(int v) { return v >= 1 && v <= kMaxBlocksPerCu; }

}  // namespace

extern "C" {

mls_status mls_tune_get(mls_ctx *ctx, mls_tune *out)
{
    if (!ctx || !out) return MLS_E_ARG;
    const Ctx &c = ctx->c;
    out->spread_tile = c.opts.spread_tile;
    out->spread_blocks_per_cu = c.spread_blocks_per_cu_req;
    out->build_blocks_per_cu = c.build_blocks_per_cu;
    out->interp_blocks_per_cu = c.interp_blocks_per_cu;
    out->spread_threads = c.spread_threads;
    return MLS_OK;
}

mls_status mls_tune_set(mls_ctx *ctx, const mls_tune *in)
{
    if (!ctx || !in) return MLS_E_ARG;
    Ctx &c = ctx->c;
    if (!bpc_ok(in->spread_blocks_per_cu) || !bpc_ok(in->build_blocks_per_cu) || !bpc_ok(in->interp_blocks_per_cu) ||
        in->spread_tile < 4 || in->spread_tile > kMaxBoxTile ||
        (in->spread_threads != 128 && in->spread_threads != 192 && in->spread_threads != 256))
        return MLS_E_ARG;
    c.spread_blocks_per_cu_req = in->spread_blocks_per_cu;
    c.spread_threads = in->spread_threads;
    c.build_blocks_per_cu = in->build_blocks_per_cu;
    c.interp_blocks_per_cu = in->interp_blocks_per_cu;
    if (in->spread_tile != c.opts.spread_tile) {
        const mls_status st = setup_tiles(c, in->spread_tile);
        if (st != MLS_OK) return st;
    } else {
        const int64_t lds = (int64_t)spread_lds_bytes(c);
        c.spread_blocks_per_cu = std::max(1, std::min(c.spread_blocks_per_cu_req, (int)((160 * 1024) / (lds + 512))));
    }
    return MLS_OK;
}

mls_status mls_autotune(mls_ctx *ctx, int32_t method, int32_t flags, const mls_step_buffers *b,
                        const char *cache_path, mls_tune_report *out, void *stream)
{
    if (!ctx || !b || !out || (flags & ~MLS_STEP_COMPACT) != 0) return MLS_E_ARG;
    Ctx &c = ctx->c;
    const int64_t n = b->n;
    if (n < 1 || !b->x0 || !b->y0 || !b->z0 || !b->area || !b->home || !b->phi || !b->u || !b->v || !b->w || !b->U ||
        !b->F || !b->fx || !b->fy || !b->fz)
        return MLS_E_ARG;
    if (method < MLS_EXACT || method > MLS_FAST_LINEAR || (method == MLS_LEARNED && !c.mlp.loaded)) return MLS_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    memset(out, 0, sizeof(*out));
    mls_tune cur;
    mls_tune_get(ctx, &cur);
    // the compact rows apply to exact MLS only; other methods tune as without them
    if (method != MLS_EXACT) flags = 0;
    const std::string key = tune_key(c, method, flags, n);
    if (cache_lookup(cache_path, key, *out)) {
        out->from_cache = 1;
        const mls_status st = mls_tune_set(ctx, &out->best);
        if (st == MLS_OK) return MLS_OK;
        memset(out, 0, sizeof(*out));   // a stale entry: tune again
    }
    mls_status st = mls_reserve(ctx, n);
    if (st != MLS_OK) return st;
    const bool compact = (flags & MLS_STEP_COMPACT) != 0;
    if (compact) {
        st = reserve_compact(ctx, n);
        if (st != MLS_OK) return st;
    }
    // the build and spreading launches below use the row width of the step
    // being tuned, and only during tuning
    struct NfReset {
        Ctx &c;
        ~NfReset() { c.step_nf = 0; }
    } nf_reset{c};
    c.step_nf = compact ? compact_nf(c) : 0;
    const bool timing = c.timing;
    c.timing = false;
    float *U = b->U, *V = b->U + n, *Wv = b->U + 2 * n;
    const float *F = b->F;
    // the exact step bins the markers and runs the build fused with
    // interpolation and forcing, then spreads in tile order
    const bool fast = method == MLS_FAST || method == MLS_FAST_LINEAR;
    if (fast) {
        st = mls_fast_tables(ctx, nullptr, nullptr, nullptr, nullptr, nullptr, stream);
        if (st != MLS_OK) { c.timing = timing; return st; }
    }
    // exact and (on uniform grids) fast-MLS run fused and in tile order; the
    // learned step runs in tile order too (the network fused with the
    // interpolation, forcing and c_l F_l of its rows)
    const bool learned = method == MLS_LEARNED;
    const bool exact = method == MLS_EXACT || (fast && fast_fused_ok(c)) || learned;
    auto build = [&]() {
        if (!exact) return mls_build(ctx, n, b->x0, b->y0, b->z0, method, b->home, b->phi, nullptr, stream);
        hipError_t e = launch_sort_positions(c, n, b->x0, b->y0, b->z0, s);
        if (e == hipSuccess) {
            if (learned) {
                const LearnedInterp li = learned_interp(c, b->u, b->v, b->w, b->vb, b->area, 1.0f, b->U, b->F);
                e = launch_build_learned(c, n, b->x0, b->y0, b->z0, b->home, b->phi, nullptr, s, c.entries, &li);
            } else if (fast)
                e = launch_fast_interp(c, n, b->x0, b->y0, b->z0, b->home, b->phi, nullptr, b->u, b->v, b->w, b->vb,
                                       b->area, 1.0f, b->U, b->F, s, method == MLS_FAST_LINEAR);
            else
                e = launch_build_interp(c, n, b->x0, b->y0, b->z0, b->home, b->phi, nullptr, b->u, b->v, b->w, b->vb,
                                        b->area, 1.0f, b->U, b->F, s);
        }
        return e == hipSuccess ? MLS_OK : MLS_E_HIP;
    };
    auto interp = [&]() {
        if (learned) return MLS_OK;   // fused into the learned build
        return mls_interp(ctx, n, b->home, b->phi, b->u, b->v, b->w, U, V, Wv, stream);
    };
    auto spread = [&]() {
        if (exact)
            return launch_spread_sorted(c, n, b->home, b->phi, b->fx, b->fy, b->fz, s) == hipSuccess ? MLS_OK
                                                                                                     : MLS_E_HIP;
        return mls_spread(ctx, n, b->home, b->phi, b->area, F, F + n, F + 2 * n, b->fx, b->fy, b->fz, stream);
    };
    bool ok = true;
    int cand = 0;
    mls_tune best = cur;
    // build shapes (the learned build has one workgroup per compute unit)
    double t_build = 1e30;
    const int bpcs[] = {8, 16, 32, 64};
    if (method != MLS_LEARNED) {
        for (int v : bpcs) {
            c.build_blocks_per_cu = v;
            const double t = time_call(s, 3, build, ok);
            if (!ok) break;
            ++cand;
            if (t < t_build) { t_build = t; best.build_blocks_per_cu = v; }
        }
        c.build_blocks_per_cu = best.build_blocks_per_cu;
    } else {
        t_build = time_call(s, 3, build, ok);
    }
    // interpolation shapes (needs valid home / phi from the build above)
    double t_interp = 1e30;
    const int ipcs[] = {8, 16, 32, 64};
    for (int v : ipcs) {
        if (!ok) break;
        c.interp_blocks_per_cu = v;
        const double t = time_call(s, 3, interp, ok);
        if (!ok) break;
        ++cand;
        if (t < t_interp) { t_interp = t; best.interp_blocks_per_cu = v; }
    }
    c.interp_blocks_per_cu = best.interp_blocks_per_cu;
    // forces F = (V_b - U) / 1 for the spreading candidates (the exact build
    // writes them itself)
    if (ok && !exact) ok = launch_force(c, n, b->vb, b->U, 1.0f, b->F, s) == hipSuccess;
    // spreading: tile edge x resident workgroups
    double t_spread = 1e30;
    const int tiles[] = {4, 6, 8, 10, 12, 16};
    const int spcs[] = {1, 2, 4, 8, 16, 32};
    const int sthreads[] = {128, 192, 256};
    std::vector<std::vector<int>> seen;
    for (int tile : tiles) {
        if (!ok) break;
        if (setup_tiles(c, tile) != MLS_OK) continue;
        std::vector<int> shape = {c.g.ax[0].tile, c.g.ax[1].tile, c.g.ax[2].tile};
        if (std::find(seen.begin(), seen.end(), shape) != seen.end()) continue;
        seen.push_back(shape);
        if (exact) ok = build() == MLS_OK;   // bin for this tiling (untimed)
        for (int th : sthreads) {
            int last_eff = -1;
            c.spread_threads = th;
            for (int v : spcs) {
                const int64_t lds = (int64_t)spread_lds_bytes(c);
                const int eff = std::max(1, std::min(v, (int)((160 * 1024) / (lds + 512))));
                if (eff == last_eff) continue;
                last_eff = eff;
                c.spread_blocks_per_cu_req = v;
                c.spread_blocks_per_cu = eff;
                const double t = time_call(s, 3, spread, ok);
                if (!ok) break;
                ++cand;
                if (t < t_spread) {
                    t_spread = t;
                    best.spread_tile = tile;
                    best.spread_blocks_per_cu = v;
                    best.spread_threads = th;
                }
            }
        }
    }
    c.timing = timing;
    if (!ok) {
        mls_tune_set(ctx, &cur);
        return MLS_E_HIP;
    }
    st = mls_tune_set(ctx, &best);
    if (st != MLS_OK) return st;
    out->best = best;
    out->ms_build = t_build;
    out->ms_interp = t_interp;
    out->ms_spread = t_spread;
    out->candidates = cand;
    cache_append(cache_path, key, *out);
    return MLS_OK;
}

}  // extern "C"
