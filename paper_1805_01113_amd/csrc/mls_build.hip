// Transfer-function build kernels: exact MLS (eq. 3-6) and fast-MLS
// (eq. 9-10), one lane per marker.
//
// A lane locates its marker on the six (axis, staggering type) node sets,
// evaluates the 1-D weights and moments once per set, and then, for each of
// the three velocity components, assembles the 4x4 moment matrix from the
// 1-D moments, solves it in FP32 (FP64 if its condition number exceeds the
// routing threshold) and writes the 27 shape-function values.  Stores are
// SoA, so a wavefront writes 64 consecutive floats per (component, node).
#include "mls_exact.h"

namespace mls {

namespace {

constexpr int kBlock = 256;

// Work split of the build kernels.  64 consecutive markers (rows) form an
// item, and each item is handled by three wavefronts, one per velocity
// component, so a wavefront stores 64 consecutive floats per support node and
// its component is uniform.  The wavefronts of the grid are numbered
// XCD-contiguously (workgroup xcd_block(), then wavefront within it);
// wavefront gw takes component gw % 3 of the items gw / 3, gw / 3 + S, ...,
// where S is a third of the grid's wavefronts.  A workgroup is kBuildWaves
// wavefronts whatever the register budget, so the compute unit's wavefront
// slots fill completely (a workgroup of two whole items, six wavefronts, left
// two of eight slots idle at two wavefronts per SIMD).  The grid is a multiple
// of 24 workgroups: the three wavefronts of an item then run on one XCD.
constexpr int kBuildWaves = 4;
constexpr int kBuildBlock = 64 * kBuildWaves;

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

struct WaveWork {
    int c;            // velocity component
    int64_t base;     // first row of the first item
    int64_t stride;   // rows between successive items of the wavefront
};

__device__ __forceinline__ WaveWork wave_work()
{
    const int gw = (int)xcd_block() * kBuildWaves + wave_id();
    const int tw = (int)gridDim.x * kBuildWaves;
    return {gw % 3, (int64_t)(gw / 3) * 64, (int64_t)(tw / 3) * 64};
}

__global__ void __launch_bounds__(kBuildBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_build_exact(const Grid *__restrict__ gp, const Weight W, float tau, int64_t n,
              const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z,
              uint32_t *__restrict__ home, float *__restrict__ phi, uint8_t *__restrict__ route,
              ErrWord *err, DevStats *st)
{
    const Grid &g = *gp;
    const int lane = threadIdx.x & 63;
    const WaveWork ww = wave_work();
    const int c = ww.c;
    const int64_t gstride = ww.stride;
    unsigned long long routed = 0;
    float kmax = 0.f;
    // the next item's coordinates are loaded one iteration ahead
    int64_t base = ww.base;
    float nx = 0.f, ny = 0.f, nz = 0.f;
    if (base + lane < n) { nx = x[base + lane]; ny = y[base + lane]; nz = z[base + lane]; }
    for (; base < n; base += gstride) {
        const int64_t l = base + lane;
        const float cx = nx, cy = ny, cz = nz;
        if (base + gstride + lane < n) {
            nx = x[base + gstride + lane];
            ny = y[base + gstride + lane];
            nz = z[base + gstride + lane];
        }
        if (l >= n) continue;
        // this wavefront's contiguous slice of the outputs (wave-uniform base)
        float *out = phi + ((((base >> 6) * 3 + c) * kNe) << 6) + lane;
        uint32_t *hout = home + (((base >> 6) * 3 + c) << 6) + lane;
        uint8_t *rout = route ? route + (((base >> 6) * 3 + c) << 6) + lane : nullptr;
        const double px = (double)cx, py = (double)cy, pz = (double)cz;
        AxisGeo G[3];
        bool ok = axis_geo(g.ax[0], c == 0, px, G[0]);
        ok = ok && axis_geo(g.ax[1], c == 1, py, G[1]);
        ok = ok && axis_geo(g.ax[2], c == 2, pz, G[2]);
        if (!ok) {
            mark_failed(err, l, px, py, pz, hout, out, rout);
            continue;
        }
        *hout = pack_home(G[0].ih, G[1].ih, G[2].ih);
        float ph[kNe];
        exact_from_geo(g, W, tau, c, l, px, py, pz, G, out, rout, 0, err, routed, kmax, ph);
    }
    // one atomic per wavefront for the statistics
    unsigned long long tot = routed;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    float km = kmax;
    for (int off = 32; off > 0; off >>= 1) km = fmaxf(km, __shfl_xor(km, off));
    if (lane == 0) {
        if (tot) atomicAdd(&st->fp64_solves, tot);
        if (km > 0.f) atomicMax(&st->kappa_max_bits, __float_as_uint(km));
    }
}

// Exact build fused with the interpolation (eq. 6) and the direct forcing of
// a time step, over the markers in spreading-tile order: row p of the
// blocked home / phi / route layout belongs to marker m = order[p].  After a
// lane has the shape function of its (marker, component) it gathers the 27
// support values of that component's velocity and writes U[c][m] and
// F[c][m] = (V_b - U) / dt, so phi is not read back (the FP64 route reads its
// own stored values).  It also writes c_m F_m of eq. 8 by row (cf_rows), the
// value the spreading scatters with the shape function.
//
// NF = 0 stores the 27 values of phi per row and c_l F_l in cf_rows.  NF = 7
// or 13 stores the compact transfer function instead, with c_l F_l after it
// (rows of kCoefStride<NF> floats, one lane's row in 16-byte words, see
// coef_word): gamma = A^{-1} e_0, then per axis the centre offset s_1 (NF = 7,
// every axis uniform: the outer offsets are s_1 -+ 1 in FP32) or the three
// offsets s_a (NF = 13).  phi_k = W_k (gamma . p_k) follows from them with the
// weights; a row solved in FP64 is marked by a NaN gamma_0 and its position in
// tile order is queued in rq (count first), so that k_route_rows stores its
// phi and its c_l F_l.
template <int NF>
__global__ void __launch_bounds__(kBuildBlock) __attribute__((amdgpu_waves_per_eu(NF == 0 ? 2 : 3)))
k_build_interp(const Grid *__restrict__ gp, const Weight W, float tau, int64_t n, const uint32_t *__restrict__ order,
               const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z,
               uint32_t *__restrict__ home, float *__restrict__ phi, uint8_t *__restrict__ route,
               const float *__restrict__ u, const float *__restrict__ v, const float *__restrict__ w,
               const float *__restrict__ vb, const float *__restrict__ area, float inv_dt, float *__restrict__ U,
               float *__restrict__ F, float *__restrict__ cf_rows, int64_t cf_stride, float *__restrict__ coef,
               uint32_t *__restrict__ rq, uint32_t *__restrict__ tmax, int64_t tstride, ErrWord *err,
               DevStats *st)
{
    const Grid &g = *gp;
    const int lane = threadIdx.x & 63;
    const WaveWork ww = wave_work();
    const int c = ww.c;
    const int64_t gstride = ww.stride;
    const float *q = c == 0 ? u : (c == 1 ? v : w);
    const int nxc = g.dims[c][0], nyc = g.dims[c][1], nzc = g.dims[c][2];
    unsigned long long routed = 0;
    float kmax = 0.f;
    int64_t base = ww.base;
    // Pipelined operand loads: the marker of the item after next, and the
    // position and area of the next item, are requested an iteration ahead.
    // Loads and stores share one completion counter that drains in order, so
    // every path through the loop issues the same memory operations: a lane
    // past the end repeats the last marker (writing identical values, its
    // shape function into a padding row) and a marker without a support is
    // computed on a neutral stencil at node 0 and stored as NaN.  A branch
    // around stores would make the compiler wait for all of them before the
    // next item's operands.
    const int64_t last = n - 1;
    uint32_t nm = order[min(base + lane, last)];
    float nx = x[nm], ny = y[nm], nz = z[nm], na = area[nm];
    uint32_t nm2 = order[min(base + gstride + lane, last)];
    for (; base < n; base += gstride) {
        const bool valid = base + lane < n;
        const int64_t m = nm;
        const float cx = nx, cy = ny, cz = nz, ca = na;
        nm = nm2;
        nx = x[nm]; ny = y[nm]; nz = z[nm]; na = area[nm];
        nm2 = order[min(base + 2 * gstride + lane, last)];
        float *out = phi + ((((base >> 6) * 3 + c) * kNe) << 6) + lane;
        uint32_t *hout = home + (((base >> 6) * 3 + c) << 6) + lane;
        uint8_t *rout = route ? route + (((base >> 6) * 3 + c) << 6) + lane : nullptr;
        const double px = (double)cx, py = (double)cy, pz = (double)cz;
        AxisGeo G[3];
        bool ok = axis_geo(g.ax[0], c == 0, px, G[0]);
        ok = ok && axis_geo(g.ax[1], c == 1, py, G[1]);
        ok = ok && axis_geo(g.ax[2], c == 2, pz, G[2]);
        neutral_geo_unless(ok, G);
        st_stream(hout, ok ? pack_home(G[0].ih, G[1].ih, G[2].ih) : 0xffffffffu);
        // the 27 field values are requested before the solve, which hides
        // their latency
        uint32_t oy[3], oz[3];
        support_rows(ok, G[1].ih, G[2].ih, nxc, nyc, nzc, g.ax[1].periodic, g.ax[2].periodic, oy, oz);
        Support sp;
        load_support(q, ok ? G[0].ih : 1, nxc, oy, oz, sp);
        const float vbv = vb ? vb[c * n + m] : 0.0f;
        float ph[kNe];
        float gam[4] = {0.f, 0.f, 0.f, 0.f};
        bool fp64 = false;
        if (!exact_fp32(W, tau, G, ph, kmax, gam)) {
            // rare: FP64 re-solve from the position
            fp64 = true;
            if (valid) ++routed;
            // full rows solve in FP64 here; compact rows leave it to k_route_rows
            if constexpr (NF == 0)
                if (!solve_fp64_regs(g, W, c, px, py, pz, ph)) raise_error(err, m, MLS_E_SINGULAR);
        }
        if (rout) *rout = fp64 ? 1 : 0;
        const float nan = __builtin_nanf("");
        if constexpr (NF == 0) {
#pragma unroll
            for (int k = 0; k < kNe; ++k) st_stream(&out[k * kLanes], ok ? ph[k] : nan);
        } else {
            // queue the rows solved in FP64 (rare; one reservation per wavefront)
            const unsigned long long rmask = __ballot(fp64 && ok && valid);
            if (rmask) {
                uint32_t slot = 0;
                if (lane == 0) slot = atomicAdd(rq, (uint32_t)__popcll(rmask));
                slot = __shfl(slot, 0);
                if (fp64 && ok && valid)
                    rq[1 + slot + __popcll(rmask & ((1ull << lane) - 1ull))] = (uint32_t)((base + lane) << 2) | c;
            }
        }
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kNe; ++k) acc += ph[k] * sp.at(k);
        const float f = (vbv - acc) * inv_dt;
        st_stream(&U[c * n + m], ok ? acc : nan);
        st_stream(&F[c * n + m], ok ? f : nan);
        // c_l F_l (eq. 8) by row for the spreading (padding rows too); a queued
        // compact row gets its U, F and c F from k_route_rows
        const float cfv = eq8_coef_built(g, c, G[0].ih, G[1].ih, G[2].ih, ph, ca * f);
        if constexpr (NF == 0) {
            st_stream(&cf_rows[c * cf_stride + base + lane], ok ? cfv : 0.0f);
        } else {
            // the compact row: gamma (NaN gamma_0 marks a row solved in FP64),
            // the offsets and c_l F_l, in 16-byte words
            constexpr int rs = kCoefStride<NF>;
            const int64_t row = base + lane;
            auto word = [&](int q) { return reinterpret_cast<f32x4 *>(coef + coef_word(row, c, rs, q)); };
            const float cfs = ok ? cfv : 0.0f;
            st_stream(word(0), f32x4{ok && !fp64 ? gam[0] : nan, gam[1], gam[2], gam[3]});
            if constexpr (NF == 7) {
                st_stream(word(1), f32x4{G[0].s[1], G[1].s[1], G[2].s[1], cfs});
            } else {
                st_stream(word(1), f32x4{G[0].s[0], G[0].s[1], G[0].s[2], G[1].s[0]});
                st_stream(word(2), f32x4{G[1].s[1], G[1].s[2], G[2].s[0], G[2].s[1]});
                st_stream(word(3), f32x4{G[2].s[2], cfs, 0.0f, 0.0f});
            }
        }
        if (!ok) {
            raise_error(err, m, isfinite(px) && isfinite(py) && isfinite(pz) ? MLS_E_SUPPORT : MLS_E_NONFINITE);
        } else if (NF == 0 || !fp64) {
            // a non-finite force or coefficient (NaN fails too)
            if (!(fabsf(cfv) <= 3.0e38f)) raise_error(err, m, MLS_E_RANGE);
        }
        // the spreading tile's largest |c F| (rows come in tile order, so a
        // wavefront holds one or two tiles)
        const bool counted = valid && ok && (NF == 0 || !fp64);
        wave_key_max(tmax + c * tstride, counted ? (int64_t)tile_from_geo(g, c, G) : -1, finite_abs(cfv));
    }
    unsigned long long tot = routed;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    float km = kmax;
    for (int off = 32; off > 0; off >>= 1) km = fmaxf(km, __shfl_xor(km, off));
    if (lane == 0) {
        if (tot) atomicAdd(&st->fp64_solves, tot);
        if (km > 0.f) atomicMax(&st->kappa_max_bits, __float_as_uint(km));
    }
}

// Zeroes n words (a kernel rather than a memset node, for graph capture).
__global__ void k_clear_words(uint32_t *p, int64_t n)
{
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// The rows that the compact step build left to FP64: entry i of rq (after the
// count) is row << 2 | component, row in tile order.  For each, the FP64
// re-solve of the pair, its phi stored into the blocked rows, and the
// interpolation and direct forcing that the build skipped: U and F by marker,
// c F (eq. 8) into the row's compact slot (index nf of the row).
__global__ void __launch_bounds__(kBlock)
k_route_rows(const Grid *__restrict__ gp, const Weight W, int64_t n, const uint32_t *__restrict__ order,
             const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z,
             const uint32_t *__restrict__ home, const uint32_t *__restrict__ rq, float *__restrict__ phi,
             const float *__restrict__ u, const float *__restrict__ v, const float *__restrict__ w,
             const float *__restrict__ vb, const float *__restrict__ area, float inv_dt, float *__restrict__ U,
             float *__restrict__ F, float *__restrict__ coef, int nf, const uint32_t *__restrict__ marker_tile,
             uint32_t *__restrict__ tmax, int64_t tstride, ErrWord *err)
{
    const Grid &g = *gp;
    const uint32_t cnt = rq[0];
    const int rs = nf == 7 ? kCoefStride<7> : kCoefStride<13>;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const uint32_t e = rq[1 + i];
        const int64_t row = e >> 2;
        const int c = (int)(e & 3u);
        const uint32_t m = order[row];
        float ph[kNe];
        if (!solve_fp64_regs(g, W, c, (double)x[m], (double)y[m], (double)z[m], ph)) raise_error(err, m, MLS_E_SINGULAR);
        float *out = phi + phi_at(row, c);
#pragma unroll
        for (int k = 0; k < kNe; ++k) out[k * kLanes] = ph[k];
        int hi, hj, hk;
        unpack_home(home[home_at(row, c)], hi, hj, hk);
        const float *q = c == 0 ? u : (c == 1 ? v : w);
        const int nxc = g.dims[c][0], nyc = g.dims[c][1], nzc = g.dims[c][2];
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kNe; ++k) {
            const int64_t gx = nb_index(hi, k % 3 - 1, nxc, g.ax[0].periodic);
            const int64_t gy = nb_index(hj, (k / 3) % 3 - 1, nyc, g.ax[1].periodic);
            const int64_t gz = nb_index(hk, k / 9 - 1, nzc, g.ax[2].periodic);
            acc += ph[k] * q[(gz * nyc + gy) * nxc + gx];
        }
        const float vbv = vb ? vb[c * n + m] : 0.0f;
        const float f = (vbv - acc) * inv_dt;
        const float ca = area[m];
        U[c * n + m] = acc;
        F[c * n + m] = f;
        const float cfv = eq8_coef_built(g, c, hi, hj, hk, ph, ca * f);
        coef[coef_word(row, c, rs, nf >> 2) + (nf & 3)] = cfv;
        if (!(fabsf(cfv) <= 3.0e38f)) raise_error(err, m, MLS_E_RANGE);
        const float av = finite_abs(cfv);
        if (av > 0.f) atomicMax(&tmax[c * tstride + marker_tile[m]], __float_as_uint(av));
    }
}

// ---- fast-MLS --------------------------------------------------------------

// Shepard blend of one component from its table.  xi: in-cell offsets,
// geo: table's normalised home control volume [lo, hi) per axis.
__device__ __forceinline__ void shepard(const float *__restrict__ tab, const float *__restrict__ geo,
                                        int nsub, const float xi[3], float *__restrict__ out)
{
    int j0[3];
    float t0[3], step[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float lo = geo[2 * d], hi = geo[2 * d + 1];
        step[d] = (hi - lo) / (float)(nsub - 1);
        float t = (xi[d] - lo) / (hi - lo) * (float)(nsub - 1);
        int j = (int)floorf(t);
        j = min(max(j, 0), nsub - 2);
        j0[d] = j;
        t0[d] = lo + (float)j * step[d];
    }
    // squared distances to the 8 corners (normalised units)
    float d2[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float xs = t0[d] + (float)((i >> d) & 1) * step[d];
            float e = xi[d] - xs;
            acc += e * e;
        }
        d2[i] = acc;
    }
    // alpha_i = prod_{j != i} d_j^2 / sum_m prod_{j != m} d_j^2 (eq. 10 in a
    // form that stays finite when the marker sits on a sub-node)
    float pre[8], suf[8];
    pre[0] = 1.f;
#pragma unroll
    for (int i = 1; i < 8; ++i) pre[i] = pre[i - 1] * d2[i - 1];
    suf[7] = 1.f;
#pragma unroll
    for (int i = 6; i >= 0; --i) suf[i] = suf[i + 1] * d2[i + 1];
    float alpha[8], den = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) { alpha[i] = pre[i] * suf[i]; den += alpha[i]; }
    const float rden = 1.f / den;
    const float *row[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int s = (j0[0] + (i & 1)) + nsub * ((j0[1] + ((i >> 1) & 1)) + nsub * (j0[2] + ((i >> 2) & 1)));
        row[i] = tab + (int64_t)s * kTableStride;
        alpha[i] *= rden;
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float4 v = *reinterpret_cast<const float4 *>(row[i] + 4 * q);
            acc.x += alpha[i] * v.x; acc.y += alpha[i] * v.y; acc.z += alpha[i] * v.z; acc.w += alpha[i] * v.w;
        }
        const float vals[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * q + e;
            if (k < kNe) st_stream(&out[k * kLanes], vals[e]);
        }
    }
}

// Trilinear blend of the same table (the first "next" item beyond eq. 9-10):
// the 8 corners of the enclosing sub-cell weighted by the multilinear
// coordinates t_d of xi inside it.  The weights sum to one and reproduce xi,
// so the exact tables' partition of unity and linear reproduction carry over.
__device__ __forceinline__ void trilinear(const float *__restrict__ tab, const float *__restrict__ geo, int nsub,
                                          const float xi[3], float *__restrict__ out)
{
    int j0[3];
    float t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float lo = geo[2 * d], hi = geo[2 * d + 1];
        const float step = (hi - lo) / (float)(nsub - 1);
        int j = (int)floorf((xi[d] - lo) / (hi - lo) * (float)(nsub - 1));
        j = min(max(j, 0), nsub - 2);
        j0[d] = j;
        t[d] = (xi[d] - (lo + (float)j * step)) / step;
    }
    float alpha[8];
    const float *row[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        alpha[i] = ((i & 1) ? t[0] : 1.f - t[0]) * (((i >> 1) & 1) ? t[1] : 1.f - t[1]) *
                   (((i >> 2) & 1) ? t[2] : 1.f - t[2]);
        const int s = (j0[0] + (i & 1)) + nsub * ((j0[1] + ((i >> 1) & 1)) + nsub * (j0[2] + ((i >> 2) & 1)));
        row[i] = tab + (int64_t)s * kTableStride;
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float4 v = *reinterpret_cast<const float4 *>(row[i] + 4 * q);
            acc.x += alpha[i] * v.x; acc.y += alpha[i] * v.y; acc.z += alpha[i] * v.z; acc.w += alpha[i] * v.w;
        }
        const float vals[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * q + e;
            if (k < kNe) st_stream(&out[k * kLanes], vals[e]);
        }
    }
}

template <bool TRILINEAR>
__global__ void __launch_bounds__(kBuildBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_build_fast(const Grid *__restrict__ gp, const FastTables T, int64_t n,
             const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z,
             uint32_t *__restrict__ home, float *__restrict__ phi, uint8_t *__restrict__ route, ErrWord *err)
{
    const Grid &g = *gp;
    const int lane = threadIdx.x & 63;
    const WaveWork ww = wave_work();
    const int c = ww.c;
    const int64_t gstride = ww.stride;
    const int64_t rows = (int64_t)T.n_sub * T.n_sub * T.n_sub;
    // the next item's coordinates are loaded one iteration ahead
    int64_t base = ww.base;
    float nx = 0.f, ny = 0.f, nz = 0.f;
    if (base + lane < n) { nx = x[base + lane]; ny = y[base + lane]; nz = z[base + lane]; }
    for (; base < n; base += gstride) {
        const int64_t l = base + lane;
        const float cx = nx, cy = ny, cz = nz;
        if (base + gstride + lane < n) {
            nx = x[base + gstride + lane];
            ny = y[base + gstride + lane];
            nz = z[base + gstride + lane];
        }
        if (l >= n) continue;
        float *out = phi + ((((base >> 6) * 3 + c) * kNe) << 6) + lane;
        uint32_t *hout = home + (((base >> 6) * 3 + c) << 6) + lane;
        uint8_t *rout = route ? route + (((base >> 6) * 3 + c) << 6) + lane : nullptr;
        const double px = (double)cx, py = (double)cy, pz = (double)cz;
        AxisGeo G[3];
        bool ok = axis_geo(g.ax[0], c == 0, px, G[0]);
        ok = ok && axis_geo(g.ax[1], c == 1, py, G[1]);
        ok = ok && axis_geo(g.ax[2], c == 2, pz, G[2]);
        if (!ok) {
            mark_failed(err, l, px, py, pz, hout, out, rout);
            continue;
        }
        *hout = pack_home(G[0].ih, G[1].ih, G[2].ih);
        int t = 0;
        if (T.stretched_axis >= 0) {
            const int d = T.stretched_axis;
            t = T.first[c == d] + G[d].ih;
        }
        const float xi[3] = {G[0].xi, G[1].xi, G[2].xi};
        if (TRILINEAR) trilinear(T.tab + (int64_t)t * rows * kTableStride, T.geo + (int64_t)t * 6, T.n_sub, xi, out);
        else shepard(T.tab + (int64_t)t * rows * kTableStride, T.geo + (int64_t)t * 6, T.n_sub, xi, out);
        if (rout) *rout = 0;
    }
}

// fast-MLS fused with the interpolation and forcing of a time step, in
// spreading-tile order like k_build_interp, for a grid whose axes are all
// uniform (one table).  There the shape functions are mirror-symmetric in
// each axis: phi at -xi_d is phi at xi_d with the support nodes a and 2 - a
// of that axis exchanged, and with an odd sub-node count the sub-cells of the
// table never straddle xi_d = 0.  So the kernel keeps only the octant
// xi >= 0 of the table (nh^3 rows, nh = (n_sub + 1)/2: 14 KB for n_sub = 9)
// in LDS.  The sub-cell and the weights (Shepard of eq. 10, or trilinear) are
// those of the whole-table lookup; a corner in the negative half of an axis
// reads the row of its mirror image, and the blended nodes of every such axis
// are put back in place with a layer of conditional swaps.
template <bool TRILINEAR>
__global__ void __launch_bounds__(kBuildBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_fast_interp(const Grid *__restrict__ gp, const float4 *__restrict__ tab, int nsub, int64_t n,
              const uint32_t *__restrict__ order, const float *__restrict__ x, const float *__restrict__ y,
              const float *__restrict__ z, uint32_t *__restrict__ home, float *__restrict__ phi,
              uint8_t *__restrict__ route, const float *__restrict__ u, const float *__restrict__ v,
              const float *__restrict__ w, const float *__restrict__ vb, const float *__restrict__ area, float inv_dt,
              float *__restrict__ U, float *__restrict__ F, float *__restrict__ cf_rows, int64_t cf_stride,
              uint32_t *__restrict__ tmax, int64_t tstride, ErrWord *err)
{
    extern __shared__ float4 oct[];   // [nh^3][7]
    const Grid &g = *gp;
    const int nh = (nsub + 1) / 2, mid = (nsub - 1) / 2;
    {
        const int total = nh * nh * nh * 7;
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const int r = i / 7, q4 = i % 7;
            const int jx = r % nh, jy = (r / nh) % nh, jz = r / (nh * nh);
            const int s = (mid + jx) + nsub * ((mid + jy) + nsub * (mid + jz));
            oct[i] = tab[(int64_t)s * 7 + q4];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const WaveWork ww = wave_work();
    const int c = ww.c;
    const int64_t gstride = ww.stride;
    const float *q = c == 0 ? u : (c == 1 ? v : w);
    const int nxc = g.dims[c][0], nyc = g.dims[c][1], nzc = g.dims[c][2];
    const float scale = (float)(nsub - 1);   // sub-cells per unit of xi (home CV [-1/2, 1/2))
    const float step = 1.0f / scale;         // sub-cell width, (hi - lo) / (n_sub - 1)
    int64_t base = ww.base;
    // Operand loads pipelined an iteration ahead and one sequence of memory
    // operations on every path, as in k_build_interp.
    const int64_t last = n - 1;
    uint32_t nm = order[min(base + lane, last)];
    float nx = x[nm], ny = y[nm], nz = z[nm], na = area[nm];
    uint32_t nm2 = order[min(base + gstride + lane, last)];
    for (; base < n; base += gstride) {
        const int64_t m = nm;
        const float cx = nx, cy = ny, cz = nz, ca = na;
        nm = nm2;
        nx = x[nm]; ny = y[nm]; nz = z[nm]; na = area[nm];
        nm2 = order[min(base + 2 * gstride + lane, last)];
        float *out = phi + ((((base >> 6) * 3 + c) * kNe) << 6) + lane;
        uint32_t *hout = home + (((base >> 6) * 3 + c) << 6) + lane;
        uint8_t *rout = route ? route + (((base >> 6) * 3 + c) << 6) + lane : nullptr;
        const double px = (double)cx, py = (double)cy, pz = (double)cz;
        AxisGeo G[3];
        bool ok = axis_geo(g.ax[0], c == 0, px, G[0]);
        ok = ok && axis_geo(g.ax[1], c == 1, py, G[1]);
        ok = ok && axis_geo(g.ax[2], c == 2, pz, G[2]);
        neutral_geo_unless(ok, G);
        st_stream(hout, ok ? pack_home(G[0].ih, G[1].ih, G[2].ih) : 0xffffffffu);
        uint32_t oy[3], oz[3];
        support_rows(ok, G[1].ih, G[2].ih, nxc, nyc, nzc, g.ax[1].periodic, g.ax[2].periodic, oy, oz);
        float qv[kNe];
        load_support(q, ok ? G[0].ih : 1, nxc, oy, oz, qv);
        const float vbv = vb ? vb[c * n + m] : 0.0f;
        // the sub-cell and the blend weights in the true frame, as the
        // whole-table lookup computes them (so a marker on a sub-cell face
        // gets the same sub-cell); only the rows come from the mirror image
        bool flip[3];
        int jj[3];
        float tf[3], t0[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float xi = G[d].xi;
            int j = (int)floorf((xi + 0.5f) * scale);
            j = min(max(j, 0), nsub - 2);
            jj[d] = j;
            flip[d] = j < mid;
            t0[d] = -0.5f + (float)j * step;
            tf[d] = (xi - t0[d]) / step;
        }
        float alpha[8];
        if (TRILINEAR) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                alpha[i] = ((i & 1) ? tf[0] : 1.f - tf[0]) * (((i >> 1) & 1) ? tf[1] : 1.f - tf[1]) *
                           (((i >> 2) & 1) ? tf[2] : 1.f - tf[2]);
        } else {
            float d2[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float acc = 0.f;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const float e = G[d].xi - (t0[d] + (float)((i >> d) & 1) * step);
                    acc += e * e;
                }
                d2[i] = acc;
            }
            float pre[8], suf[8];
            pre[0] = 1.f;
#pragma unroll
            for (int i = 1; i < 8; ++i) pre[i] = pre[i - 1] * d2[i - 1];
            suf[7] = 1.f;
#pragma unroll
            for (int i = 6; i >= 0; --i) suf[i] = suf[i + 1] * d2[i + 1];
            float den = 0.f;
#pragma unroll
            for (int i = 0; i < 8; ++i) { alpha[i] = pre[i] * suf[i]; den += alpha[i]; }
            const float rden = 1.f / den;
#pragma unroll
            for (int i = 0; i < 8; ++i) alpha[i] *= rden;
        }
        float ph[28];
#pragma unroll
        for (int k = 0; k < 28; ++k) ph[k] = 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            // octant row of corner i: sub-node j + bit, mirrored on flipped axes
            int oj[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int jn = jj[d] + ((i >> d) & 1);
                oj[d] = flip[d] ? mid - jn : jn - mid;
            }
            const int r = oj[0] + nh * (oj[1] + nh * oj[2]);
            const float4 *row = oct + r * 7;
#pragma unroll
            for (int q4 = 0; q4 < 7; ++q4) {
                const float4 t = row[q4];
                ph[4 * q4] += alpha[i] * t.x;
                ph[4 * q4 + 1] += alpha[i] * t.y;
                ph[4 * q4 + 2] += alpha[i] * t.z;
                ph[4 * q4 + 3] += alpha[i] * t.w;
            }
        }
        // back from the octant: exchange nodes a and 2 - a of every mirrored axis
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            const int k0 = 3 * o;                      // x: (0, b, c) <-> (2, b, c)
            const float t0 = ph[k0], t2 = ph[k0 + 2];
            ph[k0] = flip[0] ? t2 : t0;
            ph[k0 + 2] = flip[0] ? t0 : t2;
        }
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            const int k0 = (o % 3) + 9 * (o / 3);      // y: (a, 0, c) <-> (a, 2, c)
            const float t0 = ph[k0], t2 = ph[k0 + 6];
            ph[k0] = flip[1] ? t2 : t0;
            ph[k0 + 6] = flip[1] ? t0 : t2;
        }
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            const int k0 = o;                          // z: (a, b, 0) <-> (a, b, 2)
            const float t0 = ph[k0], t2 = ph[k0 + 18];
            ph[k0] = flip[2] ? t2 : t0;
            ph[k0 + 18] = flip[2] ? t0 : t2;
        }
        const float nan = __builtin_nanf("");
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kNe; ++k) {
            st_stream(&out[k * kLanes], ok ? ph[k] : nan);
            acc += ph[k] * qv[k];
        }
        if (rout) *rout = 0;
        const float f = (vbv - acc) * inv_dt;
        st_stream(&U[c * n + m], ok ? acc : nan);
        st_stream(&F[c * n + m], ok ? f : nan);
        // c_l F_l (eq. 8) by row for the spreading (row p < cf_stride: padding rows too)
        const float cfv = eq8_coef_built(g, c, G[0].ih, G[1].ih, G[2].ih, ph, ca * f);
        st_stream(&cf_rows[c * cf_stride + base + lane], ok ? cfv : 0.0f);
        if (!ok) {
            raise_error(err, m, isfinite(px) && isfinite(py) && isfinite(pz) ? MLS_E_SUPPORT : MLS_E_NONFINITE);
        } else if (!(fabsf(cfv) <= 3.0e38f)) {
            raise_error(err, m, MLS_E_RANGE);
        }
        const bool counted = base + lane < n && ok;
        wave_key_max(tmax + c * tstride, counted ? (int64_t)tile_from_geo(g, c, G) : -1, finite_abs(cfv));
    }
}

// Table build: one lane per (table, sub-node); exact MLS in FP64 at the
// sub-node from the table's normalised support geometry.
//   geo_in[t][d][0..2]: support node positions relative to the home node (units of H)
//   geo_in[t][d][3..4]: home control volume lo, hi in the same units
__global__ void __launch_bounds__(kBlock)
k_table_build(const Weight W, int64_t count, int nsub, const double *__restrict__ geo_in,
              float *__restrict__ tab, float *__restrict__ geo_out)
{
    const int64_t rows = (int64_t)nsub * nsub * nsub;
    const int64_t total = count * rows;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / rows;
        const int64_t s = i % rows;
        const double *G = geo_in + t * 15;
        int j[3] = {(int)(s % nsub), (int)((s / nsub) % nsub), (int)(s / ((int64_t)nsub * nsub))};
        double off[3][3], w[3][3];
        Moments<double> m[3];
        for (int d = 0; d < 3; ++d) {
            const double lo = G[d * 5 + 3], hi = G[d * 5 + 4];
            const double xs = lo + (double)j[d] * (hi - lo) / (double)(nsub - 1);
            double m0 = 0, m1 = 0, m2 = 0;
            for (int a = 0; a < 3; ++a) {
                off[d][a] = G[d * 5 + a] - xs;
                w[d][a] = weight1_d(W, off[d][a]);
                m0 += w[d][a]; m1 += w[d][a] * off[d][a]; m2 += w[d][a] * off[d][a] * off[d][a];
            }
            m[d] = {m0, m1, m2};
        }
        double A[10], L[10], gam[4] = {0, 0, 0, 0};
        assemble(m[0], m[1], m[2], A);
        const bool ok = cholesky4(A, L);
        const double e0[4] = {1.0, 0.0, 0.0, 0.0};
        if (ok) chol_solve(L, e0, gam);
        float *row = tab + i * kTableStride;
        for (int k = 0; k < kNe; ++k) {
            int a = k % 3, b = (k / 3) % 3, cc = k / 9;
            double v = w[0][a] * w[1][b] * w[2][cc] *
                       (gam[0] + gam[1] * off[0][a] + gam[2] * off[1][b] + gam[3] * off[2][cc]);
            row[k] = ok ? (float)v : __builtin_nanf("");
        }
        row[kNe] = 0.f;
        if (s == 0) {
            for (int d = 0; d < 3; ++d) {
                geo_out[t * 6 + 2 * d] = (float)G[d * 5 + 3];
                geo_out[t * 6 + 2 * d + 1] = (float)G[d * 5 + 4];
            }
        }
    }
}

// Workgroups of a build launch: enough for three wavefronts per item of 64
// markers, at most blocks_per_cu per compute unit (the rest is covered by the
// grid stride), rounded up to a multiple of 24 (8 XCDs x 3 components).
int build_grid(int64_t n, int cu, int blocks_per_cu)
{
    const int64_t items = (n + 63) / 64;
    int64_t b = (3 * items + kBuildWaves - 1) / kBuildWaves;
    const int64_t cap = (int64_t)cu * blocks_per_cu;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)((b + kBuildGridMultiple - 1) / kBuildGridMultiple * kBuildGridMultiple);
}

}  // namespace

int build_blocks(const Ctx &c, int64_t n) { return build_grid(n, c.cu_count, c.build_blocks_per_cu); }

namespace {

int grid_for(int64_t work, int cu)
{
    int64_t b = (work + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cu * 32;   // enough resident waves; lanes loop beyond
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_build_exact(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                              uint32_t *home, float *phi, uint8_t *route, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const float tau = (float)(c.opts.kappa_tau > 3.0e38 ? 3.0e38 : c.opts.kappa_tau);
    hipLaunchKernelGGL(k_build_exact, dim3(build_grid(n, c.cu_count, c.build_blocks_per_cu)), dim3(kBuildBlock), 0, s, c.d_grid, c.w, tau, n,
                       x, y, z, home, phi, route, c.err, c.stats);
    return hipGetLastError();
}

hipError_t launch_build_interp(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                               uint32_t *home, float *phi, uint8_t *route, const float *u, const float *v,
                               const float *w, const float *vb, const float *area, float dt, float *U, float *F,
                               hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const float tau = (float)(c.opts.kappa_tau > 3.0e38 ? 3.0e38 : c.opts.kappa_tau);
    const dim3 grid(build_grid(n, c.cu_count, c.build_blocks_per_cu));
    if (c.step_nf == 0) {
        hipLaunchKernelGGL(k_build_interp<0>, grid, dim3(kBuildBlock), 0, s, c.d_grid, c.w, tau, n, c.entries, x, y, z,
                           home, phi, route, u, v, w, vb, area, 1.0f / dt, U, F, c.cf_rows, c.cf_stride, nullptr,
                           nullptr, c.tile_fmax, c.g.ntiles + 1, c.err, c.stats);
        return hipGetLastError();
    }
    // compact rows: clear the FP64 queue count, build, then finish the queued rows
    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, s, c.route_queue, (int64_t)1);
    if (c.step_nf == 7)
        hipLaunchKernelGGL(k_build_interp<7>, grid, dim3(kBuildBlock), 0, s, c.d_grid, c.w, tau, n, c.entries, x, y,
                           z, home, phi, route, u, v, w, vb, area, 1.0f / dt, U, F, c.cf_rows, c.cf_stride,
                           c.coef_rows, c.route_queue, c.tile_fmax, c.g.ntiles + 1, c.err, c.stats);
    else
        hipLaunchKernelGGL(k_build_interp<13>, grid, dim3(kBuildBlock), 0, s, c.d_grid, c.w, tau, n, c.entries, x, y,
                           z, home, phi, route, u, v, w, vb, area, 1.0f / dt, U, F, c.cf_rows, c.cf_stride,
                           c.coef_rows, c.route_queue, c.tile_fmax, c.g.ntiles + 1, c.err, c.stats);
    hipLaunchKernelGGL(k_route_rows, dim3(c.cu_count), dim3(kBlock), 0, s, c.d_grid, c.w, n, c.entries, x, y, z,
                       home, c.route_queue, phi, u, v, w, vb, area, 1.0f / dt, U, F, c.coef_rows, c.step_nf,
                       c.marker_tile, c.tile_fmax, c.g.ntiles + 1, c.err);
    return hipGetLastError();
}

bool fast_fused_ok(const Ctx &c)
{
    const int nsub = c.opts.n_sub;
    const int nh = (nsub + 1) / 2;
    return c.tables && c.n_tables == 1 && c.stretched_axis < 0 && (nsub & 1) &&
           (int64_t)nh * nh * nh * kTableStride * 4 <= 64 * 1024;
}

hipError_t launch_fast_interp(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                              uint32_t *home, float *phi, uint8_t *route, const float *u, const float *v,
                              const float *w, const float *vb, const float *area, float dt, float *U, float *F,
                              hipStream_t s, bool trilinear_blend)
{
    if (n == 0) return hipSuccess;
    if (!fast_fused_ok(c)) return hipErrorInvalidValue;
    const int nsub = c.opts.n_sub, nh = (nsub + 1) / 2;
    const size_t lds = (size_t)nh * nh * nh * kTableStride * sizeof(float);
    const dim3 grid(build_grid(n, c.cu_count, c.build_blocks_per_cu));
    const float4 *tab = reinterpret_cast<const float4 *>(c.tables);
    if (trilinear_blend)
        hipLaunchKernelGGL(k_fast_interp<true>, grid, dim3(kBuildBlock), lds, s, c.d_grid, tab, nsub, n, c.entries, x,
                           y, z, home, phi, route, u, v, w, vb, area, 1.0f / dt, U, F, c.cf_rows, c.cf_stride,
                           c.tile_fmax, c.g.ntiles + 1, c.err);
    else
        hipLaunchKernelGGL(k_fast_interp<false>, grid, dim3(kBuildBlock), lds, s, c.d_grid, tab, nsub, n, c.entries, x,
                           y, z, home, phi, route, u, v, w, vb, area, 1.0f / dt, U, F, c.cf_rows, c.cf_stride,
                           c.tile_fmax, c.g.ntiles + 1, c.err);
    return hipGetLastError();
}

hipError_t launch_build_fast(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                             uint32_t *home, float *phi, uint8_t *route, hipStream_t s, bool trilinear_blend)
{
    if (n == 0) return hipSuccess;
    const dim3 grid(build_grid(n, c.cu_count, c.build_blocks_per_cu));
    if (trilinear_blend)
        hipLaunchKernelGGL(k_build_fast<true>, grid, dim3(kBuildBlock), 0, s, c.d_grid, fast_tables(c), n, x, y, z,
                           home, phi, route, c.err);
    else
        hipLaunchKernelGGL(k_build_fast<false>, grid, dim3(kBuildBlock), 0, s, c.d_grid, fast_tables(c), n, x, y, z,
                           home, phi, route, c.err);
    return hipGetLastError();
}

// Host side of the table build: the normalised support geometry of every
// table (uniform grid: one table; stretched axis: one per home plane and
// staggering type) is derived from the host copy of the grid, then the
// device computes the shape functions at the sub-nodes.
hipError_t launch_table_build(const Ctx &c, hipStream_t s)
{
    const Grid &g = c.g;
    const int d_s = c.stretched_axis;
    std::vector<double> geo((size_t)c.n_tables * 15);
    auto host_node = [&](int d, int is_face, long i) -> double {
        const Axis &a = g.ax[d];
        double shift = 0.0;
        if (a.periodic) {
            if (i < 0) { i += a.n; shift = -1.0; }
            else if (i >= a.n) { i -= a.n; shift = 1.0; }
        }
        double v = is_face ? c.h_faces[d][i] : c.h_centres[d][i];
        return v + shift * a.L;
    };
    auto fill = [&](int64_t t, const long ih[3], const int is_face[3]) {
        for (int d = 0; d < 3; ++d) {
            const Axis &a = g.ax[d];
            double xm = host_node(d, is_face[d], ih[d] - 1);
            double x0 = host_node(d, is_face[d], ih[d]);
            double xp = host_node(d, is_face[d], ih[d] + 1);
            double H = 0.5 * (xp - xm);
            double lo, hi;
            if (!is_face[d]) {
                lo = host_node(d, 1, ih[d]);
                hi = host_node(d, 1, ih[d] + 1);
            } else {
                lo = (!a.periodic && ih[d] == 0) ? c.h_faces[d][0] : host_node(d, 0, ih[d] - 1);
                hi = (!a.periodic && ih[d] == a.n) ? c.h_faces[d][a.n] : host_node(d, 0, ih[d]);
            }
            double *G = &geo[(size_t)t * 15 + d * 5];
            G[0] = (xm - x0) / H;
            G[1] = 0.0;
            G[2] = (xp - x0) / H;
            G[3] = (lo - x0) / H;
            G[4] = (hi - x0) / H;
        }
    };
    if (d_s < 0) {
        long ih[3] = {1, 1, 1};
        int tf[3] = {0, 0, 0};
        fill(0, ih, tf);
    } else {
        for (int type = 0; type < 2; ++type) {
            const Axis &a = g.ax[d_s];
            const int nodes = (type && !a.periodic) ? a.n + 1 : a.n;
            for (int p = 0; p < nodes; ++p) {
                long ih[3] = {1, 1, 1};
                int tf[3] = {0, 0, 0};
                ih[d_s] = p;
                tf[d_s] = type;
                // planes whose support would leave a wall get a table that is never used
                if (!a.periodic && (p < 1 || p + 1 > (type ? a.n : a.n - 1))) ih[d_s] = 1;
                fill(c.table_first[type] + p, ih, tf);
            }
        }
    }
    double *d_geo = nullptr;
    hipError_t e = hipMalloc((void **)&d_geo, geo.size() * sizeof(double));
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(d_geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) { hipFree(d_geo); return e; }
    const int64_t rows = (int64_t)c.opts.n_sub * c.opts.n_sub * c.opts.n_sub;
    hipLaunchKernelGGL(k_table_build, dim3(grid_for(c.n_tables * rows, c.cu_count)), dim3(kBlock), 0, s, c.w,
                       c.n_tables, (int)c.opts.n_sub, d_geo, c.tables, c.table_geo);
    e = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    hipFree(d_geo);
    return e != hipSuccess ? e : e2;
}

FastTables fast_tables(const Ctx &c)
{
    FastTables t;
    t.tab = c.tables;
    t.geo = c.table_geo;
    t.n_sub = c.opts.n_sub;
    t.stretched_axis = c.stretched_axis;
    t.first[0] = c.table_first[0];
    t.first[1] = c.table_first[1];
    return t;
}

}  // namespace mls
