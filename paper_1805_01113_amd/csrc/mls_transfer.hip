// Interpolation (eq. 6) and conservative spreading (eq. 7-8).
//
// Interpolation: one lane per marker gathers the 27 support values of each
// component and contracts them with its shape function (SoA loads).
//
// Spreading is deterministic without floating-point atomics:
//   1. every marker is binned into the tiles of the forcing grid that its
//      supports touch (a counting sort: count, exclusive scan, fill);
//   2. one workgroup owns a tile: it accumulates all contributions landing in
//      the tile in LDS as 64-bit fixed-point integers (integer addition is
//      associative, so the sum does not depend on the order in which lanes or
//      markers arrive) and finally adds the tile, converted back to FP32, into
//      the caller's field.  Each node belongs to exactly one tile, so the
//      global update is a plain read-modify-write.
// The fixed-point scale of a tile is a power of two chosen from the largest
// |c_l F_l| (eq. 8) among the tile's markers, so that no sum can overflow and
// the quantum follows the tile's own forces.
#include <mutex>

#include "mls_exact.h"

namespace mls {

namespace {

constexpr int kBlock = 256;
constexpr int kSpreadBlock = 256;   // most threads of a spreading tile workgroup

__global__ void __launch_bounds__(kBlock)
k_interp(const Grid *__restrict__ gp, int64_t n, const uint32_t *__restrict__ home, const float *__restrict__ phi,
         const float *__restrict__ u, const float *__restrict__ v, const float *__restrict__ w,
         float *__restrict__ U, float *__restrict__ V, float *__restrict__ W, ErrWord *err)
{
    const Grid &g = *gp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t l = xcd_block() * blockDim.x + threadIdx.x; l < n; l += stride) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float *q = c == 0 ? u : (c == 1 ? v : w);
            const uint32_t h = home[home_at(l, c)];
            int i, j, k;
            unpack_home(h, i, j, k);
            float *out = c == 0 ? U : (c == 1 ? V : W);
            if (!home_ok(g, c, i, j, k)) {
                raise_error(err, l, MLS_E_SUPPORT);
                out[l] = __builtin_nanf("");
                continue;
            }
            uint32_t oy[3], oz[3];
            support_rows(true, j, k, g.dims[c][0], g.dims[c][1], g.dims[c][2], g.ax[1].periodic, g.ax[2].periodic,
                         oy, oz);
            Support sp;
            load_support(q, i, g.dims[c][0], oy, oz, sp);
            const float *p = phi + phi_at(l, c);
            float acc = 0.f;
#pragma unroll
            for (int kk = 0; kk < kNe; ++kk) acc += p[kk * kLanes] * sp.at(kk);
            out[l] = acc;
        }
    }
}

// ---- spreading: tile binning -------------------------------------------------
//
// Every marker belongs to exactly one tile of the grid: the tile holding its
// cell (the home of a centre-staggered component on each axis).  A tile's
// markers spread into an LDS box that covers the tile plus the one-node halo
// of their supports (tile + 3 nodes per axis).  Tiles are coloured by the
// parity of their index per axis (a third colour for the last tile of a
// periodic axis with an odd tile count); boxes of tiles of one colour never
// overlap, so a colour's tiles add their boxes into the field with plain
// read-modify-writes, and the colours run one after another.  Each node thus
// receives its additions in the fixed colour order, and inside a box the
// contributions are summed in 64-bit fixed point, whose sum does not depend on
// the order of the markers: the result is bitwise reproducible.


__device__ __forceinline__ int64_t marker_tile(const Grid &g, const uint32_t *__restrict__ home, int64_t l,
                                               bool &valid)
{
    int hc[3][3];
    valid = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        unpack_home(home[home_at(l, c)], hc[c][0], hc[c][1], hc[c][2]);
        valid = valid && home_ok(g, c, hc[c][0], hc[c][1], hc[c][2]);
    }
    // the cell on axis d is the home of component (d + 1) % 3 (centre-staggered on d)
    const int tx = tile_of(hc[1][0], g.ax[0].inv_tile);
    const int ty = tile_of(hc[2][1], g.ax[1].inv_tile);
    const int tz = tile_of(hc[0][2], g.ax[2].inv_tile);
    return ((int64_t)tz * g.ntile[1] + ty) * g.ntile[0] + tx;
}

// Lanes of a wavefront that hit the same tile are combined into one atomic:
// the leader adds the count and the others take consecutive slots in lane
// order, so a tile's marker list is made of runs of consecutive markers.
// The counting pass also records each marker's tile (ntiles for a marker
// without a usable support) for the per-tile force maxima.
// Counting sort step of one wavefront (all lanes active): lanes with tile
// t >= 0 are grouped by tile; the counting pass adds each group's size to
// count[t], the filling pass reserves a range of cursor[t] per group and
// writes the group's markers there in lane order.  The groups are found with
// ballots first, then every group leader issues its atomic in one
// instruction, so the wavefront waits for one round trip, not one per tile.
template <bool FILL>
__device__ __forceinline__ void wave_bin(int64_t t, int lane, uint32_t *count, uint32_t *cursor, uint32_t *entries,
                                         uint32_t marker)
{
    unsigned long long pending = __ballot(t >= 0);
    unsigned long long group = 0;   // lanes of this lane's tile
    int leader = 0;
    while (pending) {
        const int lead = __ffsll((long long)pending) - 1;
        const int64_t tl = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)((uint64_t)t >> 32), lead)
                                      << 32) |
                                     (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)t, lead));
        const unsigned long long mask = __ballot(t == tl) & pending;
        if (t == tl) { group = mask; leader = lead; }
        pending &= ~mask;
    }
    if (t < 0) return;
    const uint32_t cnt = (uint32_t)__popcll(group);
    if (!FILL) {
        if (lane == leader) atomicAdd(&count[t], cnt);
    } else {
        uint32_t pos = 0;
        if (lane == leader) pos = atomicAdd(&cursor[t], cnt);
        pos = __shfl(pos, leader);
        entries[pos + __popcll(group & ((1ull << lane) - 1ull))] = marker;
    }
}

template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_bin(const Grid *__restrict__ gp, int64_t n, const uint32_t *__restrict__ home, uint32_t *__restrict__ count,
      uint32_t *__restrict__ cursor, uint32_t *__restrict__ entries, uint32_t *__restrict__ tile_of_marker,
      ErrWord *err)
{
    const Grid &g = *gp;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the loop bound is wave-uniform so that the ballots see the whole wave
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t l = base + lane;
        int64_t t = -1;
        if (l < n) {
            bool valid;
            const int64_t tt = marker_tile(g, home, l, valid);
            if (valid) t = tt;
            else if (!FILL) raise_error(err, l, MLS_E_SUPPORT);   // contributes nothing
            if (!FILL) tile_of_marker[l] = valid ? (uint32_t)tt : (uint32_t)g.ntiles;
        }
        wave_bin<FILL>(t, lane, count, cursor, entries, (uint32_t)l);
    }
}

// Binning straight from the marker positions (the exact time step): the
// tile of the cell that holds the marker (centre-staggered home on each
// axis); a marker whose cell support leaves a wall axis, or whose position is
// not finite, goes to the extra bucket ntiles, after all tiles.  The counting
// pass locates the markers and records each one's tile in tiles[]; the
// filling pass reads it back.  With jitter (amp2 > 0) the counting pass reads
// the rest positions x, y, z, jitters them (the time step's generator) and
// stores the result in jx, jy, jz, which it then locates.
template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_bin_pos(const Grid *__restrict__ gp, int64_t n, const float *__restrict__ x, const float *__restrict__ y,
          const float *__restrict__ z, uint32_t *__restrict__ count, uint32_t *__restrict__ cursor,
          uint32_t *__restrict__ entries, uint32_t *__restrict__ tiles, float *__restrict__ jx,
          float *__restrict__ jy, float *__restrict__ jz, float amp2, uint64_t seed,
          const unsigned long long *__restrict__ step_ctr)
{
    const Grid &g = *gp;
    const uint64_t step = (!FILL && amp2 > 0.0f) ? *step_ctr : 0ull;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const float itx = g.ax[0].inv_tile, ity = g.ax[1].inv_tile, itz = g.ax[2].inv_tile;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t l = base + lane;
        int64_t t = -1;
        if (l < n) {
            if (FILL) {
                t = tiles[l];
            } else {
                float px = x[l], py = y[l], pz = z[l];
                if (amp2 > 0.0f) {
                    jitter_marker(seed, step, n, l, amp2, px, py, pz, px, py, pz);
                    jx[l] = px;
                    jy[l] = py;
                    jz[l] = pz;
                }
                const double p[3] = {(double)px, (double)py, (double)pz};
                int cell[3];
                bool ok = true;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    int ih = 0;
                    double X;
                    ok = ok && locate(g.ax[d], 0, p[d], ih, X);
                    cell[d] = ih;
                }
                t = ok ? ((int64_t)tile_of(cell[2], itz) * g.ntile[1] + tile_of(cell[1], ity)) * g.ntile[0] +
                             tile_of(cell[0], itx)
                       : g.ntiles;
                tiles[l] = (uint32_t)t;
            }
        }
        wave_bin<FILL>(t, lane, count, cursor, entries, (uint32_t)l);
    }
}

__global__ void k_zero_u32(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Exclusive scan of the tile counts: block partial sums, one workgroup scans
// the partials, then each block scans its chunk.  off[ntiles] = total.
constexpr int kScanChunk = 2048;   // elements per block (256 threads x 8)

__global__ void __launch_bounds__(kBlock) k_scan_partials(const uint32_t *__restrict__ count, int64_t nt,
                                                          uint32_t *__restrict__ partial)
{
    __shared__ uint32_t sh[4];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint32_t s = 0;
    for (int q = 0; q < kScanChunk / kBlock; ++q) {
        const int64_t i = base + (int64_t)q * kBlock + threadIdx.x;
        if (i < nt) s += count[i];
    }
    uint32_t total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) k_scan_top(uint32_t *__restrict__ partial, int64_t nb)
{
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? partial[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, sh, total);
        if (i < nb) partial[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
}

// Also clears the per-tile force maxima tmax[3][tstride] of the scanned
// tiles, ahead of the kernels that write c_l F_l.  Each thread scans 8
// consecutive counts; the counts come in and the offsets go out through LDS
// so that every global access of a wavefront is one contiguous run (8-element
// strided stores leave partial lines that reach memory several times over).
__global__ void __launch_bounds__(kBlock) k_scan_final(const uint32_t *__restrict__ count, int64_t nt,
                                                       const uint32_t *__restrict__ partial,
                                                       uint32_t *__restrict__ off, uint32_t *__restrict__ cursor,
                                                       uint32_t *__restrict__ work, uint32_t *__restrict__ tmax,
                                                       int64_t tstride)
{
    __shared__ uint32_t sh[4];
    __shared__ uint32_t buf[kScanChunk];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    const int per = kScanChunk / kBlock;
    for (int q = 0; q < per; ++q) {
        const int64_t i = base + q * kBlock + threadIdx.x;
        buf[q * kBlock + threadIdx.x] = i < nt ? count[i] : 0u;
    }
    __syncthreads();
    uint32_t vals[kScanChunk / kBlock];
    uint32_t s = 0;
    for (int q = 0; q < per; ++q) {
        vals[q] = buf[threadIdx.x * per + q];
        s += vals[q];
    }
    uint32_t total;
    uint32_t run = partial[blockIdx.x] + block_exclusive_scan(s, sh, total);
    for (int q = 0; q < per; ++q) {
        buf[threadIdx.x * per + q] = run;
        run += vals[q];
    }
    // the owner of the last tile also writes off[nt] = total
    const int64_t first = base + (int64_t)threadIdx.x * per;
    if (first <= nt - 1 && nt - 1 < first + per) off[nt] = run;
    __syncthreads();
    for (int q = 0; q < per; ++q) {
        const int64_t i = base + q * kBlock + threadIdx.x;
        if (i < nt) {
            const uint32_t o = buf[q * kBlock + threadIdx.x];
            off[i] = o;
            cursor[i] = o;
            tmax[i] = 0u;
            tmax[tstride + i] = 0u;
            tmax[2 * tstride + i] = 0u;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 64) work[threadIdx.x] = 0u;   // colour list sizes and cursors
}

__device__ __forceinline__ int axis_colour(const Grid &g, int d, int t)
{
    const int k = g.ncol[d];
    return k == 1 ? 0 : ((k == 3 && t == g.ntile[d] - 1) ? 2 : (t & 1));
}

// One past the last slot of colour col in the active-tile list (the colours
// in use are 0 .. ncol_x ncol_y ncol_z - 1, their slots consecutive).
__device__ __forceinline__ int64_t colour_end(const Grid &g, int col)
{
    const int used = g.ncol[0] * g.ncol[1] * g.ncol[2];
    return col + 1 < used ? g.colour_base[col + 1] : g.ntiles;
}

// Non-empty tiles listed per colour: work[col] counts them and
// active[colour_base[col] + i] lists them.  A block gathers its 2048 tiles
// per colour in LDS and takes its slots with one atomic per colour.
constexpr int kActiveChunk = 2048;
__global__ void __launch_bounds__(kBlock)
k_active_tiles(const Grid *__restrict__ gp, const uint32_t *__restrict__ off, uint32_t *__restrict__ active,
               uint32_t *work)
{
    const Grid &g = *gp;
    __shared__ uint32_t lcount[27], lbase[27];
    if (threadIdx.x < 27) lcount[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kActiveChunk + (int64_t)threadIdx.x * (kActiveChunk / kBlock);
    int col[kActiveChunk / kBlock];
    uint32_t pos[kActiveChunk / kBlock];
#pragma unroll
    for (int q = 0; q < kActiveChunk / kBlock; ++q) {
        const int64_t t = t0 + q;
        col[q] = -1;
        if (t < g.ntiles && off[t + 1] > off[t]) {
            const int tx = (int)(t % g.ntile[0]);
            const int ty = (int)((t / g.ntile[0]) % g.ntile[1]);
            const int tz = (int)(t / ((int64_t)g.ntile[0] * g.ntile[1]));
            col[q] = axis_colour(g, 0, tx) + g.ncol[0] * (axis_colour(g, 1, ty) + g.ncol[1] * axis_colour(g, 2, tz));
            pos[q] = atomicAdd(&lcount[col[q]], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < 27) lbase[threadIdx.x] = lcount[threadIdx.x] ? atomicAdd(&work[threadIdx.x], lcount[threadIdx.x]) : 0u;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kActiveChunk / kBlock; ++q)
        if (col[q] >= 0) {
            const int64_t slot = g.colour_base[col[q]] + lbase[col[q]] + pos[q];
            if (slot < colour_end(g, col[q])) active[slot] = (uint32_t)(t0 + q);
        }
}

// ---- spreading: per-tile fixed-point accumulation ------------------------------

// Box-local index of node i (wrapped) on axis a for a box starting at node b0.
__device__ __forceinline__ int box_local(const Axis &a, int ntile, int nodes, int b0, int i)
{
    if (a.periodic && ntile == 1) return i;            // the box is the whole (short) axis
    int l = i - b0;
    if (a.periodic) l = l < 0 ? l + nodes : (l >= nodes ? l - nodes : l);
    return l;
}

// Workgroup barrier for LDS only.  The phases of a tile share data through
// LDS alone: each field node is flushed by one thread and same-colour tiles
// never overlap, so no thread needs another's global stores.  A full
// __syncthreads would also wait for every outstanding global store (the
// flush of the previous component) before the next phase could start.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this thread's LDS operations are done
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Adds a tile's box (64-bit fixed point, scale qscale) into the FP32 field f
// and returns its nodes to zero.  Consecutive threads take consecutive box
// nodes (their field accesses coalesce along x rows), kFlush per thread at a
// time: the kFlush sums are read from LDS together, then the nonzero ones are
// decoded into box coordinates, their field values loaded together and
// written back.  Box coordinates come from the compile-time row length BX
// (BX > 0) or FP32 reciprocals of the box edges (exact below 2^22 nodes).
// INSIDE: the box lies inside the grid, so a node's index is the origin's
// plus an affine offset; otherwise periodic axes wrap and nodes past a wall
// are skipped.
template <bool INSIDE, int BX>
__device__ __forceinline__ void flush_box(const Grid &g, int c, unsigned long long *acc, int bnodes, int bx_rt,
                                          int by, int b0x, int b0y, int b0z, int nxc, int nyc, int nzc, float inv_bx,
                                          float inv_by, float inv_bxy, double qscale, float *__restrict__ f)
{
    constexpr int kFlush = 8;
    const int bx = BX > 0 ? BX : bx_rt;
    const Axis &AX = g.ax[0], &AY = g.ax[1], &AZ = g.ax[2];
    float *const fo = INSIDE ? f + field_index(g, c, b0x, b0y, b0z) : f;
    const int sz = nxc * nyc;
    for (int q0 = threadIdx.x; q0 < bnodes; q0 += kFlush * blockDim.x) {
        long long sv[kFlush];
#pragma unroll
        for (int u = 0; u < kFlush; ++u) {
            const int q = q0 + u * (int)blockDim.x;
            sv[u] = q < bnodes ? (long long)acc[q] : 0;
        }
        float *dst[kFlush];
        float add[kFlush];
        float old[kFlush];
#pragma unroll
        for (int u = 0; u < kFlush; ++u) {
            dst[u] = nullptr;
            add[u] = 0.f;
            const int q = q0 + u * (int)blockDim.x;
            if (sv[u] == 0) continue;
            acc[q] = 0ull;
            int lx, ly, lz;
            if constexpr (BX > 0) {
                const int rq = q / BX;
                lx = q - rq * BX;
                lz = (int)(((float)rq + 0.5f) * inv_by);
                ly = rq - lz * by;
            } else {
                lz = (int)(((float)q + 0.5f) * inv_bxy);
                const int rq = q - lz * (bx * by);
                ly = (int)(((float)rq + 0.5f) * inv_bx);
                lx = rq - ly * bx;
            }
            if constexpr (INSIDE) {
                dst[u] = fo + (lz * sz + ly * nxc + lx);
            } else {
                int gx = b0x + lx, gy = b0y + ly, gz = b0z + lz;
                if (AX.periodic) gx = gx < 0 ? gx + nxc : (gx >= nxc ? gx - nxc : gx);
                if (AY.periodic) gy = gy < 0 ? gy + nyc : (gy >= nyc ? gy - nyc : gy);
                if (AZ.periodic) gz = gz < 0 ? gz + nzc : (gz >= nzc ? gz - nzc : gz);
                if ((unsigned)gx >= (unsigned)nxc || (unsigned)gy >= (unsigned)nyc || (unsigned)gz >= (unsigned)nzc)
                    continue;
                dst[u] = f + field_index(g, c, gx, gy, gz);
            }
            add[u] = (float)((double)sv[u] * qscale);
        }
#pragma unroll
        for (int u = 0; u < kFlush; ++u) old[u] = dst[u] ? *dst[u] : 0.f;
#pragma unroll
        for (int u = 0; u < kFlush; ++u)
            if (dst[u]) *dst[u] = old[u] + add[u];
    }
}

// NF > 0 (sorted rows of a compact exact step): phi is evaluated from the
// row's compact transfer function (gamma and the support offsets, NF = 7 or
// 13 floats, see k_build_interp) with the build's own arithmetic, or read
// from phi for a row the build solved in FP64 (NaN gamma_0).
// c_l F_l of eq. 8 per component comes with a compact row (NF > 0), or from
// cf: by row in tile order (SORTED with full rows, the time step's fused
// builds write them) or by marker (a standalone call: k_spread_coef).  Per tile, the largest finite |c_l F_l|
// of its rows sets the fixed-point scale of each component.
// Workgroups of 128, 192 or 256 threads (tuned, at most kSpreadBlock).  A tile
// holds some 200 rows: when each workgroup handles many tiles, 128 threads
// leave fewer lanes idle, pay cheaper barriers and keep more tiles in flight
// per compute unit; when a colour has only a tile or two per workgroup, 256
// threads finish each tile sooner.
// BX > 0: every axis has more than one tile and the box rows hold BX nodes.
// Then the 27 support nodes of a row are three consecutive nodes on each box
// axis, so one box address per row serves all 27 atomics (the others are
// immediate offsets) and the flush decodes box coordinates with it.
// BX = 0: any tiling (a short periodic axis kept whole wraps inside its box).
template <bool SORTED, int NF, int BX>
__global__ void __launch_bounds__(kSpreadBlock) __attribute__((amdgpu_waves_per_eu(SORTED ? 6 : 5)))
k_spread_colour(const Grid *__restrict__ gp, int colour, const uint32_t *__restrict__ home,
                const float *__restrict__ phi, const float *__restrict__ cf, int64_t cf_stride,
                float *__restrict__ fx, float *__restrict__ fy, float *__restrict__ fz,
                const uint32_t *__restrict__ off, const uint32_t *__restrict__ entries,
                const uint32_t *__restrict__ active, uint32_t *work, const float *__restrict__ coef, const Weight W,
                const uint32_t *__restrict__ tmax, int64_t tstride, ErrWord *err)
{
    const Grid &g = *gp;
    extern __shared__ unsigned long long acc[];     // the box of one component
    const Axis &AX = g.ax[0], &AY = g.ax[1], &AZ = g.ax[2];
    const int bx = BX > 0 ? BX : g.box[0], by = g.box[1], bz = g.box[2];
    const int bnodes = bx * by * bz;
    const float inv_by = 1.0f / (float)by;
    const int64_t abase = g.colour_base[colour];
    const uint32_t nact = (uint32_t)min((int64_t)work[colour], colour_end(g, colour) - abase);
    __shared__ int64_t tile_sh;
    // The box is cleared once here; afterwards every flush returns the nodes
    // it reads to zero, so each component and tile starts from a clear box.
    for (int q = threadIdx.x; q < bnodes; q += blockDim.x) acc[q] = 0ull;
    // box-local coordinates of a node index without integer division: with
    // fewer than 2^22 nodes, (q + 1/2) times the FP32 reciprocal of the divisor
    // stays within 1/2 of a quotient's interval from its floor
    const float inv_bx = 1.0f / (float)bx, inv_bxy = 1.0f / (float)(bx * by);
    // Tiles are claimed through one device-wide counter, whose atomics are
    // served one after another.  A colour with only a few tiles per workgroup
    // would have every workgroup queue on it at the start, and the last one to
    // get its tile sets the launch's end; there the first round is handed out
    // by position (tile b to workgroup b) and only the rest is claimed.
    const uint32_t G = gridDim.x;
    const uint32_t nfixed = nact < 4u * G ? min(nact, G) : 0u;
    bool first = true;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t i = first && blockIdx.x < nfixed ? blockIdx.x : nfixed + atomicAdd(&work[32 + colour], 1u);
            first = false;
            const int64_t t = i < nact ? (int64_t)active[abase + i] : -1;
            tile_sh = t < g.ntiles ? t : -1;
        }
        lds_barrier();
        const int64_t t = tile_sh;
        if (t < 0) break;
        const uint32_t beg = off[t], end = off[t + 1];
        const int tx = (int)(t % g.ntile[0]);
        const int ty = (int)((t / g.ntile[0]) % g.ntile[1]);
        const int tz = (int)(t / ((int64_t)g.ntile[0] * g.ntile[1]));
        // box origin: one node below the tile (a single-tile periodic axis keeps the whole axis)
        const int b0x = (AX.periodic && g.ntile[0] == 1) ? 0 : tx * AX.tile - 1;
        const int b0y = (AY.periodic && g.ntile[1] == 1) ? 0 : ty * AY.tile - 1;
        const int b0z = (AZ.periodic && g.ntile[2] == 1) ? 0 : tz * AZ.tile - 1;
        // one component at a time: a third of the LDS per workgroup, so more
        // workgroups fit a compute unit and tiles can be larger
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            lds_barrier();
            // The tile's largest finite |c_l F_l| (written with c_l F_l by the
            // build, or k_spread_coef) sets its scale: with |phi_k| <= 4 every
            // scaled contribution stays below 2^30 (converted to int32, summed
            // in int64), |c_l F_l| is scaled below 2^28, and the quantum is
            // 2^-30 of 4 max |c_l F_l| over the tile.  A non-finite c_l F_l is
            // left out of the maximum and fails the range test below.
            const float fm = __uint_as_float(tmax[c * tstride + t]);
            int ebits = 0;
            frexpf(fm, &ebits);                    // fm < 2^ebits
            const int S = min(28 - ebits, 126);
            const float scale_f = fm > 0.f ? ldexpf(1.0f, S) : 0.0f;
            const float lim = 1073741824.0f;       // 2^30
            const int nxc = g.dims[c][0], nyc = g.dims[c][1], nzc = g.dims[c][2];
            for (uint32_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
                // tile order: the row is the entry, so no load waits for the
                // marker index (read on the error path only)
                const int64_t row = SORTED ? (int64_t)e : (int64_t)entries[e];
                int hi, hj, hk;
                unpack_home(home[home_at(row, c)], hi, hj, hk);
                float cfv;
                float ph[kNe];
                if constexpr (NF == 0) {
                    cfv = cf[c * cf_stride + row];
                    const float *p = phi + phi_at(row, c);
#pragma unroll
                    for (int k = 0; k < kNe; ++k) ph[k] = p[k * kLanes];
                } else {
                    // the compact row and c_l F_l in two or four 16-byte loads
                    float cfr[kCoefStride<NF>];
#pragma unroll
                    for (int q = 0; q < kCoefStride<NF> / 4; ++q) {
                        const f32x4 t =
                            *reinterpret_cast<const f32x4 *>(coef + coef_word(row, c, kCoefStride<NF>, q));
                        cfr[4 * q] = t.x; cfr[4 * q + 1] = t.y; cfr[4 * q + 2] = t.z; cfr[4 * q + 3] = t.w;
                    }
                    cfv = cfr[NF];
                    // evaluated for every row (all loads issue at once); a row the
                    // build solved in FP64 has a NaN gamma_0 and its stored phi is
                    // read instead, under a wavefront-wide test
                    float sv[3][3], wv[3][3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if constexpr (NF == 7) {
                            sv[d][1] = cfr[4 + d];
                            sv[d][0] = sv[d][1] - 1.0f;
                            sv[d][2] = sv[d][1] + 1.0f;
                        } else {
#pragma unroll
                            for (int a = 0; a < 3; ++a) sv[d][a] = cfr[4 + 3 * d + a];
                        }
#pragma unroll
                        for (int a = 0; a < 3; ++a) wv[d][a] = weight1(W, sv[d][a]);
                    }
                    phi_from_gamma(wv, sv, cfr, ph);
                    const bool stored = cfr[0] != cfr[0];
                    if (__any(stored)) {
                        if (stored) {
                            const float *p = phi + phi_at(row, c);
#pragma unroll
                            for (int k = 0; k < kNe; ++k) ph[k] = p[k * kLanes];
                        }
                    }
                }
                int ix[3], iy[3], iz[3];
                bool inbox = true;
                if constexpr (BX > 0) {
                    // the support's first node on each axis; the others follow it
                    ix[0] = box_local(AX, g.ntile[0], nxc, b0x, nb_index(hi, -1, nxc, AX.periodic));
                    iy[0] = box_local(AY, g.ntile[1], nyc, b0y, nb_index(hj, -1, nyc, AY.periodic));
                    iz[0] = box_local(AZ, g.ntile[2], nzc, b0z, nb_index(hk, -1, nzc, AZ.periodic));
                    inbox = (unsigned)ix[0] <= (unsigned)(BX - 3) && (unsigned)iy[0] <= (unsigned)(by - 3) &&
                            (unsigned)iz[0] <= (unsigned)(bz - 3);
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        ix[a] = box_local(AX, g.ntile[0], nxc, b0x, nb_index(hi, a - 1, nxc, AX.periodic));
                        iy[a] = box_local(AY, g.ntile[1], nyc, b0y, nb_index(hj, a - 1, nyc, AY.periodic));
                        iz[a] = box_local(AZ, g.ntile[2], nzc, b0z, nb_index(hk, a - 1, nzc, AZ.periodic));
                        inbox = inbox && (unsigned)ix[a] < (unsigned)bx && (unsigned)iy[a] < (unsigned)by &&
                                (unsigned)iz[a] < (unsigned)bz;
                    }
                }
                if (!inbox) {           // cannot happen for a home written by the build
                    raise_error(err, SORTED ? (int64_t)entries[e] : row, MLS_E_RANGE);
                    continue;
                }
                // c_l F_l (eq. 8), pre-scaled
                const float vsc = cfv * scale_f;
                // Rounding is monotonic, so |phi_k vsc| <= max_k |phi_k| |vsc| for
                // every k, with equality at the largest: one comparison bounds all
                // 27 scaled contributions.  A NaN or infinity in the force or the
                // coefficient reaches vsc and fails it too.  Sorted rows hold the
                // library's own shape functions (finite for a usable support);
                // a caller's phi is checked here.
                float pm = 0.f;
#pragma unroll
                for (int k = 0; k < kNe; ++k) pm = fmaxf(pm, fabsf(ph[k]));
                if constexpr (!SORTED) {
                    // caller-provided phi: a NaN or infinite value fails through
                    // the sum (fmaxf above ignores a NaN operand); c_l of a grid
                    // with equal widths does not depend on phi
                    float ps = 0.f;
#pragma unroll
                    for (int k = 0; k < kNe; ++k) ps += ph[k];
                    if (!(fabsf(ps) <= 3.0e38f)) pm = __builtin_inff();
                }
                if (!(fabsf(vsc) * pm < lim)) {
                    raise_error(err, SORTED ? (int64_t)entries[e] : row, MLS_E_RANGE);
                    continue;
                }
                // truncation toward zero: within one quantum, the same on every run
                if constexpr (BX > 0) {
                    // byte address of the first node per z layer; node (a, b) of a
                    // layer sits (b BX + a) nodes further
                    char *const a0 = reinterpret_cast<char *>(acc) +
                                     (uint32_t)__umul24(__umul24(iz[0], by) + iy[0], BX) * 8u + (uint32_t)ix[0] * 8u;
                    const uint32_t zs = (uint32_t)(by * BX) * 8u;
#pragma unroll
                    for (int k = 0; k < kNe; ++k) {
                        const long long qv = (long long)(int)(ph[k] * vsc);
                        char *const p = a0 + (k / 9) * zs + (((k / 3) % 3) * BX + (k % 3)) * 8;
                        atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)qv);
                    }
                } else {
                    // byte offsets of the box rows (b, cz) and columns a
                    uint32_t rowo[9], colo[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) colo[a] = (uint32_t)ix[a] * 8u;
#pragma unroll
                    for (int r = 0; r < 9; ++r) rowo[r] = (uint32_t)((iz[r / 3] * by + iy[r % 3]) * bx) * 8u;
#pragma unroll
                    for (int k = 0; k < kNe; ++k) {
                        const long long qv = (long long)(int)(ph[k] * vsc);
                        atomicAdd(reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(acc) +
                                                                         rowo[k / 3] + colo[k % 3]),
                                  (unsigned long long)qv);
                    }
                }
            }
            lds_barrier();
            // flush: the box nodes of a thread are read in batches of kFlush
            // before any is written back, so their loads overlap
            float *f = c == 0 ? fx : (c == 1 ? fy : fz);
            const double qscale = ldexp(1.0, -S);
            // a box inside the component's grid on every axis (no wrap, no node
            // past a wall) addresses its nodes as offsets from its origin
            const bool inside = b0x >= 0 && b0y >= 0 && b0z >= 0 && b0x + bx <= nxc && b0y + by <= nyc &&
                                b0z + bz <= nzc;
            if (inside)
                flush_box<true, BX>(g, c, acc, bnodes, bx, by, b0x, b0y, b0z, nxc, nyc, nzc, inv_bx, inv_by, inv_bxy,
                                    qscale, f);
            else
                flush_box<false, BX>(g, c, acc, bnodes, bx, by, b0x, b0y, b0z, nxc, nyc, nzc, inv_bx, inv_by, inv_bxy,
                                     qscale, f);
        }
        lds_barrier();
    }
}

// c_l F_l (eq. 8) by marker for a standalone spreading call, from the stored
// shape functions, homes, areas and forces.  A marker whose homes are not
// usable gets 0 (the binning leaves it out).
// It also records the largest finite |c_l F_l| per tile (marker_tile from
// the binning) and component in tmax.
__global__ void __launch_bounds__(kBlock)
k_spread_coef(const Grid *__restrict__ gp, int64_t n, const uint32_t *__restrict__ home,
              const float *__restrict__ phi, const float *__restrict__ area, const float *__restrict__ Fx,
              const float *__restrict__ Fy, const float *__restrict__ Fz, float *__restrict__ cf, int64_t cf_stride,
              const uint32_t *__restrict__ marker_tile, uint32_t *__restrict__ tmax, int64_t tstride)
{
    const Grid &g = *gp;
    // wave-uniform loop bound: every lane takes part in the per-tile maxima
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = xcd_block() * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t l = base + (threadIdx.x & 63);
        const bool in = l < n;
        const float a = in ? area[l] : 0.f;
        const uint32_t tl = in ? marker_tile[l] : (uint32_t)g.ntiles;
        const int64_t key = tl < (uint32_t)g.ntiles ? (int64_t)tl : -1;
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            int hi = 0, hj = 0, hk = 0;
            if (in) unpack_home(home[home_at(l, c)], hi, hj, hk);
            float v = 0.0f;
            if (in && home_ok(g, c, hi, hj, hk)) {
                const float Fc = c == 0 ? Fx[l] : (c == 1 ? Fy[l] : Fz[l]);
                if (g.inv_cw2 > 0.f) {
                    // equal control-volume widths w: c_l = A_l / w^2 whatever
                    // the shape functions (a non-finite phi is caught by the
                    // tile kernel, which reads phi anyway)
                    v = a * Fc * g.inv_cw2;
                } else {
                    const float *p = phi + phi_at(l, c);
                    float ph[kNe];
#pragma unroll
                    for (int k = 0; k < kNe; ++k) ph[k] = p[k * kLanes];
                    v = eq8_coef(g, c, hi, hj, hk, ph, a * Fc);
                }
            }
            if (in) cf[c * cf_stride + l] = v;
            wave_key_max(tmax + c * tstride, key, finite_abs(v));
        }
    }
}

int grid_for(int64_t work, int cu)
{
    int64_t b = (work + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cu * 32;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

size_t spread_lds_bytes(const Ctx &c)
{
    return (size_t)c.g.box[0] * c.g.box[1] * c.g.box[2] * sizeof(unsigned long long);
}

// Device buffers of one spreading call: the context's own (mls_spread, the
// time step) or carved out of the library's fixed array (mls_spread_noalloc).
struct SpreadScratch {
    uint32_t *tile_count, *tile_off, *tile_cursor, *tile_active, *block_sums, *work, *tile_fmax, *marker_tile,
        *entries;
    float *cf;
    int64_t cf_stride;
};

static SpreadScratch ctx_scratch(Ctx &c)
{
    return {c.tile_count, c.tile_off, c.tile_cursor, c.tile_active, c.block_sums, c.work, c.tile_fmax,
            c.marker_tile, c.entries, c.cf_rows, c.cf_stride};
}

template <bool SORTED, int NF, int BX>
static hipError_t launch_tiles_bx(Ctx &c, const SpreadScratch &sc, const uint32_t *home, const float *phi, float *fx,
                                  float *fy, float *fz, hipStream_t s, bool timed)
{
    const size_t lds = spread_lds_bytes(c);
    const int persist = c.cu_count * c.spread_blocks_per_cu;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_spread_colour<SORTED, NF, BX>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    TimedLaunch tt(c, timed ? MLS_K_SPREAD_TILES : -1, s);
    for (int col = 0; col < 27; ++col) {
        if (c.colour_tiles[col] == 0) continue;
        hipLaunchKernelGGL((k_spread_colour<SORTED, NF, BX>), dim3(persist), dim3(c.spread_threads), lds, s, c.d_grid,
                           col, home, phi, sc.cf, sc.cf_stride, fx, fy, fz, sc.tile_off, sc.entries, sc.tile_active,
                           sc.work, NF ? c.coef_rows : nullptr, c.w, sc.tile_fmax, c.g.ntiles + 1, c.err);
    }
    return hipGetLastError();
}

// The box-row length the tile kernels are specialised for: the boxes of tile
// edges 4, 6, 8, 10, 12 and 16 on grids whose every axis has several tiles;
// 0 (the general kernel) otherwise.
static int box_row_template(const Ctx &c)
{
    const Grid &g = c.g;
    if (g.ntile[0] < 2 || g.ntile[1] < 2 || g.ntile[2] < 2) return 0;
    switch (g.box[0]) {
    case 7: case 9: case 11: case 13: case 15: case 19: return g.box[0];
    default: return 0;
    }
}

template <bool SORTED, int NF>
static hipError_t launch_tiles(Ctx &c, const SpreadScratch &sc, const uint32_t *home, const float *phi, float *fx,
                               float *fy, float *fz, hipStream_t s, bool timed = true)
{
    switch (box_row_template(c)) {
    case 7: return launch_tiles_bx<SORTED, NF, 7>(c, sc, home, phi, fx, fy, fz, s, timed);
    case 9: return launch_tiles_bx<SORTED, NF, 9>(c, sc, home, phi, fx, fy, fz, s, timed);
    case 11: return launch_tiles_bx<SORTED, NF, 11>(c, sc, home, phi, fx, fy, fz, s, timed);
    case 13: return launch_tiles_bx<SORTED, NF, 13>(c, sc, home, phi, fx, fy, fz, s, timed);
    case 15: return launch_tiles_bx<SORTED, NF, 15>(c, sc, home, phi, fx, fy, fz, s, timed);
    case 19: return launch_tiles_bx<SORTED, NF, 19>(c, sc, home, phi, fx, fy, fz, s, timed);
    default: return launch_tiles_bx<SORTED, NF, 0>(c, sc, home, phi, fx, fy, fz, s, timed);
    }
}

hipError_t launch_interp(const Ctx &c, int64_t n, const uint32_t *home, const float *phi,
                         const float *u, const float *v, const float *w,
                         float *U, float *V, float *W, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + kBlock - 1) / kBlock;
    blocks = round_up8(std::min(blocks, (int64_t)c.cu_count * c.interp_blocks_per_cu));
    hipLaunchKernelGGL(k_interp, dim3((unsigned)blocks), dim3(kBlock), 0, s, c.d_grid, n, home, phi,
                       u, v, w, U, V, W, c.err);
    return hipGetLastError();
}

// The standalone spreading on the buffers sc: binning from the homes, c_l F_l
// and the per-tile maxima by marker, then the coloured tile launches.  timed:
// per-kernel timing marks (they may create HIP events).
static hipError_t launch_spread_with(Ctx &c, const SpreadScratch &sc, int64_t n, const uint32_t *home,
                                     const float *phi, const float *area, const float *Fx, const float *Fy,
                                     const float *Fz, float *fx, float *fy, float *fz, hipStream_t s, bool timed)
{
    if (n == 0) return hipSuccess;
    const int64_t nt = c.g.ntiles;
    const int64_t nb = (nt + kScanChunk - 1) / kScanChunk;
    {
        TimedLaunch tb(c, timed ? MLS_K_SPREAD_BIN : -1, s);
        hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(nt, c.cu_count)), dim3(kBlock), 0, s, sc.tile_count, nt);
        const int gbin = grid_for(n, c.cu_count);
        hipLaunchKernelGGL(k_bin<false>, dim3(gbin), dim3(kBlock), 0, s, c.d_grid, n, home, sc.tile_count,
                           sc.tile_cursor, sc.entries, sc.marker_tile, c.err);
        hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(kBlock), 0, s, sc.tile_count, nt,
                           sc.block_sums);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, sc.block_sums, nb);
        hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kBlock), 0, s, sc.tile_count, nt, sc.block_sums,
                           sc.tile_off, sc.tile_cursor, sc.work, sc.tile_fmax, nt + 1);
        hipLaunchKernelGGL(k_bin<true>, dim3(grid_for(n, c.cu_count)), dim3(kBlock), 0, s, c.d_grid, n, home,
                           sc.tile_count, sc.tile_cursor, sc.entries, sc.marker_tile, c.err);
        hipLaunchKernelGGL(k_active_tiles, dim3((unsigned)((nt + kActiveChunk - 1) / kActiveChunk)), dim3(kBlock), 0,
                           s, c.d_grid, sc.tile_off, sc.tile_active, sc.work);
        hipLaunchKernelGGL(k_spread_coef, dim3((unsigned)round_up8(grid_for(n, c.cu_count))), dim3(kBlock), 0, s,
                           c.d_grid, n, home, phi, area, Fx, Fy, Fz, sc.cf, sc.cf_stride, sc.marker_tile,
                           sc.tile_fmax, nt + 1);
    }
    return launch_tiles<false, 0>(c, sc, home, phi, fx, fy, fz, s, timed);
}

hipError_t launch_spread(Ctx &c, int64_t n, const uint32_t *home, const float *phi,
                         const float *area, const float *Fx, const float *Fy, const float *Fz,
                         float *fx, float *fy, float *fz, hipStream_t s)
{
    return launch_spread_with(c, ctx_scratch(c), n, home, phi, area, Fx, Fy, Fz, fx, fy, fz, s, true);
}

hipError_t launch_sort_positions(Ctx &c, int64_t n, const float *x, const float *y, const float *z, hipStream_t s,
                                 float *jx, float *jy, float *jz, float jitter, uint64_t seed)
{
    const float amp2 = jx ? 2.0f * jitter : 0.0f;
    if (n == 0) return hipSuccess;
    const int64_t nt = c.g.ntiles + 1;   // tiles and the bucket of markers without a valid support
    const int64_t nb = (nt + kScanChunk - 1) / kScanChunk;
    TimedLaunch tb(c, MLS_K_SPREAD_BIN, s);
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(nt, c.cu_count)), dim3(kBlock), 0, s, c.tile_count, nt);
    hipLaunchKernelGGL(k_bin_pos<false>, dim3(grid_for(n, c.cu_count)), dim3(kBlock), 0, s, c.d_grid, n, x, y, z,
                       c.tile_count, c.tile_cursor, c.entries, c.marker_tile, jx, jy, jz, amp2, seed, c.step_ctr);
    hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(kBlock), 0, s, c.tile_count, nt, c.block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, c.block_sums, nb);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kBlock), 0, s, c.tile_count, nt, c.block_sums,
                       c.tile_off, c.tile_cursor, c.work, c.tile_fmax, c.g.ntiles + 1);
    hipLaunchKernelGGL(k_bin_pos<true>, dim3(grid_for(n, c.cu_count)), dim3(kBlock), 0, s, c.d_grid, n, x, y, z,
                       c.tile_count, c.tile_cursor, c.entries, c.marker_tile, nullptr, nullptr, nullptr, 0.0f,
                       (uint64_t)0, c.step_ctr);
    return hipGetLastError();
}

hipError_t launch_spread_sorted(Ctx &c, int64_t n, const uint32_t *home, const float *phi, float *fx, float *fy,
                                float *fz, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t nt = c.g.ntiles;
    {
        TimedLaunch tb(c, MLS_K_SPREAD_BIN, s);
        // colour list sizes and tile cursors start at zero on every call (the
        // call may follow another spreading of the same sort)
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kBlock), 0, s, c.work, (int64_t)64);
        hipLaunchKernelGGL(k_active_tiles, dim3((unsigned)((nt + kActiveChunk - 1) / kActiveChunk)), dim3(kBlock), 0,
                           s, c.d_grid, c.tile_off, c.tile_active, c.work);
    }
    const SpreadScratch sc = ctx_scratch(c);
    if (c.step_nf == 7) return launch_tiles<true, 7>(c, sc, home, phi, fx, fy, fz, s);
    if (c.step_nf == 13) return launch_tiles<true, 13>(c, sc, home, phi, fx, fy, fz, s);
    return launch_tiles<true, 0>(c, sc, home, phi, fx, fy, fz, s);
}


// ---- allocation-free spreading --------------------------------------------
//
// The scratch of mls_spread_noalloc lives in one fixed array in the library's
// code object.  Each GPU the library runs on holds its own copy, allocated
// when the code object is loaded on that device and kept until the process
// ends.  In host code the array's name only stands for the symbol: its
// address on a device comes from hipGetSymbolAddress, taken once per device
// by noalloc_setup (called from mls_ctx_create, with that device current) and
// kept in noalloc_ptr[]; every use on the host goes through that pointer.

static __device__ __align__(256) unsigned char scratch[MLS_SPREAD_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void *noalloc_ptr[kMaxDevices] = {};
std::mutex noalloc_mu;

// Carves the buffers of a standalone spreading of n markers over nt tiles out
// of base (or only measures them when base is NULL); returns the bytes needed.
size_t carve(int64_t nt, int64_t n, unsigned char *base, SpreadScratch &sc)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const int64_t nb = (nt + 1 + kScanChunk - 1) / kScanChunk;
    const int64_t stride = (n + 63) / 64 * 64;
    sc.tile_count = (uint32_t *)take((size_t)(nt + 1) * 4);
    sc.tile_off = (uint32_t *)take((size_t)(nt + 2) * 4);
    sc.tile_cursor = (uint32_t *)take((size_t)(nt + 1) * 4);
    sc.tile_active = (uint32_t *)take((size_t)nt * 4);
    sc.block_sums = (uint32_t *)take((size_t)(nb + 1) * 4);
    sc.work = (uint32_t *)take(128 * 4);
    sc.tile_fmax = (uint32_t *)take((size_t)3 * (nt + 1) * 4);
    sc.marker_tile = (uint32_t *)take((size_t)n * 4);
    sc.entries = (uint32_t *)take((size_t)n * 4);
    sc.cf = (float *)take((size_t)3 * stride * 4);
    sc.cf_stride = stride;
    return off;
}
}  // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    noalloc_ptr[device] = p;
    return hipSuccess;
}

size_t noalloc_bytes(const Ctx &c, int64_t n)
{
    SpreadScratch sc;
    return carve(c.g.ntiles, n, nullptr, sc);
}

hipError_t launch_spread_noalloc(Ctx &c, int64_t n, const uint32_t *home, const float *phi, const float *area,
                                 const float *Fx, const float *Fy, const float *Fz, float *fx, float *fy, float *fz,
                                 hipStream_t s)
{
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(noalloc_mu);
        if (c.device >= 0 && c.device < kMaxDevices) base = noalloc_ptr[c.device];
    }
    if (!base) return hipErrorInvalidDevicePointer;
    SpreadScratch sc;
    carve(c.g.ntiles, n, static_cast<unsigned char *>(base), sc);
    return launch_spread_with(c, sc, n, home, phi, area, Fx, Fy, Fz, fx, fy, fz, s, false);
}

}  // namespace mls
