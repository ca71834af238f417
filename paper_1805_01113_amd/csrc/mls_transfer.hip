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
// |A_l F_l| among the tile's markers, so that no sum can overflow.
#include "mls_device.h"

namespace mls {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int64_t field_index(const Grid &g, int c, int i, int j, int k)
{
    return ((int64_t)k * g.dims[c][1] + j) * g.dims[c][0] + i;
}

__global__ void __launch_bounds__(kBlock)
k_interp(const Grid *__restrict__ gp, int64_t n, const uint32_t *__restrict__ home, const float *__restrict__ phi,
         const float *__restrict__ u, const float *__restrict__ v, const float *__restrict__ w,
         float *__restrict__ U, float *__restrict__ V, float *__restrict__ W, ErrWord *err)
{
    const Grid &g = *gp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n; l += stride) {
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
            int64_t ox[3], oy[3], oz[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ox[a] = nb_index(i, a - 1, g.dims[c][0], g.ax[0].periodic);
                oy[a] = (int64_t)nb_index(j, a - 1, g.dims[c][1], g.ax[1].periodic) * g.dims[c][0];
                oz[a] = (int64_t)nb_index(k, a - 1, g.dims[c][2], g.ax[2].periodic) * g.dims[c][0] * g.dims[c][1];
            }
            const float *p = phi + phi_at(l, c);
            float acc = 0.f;
#pragma unroll
            for (int kk = 0; kk < kNe; ++kk) {
                const int a = kk % 3, b = (kk / 3) % 3, cz = kk / 9;
                acc += p[kk * kLanes] * q[oz[cz] + oy[b] + ox[a]];
            }
            out[l] = acc;
        }
    }
}

// ---- spreading: tile binning -------------------------------------------------

// Distinct tiles along one axis touched by the union of the three
// components' supports of a marker.  cell: home of a centre-staggered
// component on this axis; face: home of the face-staggered one (cell or
// cell + 1).  Writes up to 2 tile indices, returns the count.
__device__ __forceinline__ int axis_tiles(const Grid &g, int d, int cell, int face, int t[2])
{
    const Axis &a = g.ax[d];
    const int nn = a.periodic ? a.n : a.n + 1;   // node count covering all components
    int lo = cell - 1;
    int hi = cell + 1;
    const int cell1 = a.periodic ? (cell + 1 == a.n ? 0 : cell + 1) : cell + 1;
    if (face == cell1) hi = cell + 2;
    int cnt = 0;
    for (int i = lo; i <= hi; ++i) {
        int w = i;
        if (a.periodic) w = w < 0 ? w + nn : (w >= nn ? w - nn : w);
        if (w < 0 || w >= nn) continue;
        const int tile = w / a.tile;
        bool seen = false;
        for (int q = 0; q < cnt; ++q) seen = seen || (t[q] == tile);
        if (!seen && cnt < 2) t[cnt++] = tile;
    }
    return cnt;
}

// Binning of markers into tiles.  Lanes of a wavefront that hit the same tile
// are combined into one atomic (the leader adds the count, the others take
// consecutive slots after it in lane order), so a tile's entry list consists
// of runs of consecutive marker indices and the accumulation kernel reads the
// shape functions of a run with coalesced loads.
template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_bin(const Grid *__restrict__ gp, int64_t n, const uint32_t *__restrict__ home, uint32_t *__restrict__ count,
      uint32_t *__restrict__ cursor, uint32_t *__restrict__ entries, ErrWord *err)
{
    const Grid &g = *gp;
    const int lane = threadIdx.x & 63;
    const unsigned long long lower = (1ull << lane) - 1ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the loop bound is wave-uniform so that the ballots below see the whole wave
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t l = base + lane;
        int nt = 0;
        int64_t tl[8];
        if (l < n) {
            int hc[3][3];
            bool valid = true;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                unpack_home(home[home_at(l, c)], hc[c][0], hc[c][1], hc[c][2]);
                valid = valid && home_ok(g, c, hc[c][0], hc[c][1], hc[c][2]);
            }
            if (valid) {
                int tx[2], ty[2], tz[2];
                // centre-staggered home on axis d comes from component (d+1)%3
                const int nx = axis_tiles(g, 0, hc[1][0], hc[0][0], tx);
                const int ny = axis_tiles(g, 1, hc[2][1], hc[1][1], ty);
                const int nz = axis_tiles(g, 2, hc[0][2], hc[2][2], tz);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int a = q >> 2, b = (q >> 1) & 1, cc = q & 1;
                    const bool use = a < nz && b < ny && cc < nx;
                    tl[q] = use ? ((int64_t)tz[a] * g.ntile[1] + ty[b]) * g.ntile[0] + tx[cc] : -1;
                }
                nt = 8;
            } else if (!FILL) {
                raise_error(err, l, MLS_E_SUPPORT);   // contributes nothing
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t t = nt ? tl[q] : -1;
            unsigned long long pending = __ballot(t >= 0);
            while (pending) {
                const int leader = __ffsll((long long)pending) - 1;
                const int64_t tlead = __shfl(t, leader);
                const unsigned long long mask = __ballot(t == tlead) & pending;
                uint32_t pos = 0;
                if (lane == leader)
                    pos = atomicAdd(FILL ? &cursor[tlead] : &count[tlead], (uint32_t)__popcll(mask));
                pos = __shfl(pos, leader);
                if (FILL && ((mask >> lane) & 1ull)) entries[pos + __popcll(mask & lower)] = (uint32_t)l;
                pending &= ~mask;
            }
        }
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

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    // inclusive scan within the wavefront, then across the 4 wavefronts
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int q = 0; q < wid; ++q) base += sh[q];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return base + x - v;
}

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

__global__ void __launch_bounds__(kBlock) k_scan_final(const uint32_t *__restrict__ count, int64_t nt,
                                                       const uint32_t *__restrict__ partial,
                                                       uint32_t *__restrict__ off, uint32_t *__restrict__ cursor,
                                                       uint32_t *__restrict__ work)
{
    __shared__ uint32_t sh[4];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    // each thread owns 8 consecutive elements
    const int per = kScanChunk / kBlock;
    uint32_t vals[kScanChunk / kBlock];
    uint32_t s = 0;
    for (int q = 0; q < per; ++q) {
        const int64_t i = base + (int64_t)threadIdx.x * per + q;
        vals[q] = i < nt ? count[i] : 0u;
        s += vals[q];
    }
    uint32_t total;
    uint32_t run = partial[blockIdx.x] + block_exclusive_scan(s, sh, total);
    for (int q = 0; q < per; ++q) {
        const int64_t i = base + (int64_t)threadIdx.x * per + q;
        if (i < nt) {
            off[i] = run;
            cursor[i] = run;
        }
        run += vals[q];
    }
    const int64_t first = base + (int64_t)threadIdx.x * per;
    if (first <= nt - 1 && nt - 1 < first + per) off[nt] = run;   // the owner of the last tile
    if (blockIdx.x == 0 && threadIdx.x < 16) work[threadIdx.x] = 0u;   // active-list sizes and cursors
}

// Non-empty tiles, listed per XCD slab: the tiles are split into 8 contiguous
// slabs (one per XCD); work[x] counts the non-empty tiles of slab x and
// active[x * chunk + i] lists them.
__global__ void __launch_bounds__(kBlock)
k_active_tiles(const uint32_t *__restrict__ count, int64_t nt, uint32_t *__restrict__ active, uint32_t *work)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long lower = (1ull << lane) - 1ull;
    const int64_t chunk = (nt + 7) >> 3;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < nt; base += stride) {
        const int64_t t = base + lane;
        const int x = (t < nt && count[t] > 0u) ? (int)(t / chunk) : -1;
        unsigned long long pending = __ballot(x >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int xl = __shfl(x, leader);
            const unsigned long long mask = __ballot(x == xl) & pending;
            uint32_t pos = 0;
            if (lane == leader) pos = atomicAdd(&work[xl], (uint32_t)__popcll(mask));
            pos = __shfl(pos, leader);
            if ((mask >> lane) & 1ull) active[(int64_t)xl * chunk + pos + __popcll(mask & lower)] = (uint32_t)t;
            pending &= ~mask;
        }
    }
}

// ---- spreading: per-tile fixed-point accumulation ------------------------------

constexpr int kTileNodes = kMaxTile * kMaxTile * kMaxTile;   // 4096

__device__ __forceinline__ float width_of(const Axis &a, int is_face, int i)
{
    return is_face ? a.width_f[i] : a.width_c[i];
}

__global__ void __launch_bounds__(kBlock)
k_spread_tiles(const Grid *__restrict__ gp, int64_t n, const uint32_t *__restrict__ home, const float *__restrict__ phi,
               const float *__restrict__ area, const float *__restrict__ Fx, const float *__restrict__ Fy,
               const float *__restrict__ Fz, float *__restrict__ fx, float *__restrict__ fy,
               float *__restrict__ fz, const uint32_t *__restrict__ off, const uint32_t *__restrict__ entries,
               const uint32_t *__restrict__ active, uint32_t *work, ErrWord *err)
{
    const Grid &g = *gp;
    __shared__ unsigned long long acc[kTileNodes];
    __shared__ float red[3][kBlock / 64];
    const int tsx = g.ax[0].tile, tsy = g.ax[1].tile, tsz = g.ax[2].tile;
    const int tnodes = tsx * tsy * tsz;
    const Axis &AX = g.ax[0], &AY = g.ax[1], &AZ = g.ax[2];
    // XCD-aware dynamic assignment: workgroups are dispatched round-robin over
    // the 8 XCDs, so blockIdx % 8 names the XCD.  Each XCD first takes the
    // non-empty tiles of its own slab (tiles sharing markers then share that
    // XCD's L2), then helps the other slabs.
    __shared__ int64_t tile_sh;
    const int xcd = blockIdx.x & 7;
    const int64_t chunk = (g.ntiles + 7) >> 3;
    int src = xcd, rounds = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int64_t t = -1;
            while (rounds < 8) {
                const uint32_t i = atomicAdd(&work[8 + src], 1u);
                if (i < work[src]) { t = active[(int64_t)src * chunk + i]; break; }
                src = (src + 1) & 7;
                ++rounds;
            }
            tile_sh = t;
        }
        __syncthreads();
        const int64_t t = tile_sh;
        __syncthreads();
        if (t < 0) break;
        const uint32_t beg = off[t], end = off[t + 1];
        const int tx = (int)(t % g.ntile[0]);
        const int ty = (int)((t / g.ntile[0]) % g.ntile[1]);
        const int tz = (int)(t / ((int64_t)g.ntile[0] * g.ntile[1]));
        const int x0 = tx * tsx, y0 = ty * tsy, z0 = tz * tsz;

        // largest |A_l F_l| per component among the tile's markers
        float mx[3] = {0.f, 0.f, 0.f};
        for (uint32_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
            const uint32_t m = entries[e];
            const float a = fabsf(area[m]);
            mx[0] = fmaxf(mx[0], a * fabsf(Fx[m]));
            mx[1] = fmaxf(mx[1], a * fabsf(Fy[m]));
            mx[2] = fmaxf(mx[2], a * fabsf(Fz[m]));
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float v = mx[c];
            for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
            if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        float M[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) M[c] = fmaxf(fmaxf(red[c][0], red[c][1]), fmaxf(red[c][2], red[c][3]));
        // c_l <= A_l / h^2 for a shape function with sum phi dV close to dV,
        // h the smallest control-volume width near the tile; with |phi| <= 2
        // every contribution |c_l phi_k F_l| stays below bound = 8 M / h^2.
        const float hloc = fminf(fminf(AX.tile_hmin[tx], AY.tile_hmin[ty]), AZ.tile_hmin[tz]);
        const double inv_h2 = 1.0 / ((double)hloc * (double)hloc);
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            const double bound = 8.0 * (double)M[c] * inv_h2;
            if (!(bound > 0.0) || !(bound < 1e300)) {   // nothing to add, or a non-finite force
                if (!(bound >= 0.0) || bound >= 1e300)
                    for (uint32_t e = beg + threadIdx.x; e < end; e += blockDim.x) raise_error(err, entries[e], MLS_E_RANGE);
                continue;
            }
            int ebits;
            frexp(bound, &ebits);                      // bound < 2^ebits
            // each scaled contribution stays below 2^30: it converts to int32
            // exactly enough (quantum 2^-30 of the bound) and sums in int64
            const int S = 30 - ebits;
            for (int q = threadIdx.x; q < tnodes; q += blockDim.x) acc[q] = 0ull;
            __syncthreads();
            const float *F = c == 0 ? Fx : (c == 1 ? Fy : Fz);
            const float scale_f = ldexpf(1.0f, S);
            const float lim = 1073741824.0f;            // 2^30
            for (uint32_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
                const uint32_t m = entries[e];
                int hi, hj, hk;
                unpack_home(home[home_at(m, c)], hi, hj, hk);
                int ix[3], iy[3], iz[3];
                bool inx[3], iny[3], inz[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    ix[a] = nb_index(hi, a - 1, g.dims[c][0], AX.periodic);
                    iy[a] = nb_index(hj, a - 1, g.dims[c][1], AY.periodic);
                    iz[a] = nb_index(hk, a - 1, g.dims[c][2], AZ.periodic);
                    inx[a] = (unsigned)(ix[a] - x0) < (unsigned)tsx;
                    iny[a] = (unsigned)(iy[a] - y0) < (unsigned)tsy;
                    inz[a] = (unsigned)(iz[a] - z0) < (unsigned)tsz;
                }
                // this component's support may miss the tile (the entry list is
                // the union over components): then nothing is read
                if (!((inx[0] || inx[1] || inx[2]) && (iny[0] || iny[1] || iny[2]) && (inz[0] || inz[1] || inz[2])))
                    continue;
                float wx[3], wy[3], wz[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    wx[a] = width_of(AX, c == 0, ix[a]);
                    wy[a] = width_of(AY, c == 1, iy[a]);
                    wz[a] = width_of(AZ, c == 2, iz[a]);
                }
                const float *p = phi + phi_at(m, c);
                float ph[kNe];
                float hl = 0.f, den = 0.f;
#pragma unroll
                for (int k = 0; k < kNe; ++k) {
                    const int a = k % 3, b = (k / 3) % 3, cz = k / 9;
                    ph[k] = p[k * kLanes];
                    hl += ph[k] * (wx[a] + wy[b] + wz[cz]);
                    den += ph[k] * (wx[a] * wy[b] * wz[cz]);
                }
                // c_l F_l = A_l h_l F_l / sum_k phi_k dV_k   (eq. 8), pre-scaled
                const float vsc = area[m] * (hl * (1.0f / 3.0f)) * F[m] / den * scale_f;
                bool range_ok = true;
#pragma unroll
                for (int k = 0; k < kNe; ++k) {
                    const int a = k % 3, b = (k / 3) % 3, cz = k / 9;
                    if (inx[a] && iny[b] && inz[cz]) {
                        float vs = ph[k] * vsc;
                        range_ok = range_ok && (fabsf(vs) < lim);
                        vs = fminf(fmaxf(vs, -lim), lim);
                        const long long qv = (long long)(int)rintf(vs);
                        const int li = ((iz[cz] - z0) * tsy + (iy[b] - y0)) * tsx + (ix[a] - x0);
                        atomicAdd(&acc[li], (unsigned long long)qv);
                    }
                }
                if (!range_ok) raise_error(err, m, MLS_E_RANGE);
            }
            __syncthreads();
            float *f = c == 0 ? fx : (c == 1 ? fy : fz);
            const double inv_scale = ldexp(1.0, -S);
            for (int q = threadIdx.x; q < tnodes; q += blockDim.x) {
                const long long sv = (long long)acc[q];
                if (sv == 0) continue;
                const int lx = q % tsx, ly = (q / tsx) % tsy, lz = q / (tsx * tsy);
                const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
                if (gx >= g.dims[c][0] || gy >= g.dims[c][1] || gz >= g.dims[c][2]) continue;
                const int64_t idx = field_index(g, c, gx, gy, gz);
                f[idx] = f[idx] + (float)((double)sv * inv_scale);
            }
            __syncthreads();
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

hipError_t launch_interp(const Ctx &c, int64_t n, const uint32_t *home, const float *phi,
                         const float *u, const float *v, const float *w,
                         float *U, float *V, float *W, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_interp, dim3(grid_for(n, c.cu_count)), dim3(kBlock), 0, s, c.d_grid, n, home, phi,
                       u, v, w, U, V, W, c.err);
    return hipGetLastError();
}

hipError_t launch_spread(Ctx &c, int64_t n, const uint32_t *home, const float *phi,
                         const float *area, const float *Fx, const float *Fy, const float *Fz,
                         float *fx, float *fy, float *fz, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t nt = c.g.ntiles;
    const int64_t nb = (nt + kScanChunk - 1) / kScanChunk;
    TimedLaunch* tb = new TimedLaunch(c, MLS_K_SPREAD_BIN, s);
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(nt, c.cu_count)), dim3(kBlock), 0, s, c.tile_count, nt);
    hipLaunchKernelGGL(k_bin<false>, dim3(grid_for(n, c.cu_count)), dim3(kBlock), 0, s, c.d_grid, n, home,
                       c.tile_count, c.tile_cursor, c.entries, c.err);
    hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(kBlock), 0, s, c.tile_count, nt, c.block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, c.block_sums, nb);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kBlock), 0, s, c.tile_count, nt, c.block_sums,
                       c.tile_off, c.tile_cursor, c.work);
    hipLaunchKernelGGL(k_bin<true>, dim3(grid_for(n, c.cu_count)), dim3(kBlock), 0, s, c.d_grid, n, home,
                       c.tile_count, c.tile_cursor, c.entries, c.err);
    hipLaunchKernelGGL(k_active_tiles, dim3(grid_for(nt, c.cu_count)), dim3(kBlock), 0, s, c.tile_count, nt,
                       c.tile_active, c.work);
    delete tb;
    const int persist = ((c.cu_count * 4) + 7) & ~7;   // a multiple of the 8 XCDs
    TimedLaunch tt(c, MLS_K_SPREAD_TILES, s);
    hipLaunchKernelGGL(k_spread_tiles, dim3(persist), dim3(kBlock), 0, s, c.d_grid, n, home, phi, area, Fx, Fy, Fz,
                       fx, fy, fz, c.tile_off, c.entries, c.tile_active, c.work, c.err);
    return hipGetLastError();
}

}  // namespace mls
