// Coarse-grained collision detection (Sec. 4): an integer array over the
// Eulerian cells records, per cell, whether no marker, the markers of one
// body, or markers of several bodies lie in it; markers in a cell of the last
// kind are flagged for a collision force.
//
// The paper fills the array in one sequential sweep (an empty cell takes the
// body id, a cell holding another id becomes -1).  Its final state does not
// depend on the order of the sweep: -1 exactly where two or more bodies meet,
// else the one body's id.  Here every marker enters its id with one
// compare-and-swap (0 -> id); a marker that finds another body's id writes -1.
// Whatever the interleaving, the first id to land stays unless a different id
// arrives, and any different id turns the cell to -1 for good, so the result
// is that final state, bit for bit, on any schedule.  A marker whose cell
// already holds its own id or -1 skips the atomic.
#include "mls_device.h"

namespace mls {

namespace {

constexpr int kCollBlock = 256;

// Linear index [z][y][x] of the cell of marker l, or -1 (error raised).
__device__ __forceinline__ int64_t marker_cell(const Grid &g, int64_t l, const float *x, const float *y,
                                               const float *z, ErrWord *err)
{
    int i, j, k;
    if (!cell_axis(g.ax[0], x[l], i) || !cell_axis(g.ax[1], y[l], j) || !cell_axis(g.ax[2], z[l], k)) {
        raise_error(err, l, MLS_E_SUPPORT);
        return -1;
    }
    return ((int64_t)k * g.ax[1].n + j) * g.ax[0].n + i;
}

__global__ void __launch_bounds__(kCollBlock)
k_coll_enter(const Grid *__restrict__ gp, int64_t n, const float *__restrict__ x, const float *__restrict__ y,
             const float *__restrict__ z, const int32_t *__restrict__ body, int32_t *__restrict__ coll,
             ErrWord *err)
{
    const Grid &g = *gp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t l = xcd_block() * blockDim.x + threadIdx.x; l < n; l += stride) {
        const int64_t cell = marker_cell(g, l, x, y, z, err);
        if (cell < 0) continue;
        const int32_t b = body[l];
        if (b < 0 || b > 2147483646) {
            raise_error(err, l, MLS_E_ARG);
            continue;
        }
        const int32_t pid = b + 1;
        // A cell only moves 0 -> id -> -1, so a plain read that already shows
        // this body's id or -1 (possibly an earlier state) needs no atomic:
        // the marker is accounted for.
        const int32_t seen = coll[cell];
        if (seen == pid || seen == -1) continue;
        const int32_t old = atomicCAS(&coll[cell], 0, pid);
        if (old != 0 && old != pid && old != -1) atomicExch(&coll[cell], -1);
    }
}

// flags[l] = 1 where the cell of marker l holds -1 (markers of several bodies).
__global__ void __launch_bounds__(kCollBlock)
k_coll_mark(const Grid *__restrict__ gp, int64_t n, const float *__restrict__ x, const float *__restrict__ y,
            const float *__restrict__ z, const int32_t *__restrict__ coll, uint8_t *__restrict__ flags,
            ErrWord *err)
{
    const Grid &g = *gp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t l = xcd_block() * blockDim.x + threadIdx.x; l < n; l += stride) {
        int i, j, k;
        uint8_t f = 0;
        if (cell_axis(g.ax[0], x[l], i) && cell_axis(g.ax[1], y[l], j) && cell_axis(g.ax[2], z[l], k))
            f = coll[((int64_t)k * g.ax[1].n + j) * g.ax[0].n + i] == -1 ? 1 : 0;
        flags[l] = f;
    }
}

// Returns the cells of the markers to 0 (plain stores of one value: any order).
__global__ void __launch_bounds__(kCollBlock)
k_coll_clear(const Grid *__restrict__ gp, int64_t n, const float *__restrict__ x, const float *__restrict__ y,
             const float *__restrict__ z, int32_t *__restrict__ coll)
{
    const Grid &g = *gp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t l = xcd_block() * blockDim.x + threadIdx.x; l < n; l += stride) {
        int i, j, k;
        if (cell_axis(g.ax[0], x[l], i) && cell_axis(g.ax[1], y[l], j) && cell_axis(g.ax[2], z[l], k))
            coll[((int64_t)k * g.ax[1].n + j) * g.ax[0].n + i] = 0;
    }
}

unsigned coll_blocks(const Ctx &c, int64_t n)
{
    int64_t b = (n + kCollBlock - 1) / kCollBlock;
    b = std::min(b, (int64_t)c.cu_count * 16);
    return (unsigned)round_up8(std::max<int64_t>(b, 1));
}

}  // namespace

hipError_t launch_collide(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                          const int32_t *body, int32_t *coll, uint8_t *flags, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned nb = coll_blocks(c, n);
    hipLaunchKernelGGL(k_coll_enter, dim3(nb), dim3(kCollBlock), 0, s, c.d_grid, n, x, y, z, body, coll, c.err);
    if (flags)
        hipLaunchKernelGGL(k_coll_mark, dim3(nb), dim3(kCollBlock), 0, s, c.d_grid, n, x, y, z, coll, flags,
                           c.err);
    return hipGetLastError();
}

hipError_t launch_collide_clear(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                                int32_t *coll, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_coll_clear, dim3(coll_blocks(c, n)), dim3(kCollBlock), 0, s, c.d_grid, n, x, y, z, coll);
    return hipGetLastError();
}

}  // namespace mls
