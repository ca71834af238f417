// Adaptive Lagrangian mesh refinement (Sec. 3, Fig. 5): markers for the
// interfacial condition generated on the fly from a base triangle mesh.
//
// A base triangle V1 V2 V3 carries one marker at its centroid C (level 0).
// Level 1 splits it at the midpoint of V1 V2 into two triangles, level 2 at C
// into three, level 3 at the three edge midpoints into four; every
// sub-triangle carries one marker at its centroid with its flat area and
// unit normal.  A triangle's level is the smallest L with
// l^2 <= ratio^2 h^2 (L + 1) (l its mean edge length, h the mean width of the
// Eulerian cell holding C: a split into L + 1 parts shrinks the length scale
// by sqrt(L + 1)), at most 3, or one level forced for all.
//
// Three launches: the level of every triangle with per-workgroup marker
// sums; one workgroup scans the sums; every triangle writes its markers at
// its offset, so the output is in triangle order and does not depend on
// scheduling.  All geometry is FP64 from the FP32 vertices, in the order the
// construction states, and rounded to FP32 once at the store.
#include "mls_device.h"

namespace mls {

namespace {

constexpr int kRefBlock = 256;

#pragma clang fp contract(off)

__device__ __forceinline__ bool load_tri(int64_t t, const int32_t *__restrict__ tri, int64_t nvert,
                                         const float *__restrict__ xv, const float *__restrict__ yv,
                                         const float *__restrict__ zv, double V[3][3])
{
    for (int a = 0; a < 3; ++a) {
        const int32_t iv = tri[3 * t + a];
        if (iv < 0 || (int64_t)iv >= nvert) return false;
        V[a][0] = (double)xv[iv];
        V[a][1] = (double)yv[iv];
        V[a][2] = (double)zv[iv];
    }
    return true;
}

__device__ __forceinline__ void centroid(const double V[3][3], double C[3])
{
    for (int d = 0; d < 3; ++d) C[d] = (V[0][d] + V[1][d] + V[2][d]) / 3.0;
}

// Level of one triangle by the size rule; false if C has no cell.
__device__ __forceinline__ bool size_level(const Grid &g, const double V[3][3], double ratio, int &level)
{
    double C[3];
    centroid(V, C);
    double h = 0.0;
    for (int d = 0; d < 3; ++d) {
        int i;
        if (!cell_axis(g.ax[d], C[d], i)) return false;
        h += fval(g.ax[d], i + 1) - fval(g.ax[d], i);
    }
    h /= 3.0;
    double l = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double *P = V[a], *Q = V[(a + 1) % 3];
        l += sqrt((Q[0] - P[0]) * (Q[0] - P[0]) + (Q[1] - P[1]) * (Q[1] - P[1]) + (Q[2] - P[2]) * (Q[2] - P[2]));
    }
    l /= 3.0;
    level = 3;
    for (int L = 0; L <= 3; ++L) {
        if (l * l <= ratio * ratio * h * h * (double)(L + 1)) { level = L; break; }
    }
    return true;
}

__device__ __forceinline__ void put_marker(int64_t m, const double *A, const double *B, const double *Cv,
                                           int64_t cap, float *__restrict__ x, float *__restrict__ y,
                                           float *__restrict__ z, float *__restrict__ area,
                                           float *__restrict__ normal, int32_t *__restrict__ parent, int32_t t)
{
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = B[d] - A[d];
        e2[d] = Cv[d] - A[d];
    }
    const double c0 = e1[1] * e2[2] - e1[2] * e2[1];
    const double c1 = e1[2] * e2[0] - e1[0] * e2[2];
    const double c2 = e1[0] * e2[1] - e1[1] * e2[0];
    const double len = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    x[m] = (float)((A[0] + B[0] + Cv[0]) / 3.0);
    y[m] = (float)((A[1] + B[1] + Cv[1]) / 3.0);
    z[m] = (float)((A[2] + B[2] + Cv[2]) / 3.0);
    area[m] = (float)(0.5 * len);
    normal[m] = (float)(len > 0.0 ? c0 / len : 0.0);
    normal[cap + m] = (float)(len > 0.0 ? c1 / len : 0.0);
    normal[2 * cap + m] = (float)(len > 0.0 ? c2 / len : 0.0);
    parent[m] = t;
}

#pragma clang fp contract(on)

__global__ void __launch_bounds__(kRefBlock)
k_refine_level(const Grid *__restrict__ gp, int64_t ntri, const int32_t *__restrict__ tri, int64_t nvert,
               const float *__restrict__ xv, const float *__restrict__ yv, const float *__restrict__ zv,
               double ratio, int forced, uint8_t *__restrict__ tri_level, uint32_t *__restrict__ block_sums,
               ErrWord *err)
{
    __shared__ uint32_t sh[4];
    const int64_t t = (int64_t)blockIdx.x * kRefBlock + threadIdx.x;
    uint32_t m = 0;
    if (t < ntri) {
        int level = forced < 0 ? 0 : forced;
        double V[3][3];
        if (!load_tri(t, tri, nvert, xv, yv, zv, V)) {
            raise_error(err, t, MLS_E_ARG);
            level = 0;
        } else if (forced < 0 && !size_level(*gp, V, ratio, level)) {
            raise_error(err, t, MLS_E_SUPPORT);
            level = 0;
        }
        tri_level[t] = (uint8_t)level;
        m = (uint32_t)level + 1;
    }
    uint32_t total;
    block_exclusive_scan(m, sh, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the per-workgroup marker counts; the
// total goes to *count.
__global__ void __launch_bounds__(kRefBlock)
k_refine_scan(const uint32_t *__restrict__ block_sums, int64_t nb, uint32_t *__restrict__ block_off,
              int64_t *__restrict__ count)
{
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kRefBlock) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? block_sums[b] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, sh, total);
        if (b < nb) block_off[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *count = (int64_t)carry;
}

__global__ void __launch_bounds__(kRefBlock)
k_refine_emit(int64_t ntri, const int32_t *__restrict__ tri, int64_t nvert, const float *__restrict__ xv,
              const float *__restrict__ yv, const float *__restrict__ zv, const uint8_t *__restrict__ tri_level,
              const uint32_t *__restrict__ block_off, int64_t cap, float *__restrict__ x, float *__restrict__ y,
              float *__restrict__ z, float *__restrict__ area, float *__restrict__ normal,
              int32_t *__restrict__ parent)
{
    __shared__ uint32_t sh[4];
    const int64_t t = (int64_t)blockIdx.x * kRefBlock + threadIdx.x;
    const int level = t < ntri ? (int)tri_level[t] : -1;
    uint32_t total;
    const uint32_t local = block_exclusive_scan((uint32_t)(level + 1), sh, total);
    if (t >= ntri) return;
    const int64_t m = (int64_t)block_off[blockIdx.x] + local;
    double V[3][3];
    if (!load_tri(t, tri, nvert, xv, yv, zv, V)) {
        // reported by the level pass; one marker without geometry
        const float nan = __builtin_nanf("");
        x[m] = y[m] = z[m] = area[m] = nan;
        normal[m] = normal[cap + m] = normal[2 * cap + m] = nan;
        parent[m] = (int32_t)t;
        return;
    }
    const double *V1 = V[0], *V2 = V[1], *V3 = V[2];
    double C[3], L31[3], L32[3], L33[3];
    centroid(V, C);
    for (int d = 0; d < 3; ++d) {
        L31[d] = 0.5 * (V1[d] + V2[d]);
        L32[d] = 0.5 * (V2[d] + V3[d]);
        L33[d] = 0.5 * (V3[d] + V1[d]);
    }
    const int32_t ti = (int32_t)t;
    switch (level) {
    case 0:
        put_marker(m, V1, V2, V3, cap, x, y, z, area, normal, parent, ti);
        break;
    case 1:   // L1 = (V1 + V2)/2 = L31
        put_marker(m, V1, L31, V3, cap, x, y, z, area, normal, parent, ti);
        put_marker(m + 1, L31, V2, V3, cap, x, y, z, area, normal, parent, ti);
        break;
    case 2:   // L2 = C
        put_marker(m, V1, V2, C, cap, x, y, z, area, normal, parent, ti);
        put_marker(m + 1, V2, V3, C, cap, x, y, z, area, normal, parent, ti);
        put_marker(m + 2, V3, V1, C, cap, x, y, z, area, normal, parent, ti);
        break;
    default:
        put_marker(m, V1, L31, L33, cap, x, y, z, area, normal, parent, ti);
        put_marker(m + 1, L31, V2, L32, cap, x, y, z, area, normal, parent, ti);
        put_marker(m + 2, L33, L32, V3, cap, x, y, z, area, normal, parent, ti);
        put_marker(m + 3, L31, L32, L33, cap, x, y, z, area, normal, parent, ti);
        break;
    }
}

}  // namespace

hipError_t launch_refine(Ctx &c, int64_t ntri, const int32_t *tri, int64_t nvert, const float *xv,
                         const float *yv, const float *zv, double ratio, int level, int64_t cap, float *x,
                         float *y, float *z, float *area, float *normal, int32_t *parent, uint8_t *tri_level,
                         int64_t *count, hipStream_t s)
{
    const int64_t nb = (ntri + kRefBlock - 1) / kRefBlock;
    if (2 * std::max<int64_t>(nb, 1) > c.refine_cap) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        hipFree(c.refine_scratch);
        c.refine_scratch = nullptr;
        c.refine_cap = 0;
        e = hipMalloc((void **)&c.refine_scratch, (size_t)2 * std::max<int64_t>(nb, 1) * sizeof(uint32_t));
        if (e != hipSuccess) return e;
        c.refine_cap = 2 * std::max<int64_t>(nb, 1);
    }
    uint32_t *sums = c.refine_scratch, *off = c.refine_scratch + std::max<int64_t>(nb, 1);
    if (ntri > 0)
        hipLaunchKernelGGL(k_refine_level, dim3((unsigned)nb), dim3(kRefBlock), 0, s, c.d_grid, ntri, tri, nvert,
                           xv, yv, zv, ratio, level, tri_level, sums, c.err);
    hipLaunchKernelGGL(k_refine_scan, dim3(1), dim3(kRefBlock), 0, s, sums, nb, off, count);
    if (ntri > 0)
        hipLaunchKernelGGL(k_refine_emit, dim3((unsigned)nb), dim3(kRefBlock), 0, s, ntri, tri, nvert, xv, yv, zv,
                           tri_level, off, cap, x, y, z, area, normal, parent);
    return hipGetLastError();
}

}  // namespace mls
