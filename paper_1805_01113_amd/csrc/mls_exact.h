// Exact MLS (eq. 3-6) for one (marker, component) on one lane: the FP32
// moment-matrix assembly and Cholesky solve with its condition-number bound,
// the FP64 re-solve when the bound exceeds the routing threshold, and the
// failure marking of a marker whose support leaves the grid.  Shared by the
// exact build and the learned build's fallback.
#pragma once

#include "mls_device.h"

namespace mls {

// FP64 re-solve of one (marker, component): recompute the offsets, weights
// and moments in FP64 from the position; the 27 values are returned in
// registers.  Returns false if A is singular.
__device__ __forceinline__ bool solve_fp64_regs(const Grid &g, const Weight &W, int c, double px, double py,
                                                double pz, float ph[kNe])
{
    double s[3][3], w[3][3];
    Moments<double> m[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        axis_offsets_d(g.ax[d], d == c, d == 0 ? px : (d == 1 ? py : pz), s[d]);
        double m0 = 0, m1 = 0, m2 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            w[d][a] = weight1_d(W, s[d][a]);
            m0 += w[d][a]; m1 += w[d][a] * s[d][a]; m2 += w[d][a] * s[d][a] * s[d][a];
        }
        m[d] = {m0, m1, m2};
    }
    double A[10], L[10], gam[4] = {0.0, 0.0, 0.0, 0.0};
    assemble(m[0], m[1], m[2], A);
    const bool ok = cholesky4(A, L);
    if (ok) {
        const double e0[4] = {1.0, 0.0, 0.0, 0.0};
        chol_solve(L, e0, gam);
    }
#pragma unroll
    for (int k = 0; k < kNe; ++k) {
        const int a = k % 3, b = (k / 3) % 3, cc = k / 9;
        const double W3 = w[0][a] * w[1][b] * w[2][cc];
        ph[k] = ok ? (float)(W3 * (gam[0] + gam[1] * s[0][a] + gam[2] * s[1][b] + gam[3] * s[2][cc]))
                   : __builtin_nanf("");
    }
    return ok;
}

// Stencil for a marker without a support (where ok is false): the uniform
// node offsets -1, 0, 1 at node 0.  The fused kernels compute such a marker
// like any other (so all lanes issue the same memory operations) and store
// NaN in its place.  Selects on every field (G may hold anything there), so
// that the compiler does not first set every register to the neutral values
// and then copy the located ones over them.
__device__ __forceinline__ void neutral_geo_unless(bool ok, AxisGeo G[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        G[d].ih = ok ? G[d].ih : 0;
        G[d].s[0] = ok ? G[d].s[0] : -1.f;
        G[d].s[1] = ok ? G[d].s[1] : 0.f;
        G[d].s[2] = ok ? G[d].s[2] : 1.f;
        G[d].xi = ok ? G[d].xi : 0.f;
        G[d].rho = ok ? G[d].rho : 1.f;
    }
}

__device__ __forceinline__ void mark_failed(ErrWord *err, int64_t l, double px, double py, double pz,
                                            uint32_t *hout, float *out, uint8_t *rout)
{
    raise_error(err, l, isfinite(px) && isfinite(py) && isfinite(pz) ? MLS_E_SUPPORT : MLS_E_NONFINITE);
    *hout = 0xffffffffu;
#pragma unroll 1
    for (int k = 0; k < kNe; ++k) out[k * kLanes] = __builtin_nanf("");
    if (rout) *rout = 0;
}

// Shape functions phi_k = W_k (gamma . p_k) (eq. 5) of one (marker,
// component) from the 1-D weights w[d][a] and offsets s[d][a] of its support
// axes and gamma = A^{-1} e_0, in the node order of the blocked layout.  The
// build and the compact spreading of a time step both evaluate phi here, so
// that they obtain the same values from the same inputs.
// With wyz = w_y w_z and pyz = gamma_0 + gamma_2 s_y + gamma_3 s_z per (y, z)
// node pair, phi = wyz (w_x pyz + w_x gamma_1 s_x): one multiply-add and one
// multiply per node.
__device__ __forceinline__ void phi_from_gamma(const float w[3][3], const float s[3][3], const float gam[4],
                                               float ph[kNe])
{
    float vx[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) vx[ax] = w[0][ax] * (gam[1] * s[0][ax]);
#pragma unroll
    for (int cz = 0; cz < 3; ++cz) {
#pragma unroll
        for (int by = 0; by < 3; ++by) {
            const float wyz = w[1][by] * w[2][cz];
            const float pyz = gam[0] + gam[2] * s[1][by] + gam[3] * s[2][cz];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) ph[ax + 3 * by + 9 * cz] = wyz * fmaf(w[0][ax], pyz, vx[ax]);
        }
    }
}

// FP32 exact shape functions of one (marker, component) from its support
// geometry G: 1-D weights and moments, the 10 moment-matrix entries, Cholesky
// and the condition bound.  Returns false (ph and gam undefined) when the
// bound exceeds tau or A is not numerically positive definite: the caller then
// solves in FP64.  kmax accumulates the largest bound seen; gam receives
// A^{-1} e_0.
__device__ __forceinline__ bool exact_fp32(const Weight &W, float tau, const AxisGeo G[3], float ph[kNe],
                                           float &kmax, float gam[4])
{
    float w[3][3], sv[3][3];
    Moments<float> m[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            sv[d][a] = G[d].s[a];
            const float wa = weight1(W, G[d].s[a]);
            w[d][a] = wa;
            m0 += wa;
            m1 += wa * G[d].s[a];
            m2 += wa * G[d].s[a] * G[d].s[a];
        }
        m[d] = {m0, m1, m2};
    }
    float A[10], L[10];
    assemble(m[0], m[1], m[2], A);
    bool ok = cholesky4(A, L);
    if (ok) {
        const float kap = cond_bound_and_gamma(A, L, gam);
        ok = kap <= tau && isfinite(kap);
        kmax = fmaxf(kmax, isfinite(kap) ? kap : 3.0e38f);
    }
    if (!ok) return false;
    phi_from_gamma(w, sv, gam, ph);
    return true;
}

__device__ __forceinline__ bool exact_fp32(const Weight &W, float tau, const AxisGeo G[3], float ph[kNe],
                                           float &kmax)
{
    float gam[4];
    return exact_fp32(W, tau, G, ph, kmax, gam);
}

// Shape functions of component c from the support geometry G of a located
// marker, stored at out (the marker's first support node, nodes kLanes floats
// apart) and returned in ph.  route_bits is stored with bit 0 set when the
// solve went to FP64; routed and kmax accumulate the lane's statistics.
// Returns true if the FP32 solve was used.
__device__ __forceinline__ bool exact_from_geo(const Grid &g, const Weight &W, float tau, int c, int64_t l,
                                               double px, double py, double pz, const AxisGeo G[3], float *out,
                                               uint8_t *rout, uint8_t route_bits, ErrWord *err,
                                               unsigned long long &routed, float &kmax, float ph[kNe])
{
    if (exact_fp32(W, tau, G, ph, kmax)) {
#pragma unroll
        for (int k = 0; k < kNe; ++k) st_stream(&out[k * kLanes], ph[k]);
        if (rout) *rout = route_bits;
        return true;
    }
    ++routed;
    if (!solve_fp64_regs(g, W, c, px, py, pz, ph)) raise_error(err, l, MLS_E_SINGULAR);
#pragma unroll
    for (int k = 0; k < kNe; ++k) out[k * kLanes] = ph[k];
    if (rout) *rout = route_bits | 1;
    return false;
}

}  // namespace mls
