// Derivative shape functions: the gradient, with respect to the marker
// position, of the exact MLS approximation of eq. 6 (the weights, and so A
// and B, move with the marker), and the cell-centred staggering of the
// pressure.  These give velocity gradients and pressure at the markers, the
// further MLS operations that moving and deforming bodies need.
//
// In the marker-centred basis p = [1, s] (s = (node - x)/H) with
// gamma = A^-1 e0, beta_d = A^-1 e_{1+d} and eta_d = A^-1 dA_d gamma,
//   phi_k = W_k (gamma . p_k),
//   d phi_k / d xi_d = dW_dk (gamma . p_k) + W_k ((beta_d - eta_d) . p_k),
// where dW_dk = -w'(s_dk) prod_{e != d} w(s_ek) and dA_d = sum_k dW_dk
// p_k p_k^T, assembled from separable moments like A itself (the moments of
// axis d taken with w' in place of w).  The physical derivative divides by
// H_d.  The solve runs in FP32 with the condition bound of the exact build;
// a (marker, staggering) above the routing threshold is queued and redone in
// FP64 from the position by a second kernel, which keeps the registers of the
// double-precision state off the FP32 kernel.
#include "mls_device.h"

namespace mls {

namespace {

constexpr int kGradBlock = 256;

__device__ __forceinline__ int comp_dim(const Grid &g, int c, int d)
{
    return c < 3 ? g.dims[c][d] : g.ax[d].n;
}

template <typename T>
__device__ __forceinline__ void sym_mul(const T A[10], const T v[4], T out[4])
{
    out[0] = A[0] * v[0] + A[1] * v[1] + A[2] * v[2] + A[3] * v[3];
    out[1] = A[1] * v[0] + A[4] * v[1] + A[5] * v[2] + A[6] * v[3];
    out[2] = A[2] * v[0] + A[5] * v[1] + A[7] * v[2] + A[8] * v[3];
    out[3] = A[3] * v[0] + A[6] * v[1] + A[8] * v[2] + A[9] * v[3];
}

// Coefficients of one (marker, staggering): weights w, derivatives wd,
// gamma and cd[d] = beta_d - eta_d.  FP32: returns false (caller goes to
// FP64) if A is not numerically positive definite or the condition bound
// exceeds tau.  FP64: returns false if A is singular.
template <typename T>
struct GradCoef {
    T s[3][3], w[3][3], wd[3][3], gam[4], cd[3][4], rH[3];
};

template <typename T>
__device__ __forceinline__ bool grad_coef(const Weight &Wt, T tau, GradCoef<T> &q, float &kmax)
{
    Moments<T> m[3], md[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T m0 = 0, m1 = 0, m2 = 0, d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T v, dv;
            weight1_ds(Wt, q.s[d][a], v, dv);
            q.w[d][a] = v;
            q.wd[d][a] = dv;
            const T sa = q.s[d][a];
            m0 += v; m1 += v * sa; m2 += v * sa * sa;
            d0 += dv; d1 += dv * sa; d2 += dv * sa * sa;
        }
        m[d] = {m0, m1, m2};
        md[d] = {-d0, -d1, -d2};   // dW_dk carries -w'
    }
    T A[10], L[10];
    assemble(m[0], m[1], m[2], A);
    if (!cholesky4(A, L)) return false;
    if (sizeof(T) == 4) {
        const T kap = cond_bound_and_gamma(A, L, q.gam);
        kmax = fmaxf(kmax, isfinite((float)kap) ? (float)kap : 3.0e38f);
        if (!(kap <= tau)) return false;
    } else {
        const T e0[4] = {1, 0, 0, 0};
        chol_solve(L, e0, q.gam);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T e[4] = {0, 0, 0, 0};
        e[1 + d] = 1;
        T beta[4], dA[10], v[4], eta[4];
        chol_solve(L, e, beta);
        assemble(d == 0 ? md[0] : m[0], d == 1 ? md[1] : m[1], d == 2 ? md[2] : m[2], dA);
        sym_mul(dA, q.gam, v);
        chol_solve(L, v, eta);
#pragma unroll
        for (int i = 0; i < 4; ++i) q.cd[d][i] = beta[i] - eta[i];
    }
    return true;
}

// Visits the 27 support nodes (x fastest) with phi_k and the physical
// derivatives; the loops unroll fully so every index is a constant.  With
// RECOMPUTE the 1-D weights are evaluated again from the offsets instead of
// read from q (fewer live registers for the FP64 route).
template <bool RECOMPUTE, typename T, typename F>
__device__ __forceinline__ void for_each_node(const GradCoef<T> &q, const Weight &Wt, F &&f)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const T sx = q.s[0][a], sy = q.s[1][b], sz = q.s[2][c];
                T wx, wy, wz, dx, dy, dz;
                if (RECOMPUTE) {
                    weight1_ds(Wt, sx, wx, dx);
                    weight1_ds(Wt, sy, wy, dy);
                    weight1_ds(Wt, sz, wz, dz);
                } else {
                    wx = q.w[0][a]; wy = q.w[1][b]; wz = q.w[2][c];
                    dx = q.wd[0][a]; dy = q.wd[1][b]; dz = q.wd[2][c];
                }
                const T W = wx * wy * wz;
                const T gp = q.gam[0] + q.gam[1] * sx + q.gam[2] * sy + q.gam[3] * sz;
                const T dW[3] = {-dx * wy * wz, -wx * dy * wz, -wx * wy * dz};
                T dph[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const T cp = q.cd[d][0] + q.cd[d][1] * sx + q.cd[d][2] * sy + q.cd[d][3] * sz;
                    dph[d] = (dW[d] * gp + W * cp) * q.rH[d];
                }
                f(a, b, c, W * gp, dph);
            }
        }
    }
}

// Geometry of one (marker, staggering c): FP32 offsets and 1/H; false if a
// support leaves a wall axis.  ih receives the wrapped home per axis.
__device__ __forceinline__ bool grad_geo(const Grid &g, int c, const double p[3], GradCoef<float> &q, int ih[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        AxisGeo G;
        double rH;
        if (!axis_geo(g.ax[d], d == c, p[d], G, rH)) return false;
        q.s[d][0] = G.s[0]; q.s[d][1] = G.s[1]; q.s[d][2] = G.s[2];
        q.rH[d] = (float)rH;
        ih[d] = G.ih;
    }
    return true;
}

__device__ __forceinline__ void grad_geo_d(const Grid &g, int c, const double p[3], GradCoef<double> &q)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double H;
        axis_offsets_d(g.ax[d], d == c, p[d], q.s[d], H);
        q.rH[d] = 1.0 / H;
    }
}

// FP64 route of one (marker, staggering).  Shape functions: phi/dphi at the
// marker's first entries, kLanes apart.
__device__ __forceinline__ bool build_grad_fp64(const Grid &g, const Weight &Wt, int c, double px, double py, double pz,
                                             float *ph, float *dp)
{
    const double p[3] = {px, py, pz};
    GradCoef<double> qd;
    grad_geo_d(g, c, p, qd);
    float kmax = 0.f;
    const bool ok = grad_coef(Wt, 0.0, qd, kmax);
    const float nan = __builtin_nanf("");
    for_each_node<true>(qd, Wt, [&](int a, int b, int cz, double v, const double dv[3]) {
        const int k = a + 3 * b + 9 * cz;
        ph[k * kLanes] = ok ? (float)v : nan;
        dp[k * kLanes] = ok ? (float)dv[0] : nan;
        dp[(kNe + k) * kLanes] = ok ? (float)dv[1] : nan;
        dp[(2 * kNe + k) * kLanes] = ok ? (float)dv[2] : nan;
    });
    return ok;
}

// Value and gradient: out[0] = sum phi q, out[1 + d] = sum dphi_d q.
__device__ __forceinline__ bool interp_grad_fp64(const Grid &g, const Weight &Wt, int c, double px, double py,
                                              double pz, const float *fq, const int64_t ox[3], const int64_t oy[3],
                                              const int64_t oz[3], float out[4])
{
    const double p[3] = {px, py, pz};
    GradCoef<double> qd;
    grad_geo_d(g, c, p, qd);
    float kmax = 0.f;
    const bool ok = grad_coef(Wt, 0.0, qd, kmax);
    double ad = 0.0, gd[3] = {0.0, 0.0, 0.0};
    for_each_node<true>(qd, Wt, [&](int a, int b, int cz, double ph, const double dv[3]) {
        const double fv = (double)fq[oz[cz] + oy[b] + ox[a]];
        ad += ph * fv;
        gd[0] += dv[0] * fv; gd[1] += dv[1] * fv; gd[2] += dv[2] * fv;
    });
    const float nan = __builtin_nanf("");
    out[0] = ok ? (float)ad : nan;
    for (int d = 0; d < 3; ++d) out[1 + d] = ok ? (float)gd[d] : nan;
    return ok;
}

__device__ __forceinline__ void count_fp64(DevStats *stats, unsigned long long routed)
{
    if (routed) atomicAdd(&stats->fp64_solves, routed);
}

// FP64 queue: q[0] = entries, q[1 + i] = 4 l + c.
__device__ __forceinline__ void enqueue(uint32_t *queue, int64_t l, int c)
{
    const uint32_t i = atomicAdd(&queue[0], 1u);
    queue[1 + i] = (uint32_t)(4 * l + c);
}

__global__ void k_queue_clear(uint32_t *queue) { if (threadIdx.x == 0) queue[0] = 0u; }

// Shape functions and derivatives of one staggering, blocked by 64 markers:
// home[l], phi[(b*27 + k)*64 + r], dphi[((b*3 + d)*27 + k)*64 + r].
__global__ void __launch_bounds__(kGradBlock)
k_build_grad(const Grid *__restrict__ gp, Weight Wt, float tau, int c, int64_t n, const float *__restrict__ x,
             const float *__restrict__ y, const float *__restrict__ z, uint32_t *__restrict__ home,
             float *__restrict__ phi, float *__restrict__ dphi, uint32_t *queue, ErrWord *err, DevStats *stats)
{
    const Grid &g = *gp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long routed = 0;
    float kmax = 0.f;
    const int64_t npad = (n + kLanes - 1) / kLanes * kLanes;
    for (int64_t l = xcd_block() * blockDim.x + threadIdx.x; l < npad; l += stride) {
        const int64_t b = l / kLanes, r = l % kLanes;
        float *ph = phi + b * kNe * kLanes + r;
        float *dp = dphi + b * 3 * kNe * kLanes + r;
        if (l >= n) {   // padding lanes of the last block
            home[l] = 0xffffffffu;
            for (int k = 0; k < kNe; ++k) ph[k * kLanes] = 0.f;
            for (int k = 0; k < 3 * kNe; ++k) dp[k * kLanes] = 0.f;
            continue;
        }
        const double p[3] = {(double)x[l], (double)y[l], (double)z[l]};
        GradCoef<float> q;
        int ih[3];
        if (!grad_geo(g, c, p, q, ih)) {
            raise_error(err, l, isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) ? MLS_E_SUPPORT
                                                                                      : MLS_E_NONFINITE);
            home[l] = 0xffffffffu;
            for (int k = 0; k < kNe; ++k) ph[k * kLanes] = __builtin_nanf("");
            for (int k = 0; k < 3 * kNe; ++k) dp[k * kLanes] = __builtin_nanf("");
            continue;
        }
        st_stream(&home[l], (uint32_t)ih[0] | ((uint32_t)ih[1] << 11) | ((uint32_t)ih[2] << 22));
        if (grad_coef(Wt, tau, q, kmax)) {
            for_each_node<false>(q, Wt, [&](int a, int b, int cz, float v, const float dv[3]) {
                const int k = a + 3 * b + 9 * cz;
                st_stream(&ph[k * kLanes], v);
                st_stream(&dp[k * kLanes], dv[0]);
                st_stream(&dp[(kNe + k) * kLanes], dv[1]);
                st_stream(&dp[(2 * kNe + k) * kLanes], dv[2]);
            });
        } else {
            ++routed;
            enqueue(queue, l, c);
        }
    }
    count_fp64(stats, routed);
}

// Value and gradient of the MLS approximation of the fields at the markers:
// for c in 0..nc-1 (u, v, w, then the cell-centred p when given),
// val[c][l] = sum_k phi_k q_c[node_k], grad[3c + d][l] = sum_k dphi_dk q_c.
__global__ void __launch_bounds__(kGradBlock)
k_interp_grad(const Grid *__restrict__ gp, Weight Wt, float tau, int64_t n, const float *__restrict__ x,
              const float *__restrict__ y, const float *__restrict__ z, const float *__restrict__ u,
              const float *__restrict__ v, const float *__restrict__ w, const float *__restrict__ pf,
              float *__restrict__ val, float *__restrict__ grad, float *__restrict__ pval,
              float *__restrict__ pgrad, uint32_t *queue, ErrWord *err, DevStats *stats)
{
    const Grid &g = *gp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int nc = pf ? 4 : 3;
    unsigned long long routed = 0;
    float kmax = 0.f;
    for (int64_t l = xcd_block() * blockDim.x + threadIdx.x; l < n; l += stride) {
        const double p[3] = {(double)x[l], (double)y[l], (double)z[l]};
        for (int c = 0; c < nc; ++c) {
            const float *fq = c == 0 ? u : (c == 1 ? v : (c == 2 ? w : pf));
            float *vo = c < 3 ? val : pval;
            float *go = c < 3 ? grad + (int64_t)3 * c * n : pgrad;
            const int64_t vi = c < 3 ? (int64_t)c * n + l : l;
            GradCoef<float> q;
            int ih[3];
            if (!grad_geo(g, c, p, q, ih)) {
                raise_error(err, l, isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) ? MLS_E_SUPPORT
                                                                                          : MLS_E_NONFINITE);
                const float nan = __builtin_nanf("");
                if (vo) vo[vi] = nan;
                if (go) { go[l] = nan; go[n + l] = nan; go[2 * n + l] = nan; }
                continue;
            }
            const int nx = comp_dim(g, c, 0), ny = comp_dim(g, c, 1), nz = comp_dim(g, c, 2);
            uint32_t oy[3], oz[3];
            support_rows(true, ih[1], ih[2], nx, ny, nz, g.ax[1].periodic, g.ax[2].periodic, oy, oz);
            // the 27 field values are requested before the solve, which hides
            // their latency
            float qv[kNe];
            load_support(fq, ih[0], nx, oy, oz, qv);
            float acc = 0.f, ga[3] = {0.f, 0.f, 0.f};
            if (grad_coef(Wt, tau, q, kmax)) {
                // sum_k dphi_dk = 0, so the gradient is summed over q_k - q_home:
                // the terms are O(h |grad q|) instead of O(|q|), which spares
                // FP32 the cancellation of an O(|q|/h) sum down to O(|grad q|)
                const float fh = qv[13];
                for_each_node<false>(q, Wt, [&](int a, int b, int cz, float ph, const float dv[3]) {
                    const float fv = qv[a + 3 * b + 9 * cz];
                    const float df = fv - fh;
                    acc += ph * fv;
                    ga[0] += dv[0] * df; ga[1] += dv[1] * df; ga[2] += dv[2] * df;
                });
            } else {
                ++routed;
                enqueue(queue, l, c);
                continue;   // the FP64 kernel writes this (marker, staggering)
            }
            if (vo) vo[vi] = acc;
            if (go) { go[l] = ga[0]; go[n + l] = ga[1]; go[2 * n + l] = ga[2]; }
        }
    }
    count_fp64(stats, routed);
}

// FP64 redo of the queued (marker, staggering) pairs.
__global__ void __launch_bounds__(kGradBlock)
k_build_grad_fp64(const Grid *__restrict__ gp, Weight Wt, int64_t n, const float *__restrict__ x,
                  const float *__restrict__ y, const float *__restrict__ z, float *__restrict__ phi,
                  float *__restrict__ dphi, const uint32_t *__restrict__ queue, ErrWord *err)
{
    const Grid &g = *gp;
    const uint32_t cnt = queue[0];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const uint32_t e = queue[1 + i];
        const int64_t l = e >> 2;
        const int c = (int)(e & 3u);
        if (l >= n) continue;
        const int64_t b = l / kLanes, r = l % kLanes;
        if (!build_grad_fp64(g, Wt, c, (double)x[l], (double)y[l], (double)z[l], phi + b * kNe * kLanes + r,
                             dphi + b * 3 * kNe * kLanes + r))
            raise_error(err, l, MLS_E_SINGULAR);
    }
}

__global__ void __launch_bounds__(kGradBlock)
k_interp_grad_fp64(const Grid *__restrict__ gp, Weight Wt, int64_t n, const float *__restrict__ x,
                   const float *__restrict__ y, const float *__restrict__ z, const float *__restrict__ u,
                   const float *__restrict__ v, const float *__restrict__ w, const float *__restrict__ pf,
                   float *__restrict__ val, float *__restrict__ grad, float *__restrict__ pval,
                   float *__restrict__ pgrad, const uint32_t *__restrict__ queue, ErrWord *err)
{
    const Grid &g = *gp;
    const uint32_t cnt = queue[0];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const uint32_t e = queue[1 + i];
        const int64_t l = e >> 2;
        const int c = (int)(e & 3u);
        if (l >= n) continue;
        const double p[3] = {(double)x[l], (double)y[l], (double)z[l]};
        int ih[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            AxisGeo G;
            axis_geo(g.ax[d], d == c, p[d], G);   // located by the FP32 pass
            ih[d] = G.ih;
        }
        const int nx = comp_dim(g, c, 0), ny = comp_dim(g, c, 1), nz = comp_dim(g, c, 2);
        int64_t ox[3], oy[3], oz[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ox[a] = nb_index(ih[0], a - 1, nx, g.ax[0].periodic);
            oy[a] = (int64_t)nb_index(ih[1], a - 1, ny, g.ax[1].periodic) * nx;
            oz[a] = (int64_t)nb_index(ih[2], a - 1, nz, g.ax[2].periodic) * nx * ny;
        }
        const float *fq = c == 0 ? u : (c == 1 ? v : (c == 2 ? w : pf));
        float o4[4];
        if (!interp_grad_fp64(g, Wt, c, p[0], p[1], p[2], fq, ox, oy, oz, o4)) raise_error(err, l, MLS_E_SINGULAR);
        float *vo = c < 3 ? val : pval;
        float *go = c < 3 ? grad + (int64_t)3 * c * n : pgrad;
        if (vo) vo[c < 3 ? (int64_t)c * n + l : l] = o4[0];
        if (go) { go[l] = o4[1]; go[n + l] = o4[2]; go[2 * n + l] = o4[3]; }
    }
}

unsigned grad_blocks(const Ctx &c, int64_t work)
{
    int64_t b = (work + kGradBlock - 1) / kGradBlock;
    b = std::min(b, (int64_t)c.cu_count * 16);
    return (unsigned)round_up8(std::max<int64_t>(b, 1));
}

}  // namespace

// The FP64 queue holds up to 4 n entries (one per marker and staggering).
static hipError_t reserve_queue(Ctx &c, int64_t n, hipStream_t s)
{
    const int64_t need = 1 + 4 * n;
    if (need <= c.grad_queue_cap) return hipSuccess;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    hipFree(c.grad_queue);
    c.grad_queue = nullptr;
    c.grad_queue_cap = 0;
    e = hipMalloc((void **)&c.grad_queue, (size_t)need * sizeof(uint32_t));
    if (e != hipSuccess) return e;
    c.grad_queue_cap = need;
    return hipSuccess;
}

hipError_t launch_build_grad(Ctx &c, int64_t n, const float *x, const float *y, const float *z, int stagger,
                             uint32_t *home, float *phi, float *dphi, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipError_t e = reserve_queue(c, n, s);
    if (e != hipSuccess) return e;
    const int64_t npad = (n + kLanes - 1) / kLanes * kLanes;
    hipLaunchKernelGGL(k_queue_clear, dim3(1), dim3(64), 0, s, c.grad_queue);
    hipLaunchKernelGGL(k_build_grad, dim3(grad_blocks(c, npad)), dim3(kGradBlock), 0, s, c.d_grid, c.w,
                       (float)c.opts.kappa_tau, stagger, n, x, y, z, home, phi, dphi, c.grad_queue, c.err, c.stats);
    hipLaunchKernelGGL(k_build_grad_fp64, dim3(round_up8(c.cu_count)), dim3(kGradBlock), 0, s, c.d_grid, c.w, n, x, y,
                       z, phi, dphi, c.grad_queue, c.err);
    return hipGetLastError();
}

hipError_t launch_interp_grad(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *u,
                              const float *v, const float *w, const float *p, float *U, float *G, float *P, float *GP,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipError_t e = reserve_queue(c, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_queue_clear, dim3(1), dim3(64), 0, s, c.grad_queue);
    hipLaunchKernelGGL(k_interp_grad, dim3(grad_blocks(c, n)), dim3(kGradBlock), 0, s, c.d_grid, c.w,
                       (float)c.opts.kappa_tau, n, x, y, z, u, v, w, p, U, G, P, GP, c.grad_queue, c.err, c.stats);
    hipLaunchKernelGGL(k_interp_grad_fp64, dim3(round_up8(c.cu_count)), dim3(kGradBlock), 0, s, c.d_grid, c.w, n, x,
                       y, z, u, v, w, p, U, G, P, GP, c.grad_queue, c.err);
    return hipGetLastError();
}

}  // namespace mls
