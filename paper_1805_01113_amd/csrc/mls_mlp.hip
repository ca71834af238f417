// Learned shape-function surrogate (an addition to the paper's method).
//
// A 6 -> 128 -> 128 -> 27 GELU network maps the features of one (marker,
// component) support -- the in-cell offsets xi_d = (X - X_0)/H_d and the
// spacing ratios rho_d = (X_{+1} - X_0)/(X_0 - X_{-1}), which fix the exact
// MLS shape function of eq. 3-6 -- to its 27 shape-function values.
//
// Arithmetic: every matrix product runs on the matrix cores as "split BF16":
// an FP32 operand v is held as hi = bf16(v) and lo = bf16(v - hi), and
// hi*hi + hi*lo + lo*hi is accumulated in FP32 (the dropped lo*lo term and
// the rounding of lo leave a relative error near 2^-17 per product).
//
// Training: a general matrix-product kernel (optionally split along k, with
// the chunks summed in a fixed order), elementwise GELU / loss kernels and
// Adam; every reduction has a fixed order, so a training run is reproducible.
// Bias gradients come out of the weight-gradient products by appending a row
// of ones to the activations (b follows W in the parameter vector).
//
// Inference (mls_build with MLS_LEARNED): one wavefront per (64-marker block,
// component) computes the features, evaluates the network for 32 markers at a
// time with the three layers chained through registers, and checks the
// result against the consistency conditions of MLS with a linear basis:
//   r0 = |sum_k phi_k - 1|,  r1 = max_d |sum_k phi_k s_dk|
// (partition of unity, reproduction of linear fields; s_dk the offset of node
// k from the marker along d in units of H_d).  A marker whose residual is not
// below the tolerance is rebuilt with exact MLS on the same wavefront.
#include <cmath>
#include <cstring>

#include "mls_exact.h"

namespace mls {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBlock = 256;
constexpr int kLearnBlock = 512;        // 8 wavefronts share one copy of the network in LDS
constexpr int kSplitChunk = 2048;       // k-chunk of the weight-gradient products

// ---- activation ------------------------------------------------------------
// The standard normal tail Q(x) = 1 - Phi(x) = erfc(x / sqrt 2) / 2 for x >= 0
// from the rational approximation of Abramowitz & Stegun, Handbook of
// Mathematical Functions, formula 7.1.26 (|error of erf| <= 1.5e-7):
//   erfc(y) ~ t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-y^2),  t = 1 / (1 + p y).
// ez receives exp(-x^2 / 2).
__device__ __forceinline__ float normal_tail(float x, float &ez)
{
    const float yv = x * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, yv, 1.0f));
    const float poly =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
    ez = __builtin_amdgcn_exp2f(x * x * -0.72134752044448170f);   // exp(-x^2/2) = 2^(-x^2 log2(e) / 2)
    return 0.5f * poly * ez;
}

// gelu(z) = z Phi(z)
__device__ __forceinline__ float gelu(float z)
{
    float ez;
    const float q = normal_tail(fabsf(z), ez);
    return z * (z >= 0.0f ? 1.0f - q : q);
}

// gelu'(z) = Phi(z) + z phi(z), phi(z) = exp(-z^2/2) / sqrt(2 pi)
__device__ __forceinline__ float gelu_grad(float z)
{
    float ez;
    const float q = normal_tail(fabsf(z), ez);
    return (z >= 0.0f ? 1.0f - q : q) + z * ez * 0.39894228040143268f;
}

// gelu(z) = max(z, 0) - |z| Q(|z|) from the cubic table of the network image
// (inference only; training keeps the closed form above).  Beyond |z| = 6 the
// last interval's end value, 6 Q(6) < 6e-9, stands in for |z| Q(|z|).
// max(z, 0) is taken as z - min(z, 0), which passes a NaN argument on to the
// result (min returns its other operand for a NaN).
__device__ __forceinline__ float gelu_tab(float z, const float4 *__restrict__ tab)
{
    const float t = fminf(fabsf(z) * (float)kGeluPerUnit, 95.99999f);
    const float4 c = tab[(int)t];
    const float sv = __builtin_amdgcn_fractf(t);
    const float p = fmaf(fmaf(fmaf(c.w, sv, c.z), sv, c.y), sv, c.x);
    return (z - fminf(z, 0.0f)) - p;
}

__device__ __forceinline__ void split_bf16(float v, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

__device__ __forceinline__ f32x16 mfma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, f32x16 c)
{
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c, 0, 0, 0);
    return c;
}

// ---- general matrix product (training) --------------------------------------
// C(m, n) = sum_{k in chunk} A(m, k) B(k, n) with strided FP32 operands
// A(m, k) = A[m sam + k sak] for m < Ma and A(Ma, k) = 1 if ones_row (so M =
// Ma + ones_row), B(k, n) = B[k sbk + n sbn]; chunk blockIdx.y covers
// k in [y kc, min(K, (y + 1) kc)) and writes C + y cchunk, C(m, n) at
// C[m scm + n scn].  One wavefront per 32 x 32 tile of C on
// v_mfma_f32_32x32x16_bf16: operand lane l holds row (A) / column (B) l % 32
// and k = k0 + 8 (l / 32) + i, i < 8; result register j of lane l is row
// 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32.
__global__ void __launch_bounds__(kBlock)
k_gemm(int Ma, int ones_row, int N, int K, int kc, const float *__restrict__ A, int64_t sam, int64_t sak,
       const float *__restrict__ B, int64_t sbk, int64_t sbn, float *__restrict__ C, int64_t scm, int64_t scn,
       int64_t cchunk)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 31, h = lane >> 5;
    const int M = Ma + ones_row;
    const int tiles_n = (N + 31) / 32;
    const int tiles = ((M + 31) / 32) * tiles_n;
    const int wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (wave >= tiles) return;
    const int tm = wave / tiles_n, tn = wave % tiles_n;
    const int m = tm * 32 + r, n = tn * 32 + r;
    const int kbeg = blockIdx.y * kc;
    const int kend = min(K, kbeg + kc);
    f32x16 acc = {};
    for (int k0 = kbeg; k0 < kend; k0 += 16) {
        bf16x8 ahi, alo, bhi, blo;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + 8 * h + i;
            const bool kin = k < kend;
            float av = 0.0f;
            if (kin && m < Ma) av = A[(int64_t)m * sam + (int64_t)k * sak];
            else if (kin && m == Ma && ones_row) av = 1.0f;
            const float bv = (kin && n < N) ? B[(int64_t)k * sbk + (int64_t)n * sbn] : 0.0f;
            __bf16 p, q;
            split_bf16(av, p, q);
            ahi[i] = p; alo[i] = q;
            split_bf16(bv, p, q);
            bhi[i] = p; blo[i] = q;
        }
        acc = mfma3(ahi, alo, bhi, blo, acc);
    }
    float *Cc = C + (int64_t)blockIdx.y * cchunk;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = tm * 32 + 8 * (j / 4) + 4 * h + (j % 4);
        if (row < M && n < N) Cc[(int64_t)row * scm + (int64_t)n * scn] = acc[j];
    }
}

// out[i] = sum_{c < chunks} part[c * count + i], chunks in order
__global__ void k_sum_chunks(int64_t count, int chunks, const float *__restrict__ part, float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * count + i];
        out[i] = s;
    }
}

// Row of batch entry b: idx[b] if idx is given, else b.  An index outside
// [0, rows) raises MLS_E_ARG on the device and reads row 0 instead.
__device__ __forceinline__ int64_t batch_row(const int64_t *idx, int64_t b, int64_t rows, ErrWord *err)
{
    if (!idx) return b;
    const int64_t r = idx[b];
    if (r < 0 || r >= rows) {
        raise_error(err, b, MLS_E_ARG);
        return 0;
    }
    return r;
}

// U[m] = (feat[row(m)] - shift) * scale
__global__ void k_normalize(int64_t M, const float *__restrict__ feat, int64_t rows, const int64_t *__restrict__ idx,
                            const float *__restrict__ norm, float *__restrict__ U, ErrWord *err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M * 6; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i / 6;
        const int f = (int)(i - m * 6);
        const int64_t row = batch_row(idx, m, rows, err);
        U[i] = (feat[row * 6 + f] - norm[f]) * norm[6 + f];
    }
}

// Z[m][n] += bias[n]; H = gelu(Z) unless H is null
__global__ void k_bias_act(int64_t M, int N, float *__restrict__ Z, float *__restrict__ H,
                           const float *__restrict__ bias)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M * N; i += (int64_t)gridDim.x * blockDim.x) {
        const float zv = Z[i] + bias[i % N];
        Z[i] = zv;
        if (H) H[i] = gelu(zv);
    }
}

// D = D * gelu'(Z) (in place)
__global__ void k_gelu_bwd(int64_t count, float *__restrict__ D, const float *__restrict__ Z)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        D[i] *= gelu_grad(Z[i]);
}

// Offsets of the three support nodes from the marker along each axis in
// units of H, from the features: nodes at -2/(1+rho), 0, 2 rho/(1+rho)
// relative to the home node, the marker at xi.
__device__ __forceinline__ void node_offsets(const float *f, float s[3][3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float xi = f[d], rho = f[3 + d];
        const float inv = 1.0f / (1.0f + rho);
        s[d][0] = -2.0f * inv - xi;
        s[d][1] = -xi;
        s[d][2] = 2.0f * rho * inv - xi;
    }
}

// Loss L = mean_{b,k} (y - t)^2 + mu mean_b [(sum_k y - 1)^2 + sum_d (sum_k y s_dk)^2]
// and dL/dY; one thread per sample, per-block partial sums of L.
__global__ void __launch_bounds__(kBlock)
k_loss_grad(int64_t M, const float *__restrict__ Y, const float *__restrict__ T, const float *__restrict__ feat,
            int64_t rows, const int64_t *__restrict__ idx, float mu, float *__restrict__ dY, float *__restrict__ partial,
            ErrWord *err)
{
    __shared__ float red[kBlock / 64];
    float acc = 0.0f;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < M) {
        const int64_t row = batch_row(idx, b, rows, err);
        float s[3][3];
        node_offsets(feat + row * 6, s);
        const float *y = Y + b * kNe;
        const float *t = T + row * kNe;
        float sy = 0.0f, r1[3] = {0.0f, 0.0f, 0.0f}, se = 0.0f;
        for (int k = 0; k < kNe; ++k) {
            const float e = y[k] - t[k];
            se += e * e;
            sy += y[k];
            r1[0] += y[k] * s[0][k % 3];
            r1[1] += y[k] * s[1][(k / 3) % 3];
            r1[2] += y[k] * s[2][k / 9];
        }
        const float r0 = sy - 1.0f;
        const float inv_m = 1.0f / (float)M;
        acc = se * inv_m * (1.0f / kNe) + mu * inv_m * (r0 * r0 + r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
        const float ce = 2.0f * inv_m * (1.0f / kNe), cr = 2.0f * mu * inv_m;
        for (int k = 0; k < kNe; ++k)
            dY[b * kNe + k] = ce * (y[k] - t[k]) +
                              cr * (r0 + r1[0] * s[0][k % 3] + r1[1] * s[1][(k / 3) % 3] + r1[2] * s[2][k / 9]);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_sum_partials(int nb, const float *__restrict__ partial, float *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < nb; ++i) s += partial[i];
        *out = s;
    }
}

// Adam (Kingma & Ba, 2015) on the flat FP32 parameter vector; c1, c2 are the
// bias corrections 1 - beta^t.
__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float a = b1 * m1[i] + (1.0f - b1) * gi;
        const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = b;
        p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
    }
}

// Features of every (component, marker): feat[(c n + l) 6 + q] = xi_x, xi_y,
// xi_z, rho_x, rho_y, rho_z of component c's support; NaN (and a device
// error) if the support leaves the grid.
__global__ void __launch_bounds__(kBlock)
k_features(const Grid *__restrict__ gp, int64_t n, const float *__restrict__ x, const float *__restrict__ y,
           const float *__restrict__ z, float *__restrict__ feat, ErrWord *err)
{
    const Grid &g = *gp;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / n);
        const int64_t l = i - (int64_t)c * n;
        const double px = (double)x[l], py = (double)y[l], pz = (double)z[l];
        AxisGeo G[3];
        bool ok = axis_geo(g.ax[0], c == 0, px, G[0]);
        ok = ok && axis_geo(g.ax[1], c == 1, py, G[1]);
        ok = ok && axis_geo(g.ax[2], c == 2, pz, G[2]);
        float *f = feat + i * 6;
        if (!ok) {
            raise_error(err, l, isfinite(px) && isfinite(py) && isfinite(pz) ? MLS_E_SUPPORT : MLS_E_NONFINITE);
            for (int q = 0; q < 6; ++q) f[q] = __builtin_nanf("");
            continue;
        }
        f[0] = G[0].xi; f[1] = G[1].xi; f[2] = G[2].xi;
        f[3] = G[0].rho; f[4] = G[1].rho; f[5] = G[2].rho;
    }
}

// ---- inference image ---------------------------------------------------------
// Slot s of the image is (layer, output tile T, k block kb): layer 1 slots
// 0..3 (T), layer 2 slots 4 + 8 T + kb, layer 3 slots 36 + kb.  For lane l the
// A operand holds output row o = 32 T + l % 32 and, in its eight k slots, the
// inputs
//   layer 1:     8 (l / 32) + i                        (features, 6 used)
//   layers 2, 3: 32 (kb / 2) + 16 (kb % 2) + 8 (i / 4) + 4 (l / 32) + i % 4,
// the order in which the previous layer's result registers hold the hidden
// units (register j of tile T is unit 32 T + 8 (j / 4) + 4 (l / 32) + j % 4),
// so those registers serve directly as the next B operand.
__device__ __forceinline__ int layer_input(int layer, int kb, int h, int i)
{
    if (layer == 1) return 8 * h + i;
    return 32 * (kb / 2) + 16 * (kb % 2) + 8 * (i / 4) + 4 * h + (i % 4);
}

__global__ void k_pack(const float *__restrict__ P, const float *__restrict__ norm, uint4 *__restrict__ ops,
                       float *__restrict__ tail)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < kMlpImageOps) {
        const int lane = tid & 63, part = (tid >> 6) & 1, slot = tid >> 7;
        int layer, T, kb;
        if (slot < 4) { layer = 1; T = slot; kb = 0; }
        else if (slot < 36) { layer = 2; T = (slot - 4) / 8; kb = (slot - 4) % 8; }
        else { layer = 3; T = 0; kb = slot - 36; }
        const int o = 32 * T + (lane & 31), h = lane >> 5;
        uint32_t v16[8];
        for (int i = 0; i < 8; ++i) {
            const int in = layer_input(layer, kb, h, i);
            float v = 0.0f;
            if (layer == 1) v = in < kMlpIn ? P[kOffW1 + in * kMlpHidden + o] : 0.0f;
            else if (layer == 2) v = P[kOffW2 + in * kMlpHidden + o];
            else v = o < kMlpOut ? P[kOffW3 + in * kMlpOut + o] : 0.0f;
            __bf16 hi, lo;
            split_bf16(v, hi, lo);
            const __bf16 sel = part ? lo : hi;
            v16[i] = (uint32_t)__builtin_bit_cast(uint16_t, sel);
        }
        ops[tid] = make_uint4(v16[0] | v16[1] << 16, v16[2] | v16[3] << 16, v16[4] | v16[5] << 16,
                              v16[6] | v16[7] << 16);
    }
    if (tid < kMlpImageFloats) {
        float v;
        if (tid < kMlpHidden) v = P[kOffB1 + tid];
        else if (tid < 2 * kMlpHidden) v = P[kOffB2 + tid - kMlpHidden];
        else if (tid < 2 * kMlpHidden + 32)
            v = (tid - 2 * kMlpHidden) < kMlpOut ? P[kOffB3 + tid - 2 * kMlpHidden] : 0.0f;
        else v = norm[tid - 2 * kMlpHidden - 32];
        tail[tid] = v;
    }
}

// ---- fused learned build -----------------------------------------------------

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ bf16x8 op_at(const uint4 *img, int slot, int part, int lane)
{
    return __builtin_bit_cast(bf16x8, img[(slot * 2 + part) * 64 + lane]);
}

// Accumulator initialised with the bias of output tile T in result layout.
__device__ __forceinline__ f32x16 bias_tile(const float *b, int T, int h)
{
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = *reinterpret_cast<const float4 *>(b + 32 * T + 8 * q + 4 * h);
        acc[4 * q + 0] = v.x; acc[4 * q + 1] = v.y; acc[4 * q + 2] = v.z; acc[4 * q + 3] = v.w;
    }
    return acc;
}

// GELU of result registers 8 q .. 8 q + 7 as the split B operand of the next layer.
__device__ __forceinline__ void gelu_operand(const f32x16 &acc, int q, const float4 *tab, bf16x8 &hi, bf16x8 &lo)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        __bf16 p, r;
        split_bf16(gelu_tab(acc[8 * q + i], tab), p, r);
        hi[i] = p; lo[i] = r;
    }
}

// Network output for the 32 markers whose features lane l % 32 holds (ft);
// returns the 32 x 32 result tile (rows 0..26 are the outputs).
__device__ __forceinline__ f32x16 evaluate(const uint4 *img, const float *b1, const float *b2, const float *b3,
                                           const float *norm, const float4 *tab, const float ft[6], int lane)
{
    const int h = lane >> 5;
    bf16x8 uh, ul;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        float v = 0.0f;
        if (i < kMlpIn) v = (ft[i] - norm[i]) * norm[6 + i];
        v = h ? 0.0f : v;
        __bf16 p, r;
        split_bf16(v, p, r);
        uh[i] = p; ul[i] = r;
    }
    // Layer 2 is accumulated k block by k block: each 32-unit tile of layer 1
    // is computed, activated and consumed by the four layer-2 output tiles
    // at once, so only its own 16-register operand pair is live instead of
    // all of layer 1, and the four accumulators give the matrix cores four
    // independent chains.  Each accumulator still sums its k blocks in
    // order 0..7, so the result is the same as tile by tile.
    f32x16 acc[4];
#pragma unroll
    for (int T = 0; T < 4; ++T) acc[T] = bias_tile(b2, T, h);
#pragma unroll
    for (int T1 = 0; T1 < 4; ++T1) {
        f32x16 a = bias_tile(b1, T1, h);
        a = mfma3(op_at(img, T1, 0, lane), op_at(img, T1, 1, lane), uh, ul, a);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int kb = 2 * T1 + q;
            bf16x8 bh, bl;
            gelu_operand(a, q, tab, bh, bl);
#pragma unroll
            for (int T = 0; T < 4; ++T)
                acc[T] = mfma3(op_at(img, 4 + 8 * T + kb, 0, lane), op_at(img, 4 + 8 * T + kb, 1, lane), bh, bl,
                               acc[T]);
        }
    }
    f32x16 y3 = bias_tile(b3, 0, h);
#pragma unroll
    for (int T = 0; T < 4; ++T) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            bf16x8 ch, cl;
            gelu_operand(acc[T], q, tab, ch, cl);
            const int slot = 36 + 2 * T + q;
            y3 = mfma3(op_at(img, slot, 0, lane), op_at(img, slot, 1, lane), ch, cl, y3);
        }
    }
    return y3;
}

// Rows of one wavefront staged in LDS for the fused interpolation (after the
// network image): 27 values of 64 rows, node-major like the stored rows.
constexpr size_t kLearnStageBytes = (size_t)(kLearnBlock / 64) * kNe * 64 * sizeof(float);

__global__ void __launch_bounds__(kLearnBlock)
k_build_learned(const Grid *__restrict__ gp, const Weight W, float tau, float tol, int64_t n,
                const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z,
                const uint4 *__restrict__ image, uint32_t *__restrict__ home, float *__restrict__ phi,
                uint8_t *__restrict__ route, ErrWord *err, DevStats *st, const uint32_t *__restrict__ order,
                const LearnedInterp li)
{
    extern __shared__ uint4 lds[];
    // the GELU table in a static LDS array (placed first, so its rows are
    // addressed with small immediate offsets)
    __shared__ float4 tab[kGeluIntervals];
    constexpr int kWords = (int)(kMlpImageBytes / 16);
    for (int i = threadIdx.x; i < kWords; i += kLearnBlock) lds[i] = image[i];
    if (threadIdx.x < kGeluIntervals)
        tab[threadIdx.x] = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(image) +
                                                            kMlpImageTableOffset)[threadIdx.x];
    __syncthreads();
    const float *b1 = reinterpret_cast<const float *>(lds + kMlpImageOps);
    const float *b2 = b1 + kMlpHidden, *b3 = b2 + kMlpHidden, *norm = b3 + 32;

    const Grid &g = *gp;
    const int lane = threadIdx.x & 63, h = lane >> 5, r = lane & 31;
    float *const stage = reinterpret_cast<float *>(reinterpret_cast<char *>(lds) + kMlpImageBytes) +
                         wave_id() * (kNe * 64);
    const int64_t items = ((n + 63) >> 6) * 3;
    const int64_t wstride = (int64_t)gridDim.x * (kLearnBlock / 64);
    unsigned long long routed = 0, n_fb = 0, n_ok = 0;
    float kmax = 0.0f;
    for (int64_t it = (int64_t)blockIdx.x * (kLearnBlock / 64) + wave_id(); it < items; it += wstride) {
        const int64_t blk = it / 3;
        const int c = (int)(it - blk * 3);
        const int64_t l = (blk << 6) + lane;
        // the marker of row l (rows in tile order in the time step)
        const int64_t mk = l < n ? (order ? (int64_t)order[l] : l) : 0;
        float *out = phi + (((blk * 3 + c) * kNe) << 6);          // + k * 64 + marker in block
        uint32_t *hout = home + ((blk * 3 + c) << 6) + lane;
        uint8_t *rout = route ? route + ((blk * 3 + c) << 6) : nullptr;
        float f[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        bool ok = false;
        uint32_t hv = 0xffffffffu;
        if (l < n) {
            const double px = (double)x[mk], py = (double)y[mk], pz = (double)z[mk];
            AxisGeo G[3];
            ok = axis_geo(g.ax[0], c == 0, px, G[0]);
            ok = ok && axis_geo(g.ax[1], c == 1, py, G[1]);
            ok = ok && axis_geo(g.ax[2], c == 2, pz, G[2]);
            if (!ok) {
                mark_failed(err, mk, px, py, pz, hout, out + lane, rout ? rout + lane : nullptr);
            } else {
                hv = pack_home(G[0].ih, G[1].ih, G[2].ih);
                *hout = hv;
                f[0] = G[0].xi; f[1] = G[1].xi; f[2] = G[2].xi;
                f[3] = G[0].rho; f[4] = G[1].rho; f[5] = G[2].rho;
            }
        }
        const unsigned long long good = __ballot(ok);
        unsigned long long accept = 0;
#pragma unroll 1
        for (int t = 0; t < 2; ++t) {
            const uint32_t gt = (uint32_t)(good >> (32 * t));
            if (gt == 0) continue;
            const int src = 32 * t + r;
            float ft[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) ft[q] = __shfl(f[q], src);
            const f32x16 yv = evaluate(lds, b1, b2, b3, norm, tab, ft, lane);
            // consistency residuals; a marker's outputs are split between lanes r and r + 32
            float s[3][3];
            node_offsets(ft, s);
            float sy = 0.0f, r1x = 0.0f, r1y = 0.0f, r1z = 0.0f;
            // the offsets of a row are picked by a bit mask on h, so that the
            // array stays in registers (a select of two elements would become
            // a select of two addresses and put the array in scratch)
            const uint32_t hm = h ? 0xffffffffu : 0u;
            auto pick = [hm](float a0, float a1) {
                return __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, a1) & hm) |
                                                     (__builtin_bit_cast(uint32_t, a0) & ~hm));
            };
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int k0 = 8 * (j / 4) + (j % 4), k1 = k0 + 4;   // output row for h = 0, 1
                const int kk1 = k1 < kNe ? k1 : 0;
                const bool valid = h ? (k1 < kNe) : true;
                const float sx = pick(s[0][k0 % 3], s[0][kk1 % 3]);
                const float sv = pick(s[1][(k0 / 3) % 3], s[1][(kk1 / 3) % 3]);
                const float sz = pick(s[2][k0 / 9], s[2][kk1 / 9]);
                const float yj = valid ? yv[j] : 0.0f;
                sy += yj;
                r1x += yj * sx;
                r1y += yj * sv;
                r1z += yj * sz;
            }
            sy += __shfl_xor(sy, 32);
            r1x += __shfl_xor(r1x, 32);
            r1y += __shfl_xor(r1y, 32);
            r1z += __shfl_xor(r1z, 32);
            const float res = fmaxf(fmaxf(fabsf(sy - 1.0f), fabsf(r1x)), fmaxf(fabsf(r1y), fabsf(r1z)));
            const bool pass = ((gt >> r) & 1u) && res < tol;   // NaN fails
            if (pass) {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int k = 8 * (j / 4) + 4 * h + (j % 4);
                    if (k < kNe) {
                        out[k * kLanes + 32 * t + r] = yv[j];
                        if (li.U) stage[k * 64 + 32 * t + r] = yv[j];
                    }
                }
                if (rout && h == 0) rout[32 * t + r] = 2;
            }
            const unsigned long long pb = __ballot(pass);
            accept |= (pb & 0xffffffffull) << (32 * t);
        }
        const unsigned long long rej = good & ~accept;
        n_ok += (unsigned long long)__popcll(accept);
        n_fb += (unsigned long long)__popcll(rej);
        if ((rej >> lane) & 1ull) {
            const double px = (double)x[mk], py = (double)y[mk], pz = (double)z[mk];
            AxisGeo G[3];
            axis_geo(g.ax[0], c == 0, px, G[0]);
            axis_geo(g.ax[1], c == 1, py, G[1]);
            axis_geo(g.ax[2], c == 2, pz, G[2]);
            float ph[kNe];
            exact_from_geo(g, W, tau, c, mk, px, py, pz, G, out + lane, rout ? rout + lane : nullptr, 4, err, routed,
                           kmax, ph);
            if (li.U) {
#pragma unroll
                for (int k = 0; k < kNe; ++k) stage[k * 64 + lane] = ph[k];
            }
        }
        if (li.U) {
            // Interpolation (eq. 6), direct forcing and c_l F_l (eq. 8) of the
            // rows just built, from the wavefront's LDS copy of them: the same
            // arithmetic as interpolating the stored rows, without reading
            // them back from memory.  U and F go out by marker, c_l F_l by row,
            // and the largest |c_l F_l| per spreading tile into tmax.
            __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wavefront's LDS writes are done
            __builtin_amdgcn_wave_barrier();
            asm volatile("" ::: "memory");
            const bool in = l < n;
            float acc = __builtin_nanf(""), fo = __builtin_nanf(""), cfv = 0.0f;
            if (ok) {
                int i, j, k;
                unpack_home(hv, i, j, k);
                const float *q = c == 0 ? li.u : (c == 1 ? li.v : li.w);
                uint32_t oy[3], oz[3];
                support_rows(true, j, k, g.dims[c][0], g.dims[c][1], g.dims[c][2], g.ax[1].periodic,
                             g.ax[2].periodic, oy, oz);
                Support sp;
                load_support(q, i, g.dims[c][0], oy, oz, sp);
                float ph[kNe];
#pragma unroll
                for (int kk = 0; kk < kNe; ++kk) ph[kk] = stage[kk * 64 + lane];
                acc = 0.0f;
#pragma unroll
                for (int kk = 0; kk < kNe; ++kk) acc += ph[kk] * sp.at(kk);
                const float vbv = li.vb ? li.vb[c * n + mk] : 0.0f;
                fo = (vbv - acc) * li.inv_dt;
                cfv = eq8_coef_built(g, c, i, j, k, ph, li.area[mk] * fo);
                if (!(fabsf(cfv) <= 3.0e38f)) raise_error(err, mk, MLS_E_RANGE);
            }
            if (in) {
                li.U[c * n + mk] = acc;
                li.F[c * n + mk] = fo;
                li.cf[c * li.cf_stride + l] = ok ? cfv : 0.0f;
            }
            const uint32_t tl = in ? li.tile_of_marker[mk] : (uint32_t)g.ntiles;
            wave_key_max(li.tmax + c * li.tstride, ok && tl < (uint32_t)g.ntiles ? (int64_t)tl : -1,
                         finite_abs(cfv));
            // the next item's stage writes come after every lane's reads
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
            asm volatile("" ::: "memory");
        }
    }
    unsigned long long tot = routed;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    float km = kmax;
    for (int off = 32; off > 0; off >>= 1) km = fmaxf(km, __shfl_xor(km, off));
    if (lane == 0) {
        if (tot) atomicAdd(&st->fp64_solves, tot);
        if (n_fb) atomicAdd(&st->fallbacks, n_fb);
        if (n_ok) atomicAdd(&st->learned, n_ok);
        if (km > 0.0f) atomicMax(&st->kappa_max_bits, __float_as_uint(km));
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

// ---- host side ---------------------------------------------------------------

// The inference GELU table: f(a) = a Q(a), Q(a) = erfc(a / sqrt 2) / 2, on
// intervals of width 1/16 as cubic Hermite pieces in s = 16 a - i (value and
// derivative f'(a) = Q(a) - a phi(a) matched at both ends), in FP64.
static void gelu_table(float *t)
{
    auto f = [](double a) { return 0.5 * a * std::erfc(a * 0.70710678118654752440); };
    auto df = [](double a) {
        return 0.5 * std::erfc(a * 0.70710678118654752440) - a * std::exp(-0.5 * a * a) * 0.39894228040143267794;
    };
    const double h = 1.0 / kGeluPerUnit;
    for (int i = 0; i < kGeluIntervals; ++i) {
        const double a0 = i * h, a1 = (i + 1) * h;
        const double f0 = f(a0), f1 = f(a1), d0 = df(a0) * h, d1 = df(a1) * h;
        t[4 * i + 0] = (float)f0;
        t[4 * i + 1] = (float)d0;
        t[4 * i + 2] = (float)(3.0 * (f1 - f0) - 2.0 * d0 - d1);
        t[4 * i + 3] = (float)(2.0 * (f0 - f1) + d0 + d1);
    }
}

hipError_t mlp_alloc(Ctx &c)
{
    Mlp &net = c.mlp;
    if (net.params) return hipSuccess;
    const size_t floats = 4 * (size_t)kMlpParams + 12 + 4;
    const size_t head = (floats * sizeof(float) + 255) & ~(size_t)255;
    char *block = nullptr;
    hipError_t e = hipMalloc((void **)&block, head + kMlpImageBytes);
    if (e != hipSuccess) return e;
    float *fp = reinterpret_cast<float *>(block);
    net.params = fp;
    net.grad = fp + kMlpParams;
    net.m1 = fp + 2 * kMlpParams;
    net.m2 = fp + 3 * kMlpParams;
    net.norm = fp + 4 * kMlpParams;
    net.loss = net.norm + 12;
    net.image = block + head;
    float tab[4 * kGeluIntervals];
    gelu_table(tab);
    e = hipMemcpy(static_cast<char *>(net.image) + kMlpImageTableOffset, tab, sizeof(tab), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(block);
        net.params = nullptr;
        return e;
    }
    return hipFuncSetAttribute((const void *)k_build_learned, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kMlpImageBytes + kLearnStageBytes));
}

void mlp_free(Ctx &c)
{
    Mlp &net = c.mlp;
    if (net.params) hipFree(net.params);
    if (net.scratch) hipFree(net.scratch);
    net = Mlp{};
}

hipError_t mlp_pack(Ctx &c, hipStream_t s)
{
    Mlp &net = c.mlp;
    uint4 *ops = static_cast<uint4 *>(net.image);
    float *tail = reinterpret_cast<float *>(ops + kMlpImageOps);
    hipLaunchKernelGGL(k_pack, dim3((kMlpImageOps + kBlock - 1) / kBlock), dim3(kBlock), 0, s, net.params, net.norm,
                       ops, tail);
    net.image_version = net.version;
    return hipGetLastError();
}

LearnedInterp learned_interp(const Ctx &c, const float *u, const float *v, const float *w, const float *vb,
                             const float *area, float dt, float *U, float *F)
{
    LearnedInterp li;
    li.u = u; li.v = v; li.w = w; li.vb = vb; li.area = area;
    li.inv_dt = 1.0f / dt;
    li.U = U; li.F = F;
    li.cf = c.cf_rows; li.cf_stride = c.cf_stride;
    li.tile_of_marker = c.marker_tile;
    li.tmax = c.tile_fmax; li.tstride = c.g.ntiles + 1;
    return li;
}

hipError_t launch_build_learned(Ctx &c, int64_t n, const float *x, const float *y, const float *z, uint32_t *home,
                                float *phi, uint8_t *route, hipStream_t s, const uint32_t *order,
                                const LearnedInterp *interp)
{
    if (n == 0) return hipSuccess;
    Mlp &net = c.mlp;
    if (net.image_version != net.version) {
        hipError_t e = mlp_pack(c, s);
        if (e != hipSuccess) return e;
    }
    const float tau = (float)(c.opts.kappa_tau > 3.0e38 ? 3.0e38 : c.opts.kappa_tau);
    const float tol = (float)(c.opts.fallback_tol > 3.0e38 ? 3.0e38 : c.opts.fallback_tol);
    const int64_t waves = ((n + 63) / 64) * 3;
    int64_t blocks = (waves + kLearnBlock / 64 - 1) / (kLearnBlock / 64);
    if (blocks > c.cu_count) blocks = c.cu_count;
    const LearnedInterp li = interp ? *interp : LearnedInterp{};
    hipLaunchKernelGGL(k_build_learned, dim3((unsigned)blocks), dim3(kLearnBlock),
                       kMlpImageBytes + (li.U ? kLearnStageBytes : 0), s, c.d_grid, c.w, tau, tol, n, x, y, z,
                       static_cast<const uint4 *>(net.image), home, phi, route, c.err, c.stats, order, li);
    return hipGetLastError();
}

hipError_t launch_features(const Ctx &c, int64_t n, const float *x, const float *y, const float *z, float *feat,
                           hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(grid_for(3 * n, c.cu_count)), dim3(kBlock), 0, s, c.d_grid, n, x, y, z,
                       feat, c.err);
    return hipGetLastError();
}

// Scratch layout for batches of up to cap samples: split-product chunks,
// then U (6 M), Z1, H1, Z2, H2 (128 M each), Y (27 M), dY (27 M) and the
// loss partials.
static int64_t part_floats(int64_t cap)
{
    const int64_t chunks = (cap + kSplitChunk - 1) / kSplitChunk;
    return chunks * (kMlpHidden + 1) * kMlpHidden;
}

// Matrix product C = A B (+ ones row, see k_gemm).  A k range longer than
// one chunk is split when C has few tiles; the chunks go to the head of the
// training scratch and are summed in order into C, which is then row-major
// (scm = N, scn = 1).
static void gemm(Ctx &c, hipStream_t s, int Ma, int ones_row, int N, int K, const float *A, int64_t sam,
                 int64_t sak, const float *B, int64_t sbk, int64_t sbn, float *C, int64_t scm, int64_t scn)
{
    const int M = Ma + ones_row;
    const int tiles = ((M + 31) / 32) * ((N + 31) / 32);
    const int bx = (tiles + 3) / 4;
    const int chunks = (K + kSplitChunk - 1) / kSplitChunk;
    if (chunks <= 1 || tiles >= 256) {
        hipLaunchKernelGGL(k_gemm, dim3(bx, 1), dim3(kBlock), 0, s, Ma, ones_row, N, K, K > 0 ? K : 1, A, sam, sak, B,
                           sbk, sbn, C, scm, scn, (int64_t)0);
        return;
    }
    float *part = c.mlp.scratch;
    hipLaunchKernelGGL(k_gemm, dim3(bx, chunks), dim3(kBlock), 0, s, Ma, ones_row, N, K, kSplitChunk, A, sam, sak, B,
                       sbk, sbn, part, (int64_t)N, (int64_t)1, (int64_t)M * N);
    const int64_t count = (int64_t)M * N;
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, count,
                       chunks, part, C);
}

hipError_t mlp_reserve(Ctx &c, int64_t M)
{
    Mlp &net = c.mlp;
    if (M <= net.cap_batch) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    ++c.scratch_gen;
    if (net.scratch) hipFree(net.scratch);
    net.scratch = nullptr;
    net.cap_batch = 0;
    const int64_t per = 6 + 4 * kMlpHidden + 2 * kMlpOut;
    const int64_t floats = part_floats(M) + per * M + (M + kBlock - 1) / kBlock + 64;
    e = hipMalloc((void **)&net.scratch, (size_t)floats * sizeof(float));
    if (e != hipSuccess) return e;
    net.cap_batch = M;
    return hipSuccess;
}

struct Acts {
    float *U, *Z1, *H1, *Z2, *H2, *Y, *dY, *partial;
};

static Acts acts(Ctx &c, int64_t M)
{
    Acts a;
    a.U = c.mlp.scratch + part_floats(c.mlp.cap_batch);
    a.Z1 = a.U + 6 * M;
    a.H1 = a.Z1 + kMlpHidden * M;
    a.Z2 = a.H1 + kMlpHidden * M;
    a.H2 = a.Z2 + kMlpHidden * M;
    a.Y = a.H2 + kMlpHidden * M;
    a.dY = a.Y + kMlpOut * M;
    a.partial = a.dY + kMlpOut * M;
    return a;
}

hipError_t mlp_forward_batch(Ctx &c, int64_t M, const float *feat, int64_t rows, const int64_t *idx, float *Yout,
                             hipStream_t s)
{
    if (M == 0) return hipSuccess;
    Mlp &net = c.mlp;
    const int H = kMlpHidden;
    const Acts a = acts(c, M);
    float *Y = Yout ? Yout : a.Y;
    const float *P = net.params;
    const int g = grid_for(M * H, c.cu_count);
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(M * 6, c.cu_count)), dim3(kBlock), 0, s, M, feat, rows, idx,
                       net.norm, a.U, c.err);
    gemm(c, s, (int)M, 0, H, kMlpIn, a.U, kMlpIn, 1, P + kOffW1, H, 1, a.Z1, H, 1);
    hipLaunchKernelGGL(k_bias_act, dim3(g), dim3(kBlock), 0, s, M, H, a.Z1, a.H1, P + kOffB1);
    gemm(c, s, (int)M, 0, H, H, a.H1, H, 1, P + kOffW2, H, 1, a.Z2, H, 1);
    hipLaunchKernelGGL(k_bias_act, dim3(g), dim3(kBlock), 0, s, M, H, a.Z2, a.H2, P + kOffB2);
    gemm(c, s, (int)M, 0, kMlpOut, H, a.H2, H, 1, P + kOffW3, kMlpOut, 1, Y, kMlpOut, 1);
    hipLaunchKernelGGL(k_bias_act, dim3(grid_for(M * kMlpOut, c.cu_count)), dim3(kBlock), 0, s, M, kMlpOut, Y,
                       (float *)nullptr, P + kOffB3);
    return hipGetLastError();
}

hipError_t mlp_grad_batch(Ctx &c, int64_t M, const float *feat, const float *target, int64_t rows,
                          const int64_t *idx, float mu, float *grad, float *loss, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    Mlp &net = c.mlp;
    const int H = kMlpHidden;
    hipError_t e = mlp_forward_batch(c, M, feat, rows, idx, nullptr, s);
    if (e != hipSuccess) return e;
    const Acts a = acts(c, M);
    const float *P = net.params;
    const int nb = (int)((M + kBlock - 1) / kBlock);
    const int g = grid_for(M * H, c.cu_count);
    hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(kBlock), 0, s, M, a.Y, target, feat, rows, idx, mu, a.dY,
                       a.partial, c.err);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, nb, a.partial, loss);
    // layer 3: [dW3; db3] = [H2 1]^T dY; dZ2 = (dY W3^T) gelu'(Z2), written over H2
    gemm(c, s, H, 1, kMlpOut, (int)M, a.H2, 1, H, a.dY, kMlpOut, 1, grad + kOffW3, kMlpOut, 1);
    gemm(c, s, (int)M, 0, H, kMlpOut, a.dY, kMlpOut, 1, P + kOffW3, 1, kMlpOut, a.H2, H, 1);
    hipLaunchKernelGGL(k_gelu_bwd, dim3(g), dim3(kBlock), 0, s, M * H, a.H2, a.Z2);
    // layer 2: [dW2; db2] = [H1 1]^T dZ2; dZ1 = (dZ2 W2^T) gelu'(Z1), written over H1
    gemm(c, s, H, 1, H, (int)M, a.H1, 1, H, a.H2, H, 1, grad + kOffW2, H, 1);
    gemm(c, s, (int)M, 0, H, H, a.H2, H, 1, P + kOffW2, 1, H, a.H1, H, 1);
    hipLaunchKernelGGL(k_gelu_bwd, dim3(g), dim3(kBlock), 0, s, M * H, a.H1, a.Z1);
    // layer 1: [dW1; db1] = [U 1]^T dZ1
    gemm(c, s, kMlpIn, 1, H, (int)M, a.U, 1, kMlpIn, a.H1, H, 1, grad + kOffW1, H, 1);
    return hipGetLastError();
}

hipError_t mlp_adam(Ctx &c, float lr, hipStream_t s)
{
    Mlp &net = c.mlp;
    net.adam_step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, (double)net.adam_step));
    const float c2 = (float)(1.0 - std::pow(b2, (double)net.adam_step));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(kMlpParams, c.cu_count)), dim3(kBlock), 0, s, (int64_t)kMlpParams,
                       net.params, net.grad, net.m1, net.m2, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    net.version += 1;
    return hipGetLastError();
}

}  // namespace mls
