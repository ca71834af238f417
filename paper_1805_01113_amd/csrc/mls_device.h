// Device helpers: support selection on the staggered grid (Sec. 2), the
// weight function, the 4x4 moment-matrix solve and the device error word.
#pragma once

#include "mls_internal.h"

namespace mls {

// Geometry of the 3-node support along one axis for one staggering type.
struct AxisGeo {
    int32_t ih;      // wrapped home node index
    float s[3];      // (X_a - X)/H for a = -1, 0, +1
    float xi;        // (X - X_0)/H
    float rho;       // (X_{+1} - X_0)/(X_0 - X_{-1}): 1 on a uniform axis
};

__device__ __forceinline__ void raise_error(ErrWord *err, int64_t marker, int status)
{
    unsigned long long w = ((unsigned long long)marker << 8) | (unsigned long long)(-status & 0xff);
    atomicMin(&err->word, w);
}

// Unwrapped node coordinate.  i ranges over [-1, n+1] for periodic axes.
// Kept free of fused multiply-adds so that the coordinates are the plain
// IEEE results of their definitions.
#pragma clang fp contract(off)
// Face / centre coordinate of wrapped index i in [0, n] / [0, n-1].  On an
// axis whose stored coordinates equal f0 + i h (faces) and f0 + (i + 1/2) h
// (centres) bit for bit -- checked on the host -- they are recomputed here,
// which spares the locate step its dependent memory loads.
__device__ __forceinline__ double fval(const Axis &a, int i)
{
    return a.exact ? a.f0 + (double)i * a.h : a.faces[i];
}

__device__ __forceinline__ double cval(const Axis &a, int i)
{
    return a.exact ? a.f0 + ((double)i + 0.5) * a.h : a.centres[i];
}

__device__ __forceinline__ double face_x(const Axis &a, int i)
{
    double shift = 0.0;
    if (a.periodic) {
        if (i < 0) { i += a.n; shift = -1.0; }
        else if (i >= a.n) { i -= a.n; shift = 1.0; }
    }
    return fval(a, i) + shift * a.L;
}

__device__ __forceinline__ double centre_x(const Axis &a, int i)
{
    double shift = 0.0;
    if (a.periodic) {
        if (i < 0) { i += a.n; shift = -1.0; }
        else if (i >= a.n) { i -= a.n; shift = 1.0; }
    }
    return cval(a, i) + shift * a.L;
}

__device__ __forceinline__ double node_x(const Axis &a, int is_face, int i)
{
    return is_face ? face_x(a, i) : centre_x(a, i);
}

// Periodic wrap of x into [f0, f0 + L).  With f0 = 0 a coordinate already in
// [0, L) gives t = floor(x / L) = 0 exactly, so it is returned unchanged.
__device__ __forceinline__ double wrap_x(const Axis &a, double x)
{
    if (a.f0 == 0.0 && x >= 0.0 && x < a.L) return x;
    double t = floor((x - a.f0) / a.L);
    double X = x - t * a.L;
    if (X >= a.f0 + a.L) X -= a.L;
    if (X < a.f0) X += a.L;
    return X;
}

// The cell i with f[i] <= X < f[i+1] (i in [0, n-1], clamped at the ends),
// from a guess i on a uniform axis.  The FP64 guess is off by at most one
// cell unless the coordinates are close to the resolution of FP64, so one
// step is taken first and only a lane that moved walks on; the result is
// that of walking from the guess.
__device__ __forceinline__ int fix_cell(const Axis &a, double X, int i)
{
    const int n = a.n;
    const bool dn = i > 0 && X < fval(a, i);
    const bool up = !dn && i < n - 1 && X >= fval(a, i + 1);
    i += (int)up - (int)dn;
    if (dn || up) {
        while (i > 0 && X < fval(a, i)) --i;
        while (i < n - 1 && X >= fval(a, i + 1)) ++i;
    }
    return i;
}

// The face node i in [1, n-1] with c[i-1] <= X < c[i] (clamped at the
// ends), from a guess i on a uniform axis; as fix_cell.
__device__ __forceinline__ int fix_face(const Axis &a, double X, int i)
{
    const int n = a.n;
    const bool dn = i > 1 && X < cval(a, i - 1);
    const bool up = !dn && i < n - 1 && X >= cval(a, i);
    i += (int)up - (int)dn;
    if (dn || up) {
        while (i > 1 && X < cval(a, i - 1)) --i;
        while (i < n - 1 && X >= cval(a, i)) ++i;
    }
    return i;
}

// Eulerian cell along one axis that contains x: f[i] <= X < f[i+1], X wrapped
// into [f0, f0 + L) on a periodic axis.  false for a non-finite coordinate or
// one outside [f0, fn) on a wall axis.
__device__ __forceinline__ bool cell_axis(const Axis &a, double x, int &i)
{
    if (!isfinite(x)) return false;
    const int n = a.n;
    const double X = a.periodic ? wrap_x(a, x) : x;
    if (!(X >= fval(a, 0) && X < fval(a, n))) return false;
    if (a.uniform) {
        i = fix_cell(a, X, min(max((int)floor((X - a.f0) * a.inv_h), 0), n - 1));
    } else {
        int lo = 0, hi = n;   // faces[lo] <= X < faces[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.faces[mid] <= X) lo = mid; else hi = mid;
        }
        i = lo;
    }
    return true;
}

// Home node along one axis: the node whose control volume [lo, hi) contains
// the marker.  Returns false if the support leaves a wall axis or x is not
// finite.  On success ih_u is the unwrapped home index (a periodic face axis
// may return n, node 0 shifted by L) and X the wrapped coordinate.
__device__ __forceinline__ bool locate(const Axis &a, int is_face, double x, int &ih_u, double &X)
{
    if (!isfinite(x)) return false;
    const int n = a.n;
    if (a.periodic) {
        X = wrap_x(a, x);
    } else {
        X = x;
        if (!(X >= fval(a, 0) && X <= fval(a, n))) return false;
    }
    int i;
    if (!is_face) {
        if (X >= fval(a, n)) return false;
        if (a.uniform) {
            i = fix_cell(a, X, min(max((int)floor((X - a.f0) * a.inv_h), 0), n - 1));
        } else {
            int lo = 0, hi = n;   // faces[lo] <= X < faces[hi]
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (a.faces[mid] <= X) lo = mid; else hi = mid;
            }
            i = lo;
        }
    } else {
        if (X < cval(a, 0)) {
            i = 0;
        } else if (X >= cval(a, n - 1)) {
            i = n;
        } else if (a.uniform) {
            // centres[i-1] <= X < centres[i], i in [1, n-1]
            i = fix_face(a, X, min(max((int)floor((X - a.f0) * a.inv_h + 0.5), 1), n - 1));
        } else {
            int lo = 0, hi = n - 1;   // centres[lo] <= X < centres[hi]
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (a.centres[mid] <= X) lo = mid; else hi = mid;
            }
            i = hi;
        }
    }
    if (!a.periodic) {
        const int last = is_face ? n : n - 1;
        if (i - 1 < 0 || i + 1 > last) return false;
    }
    ih_u = i;
    return true;
}

// Support geometry along one axis (FP64 offsets, rounded to FP32 after the
// subtraction so that stretched axes keep their digits).
// rH_out receives 1/H (physical units).
__device__ __forceinline__ bool axis_geo(const Axis &a, int is_face, double x, AxisGeo &g, double &rH_out)
{
    int ih;
    double X;
    if (!locate(a, is_face, x, ih, X)) return false;
    const double x0 = node_x(a, is_face, ih);
    if (a.uniform) {
        // neighbours one spacing away; H = h
        // the outer offsets are formed in FP32 from the rounded centre offset,
        // so that the centre offset alone reproduces all three bit for bit
        // (the compact transfer function of a time step stores only it)
        const double d0 = (x0 - X) * a.inv_h;
        g.s[1] = (float)d0;
        g.s[0] = g.s[1] - 1.0f;
        g.s[2] = g.s[1] + 1.0f;
        g.xi = (float)(-d0);
        g.rho = 1.0f;
        rH_out = a.inv_h;
    } else {
        const double xm = node_x(a, is_face, ih - 1);
        const double xp = node_x(a, is_face, ih + 1);
        const double rH = 2.0 / (xp - xm);   // 1 / H, H = half the support width
        g.s[0] = (float)((xm - X) * rH);
        g.s[1] = (float)((x0 - X) * rH);
        g.s[2] = (float)((xp - X) * rH);
        g.xi = (float)((X - x0) * rH);
        g.rho = (float)((xp - x0) / (x0 - xm));
        rH_out = rH;
    }
    g.ih = (a.periodic && ih >= a.n) ? ih - a.n : ih;
    return true;
}

__device__ __forceinline__ bool axis_geo(const Axis &a, int is_face, double x, AxisGeo &g)
{
    double rH;
    return axis_geo(a, is_face, x, g, rH);
}

// FP64 offsets for the rare FP64 route (recomputed from the position).
__device__ __forceinline__ void axis_offsets_d(const Axis &a, int is_face, double x, double s[3], double &H)
{
    int ih;
    double X;
    locate(a, is_face, x, ih, X);
    double xm = node_x(a, is_face, ih - 1);
    double x0 = node_x(a, is_face, ih);
    double xp = node_x(a, is_face, ih + 1);
    H = 0.5 * (xp - xm);
    s[0] = (xm - X) / H;
    s[1] = (x0 - X) / H;
    s[2] = (xp - X) / H;
}

__device__ __forceinline__ void axis_offsets_d(const Axis &a, int is_face, double x, double s[3])
{
    double H;
    axis_offsets_d(a, is_face, x, s, H);
}
#pragma clang fp contract(on)

// ---- weight function ------------------------------------------------------

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator: value
// ctr is the output function applied to the state seed + (ctr + 1) * gamma
// (mod 2^64), gamma the golden-ratio increment below.
constexpr uint64_t kSplitMixGamma = 0x9E3779B97F4A7C15ull;

// The output function applied to a state z.
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

#pragma clang fp contract(off)
// Jittered position of marker l of n in step `step`: p = p0 + (u - 1/2) amp2
// per axis, u on the 2^-24 lattice of [0, 1) from counter (step n + l) 3 +
// axis; plain FP32 operations (no fused multiply-add), so every kernel that
// jitters obtains the same bits.
__device__ __forceinline__ void jitter_marker(uint64_t seed, uint64_t step, int64_t n, int64_t l, float amp2,
                                              float x0, float y0, float z0, float &x, float &y, float &z)
{
    const uint64_t base = ((uint64_t)step * (uint64_t)n + (uint64_t)l) * 3ull;
    // the states of counters base, base + 1, base + 2 are consecutive
    // multiples of the increment (mod 2^64): one multiply, two adds
    const uint64_t st = seed + (base + 1ull) * kSplitMixGamma;
    const float ux = (float)(splitmix64_mix(st) >> 40) * 0x1p-24f;
    const float uy = (float)(splitmix64_mix(st + kSplitMixGamma) >> 40) * 0x1p-24f;
    const float uz = (float)(splitmix64_mix(st + 2ull * kSplitMixGamma) >> 40) * 0x1p-24f;
    x = x0 + (ux - 0.5f) * amp2;
    y = y0 + (uy - 0.5f) * amp2;
    z = z0 + (uz - 0.5f) * amp2;
}
#pragma clang fp contract(on)

// One form for every kind, with no select: w = max(2^(s^2 e2) - cut, 0) where
// e2 = -log2(e) / eps^2 (0 for the constant weight, whose value is then
// 2^0 - 0 = 1 exactly) and cut = exp(-(R/eps)^2) for the shifted Gaussian, 0
// otherwise (max(g, 0) = g for the plain Gaussian).  Five VALU operations.
__device__ __forceinline__ float weight1(const Weight &w, float s)
{
    return fmaxf(__builtin_amdgcn_exp2f(s * s * w.e2) - w.cut, 0.0f);
}

__device__ __forceinline__ double weight1_d(const Weight &w, double s)
{
    if (w.kind == MLS_W_CONST) return 1.0;
    double t = s * w.inv_eps_d;
    double g = exp(-t * t);
    if (w.kind == MLS_W_GAUSS) return g;
    return fmax(g - w.cut_d, 0.0);
}

// Weight and its derivative dw/ds (0 where the shifted Gaussian is clipped).
__device__ __forceinline__ void weight1_ds(const Weight &w, float s, float &v, float &dv)
{
    if (w.kind == MLS_W_CONST) { v = 1.0f; dv = 0.0f; return; }
    const float t = s * w.inv_eps;
    const float g = __expf(-t * t);
    const float dg = -2.0f * t * w.inv_eps * g;
    if (w.kind == MLS_W_GAUSS) { v = g; dv = dg; return; }
    v = fmaxf(g - w.cut, 0.0f);
    dv = g - w.cut > 0.0f ? dg : 0.0f;
}

__device__ __forceinline__ void weight1_ds(const Weight &w, double s, double &v, double &dv)
{
    if (w.kind == MLS_W_CONST) { v = 1.0; dv = 0.0; return; }
    const double t = s * w.inv_eps_d;
    const double g = exp(-t * t);
    const double dg = -2.0 * t * w.inv_eps_d * g;
    if (w.kind == MLS_W_GAUSS) { v = g; dv = dg; return; }
    v = fmax(g - w.cut_d, 0.0);
    dv = g - w.cut_d > 0.0 ? dg : 0.0;
}

// ---- moment matrix --------------------------------------------------------
// With a tensor-product weight W_k = wx(a) wy(b) wz(c) the moment matrix of
// eq. 3 with p = [1, s_x, s_y, s_z] follows from three 1-D moments per axis,
// m0 = sum w, m1 = sum w s, m2 = sum w s^2:
//   A00 = m0x m0y m0z, A0x = m1x m0y m0z, Axx = m2x m0y m0z,
//   Axy = m1x m1y m0z, ... (10 unique entries of the symmetric 4x4).

template <typename T>
struct Moments { T m0, m1, m2; };

template <typename T>
__device__ __forceinline__ void assemble(const Moments<T> mx, const Moments<T> my, const Moments<T> mz, T A[10])
{
    // A stored as a00 a01 a02 a03 a11 a12 a13 a22 a23 a33
    A[0] = mx.m0 * my.m0 * mz.m0;
    A[1] = mx.m1 * my.m0 * mz.m0;
    A[2] = mx.m0 * my.m1 * mz.m0;
    A[3] = mx.m0 * my.m0 * mz.m1;
    A[4] = mx.m2 * my.m0 * mz.m0;
    A[5] = mx.m1 * my.m1 * mz.m0;
    A[6] = mx.m1 * my.m0 * mz.m1;
    A[7] = mx.m0 * my.m2 * mz.m0;
    A[8] = mx.m0 * my.m1 * mz.m1;
    A[9] = mx.m0 * my.m0 * mz.m2;
}

// Cholesky factor of the symmetric 4x4 A (10 entries).  Returns false if A is
// not numerically positive definite.  L stored row-wise lower: l00 l10 l11
// l20 l21 l22 l30 l31 l32 l33; the diagonal holds 1/l_ii.
__device__ __forceinline__ float rsqrt_t(float v) { return rsqrtf(v); }
__device__ __forceinline__ double rsqrt_t(double v) { return 1.0 / sqrt(v); }

template <typename T>
__device__ __forceinline__ bool cholesky4(const T A[10], T L[10])
{
    T d0 = A[0];
    if (!(d0 > T(0))) return false;
    T r0 = rsqrt_t(d0);
    T l10 = A[1] * r0, l20 = A[2] * r0, l30 = A[3] * r0;
    T d1 = A[4] - l10 * l10;
    if (!(d1 > T(0))) return false;
    T r1 = rsqrt_t(d1);
    T l21 = (A[5] - l20 * l10) * r1;
    T l31 = (A[6] - l30 * l10) * r1;
    T d2 = A[7] - l20 * l20 - l21 * l21;
    if (!(d2 > T(0))) return false;
    T r2 = rsqrt_t(d2);
    T l32 = (A[8] - l30 * l20 - l31 * l21) * r2;
    T d3 = A[9] - l30 * l30 - l31 * l31 - l32 * l32;
    if (!(d3 > T(0))) return false;
    T r3 = rsqrt_t(d3);
    L[0] = r0; L[1] = l10; L[2] = r1; L[3] = l20; L[4] = l21; L[5] = r2;
    L[6] = l30; L[7] = l31; L[8] = l32; L[9] = r3;
    return true;
}

// Solve A x = b with the factor above.
template <typename T>
__device__ __forceinline__ void chol_solve(const T L[10], const T b[4], T x[4])
{
    T y0 = b[0] * L[0];
    T y1 = (b[1] - L[1] * y0) * L[2];
    T y2 = (b[2] - L[3] * y0 - L[4] * y1) * L[5];
    T y3 = (b[3] - L[6] * y0 - L[7] * y1 - L[8] * y2) * L[9];
    x[3] = y3 * L[9];
    x[2] = (y2 - L[8] * x[3]) * L[5];
    x[1] = (y1 - L[4] * x[2] - L[7] * x[3]) * L[2];
    x[0] = (y0 - L[1] * x[1] - L[3] * x[2] - L[6] * x[3]) * L[0];
}

// gamma = A^-1 e_0 and an upper bound of the 2-norm condition number,
// kappa_2(A) <= ||A||_F ||L^-1||_F^2 (A^-1 = L^-T L^-1), from the explicit
// inverse M = L^-1 of the Cholesky factor.
template <typename T>
__device__ __forceinline__ T cond_bound_and_gamma(const T A[10], const T L[10], T gamma[4])
{
    // M = L^-1 (lower triangular), column by column
    const T m00 = L[0];
    const T m11 = L[2], m10 = -L[1] * m00 * m11;
    const T m22 = L[5], m21 = -L[4] * m11 * m22, m20 = -(L[3] * m00 + L[4] * m10) * m22;
    const T m33 = L[9];
    const T m32 = -L[8] * m22 * m33;
    const T m31 = -(L[7] * m11 + L[8] * m21) * m33;
    const T m30 = -(L[6] * m00 + L[7] * m10 + L[8] * m20) * m33;
    // gamma = M^T (M e_0)
    gamma[0] = m00 * m00 + m10 * m10 + m20 * m20 + m30 * m30;
    gamma[1] = m11 * m10 + m21 * m20 + m31 * m30;
    gamma[2] = m22 * m20 + m32 * m30;
    gamma[3] = m33 * m30;
    const T mf = m00 * m00 + m10 * m10 + m11 * m11 + m20 * m20 + m21 * m21 + m22 * m22 + m30 * m30 +
                 m31 * m31 + m32 * m32 + m33 * m33;
    const T af = A[0] * A[0] + A[4] * A[4] + A[7] * A[7] + A[9] * A[9] +
                 T(2) * (A[1] * A[1] + A[2] * A[2] + A[3] * A[3] + A[5] * A[5] + A[6] * A[6] + A[8] * A[8]);
    return sqrt(af) * mf;
}

// Blocked marker layout of the shape functions, home indices and route
// flags: markers are grouped in blocks of 64 (one wavefront); inside a block
// the 64 values of one (component, support node) are consecutive.  So a
// wavefront building one component of 64 markers writes one contiguous
// 27 x 256-byte stretch, and a lane's consecutive support nodes are 64
// floats apart.
constexpr int kLanes = 64;
__device__ __forceinline__ int64_t phi_at(int64_t l, int c)
{
    return ((((l >> 6) * 3 + c) * kNe) << 6) + (l & 63);   // + k * kLanes for node k
}
// Compact transfer-function rows of a compact exact step (NF = 7 or 13 values:
// gamma, the support offsets) with c_l F_l of eq. 8 after them, rs floats per
// row (kCoefStride): two or four 16-byte words per row, and for a (64-row
// block, component) the words q of its 64 rows consecutive, so that one
// wavefront instruction moves 1 KB of whole cache lines.  Float offset of
// word q of row l.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int64_t coef_word(int64_t l, int c, int rs, int q)
{
    return (((((l >> 6) * 3 + c) * (rs >> 2) + q) << 6) + (l & 63)) << 2;
}

__device__ __forceinline__ int64_t home_at(int64_t l, int c)
{
    return (((l >> 6) * 3 + c) << 6) + (l & 63);
}

// Store of an output that the kernel writes once and never reads back (shape
// functions, homes, interpolated values, forces), with the non-temporal
// (streaming) cache policy, so it does not take cache lines from the field
// values that neighbouring markers gather again.
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

__device__ __forceinline__ uint32_t pack_home(int i, int j, int k)
{
    return (uint32_t)i | ((uint32_t)j << kPackI) | ((uint32_t)k << (kPackI + kPackJ));
}

__device__ __forceinline__ void unpack_home(uint32_t h, int &i, int &j, int &k)
{
    i = (int)(h & kMaskI);
    j = (int)((h >> kPackI) & kMaskJ);
    k = (int)(h >> (kPackI + kPackJ));
}

// A packed home is usable by interpolation and spreading if every support
// node exists: the home index lies on the component grid and, on a wall axis,
// both neighbours do too.  Markers whose build failed carry 0xffffffff.
__device__ __forceinline__ bool home_ok(const Grid &g, int c, int i, int j, int k)
{
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int m = g.dims[c][d];
        if (idx[d] >= m) return false;
        if (!g.ax[d].periodic && (idx[d] < 1 || idx[d] + 1 >= m)) return false;
    }
    return true;
}

// Workgroups are dispatched to the 8 XCDs of the chip round-robin
// (workgroup b runs on XCD b % 8), and each XCD has its own L2.  For a grid
// of nb workgroups (a multiple of 8) this index gives XCD x the contiguous
// range [x nb / 8, (x + 1) nb / 8), so that neighbouring work items -- which
// gather the same field lines -- share one L2.
__device__ __forceinline__ int64_t xcd_block()
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    return (int64_t)(b & 7) * (nb >> 3) + (b >> 3);
}

// Exclusive scan of v over a workgroup of 256 threads (4 wavefronts); sh holds
// 4 words of LDS.  total receives the workgroup sum.
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

__host__ __device__ __forceinline__ int64_t round_up8(int64_t b) { return (b + 7) & ~(int64_t)7; }

// Offset of node (i, j, k) in component c's field ([z][y][x], C order).
__device__ __forceinline__ int64_t field_index(const Grid &g, int c, int i, int j, int k)
{
    return ((int64_t)k * g.dims[c][1] + j) * g.dims[c][0] + i;
}

// Wrapped neighbour index along an axis (periodic) or plain (wall axis: the
// support check guarantees it is in range).
__device__ __forceinline__ int nb_index(int i, int a, int n, int periodic)
{
    int j = i + a;
    if (periodic) { j = j < 0 ? j + n : (j >= n ? j - n : j); }
    return j;
}

// Node offsets of the three y rows (oy) and z layers (oz) of the support of
// home (., j, k) on a component grid of nx x ny x nz nodes; zero when ok is
// false (a lane without a support, which loads row 0).  The grid limits (at
// most 2048 x 2048 x 1024 nodes per component) keep every node index below
// 2^32 and nx ny at most 2^22, so the offsets are exact 24-bit products in
// 32 bits (full-rate multiplies instead of 64-bit ones).
__device__ __forceinline__ void support_rows(bool ok, int j, int k, int nx, int ny, int nz, int py, int pz,
                                             uint32_t oy[3], uint32_t oz[3])
{
    const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        oy[a] = ok ? __umul24((uint32_t)nb_index(j, a - 1, ny, py), (uint32_t)nx) : 0u;
        oz[a] = ok ? __umul24((uint32_t)nb_index(k, a - 1, nz, pz), nxy) : 0u;
    }
}

// The 27 values of a field on the support of a home node, as loaded by
// load_support: v holds the window of each row, e the far end of the row for
// a stencil that wraps round a periodic x axis.  at(k) is the value of node
// k = a + 3 b + 9 cz.
struct Support {
    float v[kNe];
    float e[9];
    bool lo, hi;   // the stencil wraps below node 0 / above node nx - 1
    __device__ __forceinline__ float at(int k) const
    {
        const int r = k / 3, a = k % 3;
        if (a == 0) return lo ? e[r] : (hi ? v[3 * r + 1] : v[3 * r]);
        if (a == 1) return lo ? v[3 * r] : (hi ? v[3 * r + 2] : v[3 * r + 1]);
        return lo ? v[3 * r + 1] : (hi ? e[r] : v[3 * r + 2]);
    }
};

// Loads the support values of field q around home node (i, ., .): x index i
// on rows of length nx >= 3, the rows of the y and z neighbours at offsets
// oy[b] + oz[cz].  The three x-neighbours of a row arrive in one 12-byte load
// from the window i - 1 .. i + 1 clamped into the row: a third of the memory
// instructions of one load per value, which matters because the vector L1
// serves each instruction cache line by cache line.  A stencil that wraps
// round a periodic axis (i = 0 or nx - 1) holds two of its values in the
// window and needs the far end of the row: in a wavefront with such a lane,
// every lane loads that one extra value per row (elsewhere e stays 0), and
// Support::at picks each node's value by selects where it is used.  The
// window registers are never rewritten, so the common path does not wait for
// the loads before the solve that follows them.  The values are those of one
// load per node.  A lane without a support passes i = 1 and row offsets 0.
__device__ __forceinline__ void load_support(const float *__restrict__ q, int i, int nx, const uint32_t oy[3],
                                             const uint32_t oz[3], Support &sp)
{
    const uint32_t sx = (uint32_t)min(max(i - 1, 0), nx - 3);
    struct Row3 { float v[3]; };
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        Row3 t;
        __builtin_memcpy(&t, q + (oz[r / 3] + oy[r % 3] + sx), sizeof t);
        sp.v[3 * r] = t.v[0]; sp.v[3 * r + 1] = t.v[1]; sp.v[3 * r + 2] = t.v[2];
    }
    sp.lo = i < 1;
    sp.hi = i > nx - 2;   // both only on a periodic axis
#pragma unroll
    for (int r = 0; r < 9; ++r) sp.e[r] = 0.f;
    if (__any(sp.lo || sp.hi)) {
#pragma unroll
        for (int r = 0; r < 9; ++r) sp.e[r] = q[oz[r / 3] + oy[r % 3] + (sp.lo ? (uint32_t)nx - 1u : 0u)];
    }
}

// The same values in a plain array, the wrapping lanes' windows rotated in
// place by the fix-up.  The compiler then moves the window values into the
// fix-up's registers on the common path and waits for the loads there, which
// costs the latency that Support hides, but the array needs 9 registers fewer
// than Support.  The fused fast-MLS kernel, at its limit of 128 registers, and
// the velocity-gradient kernel, which uses the values inside its node visitor,
// are faster this way.
__device__ __forceinline__ void load_support(const float *__restrict__ q, int i, int nx, const uint32_t oy[3],
                                             const uint32_t oz[3], float qv[kNe])
{
    const uint32_t sx = (uint32_t)min(max(i - 1, 0), nx - 3);
    struct Row3 { float v[3]; };
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        Row3 t;
        __builtin_memcpy(&t, q + (oz[r / 3] + oy[r % 3] + sx), sizeof t);
        qv[3 * r] = t.v[0]; qv[3 * r + 1] = t.v[1]; qv[3 * r + 2] = t.v[2];
    }
    const bool lo = i < 1, hi = i > nx - 2;   // only on a periodic axis
    if (__any(lo || hi)) {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const float e = q[oz[r / 3] + oy[r % 3] + (lo ? (uint32_t)nx - 1u : 0u)];
            const float a0 = qv[3 * r], a1 = qv[3 * r + 1], a2 = qv[3 * r + 2];
            qv[3 * r] = lo ? e : (hi ? a1 : a0);
            qv[3 * r + 1] = lo ? a0 : (hi ? a2 : a1);
            qv[3 * r + 2] = lo ? a1 : (hi ? e : a2);
        }
    }
}

// Control-volume width of node i along an axis: a cell width for a centre
// node, the centre-to-centre distance for a face node.
__device__ __forceinline__ float width_of(const Axis &a, int is_face, int i)
{
    return is_face ? a.width_f[i] : a.width_c[i];
}

// The factors of the spreading coefficient of eq. 8 for one (marker,
// component) with home (hi, hj, hk) and shape function ph:
// h3 = h_l / 3 = sum_k phi_k (dx_k + dy_k + dz_k) / 3 and
// den = sum_k phi_k dV_k, so that c_l F_l = A_l F_l h3 / den.  On a grid
// whose widths are all equal (const_width) the sums skip the width tables;
// they are the same floats.
__device__ __forceinline__ void eq8_sums(const Grid &g, int c, int hi, int hj, int hk, const float ph[kNe],
                                         float &h3, float &den)
{
    float hl = 0.f, dn = 0.f;
    const float cw = g.const_width;
    if (cw > 0.f) {
        const float s3 = cw + cw + cw, p3 = cw * cw * cw;
#pragma unroll
        for (int k = 0; k < kNe; ++k) {
            hl += ph[k] * s3;
            dn += ph[k] * p3;
        }
    } else {
        float wx[3], wy[3], wz[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            wx[a] = width_of(g.ax[0], c == 0, nb_index(hi, a - 1, g.dims[c][0], g.ax[0].periodic));
            wy[a] = width_of(g.ax[1], c == 1, nb_index(hj, a - 1, g.dims[c][1], g.ax[1].periodic));
            wz[a] = width_of(g.ax[2], c == 2, nb_index(hk, a - 1, g.dims[c][2], g.ax[2].periodic));
        }
#pragma unroll
        for (int k = 0; k < kNe; ++k) {
            const int a = k % 3, b = (k / 3) % 3, cz = k / 9;
            hl += ph[k] * (wx[a] + wy[b] + wz[cz]);
            dn += ph[k] * (wx[a] * wy[b] * wz[cz]);
        }
    }
    h3 = hl * (1.0f / 3.0f);
    den = dn;
}

// c_l F_l of eq. 8 from A_l F_l: the per-row value the spreading scatters as
// c_l F_l phi_k.  Computed with the sums of shape-function values given from
// outside (a standalone spreading call), so that a non-finite value among
// them reaches c_l F_l and is reported.
__device__ __forceinline__ float eq8_coef(const Grid &g, int c, int hi, int hj, int hk, const float ph[kNe], float af)
{
    float h3, den;
    eq8_sums(g, c, hi, hj, hk, ph, h3, den);
    return af * h3 / den;
}

// The same for shape functions the library has just computed.  On a grid
// whose widths all equal w, h_l = w sum_k phi_k and sum_k phi_k dV_k =
// w^3 sum_k phi_k, so c_l = A_l / w^2 exactly, whatever the (nonzero) sum of
// the shape functions; elsewhere the sums are taken.
__device__ __forceinline__ float eq8_coef_built(const Grid &g, int c, int hi, int hj, int hk, const float ph[kNe],
                                                float af)
{
    if (g.inv_cw2 > 0.f) return af * g.inv_cw2;
    return eq8_coef(g, c, hi, hj, hk, ph, af);
}

// Largest value of the 64 lanes of a wavefront (all lanes active), returned
// to every lane: four DPP steps give each 16-lane row its maximum (lane
// pairs, quads, half rows, rows), then the four row maxima are read out.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));   // row_half_mirror
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));   // row_mirror
    const uint32_t r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const uint32_t r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return max(max(r0, r1), max(r2, r3));
}

// Per-key maxima of the lanes of a wavefront: for every distinct key >= 0 the
// largest v of the lanes holding it goes into tmax[key] with one atomic max
// (v finite and >= 0; such floats order as their bit patterns do, so the
// maximum is taken on those).  Every lane of the wavefront must call it.
__device__ __forceinline__ void wave_key_max(uint32_t *tmax, int64_t key, float v)
{
    unsigned long long pending = __ballot(key >= 0);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int64_t kl = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)((uint64_t)key >> 32), leader)
                                      << 32) |
                                     (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, leader));
        const bool mine = key == kl;
        const uint32_t m = wave_max_u32(mine ? __float_as_uint(v) : 0u);
        if ((int)(threadIdx.x & 63) == leader && m > 0u) atomicMax(&tmax[kl], m);
        pending &= ~__ballot(mine);
    }
}

// |v| when finite, else 0 (a non-finite value is reported where it is used).
__device__ __forceinline__ float finite_abs(float v)
{
    const float a = fabsf(v);
    return a <= 3.0e38f ? a : 0.f;
}

// Tile index of cell i on an axis with tile edge 1/inv_tile: the exact quotient
// i / tile, since i + 1/2 stays at least 1/(2 tile) from a multiple of tile and
// the FP32 product errs by far less for cells and tiles below 2^11.
__device__ __forceinline__ int tile_of(int i, float inv_tile)
{
    return (int)(((float)i + 0.5f) * inv_tile);
}

// Spreading tile of the cell that holds a marker, from the support geometry G
// of its component c: on the axes other than c the home node is the cell (a
// centre node); on axis c it is the face node fd, and the cell is fd when the
// marker lies at or above that face (offset s_1 = (x_fd - X) / H <= 0, its
// sign exact), else fd - 1 (wrapped on a periodic axis).  The same cell as
// the locate of the binning.
__device__ __forceinline__ uint32_t tile_from_geo(const Grid &g, int c, const AxisGeo G[3])
{
    int t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int cell = G[d].ih;
        if (d == c && G[d].s[1] > 0.0f) cell = cell > 0 ? cell - 1 : g.ax[d].n - 1;
        t[d] = tile_of(cell, g.ax[d].inv_tile);
    }
    return (uint32_t)(((int64_t)t[2] * g.ntile[1] + t[1]) * g.ntile[0] + t[0]);
}

}  // namespace mls
