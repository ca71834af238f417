/*
 * mls_oracle.c -- plain FP64 CPU oracle for the MLS immersed-boundary transfer
 * (Spandan, Lohse, de Tullio, Verzicco, "A fast moving least squares
 * approximation with adaptive Lagrangian mesh refinement for large scale
 * immersed boundary simulations", arXiv:1805.01113).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP library: every definition below is written out from the paper.
 *
 * Everything is double precision and written for readability, not speed.
 *
 * Readings of the paper used here (the paper is silent or garbled on these):
 *  - weight (Sec. 2, after eq. 2: "exponential ... arbitrary"): a tensor
 *    product of 1-D shifted Gaussians w(s) = max(0, exp(-(s/eps)^2) -
 *    exp(-(R/eps)^2)), s in units of the local node spacing, eps = 1,
 *    R = 1.5; plain Gaussian and constant weights are kept for tests.
 *  - basis (eq. 1, p = [1,x,y,z]): coordinates centred at the marker and
 *    scaled per axis by the local spacing H; an invertible affine change of
 *    the basis leaves Phi = p^T A^-1 B unchanged (checked against the literal
 *    absolute-coordinate form by orc_mls_shape_literal).
 *  - eq. 4 is typeset as a row of W p^T; B is m x N_e with columns W_k p_k.
 *  - eq. 10 numerator reads 1/d_i^2 (index garbled in the paper); in 3-D the
 *    blend runs over the 8 corners of the enclosing sub-cell; at d_i = 0 the
 *    blend is the indicator of that sub-node (product form below).
 *  - sub-nodes include the home control-volume boundaries, n per axis.
 *  - support (Sec. 2, figure 1 text): home node of the marker plus its
 *    neighbours, 3 per axis, on each velocity component's own staggered grid;
 *    the home node is the one whose control volume contains the marker,
 *    half-open [lo, hi), so ties go to the upper node.
 *  - spreading (eq. 7-8): h_l, Delta V_k per component with that component's
 *    shape function and control-volume widths; forces are added into f.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_SUPPORT (-2)
#define ORC_E_SINGULAR (-3)

#define ORC_W_GAUSS_SHIFTED 0
#define ORC_W_GAUSS 1
#define ORC_W_CONST 2

/* ------------------------------------------------------------------------ */
/* Dense linear algebra (Gaussian elimination with partial pivoting).        */
/* ------------------------------------------------------------------------ */

/* Solve A X = B for X, A m x m row-major (destroyed), B m x nrhs row-major
 * (overwritten by X).  Returns ORC_E_SINGULAR if a pivot is exactly zero. */
static int gepp_solve(int m, double *A, int nrhs, double *B)
{
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(A[r * m + col]) > fabs(A[piv * m + col])) piv = r;
        if (A[piv * m + col] == 0.0) return ORC_E_SINGULAR;
        if (piv != col) {
            for (int c = 0; c < m; ++c) {
                double t = A[col * m + c]; A[col * m + c] = A[piv * m + c]; A[piv * m + c] = t;
            }
            for (int c = 0; c < nrhs; ++c) {
                double t = B[col * nrhs + c]; B[col * nrhs + c] = B[piv * nrhs + c]; B[piv * nrhs + c] = t;
            }
        }
        for (int r = col + 1; r < m; ++r) {
            double f = A[r * m + col] / A[col * m + col];
            for (int c = col; c < m; ++c) A[r * m + c] -= f * A[col * m + c];
            for (int c = 0; c < nrhs; ++c) B[r * nrhs + c] -= f * B[col * nrhs + c];
        }
    }
    for (int r = m - 1; r >= 0; --r) {
        for (int c = 0; c < nrhs; ++c) {
            double s = B[r * nrhs + c];
            for (int k = r + 1; k < m; ++k) s -= A[r * m + k] * B[k * nrhs + c];
            B[r * nrhs + c] = s / A[r * m + r];
        }
    }
    return ORC_OK;
}

/* 1-norm condition number ||A||_1 ||A^-1||_1 of an m x m matrix. */
static double cond1(int m, const double *A)
{
    double a[16], inv[16];
    memcpy(a, A, sizeof(double) * m * m);
    for (int i = 0; i < m * m; ++i) inv[i] = 0.0;
    for (int i = 0; i < m; ++i) inv[i * m + i] = 1.0;
    if (gepp_solve(m, a, m, inv) != ORC_OK) return INFINITY;
    double na = 0.0, ni = 0.0;
    for (int c = 0; c < m; ++c) {
        double sa = 0.0, si = 0.0;
        for (int r = 0; r < m; ++r) { sa += fabs(A[r * m + c]); si += fabs(inv[r * m + c]); }
        if (sa > na) na = sa;
        if (si > ni) ni = si;
    }
    return na * ni;
}

/* ------------------------------------------------------------------------ */
/* Weight function (Sec. 2, after eq. 2).                                    */
/* ------------------------------------------------------------------------ */

double orc_weight_1d(int kind, double eps, double R, double s)
{
    if (kind == ORC_W_CONST) return 1.0;
    double g = exp(-(s / eps) * (s / eps));
    if (kind == ORC_W_GAUSS) return g;
    double w = g - exp(-(R / eps) * (R / eps));
    return w > 0.0 ? w : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Exact MLS shape function (eq. 1-6).                                       */
/* ------------------------------------------------------------------------ */

/* dim = 2 or 3.  s[d*3 + a] (a = 0,1,2 for offsets -1,0,+1) is the position
 * of support node a along axis d relative to the marker, in units of the
 * local spacing.  The support is the tensor product of the three nodes per
 * axis, N_e = 3^dim, node index k = sum_d a_d 3^d (x fastest).
 * Basis p = [1, s_x, s_y(, s_z)] (centred at the marker, so p(x_l) = e_0).
 * A = sum_k W_k p_k p_k^T (eq. 3), B = [W_k p_k] (eq. 4),
 * Phi^T = p^T(x_l) A^-1 B (eq. 6).  kappa1 receives ||A||_1 ||A^-1||_1. */
int orc_mls_shape(int dim, const double *s, int kind, double eps, double R,
                  double *phi, double *kappa1)
{
    if (dim != 2 && dim != 3) return ORC_E_ARG;
    const int m = dim + 1;
    const int ne = dim == 2 ? 9 : 27;
    double A[16] = {0}, Acopy[16];
    double B[4 * 27];
    for (int k = 0; k < ne; ++k) {
        double p[4];
        double W = 1.0;
        int kk = k;
        p[0] = 1.0;
        for (int d = 0; d < dim; ++d) {
            int a = kk % 3; kk /= 3;
            p[1 + d] = s[d * 3 + a];
            W *= orc_weight_1d(kind, eps, R, s[d * 3 + a]);
        }
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) A[i * m + j] += W * p[i] * p[j];
            B[i * ne + k] = W * p[i];
        }
    }
    memcpy(Acopy, A, sizeof(A));
    if (kappa1) *kappa1 = cond1(m, A);
    int rc = gepp_solve(m, Acopy, ne, B);   /* B <- A^-1 B */
    if (rc != ORC_OK) return rc;
    /* p(x_l) = [1, 0, ..., 0] in marker-centred coordinates */
    for (int k = 0; k < ne; ++k) phi[k] = B[0 * ne + k];
    return ORC_OK;
}

/* The literal form of eq. 6 with the absolute basis p = [1, x, y(, z)]:
 * xl[d] is the marker coordinate, xn[d*3 + a] the support node coordinates,
 * H[d] the spacing used to scale the weight argument.  Used only to check the
 * centred form above. */
int orc_mls_shape_literal(int dim, const double *xl, const double *xn,
                          const double *H, int kind, double eps, double R,
                          double *phi)
{
    if (dim != 2 && dim != 3) return ORC_E_ARG;
    const int m = dim + 1;
    const int ne = dim == 2 ? 9 : 27;
    double A[16] = {0};
    double B[4 * 27];
    for (int k = 0; k < ne; ++k) {
        double p[4];
        double W = 1.0;
        int kk = k;
        p[0] = 1.0;
        for (int d = 0; d < dim; ++d) {
            int a = kk % 3; kk /= 3;
            p[1 + d] = xn[d * 3 + a];
            W *= orc_weight_1d(kind, eps, R, (xn[d * 3 + a] - xl[d]) / H[d]);
        }
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) A[i * m + j] += W * p[i] * p[j];
            B[i * ne + k] = W * p[i];
        }
    }
    int rc = gepp_solve(m, A, ne, B);
    if (rc != ORC_OK) return rc;
    double pl[4];
    pl[0] = 1.0;
    for (int d = 0; d < dim; ++d) pl[1 + d] = xl[d];
    for (int k = 0; k < ne; ++k) {
        double v = 0.0;
        for (int i = 0; i < m; ++i) v += pl[i] * B[i * ne + k];
        phi[k] = v;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Staggered grid geometry: nodes, control volumes, home node.               */
/* ------------------------------------------------------------------------ */
/* An axis has n cells with face coordinates f[0..n].  Along axis d the
 * velocity component c lives on the faces when d == c and on the cell
 * centres otherwise (marker-and-cell staggering).  On a periodic axis of
 * length L = f[n] - f[0] node indices wrap modulo n and coordinates shift by
 * multiples of L.  A cell-centre node i owns the control volume
 * [f[i], f[i+1]); a face node i owns [c(i-1), c(i)) between the neighbouring
 * centres (on a wall axis the end faces own [f[0], c(0)) and [c(n-1), f[n]]). */

static long floor_div(long a, long b)
{
    long q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

static double centre_x(const double *f, int n, int periodic, long i)
{
    long shift = 0;
    if (periodic) { shift = floor_div(i, n); i -= shift * n; }
    double L = f[n] - f[0];
    return 0.5 * (f[i] + f[i + 1]) + (double)shift * L;
}

static double face_x(const double *f, int n, int periodic, long i)
{
    long shift = 0;
    if (periodic) { shift = floor_div(i, n); i -= shift * n; }
    double L = f[n] - f[0];
    return f[i] + (double)shift * L;
}

static double node_x(const double *f, int n, int periodic, int is_face, long i)
{
    return is_face ? face_x(f, n, periodic, i) : centre_x(f, n, periodic, i);
}

/* Periodic wrap of a coordinate into [f[0], f[0] + L). */
static double wrap_x(const double *f, int n, double x)
{
    double L = f[n] - f[0];
    double t = floor((x - f[0]) / L);
    double X = x - t * L;
    if (X >= f[0] + L) X -= L;
    if (X < f[0]) X += L;
    return X;
}

/* Control volume [lo, hi) of node i (unwrapped index). */
static void node_cv(const double *f, int n, int periodic, int is_face, long i,
                    double *lo, double *hi)
{
    if (!is_face) {
        *lo = face_x(f, n, periodic, i);
        *hi = face_x(f, n, periodic, i + 1);
    } else {
        *lo = (!periodic && i == 0) ? f[0] : centre_x(f, n, periodic, i - 1);
        *hi = (!periodic && i == n) ? f[n] : centre_x(f, n, periodic, i);
    }
}

/* Number of nodes of a component's grid along an axis. */
static long axis_nodes(int n, int periodic, int is_face)
{
    return (is_face && !periodic) ? (long)n + 1 : (long)n;
}

/* Home node along one axis.  Returns the unwrapped home index ih (for a
 * periodic face axis ih may equal n, which is node 0 shifted by L) and the
 * wrapped coordinate X.  The home node is the one whose control volume
 * contains X (found by bisection over the sorted node control volumes).
 * The 3-node support ih-1..ih+1 must lie inside a wall axis, else
 * ORC_E_SUPPORT. */
int orc_locate_axis(const double *f, int n, int periodic, int is_face,
                    double x, long *ih_out, double *X_out)
{
    double X;
    if (periodic) {
        X = wrap_x(f, n, x);
    } else {
        X = x;
        if (!(X >= f[0] && X <= f[n])) return ORC_E_SUPPORT;
    }
    long ih;
    if (!is_face) {
        /* largest i in [0, n-1] with f[i] <= X */
        long lo = 0, hi = n;          /* f[lo] <= X < f[hi] */
        if (X >= f[n]) return ORC_E_SUPPORT;
        while (hi - lo > 1) {
            long mid = (lo + hi) / 2;
            if (f[mid] <= X) lo = mid; else hi = mid;
        }
        ih = lo;
    } else {
        /* i in [0, n] with c(i-1) <= X < c(i) */
        double c0 = centre_x(f, n, periodic, 0);
        double cl = centre_x(f, n, periodic, n - 1);
        if (X < c0) {
            ih = 0;
        } else if (X >= cl) {
            ih = n;
        } else {
            long lo = 0, hi = n - 1;  /* c(lo) <= X < c(hi) */
            while (hi - lo > 1) {
                long mid = (lo + hi) / 2;
                if (centre_x(f, n, periodic, mid) <= X) lo = mid; else hi = mid;
            }
            ih = hi;
        }
    }
    if (!periodic) {
        long last = axis_nodes(n, periodic, is_face) - 1;
        if (ih - 1 < 0 || ih + 1 > last) return ORC_E_SUPPORT;
    }
    *ih_out = ih;
    *X_out = X;
    return ORC_OK;
}

/* Local geometry of the 3-node support along one axis for a marker at X with
 * unwrapped home ih: offsets s[a] = (X(ih+a-1) - X)/H with
 * H = (X(ih+1) - X(ih-1))/2, the in-cell offset xi = (X - X(ih))/H, the
 * spacing ratio rho = (X(ih+1) - X(ih))/(X(ih) - X(ih-1)), the home control
 * volume in the same normalised units, and the control-volume widths of the
 * three support nodes. */
typedef struct {
    double s[3], xi, rho, H, cvlo, cvhi, width[3];
} orc_axis_geo;

static void axis_geometry(const double *f, int n, int periodic, int is_face,
                          long ih, double X, orc_axis_geo *g)
{
    double xm = node_x(f, n, periodic, is_face, ih - 1);
    double x0 = node_x(f, n, periodic, is_face, ih);
    double xp = node_x(f, n, periodic, is_face, ih + 1);
    double H = 0.5 * (xp - xm);
    g->H = H;
    g->s[0] = (xm - X) / H;
    g->s[1] = (x0 - X) / H;
    g->s[2] = (xp - X) / H;
    g->xi = (X - x0) / H;
    g->rho = (xp - x0) / (x0 - xm);
    double lo, hi;
    node_cv(f, n, periodic, is_face, ih, &lo, &hi);
    g->cvlo = (lo - x0) / H;
    g->cvhi = (hi - x0) / H;
    for (int a = 0; a < 3; ++a) {
        node_cv(f, n, periodic, is_face, ih + a - 1, &lo, &hi);
        g->width[a] = hi - lo;
    }
}

/* Grid passed as: faces = concatenation of the three face arrays
 * (n[0]+1, n[1]+1, n[2]+1 values), n[3], periodic[3]. */
typedef struct {
    const double *f[3];
    int n[3];
    int periodic[3];
} grid3;

static void grid_unpack(const double *faces, const int32_t *n, const int32_t *periodic, grid3 *g)
{
    long off = 0;
    for (int d = 0; d < 3; ++d) {
        g->f[d] = faces + off;
        g->n[d] = n[d];
        g->periodic[d] = periodic[d];
        off += n[d] + 1;
    }
}

/* Home indices (wrapped) and per-axis geometry of one marker for component
 * comp. */
static int marker_geometry(const grid3 *g, int comp, const double x[3],
                           long home[3], orc_axis_geo geo[3], long ih_unwrapped[3])
{
    for (int d = 0; d < 3; ++d) {
        long ih; double X;
        int is_face = (d == comp);
        int rc = orc_locate_axis(g->f[d], g->n[d], g->periodic[d], is_face, x[d], &ih, &X);
        if (rc != ORC_OK) return rc;
        axis_geometry(g->f[d], g->n[d], g->periodic[d], is_face, ih, X, &geo[d]);
        ih_unwrapped[d] = ih;
        home[d] = g->periodic[d] ? ih - floor_div(ih, g->n[d]) * g->n[d] : ih;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-marker exact build (support selection + eq. 3-6).                     */
/* ------------------------------------------------------------------------ */

/* For component comp and markers x,y,z (FP32, as the markers are stored),
 * writes home[l*3 + d] (wrapped node index), phi[l*27 + k], kappa[l]
 * (1-norm condition of the normalised moment matrix), and, if non-NULL,
 * xi[l*3+d] and rho[l*3+d].  Returns the first error and its marker in
 * *bad (or -1). */
int orc_build_exact(const double *faces, const int32_t *n, const int32_t *periodic,
                    int comp, int kind, double eps, double R,
                    long nm, const float *x, const float *y, const float *z,
                    int32_t *home, double *phi, double *kappa,
                    double *xi, double *rho, long *bad)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    int first_rc = ORC_OK;
    long first_bad = -1;
    #pragma omp parallel for schedule(static)
    for (long l = 0; l < nm; ++l) {
        double xl[3] = {x[l], y[l], z[l]};
        long h[3], ihu[3];
        orc_axis_geo geo[3];
        int rc = marker_geometry(&g, comp, xl, h, geo, ihu);
        double s[9];
        double kap = 0.0;
        if (rc == ORC_OK) {
            for (int d = 0; d < 3; ++d)
                for (int a = 0; a < 3; ++a) s[d * 3 + a] = geo[d].s[a];
            rc = orc_mls_shape(3, s, kind, eps, R, phi + l * 27, &kap);
        }
        if (rc != ORC_OK) {
            #pragma omp critical
            {
                if (first_bad < 0 || l < first_bad) { first_bad = l; first_rc = rc; }
            }
            for (int k = 0; k < 27; ++k) phi[l * 27 + k] = NAN;
            for (int d = 0; d < 3; ++d) home[l * 3 + d] = -1;
            continue;
        }
        for (int d = 0; d < 3; ++d) home[l * 3 + d] = (int32_t)h[d];
        if (kappa) kappa[l] = kap;
        if (xi) for (int d = 0; d < 3; ++d) xi[l * 3 + d] = geo[d].xi;
        if (rho) for (int d = 0; d < 3; ++d) rho[l * 3 + d] = geo[d].rho;
    }
    if (bad) *bad = first_bad;
    return first_rc;
}

/* ------------------------------------------------------------------------ */
/* fast-MLS (eq. 9-10).                                                      */
/* ------------------------------------------------------------------------ */

/* Sub-node coordinate j (0..nsub-1) of the home control volume [lo, hi) in
 * normalised units, boundaries included. */
static double subnode(double lo, double hi, int nsub, int j)
{
    return lo + (double)j * (hi - lo) / (double)(nsub - 1);
}

/* Table of exact shape functions at the nsub^dim sub-nodes of one home
 * control volume.  node[d*3 + a] is the position of support node a along
 * axis d relative to the home node, in units of H (so node[d*3+1] = 0),
 * cvlo[d], cvhi[d] the home control volume in the same units.
 * table[s*ne + k], sub-node index s = sum_d j_d nsub^d (x fastest). */
int orc_fast_table(int dim, const double *node, const double *cvlo, const double *cvhi,
                   int nsub, int kind, double eps, double R, double *table)
{
    if ((dim != 2 && dim != 3) || nsub < 2) return ORC_E_ARG;
    const int ne = dim == 2 ? 9 : 27;
    long ns = 1;
    for (int d = 0; d < dim; ++d) ns *= nsub;
    for (long sidx = 0; sidx < ns; ++sidx) {
        double s[9];
        long ss = sidx;
        for (int d = 0; d < dim; ++d) {
            int j = (int)(ss % nsub); ss /= nsub;
            double xs = subnode(cvlo[d], cvhi[d], nsub, j);
            for (int a = 0; a < 3; ++a) s[d * 3 + a] = node[d * 3 + a] - xs;
        }
        int rc = orc_mls_shape(dim, s, kind, eps, R, table + sidx * ne, NULL);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/* Shepard blend (eq. 9-10) of the table over the 2^dim corners of the
 * sub-cell that encloses the in-cell offset xi[d].  The inverse-square
 * distance weights alpha_i = (1/d_i^2) / sum_j (1/d_j^2) are evaluated in the
 * equivalent product form alpha_i = prod_{j!=i} d_j^2 / sum_m prod_{j!=m}
 * d_j^2, which gives the indicator of a sub-node when the marker sits on it.
 * Distances are measured in the normalised units of xi. */
int orc_fast_shape(int dim, const double *xi, const double *cvlo, const double *cvhi,
                   int nsub, const double *table, double *phi)
{
    if ((dim != 2 && dim != 3) || nsub < 2) return ORC_E_ARG;
    const int ne = dim == 2 ? 9 : 27;
    const int nc = 1 << dim;
    int j0[3];
    for (int d = 0; d < dim; ++d) {
        double t = (xi[d] - cvlo[d]) / (cvhi[d] - cvlo[d]) * (double)(nsub - 1);
        int j = (int)floor(t);
        if (j > nsub - 2) j = nsub - 2;
        if (j < 0) j = 0;
        j0[d] = j;
    }
    double d2[8];
    long sidx[8];
    for (int i = 0; i < nc; ++i) {
        double acc = 0.0;
        long idx = 0, stride = 1;
        for (int d = 0; d < dim; ++d) {
            int j = j0[d] + ((i >> d) & 1);
            double xs = subnode(cvlo[d], cvhi[d], nsub, j);
            acc += (xi[d] - xs) * (xi[d] - xs);
            idx += j * stride;
            stride *= nsub;
        }
        d2[i] = acc;
        sidx[i] = idx;
    }
    double alpha[8], den = 0.0;
    for (int i = 0; i < nc; ++i) {
        double p = 1.0;
        for (int j = 0; j < nc; ++j) if (j != i) p *= d2[j];
        alpha[i] = p;
        den += p;
    }
    for (int i = 0; i < nc; ++i) alpha[i] /= den;
    for (int k = 0; k < ne; ++k) {
        double v = 0.0;
        for (int i = 0; i < nc; ++i) v += alpha[i] * table[sidx[i] * ne + k];
        phi[k] = v;
    }
    return ORC_OK;
}

/* Trilinear variant of the fast-MLS lookup (the first "next" item beyond the
 * paper's Shepard blend): the same enclosing sub-cell and table, blended with
 * the multilinear weights of xi inside the sub-cell,
 *   alpha_i = prod_d (t_d if corner i is at the upper sub-node along d else 1 - t_d),
 * t_d = (xi_d - xs_lo,d) / (xs_hi,d - xs_lo,d).  The weights sum to one and
 * reproduce xi itself, so the blend keeps the partition of unity and the
 * exact reproduction of linear fields of the tabulated exact shape functions. */
int orc_fast_shape_trilinear(int dim, const double *xi, const double *cvlo, const double *cvhi,
                             int nsub, const double *table, double *phi)
{
    if ((dim != 2 && dim != 3) || nsub < 2) return ORC_E_ARG;
    const int ne = dim == 2 ? 9 : 27;
    const int nc = 1 << dim;
    int j0[3];
    double t[3];
    for (int d = 0; d < dim; ++d) {
        double u = (xi[d] - cvlo[d]) / (cvhi[d] - cvlo[d]) * (double)(nsub - 1);
        int j = (int)floor(u);
        if (j > nsub - 2) j = nsub - 2;
        if (j < 0) j = 0;
        j0[d] = j;
        double xa = subnode(cvlo[d], cvhi[d], nsub, j), xb = subnode(cvlo[d], cvhi[d], nsub, j + 1);
        t[d] = (xi[d] - xa) / (xb - xa);
    }
    for (int k = 0; k < ne; ++k) phi[k] = 0.0;
    for (int i = 0; i < nc; ++i) {
        double alpha = 1.0;
        long idx = 0, stride = 1;
        for (int d = 0; d < dim; ++d) {
            int up = (i >> d) & 1;
            alpha *= up ? t[d] : 1.0 - t[d];
            idx += (j0[d] + up) * stride;
            stride *= nsub;
        }
        for (int k = 0; k < ne; ++k) phi[k] += alpha * table[idx * ne + k];
    }
    return ORC_OK;
}

/* Per-marker fast-MLS build for component comp on the staggered grid.  The
 * table of a home node depends only on the support geometry; on a uniform
 * axis every cell has the same geometry, on a stretched axis each home index
 * has its own (the paper stores the extra shape functions of the cells along
 * the stretched direction).  Tables are computed here on demand, one per
 * distinct (home index along the non-uniform axes). */
/* blend 0: Shepard (eq. 9-10), 1: trilinear (orc_fast_shape_trilinear). */
int orc_build_fast_blend(const double *faces, const int32_t *n, const int32_t *periodic,
                         int comp, int kind, double eps, double R, int nsub, int blend,
                         long nm, const float *x, const float *y, const float *z,
                         int32_t *home, double *phi, long *bad)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    /* which axes are uniform: all cell widths equal (to 1e-12 relative, the
       rounding of the face coordinates) */
    int uniform[3];
    for (int d = 0; d < 3; ++d) {
        uniform[d] = 1;
        double w0 = g.f[d][1] - g.f[d][0];
        for (int i = 1; i < g.n[d]; ++i)
            if (fabs((g.f[d][i + 1] - g.f[d][i]) - w0) > 1e-12 * w0) { uniform[d] = 0; break; }
    }
    long ns = (long)nsub * nsub * nsub;
    /* table cache keyed by the home indices along non-uniform axes
       (at most one non-uniform axis is supported, as in the paper) */
    int nonuni = -1;
    for (int d = 0; d < 3; ++d) if (!uniform[d]) { if (nonuni >= 0) return ORC_E_ARG; nonuni = d; }
    long nkeys = nonuni < 0 ? 1 : axis_nodes(g.n[nonuni], g.periodic[nonuni], nonuni == comp);
    double **cache = (double **)calloc((size_t)nkeys, sizeof(double *));
    if (!cache) return ORC_E_ARG;
    int first_rc = ORC_OK;
    long first_bad = -1;
    for (long l = 0; l < nm; ++l) {
        double xl[3] = {x[l], y[l], z[l]};
        long h[3], ihu[3];
        orc_axis_geo geo[3];
        int rc = marker_geometry(&g, comp, xl, h, geo, ihu);
        if (rc != ORC_OK) {
            if (first_bad < 0) { first_bad = l; first_rc = rc; }
            for (int k = 0; k < 27; ++k) phi[l * 27 + k] = NAN;
            for (int d = 0; d < 3; ++d) home[l * 3 + d] = -1;
            continue;
        }
        long key = nonuni < 0 ? 0 : h[nonuni];
        double node[9], lo[3], hi[3], xi[3];
        for (int d = 0; d < 3; ++d) {
            /* support geometry seen from the home node itself */
            int is_face = (d == comp);
            double x0 = node_x(g.f[d], g.n[d], g.periodic[d], is_face, ihu[d]);
            orc_axis_geo hg;
            axis_geometry(g.f[d], g.n[d], g.periodic[d], is_face, ihu[d], x0, &hg);
            for (int a = 0; a < 3; ++a) node[d * 3 + a] = hg.s[a];
            lo[d] = hg.cvlo;
            hi[d] = hg.cvhi;
            xi[d] = geo[d].xi;
        }
        if (!cache[key]) {
            cache[key] = (double *)malloc(sizeof(double) * ns * 27);
            rc = orc_fast_table(3, node, lo, hi, nsub, kind, eps, R, cache[key]);
            if (rc != ORC_OK) { free(cache[key]); cache[key] = NULL; if (first_bad < 0) { first_bad = l; first_rc = rc; } continue; }
        }
        if (blend == 1) orc_fast_shape_trilinear(3, xi, lo, hi, nsub, cache[key], phi + l * 27);
        else orc_fast_shape(3, xi, lo, hi, nsub, cache[key], phi + l * 27);
        for (int d = 0; d < 3; ++d) home[l * 3 + d] = (int32_t)h[d];
    }
    for (long k = 0; k < nkeys; ++k) free(cache[k]);
    free(cache);
    if (bad) *bad = first_bad;
    return first_rc;
}

int orc_build_fast(const double *faces, const int32_t *n, const int32_t *periodic,
                   int comp, int kind, double eps, double R, int nsub,
                   long nm, const float *x, const float *y, const float *z,
                   int32_t *home, double *phi, long *bad)
{
    return orc_build_fast_blend(faces, n, periodic, comp, kind, eps, R, nsub, 0, nm, x, y, z, home, phi, bad);
}

/* Geometry of the normalised support of one home node, for table checks:
 * node[d*3+a], cvlo[d], cvhi[d] as orc_fast_table expects. */
int orc_home_support(const double *faces, const int32_t *n, const int32_t *periodic,
                     int comp, const int32_t *home, double *node, double *cvlo, double *cvhi)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    for (int d = 0; d < 3; ++d) {
        int is_face = (d == comp);
        long ih = home[d];
        double x0 = node_x(g.f[d], g.n[d], g.periodic[d], is_face, ih);
        orc_axis_geo geo;
        axis_geometry(g.f[d], g.n[d], g.periodic[d], is_face, ih, x0, &geo);
        for (int a = 0; a < 3; ++a) node[d * 3 + a] = geo.s[a];
        cvlo[d] = geo.cvlo;
        cvhi[d] = geo.cvhi;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Interpolation (eq. 6: Q = Phi^T q) and spreading (eq. 7-8).               */
/* ------------------------------------------------------------------------ */

/* Node index of support node k of a marker with wrapped home h on the
 * component-comp grid (C order [z][y][x]). */
static long support_index(const grid3 *g, const int32_t *h, int k, long dims[3])
{
    long idx[3];
    int a[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
    for (int d = 0; d < 3; ++d) {
        long i = (long)h[d] + a[d];
        if (g->periodic[d]) i = i - floor_div(i, g->n[d]) * g->n[d];
        idx[d] = i;
    }
    return (idx[2] * dims[1] + idx[1]) * dims[0] + idx[0];
}

static void comp_dims(const grid3 *g, int comp, long dims[3])
{
    for (int d = 0; d < 3; ++d) dims[d] = axis_nodes(g->n[d], g->periodic[d], d == comp);
}

/* U[l] = sum_k phi[l*27+k] q[node_k(l)], q stored as FP32 (promoted). */
int orc_interp(const double *faces, const int32_t *n, const int32_t *periodic, int comp,
               long nm, const int32_t *home, const double *phi, const float *q, double *U)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    long dims[3];
    comp_dims(&g, comp, dims);
    #pragma omp parallel for schedule(static)
    for (long l = 0; l < nm; ++l) {
        double acc = 0.0;
        for (int k = 0; k < 27; ++k)
            acc += phi[l * 27 + k] * (double)q[support_index(&g, home + l * 3, k, dims)];
        U[l] = acc;
    }
    return ORC_OK;
}

/* Spreading of marker forces F[l] (component comp) onto the grid, eq. 7-8:
 *   h_l     = sum_k phi_k (dx_k + dy_k + dz_k)/3
 *   dV_l    = A_l h_l
 *   c_l     = dV_l / sum_k phi_k dV_k
 *   f_k    += c_l phi_k F_l
 * dx_k, dy_k, dz_k are the control-volume widths of support node k on the
 * component's own grid and dV_k = dx_k dy_k dz_k.  f is a dense FP64 field
 * that is added into.  cl (optional) receives c_l. */
int orc_spread(const double *faces, const int32_t *n, const int32_t *periodic, int comp,
               long nm, const int32_t *home, const double *phi, const float *area,
               const float *F, double *f, double *cl)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    long dims[3];
    comp_dims(&g, comp, dims);
    for (long l = 0; l < nm; ++l) {
        const int32_t *h = home + l * 3;
        double wdt[3][3];
        for (int d = 0; d < 3; ++d) {
            int is_face = (d == comp);
            for (int a = 0; a < 3; ++a) {
                double lo, hi;
                node_cv(g.f[d], g.n[d], g.periodic[d], is_face, (long)h[d] + a - 1, &lo, &hi);
                wdt[d][a] = hi - lo;
            }
        }
        double hl = 0.0, den = 0.0;
        for (int k = 0; k < 27; ++k) {
            int a = k % 3, b = (k / 3) % 3, c = k / 9;
            double dx = wdt[0][a], dy = wdt[1][b], dz = wdt[2][c];
            hl += phi[l * 27 + k] * (dx + dy + dz) / 3.0;
            den += phi[l * 27 + k] * (dx * dy * dz);
        }
        double dVl = (double)area[l] * hl;
        double c_l = dVl / den;
        if (cl) cl[l] = c_l;
        for (int k = 0; k < 27; ++k)
            f[support_index(&g, h, k, dims)] += c_l * phi[l * 27 + k] * (double)F[l];
    }
    return ORC_OK;
}

/* Control-volume volume dV of every node of the component grid (for the
 * conservation check of eq. 7). */
int orc_node_volumes(const double *faces, const int32_t *n, const int32_t *periodic, int comp,
                     double *dV)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    long dims[3];
    comp_dims(&g, comp, dims);
    for (long k = 0; k < dims[2]; ++k)
        for (long j = 0; j < dims[1]; ++j)
            for (long i = 0; i < dims[0]; ++i) {
                long ii[3] = {i, j, k};
                double v = 1.0;
                for (int d = 0; d < 3; ++d) {
                    double lo, hi;
                    node_cv(g.f[d], g.n[d], g.periodic[d], d == comp, ii[d], &lo, &hi);
                    v *= hi - lo;
                }
                dV[(k * dims[1] + j) * dims[0] + i] = v;
            }
    return ORC_OK;
}

/* Node coordinates of the component grid along one axis (for tests). */
int orc_axis_nodes(const double *faces, const int32_t *n, const int32_t *periodic, int comp,
                   int axis, double *X)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    long m = axis_nodes(g.n[axis], g.periodic[axis], axis == comp);
    for (long i = 0; i < m; ++i) X[i] = node_x(g.f[axis], g.n[axis], g.periodic[axis], axis == comp, i);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Coarse-grained collision detection (Sec. 4, the integer cell array coll). */
/* ------------------------------------------------------------------------ */
/* The cell of a marker is the Eulerian cell that contains it: along each
 * axis the i with f[i] <= X < f[i+1], X being the wrapped coordinate on a
 * periodic axis.  On a wall axis a coordinate outside [f[0], f[n]) has no
 * cell (ORC_E_SUPPORT). */
static int cell_axis(const double *f, int n, int periodic, double x, long *i_out)
{
    if (!isfinite(x)) return ORC_E_SUPPORT;
    double X = periodic ? wrap_x(f, n, x) : x;
    if (!(X >= f[0] && X < f[n])) return ORC_E_SUPPORT;
    long lo = 0, hi = n;   /* f[lo] <= X < f[hi] */
    while (hi - lo > 1) {
        long mid = (lo + hi) / 2;
        if (f[mid] <= X) lo = mid; else hi = mid;
    }
    *i_out = lo;
    return ORC_OK;
}

/* The paper's two sweeps over the markers, in marker order.
 *   coll, one int32 per cell (C order [z][y][x]), starts at 0 (cleared here).
 *   Sweep 1: marker l of body b carries the id pid = b + 1.  If its cell
 *   holds 0 the cell takes pid; if the cell then holds anything but pid it
 *   becomes -1 (markers of more than one body share the cell).
 *   Sweep 2: flag[l] = 1 where the cell of marker l holds -1 (a collision
 *   force would be switched on for that marker), else 0.
 * cell[l] receives the linear cell index of marker l.  Every marker is
 * located before coll is touched: a marker without a cell returns
 * ORC_E_SUPPORT, a body id outside [0, 2^31 - 2] ORC_E_ARG, with the first
 * such marker in *bad. */
int orc_collide(const double *faces, const int32_t *n, const int32_t *periodic,
                long nm, const float *x, const float *y, const float *z, const int32_t *body,
                int32_t *coll, long *cell, uint8_t *flag, long *bad)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    *bad = -1;
    const long ncell = (long)n[0] * n[1] * n[2];
    for (long l = 0; l < nm; ++l) {
        const double p[3] = {(double)x[l], (double)y[l], (double)z[l]};
        long ic[3];
        for (int d = 0; d < 3; ++d) {
            if (cell_axis(g.f[d], g.n[d], g.periodic[d], p[d], &ic[d]) != ORC_OK) {
                *bad = l;
                return ORC_E_SUPPORT;
            }
        }
        if (body[l] < 0 || body[l] > 2147483646) {
            *bad = l;
            return ORC_E_ARG;
        }
        cell[l] = (ic[2] * n[1] + ic[1]) * n[0] + ic[0];
    }
    for (long c = 0; c < ncell; ++c) coll[c] = 0;
    for (long l = 0; l < nm; ++l) {
        const int32_t pid = body[l] + 1;
        int32_t *cv = &coll[cell[l]];
        if (*cv == 0) *cv = pid;
        if (*cv != pid) *cv = -1;
    }
    for (long l = 0; l < nm; ++l) flag[l] = coll[cell[l]] == -1 ? 1 : 0;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Adaptive Lagrangian mesh refinement (Sec. 3, Fig. 5, Table 1).            */
/* ------------------------------------------------------------------------ */
/* A base triangle V1 V2 V3 carries one marker at its centroid
 * C = (V1 + V2 + V3)/3 (level 0).  The three refinement levels split it into
 * sub-triangles and put one marker at each sub-triangle's centroid:
 *   level 1: L1 = (V1 + V2)/2 splits it in two: (V1, L1, V3), (L1, V2, V3);
 *   level 2: L2 = C splits it in three: (V1, V2, L2), (V2, V3, L2), (V3, V1, L2);
 *   level 3: the edge midpoints L31 = (V1 + V2)/2, L32 = (V2 + V3)/2,
 *            L33 = (V3 + V1)/2 split it in four: (V1, L31, L33), (L31, V2, L32),
 *            (L33, L32, V3), (L31, L32, L33).
 * So level L gives L + 1 markers per base triangle (Table 1: x2, x3, x4).
 * Each marker carries its sub-triangle's flat area and unit normal (right-hand
 * rule on the vertex order).
 * Level of a triangle (the paper asks for a Lagrangian spacing no coarser than
 * the local Eulerian one; the rule is this oracle's reading): l = mean edge
 * length, h = mean of the three widths of the Eulerian cell containing C; a
 * split into m sub-triangles shrinks the length scale by sqrt(m), so the level
 * is the smallest L in 0..3 with l^2 <= ratio^2 h^2 (L + 1), else 3.  A
 * forced level (0..3) applies to every triangle instead. */

static void tri_sub(const double *A, const double *B, const double *C, double *cen, double *area, double *nrm)
{
    double e1[3], e2[3], cr[3];
    for (int d = 0; d < 3; ++d) {
        cen[d] = (A[d] + B[d] + C[d]) / 3.0;
        e1[d] = B[d] - A[d];
        e2[d] = C[d] - A[d];
    }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    *area = 0.5 * len;
    for (int d = 0; d < 3; ++d) nrm[d] = len > 0.0 ? cr[d] / len : 0.0;
}

/* Writes, for each base triangle t (vertex indices tri[3t..3t+2] into the
 * FP32 vertex arrays), its level to tri_level[t] and its L + 1 markers, in
 * triangle order and the sub-triangle order above, to x, y, z, area,
 * normal[3 * m + d] (FP64) and parent[m] = t.  *count receives the marker
 * total.  Errors: a vertex index outside [0, nvert) is ORC_E_ARG, a centroid
 * outside a wall axis ORC_E_SUPPORT, with the triangle in *bad. */
int orc_refine(const double *faces, const int32_t *n, const int32_t *periodic,
               long ntri, const int32_t *tri, long nvert, const float *xv, const float *yv, const float *zv,
               double ratio, int forced_level, double *x, double *y, double *z, double *area, double *normal,
               int32_t *parent, uint8_t *tri_level, long *count, long *bad)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    *bad = -1;
    long m = 0;
    for (long t = 0; t < ntri; ++t) {
        double V[3][3];
        for (int a = 0; a < 3; ++a) {
            long iv = tri[3 * t + a];
            if (iv < 0 || iv >= nvert) { *bad = t; return ORC_E_ARG; }
            V[a][0] = xv[iv]; V[a][1] = yv[iv]; V[a][2] = zv[iv];
        }
        double C[3];
        for (int d = 0; d < 3; ++d) C[d] = (V[0][d] + V[1][d] + V[2][d]) / 3.0;
        int level = forced_level;
        if (level < 0) {
            double h = 0.0;
            for (int d = 0; d < 3; ++d) {
                long ic;
                if (cell_axis(g.f[d], g.n[d], g.periodic[d], C[d], &ic) != ORC_OK) { *bad = t; return ORC_E_SUPPORT; }
                h += g.f[d][ic + 1] - g.f[d][ic];
            }
            h /= 3.0;
            double l = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double *P = V[a], *Q = V[(a + 1) % 3];
                l += sqrt((Q[0] - P[0]) * (Q[0] - P[0]) + (Q[1] - P[1]) * (Q[1] - P[1]) +
                          (Q[2] - P[2]) * (Q[2] - P[2]));
            }
            l /= 3.0;
            level = 3;
            for (int L = 0; L <= 3; ++L) {
                if (l * l <= ratio * ratio * h * h * (double)(L + 1)) { level = L; break; }
            }
        }
        tri_level[t] = (uint8_t)level;
        const double *V1 = V[0], *V2 = V[1], *V3 = V[2];
        double sub[4][3][3];
        int ns = level + 1;
        double L1[3], L31[3], L32[3], L33[3];
        for (int d = 0; d < 3; ++d) {
            L1[d] = 0.5 * (V1[d] + V2[d]);
            L31[d] = 0.5 * (V1[d] + V2[d]);
            L32[d] = 0.5 * (V2[d] + V3[d]);
            L33[d] = 0.5 * (V3[d] + V1[d]);
        }
        for (int d = 0; d < 3; ++d) {
            switch (level) {
            case 0:
                sub[0][0][d] = V1[d]; sub[0][1][d] = V2[d]; sub[0][2][d] = V3[d];
                break;
            case 1:
                sub[0][0][d] = V1[d]; sub[0][1][d] = L1[d]; sub[0][2][d] = V3[d];
                sub[1][0][d] = L1[d]; sub[1][1][d] = V2[d]; sub[1][2][d] = V3[d];
                break;
            case 2:
                sub[0][0][d] = V1[d]; sub[0][1][d] = V2[d]; sub[0][2][d] = C[d];
                sub[1][0][d] = V2[d]; sub[1][1][d] = V3[d]; sub[1][2][d] = C[d];
                sub[2][0][d] = V3[d]; sub[2][1][d] = V1[d]; sub[2][2][d] = C[d];
                break;
            default:
                sub[0][0][d] = V1[d]; sub[0][1][d] = L31[d]; sub[0][2][d] = L33[d];
                sub[1][0][d] = L31[d]; sub[1][1][d] = V2[d]; sub[1][2][d] = L32[d];
                sub[2][0][d] = L33[d]; sub[2][1][d] = L32[d]; sub[2][2][d] = V3[d];
                sub[3][0][d] = L31[d]; sub[3][1][d] = L32[d]; sub[3][2][d] = L33[d];
                break;
            }
        }
        for (int s = 0; s < ns; ++s, ++m) {
            double cen[3], a, nr[3];
            tri_sub(sub[s][0], sub[s][1], sub[s][2], cen, &a, nr);
            x[m] = cen[0]; y[m] = cen[1]; z[m] = cen[2];
            area[m] = a;
            for (int d = 0; d < 3; ++d) normal[3 * m + d] = nr[d];
            parent[m] = (int32_t)t;
        }
    }
    *count = m;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Derivative shape functions (eq. 6 differentiated in the marker position). */
/* ------------------------------------------------------------------------ */
/* The paper lists velocity gradients and pressure at the markers among the
 * MLS operations a moving body needs, without formulas.  Reading used here:
 * the gradient of the MLS approximation u(x) = sum_k phi_k(x) u_k with
 * respect to the marker position x, i.e. the full derivative of eq. 6 in
 * which the weights, and so A and B, move with the marker.  With the basis
 * held fixed at the marker (p(y) = [1, (y - x_l)/H]), at y = x_l:
 *   d Phi^T = dp^T A^-1 B - p^T A^-1 dA A^-1 B + p^T A^-1 dB,
 *   p = e_0, dp = e_{1+d}, dA = sum_k dW_k p_k p_k^T, dB = [dW_k p_k],
 * derivatives taken in the normalised coordinate xi_d = x_d / H_d; a node
 * offset s = (node - x)/H moves by -d xi, so dW_k = -w'(s_{d,k}) times the
 * other two factors.  Pressure lives at cell centres on every axis: its
 * shape functions are those of "component" 3 (no face-staggered axis). */

/* dw/ds of orc_weight_1d (0 where w is clipped to 0). */
double orc_weight_1d_deriv(int kind, double eps, double R, double s)
{
    if (kind == ORC_W_CONST) return 0.0;
    double g = exp(-(s / eps) * (s / eps));
    double dg = -2.0 * s / (eps * eps) * g;
    if (kind == ORC_W_GAUSS) return dg;
    return g - exp(-(R / eps) * (R / eps)) > 0.0 ? dg : 0.0;
}

/* phi[k] as orc_mls_shape and dphi[d * ne + k] = d phi_k / d xi_d. */
int orc_mls_shape_grad(int dim, const double *s, int kind, double eps, double R, double *phi, double *dphi)
{
    if (dim != 2 && dim != 3) return ORC_E_ARG;
    const int m = dim + 1;
    const int ne = dim == 2 ? 9 : 27;
    double A[16] = {0}, dA[3][16], B[4 * 27], dB[3][4 * 27];
    memset(dA, 0, sizeof(dA));
    for (int k = 0; k < ne; ++k) {
        double p[4], w[3], wd[3];
        int kk = k;
        p[0] = 1.0;
        for (int d = 0; d < dim; ++d) {
            int a = kk % 3; kk /= 3;
            p[1 + d] = s[d * 3 + a];
            w[d] = orc_weight_1d(kind, eps, R, s[d * 3 + a]);
            wd[d] = orc_weight_1d_deriv(kind, eps, R, s[d * 3 + a]);
        }
        double W = 1.0;
        for (int d = 0; d < dim; ++d) W *= w[d];
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) A[i * m + j] += W * p[i] * p[j];
            B[i * ne + k] = W * p[i];
        }
        for (int d = 0; d < dim; ++d) {
            double dW = -wd[d];
            for (int e = 0; e < dim; ++e)
                if (e != d) dW *= w[e];
            for (int i = 0; i < m; ++i) {
                for (int j = 0; j < m; ++j) dA[d][i * m + j] += dW * p[i] * p[j];
                dB[d][i * ne + k] = dW * p[i];
            }
        }
    }
    /* T = A^-1 B, gamma = A^-1 e_0 (A symmetric, so p^T A^-1 = gamma^T) */
    double Ac[16], T[4 * 27], gam[4] = {1.0, 0.0, 0.0, 0.0};
    memcpy(Ac, A, sizeof(A));
    memcpy(T, B, sizeof(double) * m * ne);
    int rc = gepp_solve(m, Ac, ne, T);
    if (rc != ORC_OK) return rc;
    memcpy(Ac, A, sizeof(A));
    rc = gepp_solve(m, Ac, 1, gam);
    if (rc != ORC_OK) return rc;
    for (int k = 0; k < ne; ++k) phi[k] = T[k];
    for (int d = 0; d < dim; ++d) {
        for (int k = 0; k < ne; ++k) {
            double v = T[(1 + d) * ne + k];                 /* dp^T A^-1 B */
            for (int i = 0; i < m; ++i) {
                double dAT = 0.0;
                for (int j = 0; j < m; ++j) dAT += dA[d][i * m + j] * T[j * ne + k];
                v -= gam[i] * dAT;                           /* - p^T A^-1 dA A^-1 B */
                v += gam[i] * dB[d][i * ne + k];             /* + p^T A^-1 dB */
            }
            dphi[d * ne + k] = v;
        }
    }
    return ORC_OK;
}

/* Per marker, for staggering comp (0, 1, 2: the u, v, w grids; 3: cell
 * centres): home[l*3 + d], phi[l*27 + k] and dphi[(l*3 + d)*27 + k] =
 * d phi_k / d x_d in physical units.  Errors as orc_build_exact. */
int orc_build_grad(const double *faces, const int32_t *n, const int32_t *periodic,
                   int comp, int kind, double eps, double R,
                   long nm, const float *x, const float *y, const float *z,
                   int32_t *home, double *phi, double *dphi, long *bad)
{
    grid3 g;
    grid_unpack(faces, n, periodic, &g);
    int first_rc = ORC_OK;
    long first_bad = -1;
    if (comp < 0 || comp > 3) return ORC_E_ARG;
    #pragma omp parallel for schedule(static)
    for (long l = 0; l < nm; ++l) {
        double xl[3] = {x[l], y[l], z[l]};
        long h[3], ihu[3];
        orc_axis_geo geo[3];
        int rc = marker_geometry(&g, comp, xl, h, geo, ihu);
        double s[9], dxi[3 * 27];
        if (rc == ORC_OK) {
            for (int d = 0; d < 3; ++d)
                for (int a = 0; a < 3; ++a) s[d * 3 + a] = geo[d].s[a];
            rc = orc_mls_shape_grad(3, s, kind, eps, R, phi + l * 27, dxi);
        }
        if (rc != ORC_OK) {
            #pragma omp critical
            {
                if (first_bad < 0 || l < first_bad) { first_bad = l; first_rc = rc; }
            }
            for (int k = 0; k < 27; ++k) phi[l * 27 + k] = NAN;
            for (int k = 0; k < 81; ++k) dphi[l * 81 + k] = NAN;
            for (int d = 0; d < 3; ++d) home[l * 3 + d] = -1;
            continue;
        }
        for (int d = 0; d < 3; ++d) {
            home[l * 3 + d] = (int32_t)h[d];
            for (int k = 0; k < 27; ++k) dphi[(l * 3 + d) * 27 + k] = dxi[d * 27 + k] / geo[d].H;
        }
    }
    if (bad) *bad = first_bad;
    return first_rc;
}
