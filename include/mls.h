/*
 * mls.h -- C ABI of the MI355X moving-least-squares immersed-boundary
 * transfer library (libmls_hip.so).
 *
 * Method: V. Spandan, D. Lohse, M. D. de Tullio, R. Verzicco, "A fast moving
 * least squares approximation with adaptive Lagrangian mesh refinement for
 * large scale immersed boundary simulations", arXiv:1805.01113, Sec. 2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Marker and field arrays are DEVICE pointers owned by the caller; the
 *    library never frees them and never allocates caller-visible memory.
 *    Host pointers appear only in mls_grid (copied at context creation) and in
 *    the out-parameters of mls_sync / mls_stats_get / mls_*_info.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Every
 *    compute entry point only enqueues work on that stream and returns.
 *  - Argument errors are detected on the host and returned at once, nothing
 *    is enqueued.  Errors found on the device (support outside a wall axis,
 *    singular moment matrix, out-of-range force) set a sticky device error
 *    word holding the lowest offending marker index; mls_sync reports it.
 *  - Staggered grid (marker-and-cell): velocity component c (0=u, 1=v, 2=w)
 *    lives on the cell faces along axis c and on the cell centres along the
 *    other two axes.  Axis d has n[d] cells with face coordinates
 *    faces[d][0..n[d]].  On a periodic axis a component has n[d] nodes; on a
 *    wall axis the face component has n[d]+1 nodes (both walls included).
 *    Fields are C-order arrays [z][y][x] of FP32 over a component's nodes.
 *  - Support (Sec. 2, text of figure 1): the home node of the marker plus its
 *    neighbours, 3 per axis (N_e = 27), on each component's own grid.  The
 *    home node is the one whose control volume contains the marker
 *    (half-open [lo, hi): ties go to the upper node).  A centre node owns its
 *    cell; a face node owns the interval between the two adjacent centres.
 *    Periodic coordinates are wrapped in FP64.
 *  - Shape-function layout (SoA inside blocks of 64 markers, one wavefront):
 *    with npad = n rounded up to a multiple of 64, b = l / 64 and r = l % 64,
 *      phi[((b*3 + c)*27 + k)*64 + r]   (81 * npad floats)
 *    is the FP32 weight of support node k of marker l for component c, with
 *    k = (a_x+1) + 3 (a_y+1) + 9 (a_z+1) and a_d in {-1,0,1} the node offset
 *    from the home node;
 *      home[(b*3 + c)*64 + r]           (3 * npad uint32)
 *    packs the wrapped home node indices of component c as
 *    i | j << 11 | k << 22 (a component grid may have at most
 *    2048 x 2048 x 1024 nodes); route flags use the layout of home.
 *    Padding entries past n are never read or written.
 *  - Calls on one context are not thread-safe; issue them from one thread.
 */
#ifndef MLS_H
#define MLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mls_ctx mls_ctx;

typedef enum {
    MLS_OK = 0,
    MLS_E_ARG = -1,        /* invalid argument (host check) */
    MLS_E_SUPPORT = -2,    /* a 3-node support leaves a wall axis (device) */
    MLS_E_SINGULAR = -3,   /* moment matrix not positive definite even in FP64 (device) */
    MLS_E_NONFINITE = -4,  /* non-finite marker coordinate (device) */
    MLS_E_HIP = -5,        /* HIP runtime error */
    MLS_E_NOMEM = -6,      /* device allocation failed */
    MLS_E_RANGE = -7       /* a spread contribution exceeds the fixed-point range (device) */
} mls_status;

typedef enum {
    MLS_W_GAUSS_SHIFTED = 0, /* w(s) = max(0, exp(-(s/eps)^2) - exp(-(R/eps)^2)) per axis (default) */
    MLS_W_GAUSS = 1,         /* w(s) = exp(-(s/eps)^2) per axis */
    MLS_W_CONST = 2          /* w = 1 */
} mls_weight_kind;

typedef enum {
    MLS_EXACT = 0,   /* eq. 3-6 per marker */
    MLS_FAST = 1,    /* eq. 9-10: Shepard blend of a sub-node table */
    MLS_LEARNED = 2, /* MLP surrogate with exact-MLS fallback */
    MLS_FAST_LINEAR = 3  /* the fast-MLS tables with a trilinear blend (beyond the paper) */
} mls_method;

/* The Eulerian grid as the paper states the problem (Sec. 2): per axis the
 * cell count, a periodic flag and the n[d]+1 increasing face coordinates
 * (HOST pointers, FP64, copied by mls_ctx_create).  At most one axis may be
 * non-uniform (the paper's grid stretched in one direction). */
typedef struct {
    int32_t n[3];
    int32_t periodic[3];
    const double *faces[3];
} mls_grid;

/* Weight function W of eq. 2-4 as a tensor product of 1-D weights of the
 * node offset s measured in units of the local spacing H_d = half the
 * distance between the outer support nodes on axis d.  The paper leaves the
 * form open (Sec. 2, after eq. 2); eps = 1, radius = 1.5 is the default. */
typedef struct {
    int32_t kind;     /* mls_weight_kind */
    double eps;
    double radius;
} mls_weight;

typedef struct {
    double kappa_tau;     /* FP32 moment-matrix solves whose condition-number
                             bound ||A||_F ||L^-1||_F^2 (>= kappa_2(A), A = L L^T)
                             exceeds this are redone in FP64 (default 1e6;
                             0 routes every solve to FP64) */
    int32_t n_sub;        /* fast-MLS sub-nodes per axis of the home control
                             volume, boundaries included (default 9 -> 729) */
    double fallback_tol;  /* learned: a marker keeps the network's shape
                             functions only if its consistency residual is
                             below this, else it falls back to exact MLS
                             (default 1e-4; 0 sends every marker to exact) */
    int32_t spread_tile;  /* edge (cells) of the spreading tiles on axes longer
                             than 16 cells, 4..16 (0 = default 8); a periodic
                             axis uses a divisor of its length */
} mls_opts;

typedef struct {
    int64_t fp64_solves;     /* (marker, component) solves routed to FP64 */
    int64_t fallbacks;       /* learned: (marker, component) fallbacks to exact */
    int64_t learned;         /* learned: (marker, component) accepted */
    double kappa_max;        /* largest FP32 condition-number bound seen (0 if none) */
    int64_t spread_entries;  /* (tile, marker) pairs of the last spread */
    int64_t spread_tiles;    /* tiles of the forcing grid */
} mls_stats;

/* Library version string: "mls_hip <version> (gfx950) src <sha256>", the
   last field the SHA-256 of the HIP sources and this header the library was
   compiled from ("unstamped" for a build outside the package's build step).
   Static storage; never NULL. */
const char *mls_version(void);

/* Create a context on the current HIP device for one grid, weight and
 * option set.  Copies the grid (host FP64) to the device, precomputes node
 * coordinates and control-volume widths, and sizes the spreading tiles.
 * weight/opts may be NULL for the defaults.  Returns MLS_E_ARG for a grid
 * that is not increasing, has fewer than 3 cells on an axis, exceeds the
 * packed-index limits, or has a periodic axis longer than 16 cells whose cell
 * count has no divisor between 4 and 16 (the spreading tiles). */
mls_status mls_ctx_create(mls_ctx **ctx, const mls_grid *grid, const mls_weight *weight,
                          const mls_opts *opts);
void mls_ctx_destroy(mls_ctx *ctx);

/* Reserve device scratch for up to n_markers markers so that later calls
 * with at most that many markers allocate nothing (needed before capturing
 * a step in a HIP graph). */
mls_status mls_reserve(mls_ctx *ctx, int64_t n_markers);

/* Transfer-function build (Sec. 2, eq. 1-6 exact; eq. 9-10 fast).
 * For n markers at x,y,z (device FP32 SoA, any position on periodic axes):
 * writes home (3 * npad, packed home indices, see above), phi (81 * npad FP32
 * shape functions, Phi^T = p^T A^-1 B of eq. 6 in marker-centred, spacing-
 * scaled coordinates, which gives the same Phi as the paper's absolute basis)
 * and, if route != NULL, route (3 * npad; bit 0: FP64 solve, bit 1: learned
 * accepted, bit 2: learned fell back to exact).  MLS_EXACT assembles the 4x4
 * moment matrix A = sum_k W_k p_k p_k^T (eq. 3) per (marker, component),
 * solves it in FP32 (Cholesky) and redoes the solve in FP64 when the bound
 * ||A||_F ||L^-1||_F^2 of its 2-norm condition number exceeds
 * opts.kappa_tau.  MLS_FAST builds, on first use, the tables of exact
 * shape functions at the n_sub^3 sub-nodes of the home control volume (one
 * table on a uniform grid, one per plane and staggering type along a
 * stretched axis, Sec. 2 last paragraph) and blends the 8 corners of the
 * enclosing sub-cell with inverse-square-distance (Shepard) weights, eq. 9-10.
 * MLS_FAST_LINEAR blends the same 8 rows with the multilinear weights of the
 * marker inside the sub-cell; the weights sum to one and reproduce the
 * position, so the tables' partition of unity and exact reproduction of
 * linear fields carry over (second-order error in the sub-cell size).
 * MLS_LEARNED evaluates the loaded network (mls_mlp_load) and keeps its
 * output where the residual max(|sum_k phi_k - 1|, max_d |sum_k phi_k s_dk|)
 * (partition of unity and reproduction of linear fields, the consistency
 * conditions of MLS with a linear basis; s_dk the offset of node k from the
 * marker along d in units of H_d) is below opts.fallback_tol, and builds the
 * other markers with exact MLS (route bit 2).  Markers whose
 * support leaves a wall axis get NaN phi and raise MLS_E_SUPPORT. */
mls_status mls_build(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                     int32_t method, uint32_t *home, float *phi, uint8_t *route, void *stream);

/* Interpolation Q = Phi^T q (eq. 6) of the three staggered velocity fields
 * u, v, w (device FP32, component grids as above) onto the n markers:
 * U[l] = sum_k phi[0][k][l] u[node_k], likewise V from v, W from w.
 * home/phi as written by mls_build.  Outputs are FP32 device arrays of n. */
mls_status mls_interp(mls_ctx *ctx, int64_t n, const uint32_t *home, const float *phi,
                      const float *u, const float *v, const float *w,
                      float *U, float *V, float *W, void *stream);

/* Conservative spreading (eq. 7-8) of marker forces onto the grid, ADDED into
 * fx, fy, fz (device FP32 component fields; zeroing them is the caller's):
 *   h_l = sum_k phi_k (dx_k + dy_k + dz_k)/3,  dV_l = A_l h_l,
 *   c_l = dV_l / sum_k phi_k dV_k,            f_k += c_l phi_k F_l,
 * with dx_k, dy_k, dz_k the control-volume widths of support node k on the
 * component's grid and dV_k = dx_k dy_k dz_k.  area = A_l (device FP32, n).
 * The result is bitwise reproducible and independent of the marker order:
 * markers are binned (counting sort) by the tile of the forcing grid that
 * holds their cell; a tile sums its markers' contributions in 64-bit fixed
 * point in a box covering the tile and its one-node halo (one component at a
 * time); tiles are coloured by the parity of their index per axis (a third
 * colour for the last tile of a periodic axis with an odd tile count) so that
 * boxes of one colour never overlap, and the colours add their boxes into the
 * field one after another.  The fixed-point scale is chosen per tile and
 * component from the largest finite |c_l F_l| of the tile's markers (its
 * quantum is 2^-30 of 4 times that value), so weak forces keep their
 * precision beside strong ones elsewhere on the grid.  A non-finite
 * c_l F_l, or a contribution beyond the bound (a shape function with
 * |phi_k| > 4), raises MLS_E_RANGE at that marker. */
mls_status mls_spread(mls_ctx *ctx, int64_t n, const uint32_t *home, const float *phi,
                      const float *area, const float *Fx, const float *Fy, const float *Fz,
                      float *fx, float *fy, float *fz, void *stream);

/* Fixed size of the library's scratch array for mls_spread_noalloc (bytes). */
#define MLS_SPREAD_NOALLOC_BYTES (64u << 20)

/* mls_spread for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, arithmetic, result (bitwise equal to mls_spread's) and errors,
 * but it calls no hipMalloc, hipFree or allocating library routine and never
 * grows the context.  Its scratch (tile counts and offsets, binned marker
 * entries, c_l F_l per marker, per-tile maxima) lives in one fixed device
 * array of MLS_SPREAD_NOALLOC_BYTES in the library, one copy per GPU, held
 * from the first context created on that GPU (mls_ctx_create takes its
 * address) until the process ends.  It needs about
 *   20 bytes per marker + 28 bytes per spreading tile of the grid
 * (plus 256-byte alignment of each part); a call that needs more returns
 * MLS_E_ARG with a message and launches nothing.  Every call on one GPU
 * shares that GPU's array and overwrites it (whatever must start at zero is
 * cleared by the call's own kernels): calls that overlap on one GPU, from
 * any context or stream, race, so order them on one stream or synchronise
 * between them. */
mls_status mls_spread_noalloc(mls_ctx *ctx, int64_t n, const uint32_t *home, const float *phi,
                              const float *area, const float *Fx, const float *Fy, const float *Fz,
                              float *fx, float *fy, float *fz, void *stream);

/* Derivative shape functions: the gradient with respect to the marker
 * position x of the exact MLS shape functions of eq. 6, Phi(x) =
 * W(x) p^T A(x)^-1 B(x), the weights (and so A and B) moving with the marker;
 * the paper asks for velocity gradients and pressure at the markers of
 * moving bodies without giving formulas, and this is the full derivative of
 * its approximation.  stagger selects the node set: 0, 1, 2 the u, v, w grids
 * as in mls_build, 3 the cell centres on every axis (pressure).  Writes, in
 * the 64-marker blocked layout (npad = n rounded up to 64): home[l] packed as
 * in mls_build (npad entries), phi[(b*27 + k)*64 + r] (27 npad) and
 * dphi[((b*3 + d)*27 + k)*64 + r] = d phi_k / d x_d in physical units
 * (81 npad), l = 64 b + r; padding lanes get home 0xffffffff and zeros.  The
 * solve is FP32 with the condition bound of mls_build, redone in FP64 from
 * the position above opts.kappa_tau (counted in mls_stats fp64_solves).
 * Support errors as mls_build. */
mls_status mls_build_grad(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                          int32_t stagger, uint32_t *home, float *phi, float *dphi, void *stream);

/* Fused value and gradient of the MLS approximation at the markers (no shape
 * functions stored): for the staggered velocity fields u, v, w (device FP32,
 * component grids as in mls_interp) U[c][l] (if U != NULL, [3][n]) and
 * G[3c + d][l] = d u_c / d x_d ([9][n]); if p != NULL (device FP32 cell-centred
 * field, [n_z][n_y][n_x] over the cells) also P[l] = p at the marker and
 * GP[d][l] = d p / d x_d (either may be NULL).  Same arithmetic and errors as
 * mls_build_grad. */
mls_status mls_interp_grad(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                           const float *u, const float *v, const float *w, float *U, float *G, const float *p,
                           float *P, float *GP, void *stream);

/* Coarse-grained collision detection (Sec. 4, the integer cell array of its
 * detection algorithm).  coll is a device int32 array with one entry per
 * Eulerian cell, C order [z][y][x] over the n_z x n_y x n_x cells of the
 * context's grid (cells, not velocity nodes), holding only zeros on entry (a
 * fresh array, or one returned to zero by mls_collide_clear).  Marker l
 * (device FP32 x, y, z) belongs to body body[l] (device int32,
 * 0 <= body[l] <= 2^31 - 2) and lies in the cell with f[i] <= X < f[i+1]
 * along each axis (X wrapped on a periodic axis).  On return a cell holds 0
 * where no marker lies, body + 1 where markers of one body only lie and -1
 * where markers of two or more bodies lie; if flags (device uint8 of n) is
 * non-NULL, flags[l] = 1 where the cell of marker l holds -1 (the markers a
 * collision force applies to), else 0.  The result is independent of marker
 * order and scheduling, bit for bit.  Device errors (mls_sync, lowest marker
 * first): a marker with a non-finite coordinate or outside a wall axis raises
 * MLS_E_SUPPORT, a body id out of range MLS_E_ARG; such markers are left out
 * and get flag 0.  Cost O(n): three cell lookups per marker, one
 * compare-and-swap. */
mls_status mls_collide(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                       const int32_t *body, int32_t *coll, uint8_t *flags, void *stream);

/* Returns to zero the entries of coll at the cells of the n markers at x, y, z
 * (the positions given to mls_collide), so that the array can be reused
 * without clearing every cell: O(n), not O(cells). */
mls_status mls_collide_clear(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                             int32_t *coll, void *stream);

/* Adaptive Lagrangian mesh refinement (Sec. 3, Fig. 5, Table 1): markers
 * for the interfacial condition generated from a base triangle mesh.
 * tri (device int32 [ntri][3]) indexes the nvert vertices xv, yv, zv
 * (device FP32).  Base triangle V1 V2 V3 gets a level L in 0..3 and L + 1
 * markers, one at the centroid of each sub-triangle, with the sub-triangle's
 * flat area and unit normal (right-hand rule on the vertex order):
 *   L = 0: the triangle itself (marker at C = (V1 + V2 + V3)/3);
 *   L = 1: split at L1 = (V1 + V2)/2 into (V1, L1, V3), (L1, V2, V3);
 *   L = 2: split at C into (V1, V2, C), (V2, V3, C), (V3, V1, C);
 *   L = 3: split at the edge midpoints L31 = (V1 + V2)/2, L32 = (V2 + V3)/2,
 *          L33 = (V3 + V1)/2 into (V1, L31, L33), (L31, V2, L32),
 *          (L33, L32, V3), (L31, L32, L33).
 * level = -1 chooses per triangle the smallest L with
 * l^2 <= ratio^2 h^2 (L + 1), at most 3, where l is the mean edge length and
 * h the mean of the three widths of the Eulerian cell containing C (a split
 * into L + 1 parts shrinks the length scale by sqrt(L + 1); ratio is the
 * largest Lagrangian-to-Eulerian spacing kept, ratio > 0); level = 0..3
 * forces that level on every triangle.  Outputs (device, capacity >= 4 ntri
 * entries each; normal is [3][capacity]): markers in triangle order, then
 * sub-triangle order as listed, x, y, z, area, normal, parent (base triangle
 * index); tri_level (device uint8 [ntri]) the levels; *count (device int64)
 * the number of markers written.  Geometry is evaluated in FP64 from the FP32
 * vertices and rounded to FP32 once.  Device errors: a vertex index outside
 * [0, nvert) raises MLS_E_ARG, a centroid with no Eulerian cell (adaptive
 * level only) MLS_E_SUPPORT, with the lowest triangle index; such a triangle
 * gets level 0 (NaN marker for a bad index).  May allocate a small scratch
 * buffer on first use or growth (not while a graph is captured). */
mls_status mls_refine(mls_ctx *ctx, int64_t ntri, const int32_t *tri, int64_t nvert, const float *xv,
                      const float *yv, const float *zv, double ratio, int32_t level, int64_t capacity, float *x,
                      float *y, float *z, float *area, float *normal, int32_t *parent, uint8_t *tri_level,
                      int64_t *count, void *stream);

/* Synchronise `stream`, then report and clear the device error word.
 * Returns MLS_OK or the device error; *first_bad (if non-NULL) receives the
 * lowest offending marker index (or -1). */
mls_status mls_sync(mls_ctx *ctx, void *stream, int64_t *first_bad);

/* Human-readable description of the last error on this context. */
const char *mls_last_error(const mls_ctx *ctx);

/* Counters accumulated since creation or the last reset (synchronises the
 * device). */
mls_status mls_stats_get(mls_ctx *ctx, mls_stats *out);
mls_status mls_stats_reset(mls_ctx *ctx);

/* fast-MLS tables (built on first use; this call builds them if needed).
 * Reports count tables of n_sub^3 rows of row_stride floats each (the 27
 * shape-function values of a sub-node, then padding), sub-node index
 * s = jx + n_sub (jy + n_sub jz).  Table t holds home plane t - first[type]
 * along the stretched axis (type 0: centre-staggered components, 1: the
 * face-staggered one); on a uniform grid there is one table for all
 * components and *stretched_axis = -1.  If dst is not NULL, all tables are
 * copied into it (device, count * n_sub^3 * row_stride floats) on stream. */
mls_status mls_fast_tables(mls_ctx *ctx, float *dst, int64_t *count, int32_t *row_stride,
                           int32_t first[2], int32_t *stretched_axis, void *stream);

/* ---- one immersed-boundary time step (batched over all bodies) ----------
 * Markers of all bodies are stored back to back (any number of bodies of any
 * size); every phase is one grid-stride launch over the whole marker array.
 * A step runs, in order on `stream`:
 *   jitter   x = x0 + delta, delta uniform in [-jitter, jitter) per axis from a
 *            counter-based generator (the SplitMix64 output function applied to
 *            seed + (counter + 1) * 0x9E3779B97F4A7C15 with
 *            counter = (step * n + marker) * 3 + axis, top 24 bits), skipped
 *            when jitter == 0 (then x0 is built directly);
 *   build    mls_build with `method`;
 *   interp   U = Phi^T u (eq. 6);
 *   force    F = (V_b - U) / dt, the direct forcing of Sec. 2 (V_b = 0 if NULL);
 *   spread   f += c_l phi F (eq. 7-8);
 * and then increments the context's device step counter, which the jitter
 * of the next step reads.  With MLS_EXACT, with fast-MLS on a grid whose
 * axes are all uniform, and with MLS_LEARNED, the step works in
 * spreading-tile order: markers are binned by the tile of their cell (the
 * jitter runs inside that pass, with the same generator), row p of the
 * blocked home / phi / route layout holds marker order[p] (see
 * mls_step_order), so that the tiles read their rows contiguously, and U and
 * F stay indexed by marker.  The exact and fast-MLS builds run fused with the
 * interpolation and forcing (phi is not read back); the learned build
 * stores its rows and interpolates and forces from a copy of them in LDS
 * in the same kernel.  Markers whose support
 * leaves the grid come last.  The order of the markers inside a tile may
 * differ between runs; U, F and the forcing do not.  With the other methods
 * (and fast-MLS on a stretched grid) rows are in marker order.  All buffers are caller-owned device arrays:
 * x0,y0,z0 [n] (read), x,y,z [n] (written by jitter), area [n], vb [3][n] or
 * NULL, home, phi and route (or NULL) in the blocked layout above, U [3][n], F [3][n],
 * the velocity fields u,v,w and the forcing fields fx,fy,fz.
 *
 * flags MLS_STEP_COMPACT (MLS_EXACT only; ignored by the other methods): the
 * step keeps each (marker, component) transfer function in its defining
 * quantities instead of its 27 values -- gamma = A^{-1} e_0 of eq. 5 and the
 * support offsets (one per axis when all axes are uniform, else three) -- in
 * context scratch, and the spreading evaluates phi_k = W_k (gamma . p_k)
 * from them with the build's arithmetic, so it spreads with the values the
 * interpolation used.  phi then receives only the rows of the pairs solved
 * in FP64; its other rows are left as they were.  Results (U, F, forcing)
 * are those of the default step. */
enum { MLS_STEP_COMPACT = 1 };

typedef struct {
    int32_t method;
    float dt;
    float jitter;
    uint64_t seed;
    int32_t flags;     /* 0 or MLS_STEP_COMPACT */
} mls_step_desc;

typedef struct {
    int64_t n;
    const float *x0, *y0, *z0;
    float *x, *y, *z;
    const float *area;
    const float *vb;
    uint32_t *home;
    float *phi;
    uint8_t *route;
    const float *u, *v, *w;
    float *U;
    float *F;
    float *fx, *fy, *fz;
} mls_step_buffers;

/* Enqueue one step.  Reserves scratch on first use for n markers. */
mls_status mls_step(mls_ctx *ctx, const mls_step_desc *desc, const mls_step_buffers *buf, void *stream);

/* Copy the row order of the last step in spreading-tile order (MLS_EXACT,
 * fast-MLS on a uniform grid, MLS_LEARNED) of n markers into order (device,
 * n uint32): row p of its home / phi / route holds marker order[p].
 * MLS_E_ARG if that step had a different marker count. */
mls_status mls_step_order(mls_ctx *ctx, uint32_t *order, int64_t n, void *stream);

/* Set the device step counter read by the jitter (enqueued on stream). */
mls_status mls_step_counter_set(mls_ctx *ctx, uint64_t step, void *stream);

/* A step captured once as a HIP graph and replayed: the capture contains no
 * allocation, no memset node and no host synchronisation, so a replay costs
 * one graph launch.  The buffers are baked into the graph; they must stay
 * allocated until mls_graph_destroy.  So is the context's scratch: after it
 * grows (mls_reserve or a step with more markers than any before) or the
 * spreading tile changes (mls_tune_set, mls_autotune), mls_graph_launch
 * returns MLS_E_ARG and the graph must be created again. */
typedef struct mls_graph mls_graph;
mls_status mls_graph_create(mls_ctx *ctx, const mls_step_desc *desc, const mls_step_buffers *buf,
                            mls_graph **out);
mls_status mls_graph_launch(mls_graph *graph, int32_t n_steps, void *stream);
void mls_graph_destroy(mls_graph *graph);

/* ---- per-kernel timing (HIP events on the launch stream) -----------------
 * When enabled, the library records a HIP event pair around each launch of
 * the kernels below (not inside a graph capture); mls_timing_get
 * synchronises and returns the summed milliseconds and launch counts.  In a
 * step in spreading-tile order, MLS_K_SPREAD_BIN covers the binning (with
 * the jitter inside it) and MLS_K_BUILD_INTERP the fused build with, for
 * compact rows, the pass that finishes the rows solved in FP64; MLS_K_JITTER
 * then records nothing. */
enum {
    MLS_K_BUILD_EXACT = 0, MLS_K_BUILD_FAST = 1, MLS_K_BUILD_LEARNED = 2, MLS_K_INTERP = 3,
    MLS_K_SPREAD_BIN = 4, MLS_K_SPREAD_TILES = 5, MLS_K_JITTER = 6, MLS_K_FORCE = 7,
    MLS_K_BUILD_INTERP = 8,  /* exact build fused with interpolation and forcing (mls_step, MLS_EXACT) */
    MLS_K_COLLIDE = 9, MLS_K_COLLIDE_CLEAR = 10, MLS_K_REFINE = 11, MLS_K_BUILD_GRAD = 12, MLS_K_INTERP_GRAD = 13,
    MLS_K_FAST_INTERP = 14,  /* fast-MLS fused with interpolation and forcing (mls_step, uniform grids) */
    MLS_K_COUNT = 16
};
typedef struct {
    double ms[MLS_K_COUNT];
    int64_t launches[MLS_K_COUNT];
} mls_timing;
mls_status mls_timing_enable(mls_ctx *ctx, int32_t on);
mls_status mls_timing_get(mls_ctx *ctx, mls_timing *out, int32_t reset);

/* ---- launch shapes and the autotuner (an addition to the paper's method) ---
 * spread_tile: edge of the spreading tiles (4..16, as mls_opts.spread_tile);
 * *_blocks_per_cu (1..64): workgroups per compute unit in the grid of the
 * spreading tile launches (bounded further by the LDS of a tile's boxes), of
 * the exact / fast build and of the interpolation; a grid-stride loop covers
 * the work beyond the grid.  spread_threads (128, 192 or 256): threads of a
 * spreading tile workgroup (fewer suit many tiles per workgroup, more suit
 * few). */
typedef struct {
    int32_t spread_tile;
    int32_t spread_blocks_per_cu;
    int32_t build_blocks_per_cu;
    int32_t interp_blocks_per_cu;
    int32_t spread_threads;
} mls_tune;

typedef struct {
    mls_tune best;           /* the shapes now applied */
    double ms_build;         /* their time per call (ms) of each phase */
    double ms_interp;
    double ms_spread;        /* binning and tiles */
    int32_t from_cache;      /* 1: taken from the cache file, nothing timed */
    int32_t candidates;      /* shapes timed */
} mls_tune_report;

mls_status mls_tune_get(mls_ctx *ctx, mls_tune *out);

/* Apply launch shapes.  A new spread_tile re-cuts the spreading tiles
 * (capture step graphs after this call).  MLS_E_ARG for a value out of range
 * or a tile edge the grid does not allow (the previous shapes stay). */
mls_status mls_tune_set(mls_ctx *ctx, const mls_tune *in);

/* Time candidate launch shapes of the build (method), the interpolation and
 * the spreading on the caller's step buffers (n, x0, y0, z0, area, vb, home,
 * phi, u, v, w, U, F, fx, fy, fz as for mls_step; markers at x0), keep the
 * fastest of each phase and apply them.  flags are the step flags the shapes
 * are for (MLS_STEP_COMPACT times the compact exact build and spreading; other
 * methods ignore it; other bits: MLS_E_ARG).  cache_path (may be NULL) names a
 * JSON-lines file: an entry whose key (device architecture, compute units,
 * grid, periodic flags, stretched axis, method, flags, floor(log2 n)) matches
 * is applied without timing; otherwise the result is appended.  home, phi, U and
 * F are overwritten and the forcing fields receive the contributions of the
 * timed spreading calls (zero them afterwards).  Synchronises `stream`. */
mls_status mls_autotune(mls_ctx *ctx, int32_t method, int32_t flags, const mls_step_buffers *buf,
                        const char *cache_path, mls_tune_report *out, void *stream);

/* ---- learned surrogate (an addition to the paper's method) ----------------
 * A network 6 -> 128 -> 128 -> 27 maps the features of a (marker, component)
 * support -- xi_d = (X - X_0)/H_d (in-cell offset, H_d = half the support
 * width on axis d) and rho_d = (X_{+1} - X_0)/(X_0 - X_{-1}) (spacing ratio),
 * d = x, y, z, which fix the exact shape function of eq. 3-6 -- to its 27
 * shape-function values:
 *   u = (feat - shift) * scale,  h1 = gelu(u W1 + b1),  h2 = gelu(h1 W2 + b2),
 *   phi = h2 W3 + b3,            gelu(z) = z Phi(z) (Phi: standard normal CDF).
 * Parameters are one FP32 vector of MLS_MLP_PARAMS floats: W1 [6][128], b1
 * [128], W2 [128][128], b2 [128], W3 [128][27], b3 [27], each W stored
 * [input][output] row-major; the input normalisation is norm[12] = shift[6],
 * scale[6].  Matrix products run on the matrix cores in split BF16 (each FP32
 * operand as a high plus a low BF16 part, three products accumulated in FP32).
 * Training minimises
 *   L = mean_{b,k} (phi_bk - t_bk)^2
 *       + mu mean_b [(sum_k phi_bk - 1)^2 + sum_d (sum_k phi_bk s_dk)^2]
 * with Adam (beta1 0.9, beta2 0.999, eps 1e-8). */
#define MLS_MLP_PARAMS 20891

/* Load parameters and normalisation (HOST pointers, copied) and reset the
 * Adam state.  MLS_E_ARG on a non-finite value. */
mls_status mls_mlp_load(mls_ctx *ctx, const float *params, const float *norm);

/* Copy the current parameters (MLS_MLP_PARAMS floats) and normalisation (12)
 * to HOST memory (either may be NULL); synchronises the device. */
mls_status mls_mlp_get(mls_ctx *ctx, float *params, float *norm);

/* Features of n markers (device x, y, z): feat[(c n + l) 6 + q] (device FP32,
 * 3 n rows of 6) for component c = 0, 1, 2; a row whose support leaves the
 * grid is NaN and raises MLS_E_SUPPORT. */
mls_status mls_features(mls_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, float *feat,
                        void *stream);

/* Network output out[b][27] (device FP32) for a batch of m entries taken
 * from the feature rows feat[rows][6] (device FP32): entry b is row idx[b]
 * if idx (device int64, m entries) is not NULL, else row b (then m <= rows).
 * An idx entry outside [0, rows) raises MLS_E_ARG on the device (mls_sync
 * reports it) and reads row 0. */
mls_status mls_mlp_forward(mls_ctx *ctx, int64_t m, const float *feat, int64_t rows, const int64_t *idx,
                           float *out, void *stream);

/* Loss L (above) and its gradient dL/dparams of a batch of m >= 1 entries,
 * rows chosen as in mls_mlp_forward from feat [rows][6] and target
 * [rows][27] (device FP32); grad: device MLS_MLP_PARAMS floats in the
 * parameter layout, loss: device float.  Every reduction runs in a fixed
 * order, so equal inputs give equal results bit for bit. */
mls_status mls_mlp_grad(mls_ctx *ctx, int64_t m, const float *feat, const float *target, int64_t rows,
                        const int64_t *idx, float mu, float *grad, float *loss, void *stream);

/* One Adam step with learning rate lr on the gradient of the batch as in
 * mls_mlp_grad; loss (device float) may be NULL.  A later MLS_LEARNED build
 * uses the updated parameters. */
mls_status mls_mlp_train_step(mls_ctx *ctx, int64_t m, const float *feat, const float *target, int64_t rows,
                              const int64_t *idx, float mu, float lr, float *loss, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MLS_H */
