// Internal declarations of the MI355X MLS transfer library.
//
// Device-side grid description, the device error word, the context and the
// kernel launchers shared by the translation units.  Nothing here is part of
// the C ABI (include/mls.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mls.h"

namespace mls {

constexpr int kNe = 27;           // 3x3x3 support nodes
constexpr int kTableStride = 28;  // table row: 27 values + 1 pad (16-byte rows)
constexpr int kMaxTile = 16;      // a periodic axis of up to this many cells is one spreading tile
constexpr int kMaxBoxTile = 16;   // largest tile edge cut from a longer axis (an int64 box of edge + 3 in LDS)
constexpr int kMaxBlocksPerCu = 64;   // largest tunable workgroups per compute unit of a launch
constexpr int kBuildGridMultiple = 24;   // build grids are a multiple of this many workgroups
constexpr int kPackI = 11, kPackJ = 11;  // home packing i | j << 11 | k << 22
// Floats per compact transfer-function row (NF = 7 or 13 values and c_l F_l,
// padded to 16-byte words).
template <int NF>
constexpr int kCoefStride = NF == 7 ? 8 : 16;
constexpr uint32_t kMaskI = (1u << kPackI) - 1, kMaskJ = (1u << kPackJ) - 1;

// One axis of the Eulerian grid as the device sees it.
struct Axis {
    int32_t n;          // cells
    int32_t periodic;   // 1 = periodic
    int32_t uniform;    // 1 = all cell widths bitwise equal
    int32_t tile;       // tile edge (nodes) of the spreading grid along this axis
    float inv_tile;     // 1.0f / tile in FP32 (correctly rounded, as the device division gives it)
    int32_t exact;      // 1: faces[i] == f0 + i*h and centres[i] == f0 + (i+0.5)*h bit for bit
    double h;           // L / n (exactly-uniform axes)
    double f0;          // faces[0]
    double L;           // faces[n] - faces[0]
    double inv_h;       // n / L: only used to guess the home node
    const double *faces;    // n + 1
    const double *centres;  // n, 0.5 * (f[i] + f[i+1])
    const float *width_c;   // n     control-volume widths of centre nodes
    const float *width_f;   // n + 1 control-volume widths of face nodes
};

struct Weight {
    int32_t kind;
    float inv_eps;   // 1/eps
    float cut;       // exp(-(R/eps)^2) in FP32 for the shifted Gaussian, 0 for the other kinds
    float e2;        // -log2(e)/eps^2 (0 for the constant weight): w = max(2^(s^2 e2) - cut, 0)
    double inv_eps_d;
    double cut_d;
};

// Everything a kernel needs to know about the grid.
struct Grid {
    Axis ax[3];
    int32_t dims[3][3];   // dims[c][d]: nodes of component c along axis d
    int32_t ntile[3];     // tiles per axis (spreading)
    int32_t box[3];       // LDS box edge per axis: tile + 3 (whole axis for a single periodic tile)
    int32_t ncol[3];      // tile colours per axis: 1 (one tile), 2 (even count or walls), 3 (odd periodic count)
    int64_t ntiles;       // product
    int32_t ncol_tiles[3][3]; // [axis colour][axis]: tiles of that colour along the axis
    int64_t colour_base[27];  // first slot of each colour in the active-tile list
    double h_min;         // smallest node spacing over all axes and components
    float const_width;    // the control-volume width when every width of every axis and node kind is
                          // bitwise equal (uniform periodic grids), else 0
    float inv_cw2;        // 1 / const_width^2 (0 when the widths differ)
};

// Device error word: lowest offending marker index in the upper 56 bits, the
// (negated) status in the low 8 bits; all ones = no error.
struct ErrWord {
    unsigned long long word;
};

struct DevStats {
    unsigned long long fp64_solves;
    unsigned long long fallbacks;
    unsigned long long learned;
    unsigned int kappa_max_bits;  // FP32 bits of the largest kappa (positive floats order as uints)
    unsigned int pad;
};

// fast-MLS tables on the device.
struct FastTables {
    const float *tab;        // [count][n_sub^3][kTableStride]
    const float *geo;        // [count][3 axes][2]: normalised home CV lo, hi
    int32_t n_sub;
    int32_t stretched_axis;  // -1 = uniform grid, one table
    int32_t first[2];        // first table index of centre / face staggering
};

// Learned surrogate: 6 -> 128 -> 128 -> 27 GELU network.  The FP32 parameter
// vector is W1 [6][128], b1 [128], W2 [128][128], b2 [128], W3 [128][27],
// b3 [27] (weights stored [input][output]); norm = shift[6], scale[6].
constexpr int kMlpIn = 6, kMlpHidden = 128, kMlpOut = 27;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHidden;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;   // 20891
// Inference image of the network (built from the FP32 parameters): the
// matrix-core operands of every (layer, 32-row output tile, 16-wide k block)
// as split BF16 (high part, low part), 64 lanes x 8 values each, followed by
// the FP32 biases (b1, b2, b3 padded to 32) and norm, then the GELU table of
// the inference kernel: for z >= 0, z Q(z) (Q the standard normal tail) as
// one cubic in s = 16 z - i per interval [i/16, (i+1)/16), i < 96, 4 FP32
// coefficients each (value and slope matched at both ends).
constexpr int kMlpSlots = 4 + 4 * 8 + 8;                       // layer 1, 2, 3
constexpr int kMlpImageOps = kMlpSlots * 2 * 64;               // 16-byte operand words
constexpr int kMlpImageFloats = 2 * kMlpHidden + 32 + 12;      // biases + norm
constexpr int kGeluPerUnit = 16, kGeluIntervals = 96;          // table over [0, 6)
constexpr size_t kMlpImageTableOffset = (size_t)kMlpImageOps * 16 + kMlpImageFloats * sizeof(float);
constexpr size_t kMlpImageBytes = kMlpImageTableOffset + (size_t)kGeluIntervals * 4 * sizeof(float);
static_assert(kMlpImageTableOffset % 16 == 0, "GELU table rows are 16-byte aligned");

struct Mlp {
    bool loaded = false;
    float *params = nullptr;   // kMlpParams (FP32 master copy)
    float *grad = nullptr;     // kMlpParams
    float *m1 = nullptr, *m2 = nullptr;   // Adam moments
    float *norm = nullptr;     // 12
    void *image = nullptr;     // kMlpImageBytes
    float *loss = nullptr;     // 1 (device)
    float h_norm[12] = {};
    int64_t version = 0, image_version = -1;
    int64_t adam_step = 0;
    float *scratch = nullptr;  // training activations
    int64_t cap_batch = 0;
};

struct Ctx {
    int device = 0;
    Grid g{};
    Grid *d_grid = nullptr;       // device copy of g read by the kernels
    Weight w{};
    mls_opts opts{};
    std::vector<double> h_faces[3];
    std::vector<double> h_centres[3];
    std::vector<float> h_wc[3], h_wf[3];   // control-volume widths of centre / face nodes
    std::string last_error;
    // device allocations owned by the context
    void *geom_block = nullptr;   // faces, centres, widths
    ErrWord *err = nullptr;
    DevStats *stats = nullptr;
    // fast-MLS tables
    float *tables = nullptr;
    float *table_geo = nullptr;
    int64_t n_tables = 0;
    int32_t table_first[2] = {0, 0};
    int32_t stretched_axis = -1;
    // spreading scratch
    int64_t cap_markers = 0;
    uint32_t *tile_count = nullptr;    // ntiles + 1 (the last bucket: markers without a support)
    uint32_t *tile_off = nullptr;      // ntiles + 2
    uint32_t *tile_cursor = nullptr;   // ntiles + 1
    uint32_t *tile_active = nullptr;   // ntiles: non-empty tiles, grouped by colour
    uint32_t *block_sums = nullptr;    // scan partials
    uint32_t *entries = nullptr;       // cap_markers: markers sorted by tile
    float *cf_rows = nullptr;          // [3][cf_stride]: c_l F_l (eq. 8) by row (step, tile order) or by marker
    uint32_t *tile_fmax = nullptr;     // [3][ntiles + 1]: largest finite |c_l F_l| of each tile's markers (FP32
                                       // bits), the fixed-point scale of its spreading sums
    uint32_t *marker_tile = nullptr;   // [cap_markers]: spreading tile of each marker (binning from positions)
    float *coef_rows = nullptr;        // compact transfer functions of a compact exact step, rows of step_nf floats
    uint32_t *route_queue = nullptr;   // [1 + 3 cap]: count, then row << 2 | component of its FP64-solved rows
    int64_t coef_cap = 0;              // markers the two buffers above hold
    int step_nf = 0;                   // row width of the step being enqueued: 0 (full phi), 7 or 13
    uint64_t scratch_gen = 0;          // bumped whenever context scratch moves or the tiling changes
                                       // (a captured step graph holds the old addresses and tiling)
    int64_t cf_stride = 0;             // cap_markers rounded up to 64
    uint32_t *work = nullptr;          // [0..26] active-list sizes per colour, [32..58] cursors
    int64_t colour_tiles[27] = {};     // tiles of each colour
    // launch shapes (autotuned): resident workgroups per compute unit
    int spread_blocks_per_cu = 16;      // effective (bounded by the LDS of the tile boxes)
    int spread_blocks_per_cu_req = 16;  // requested
    int spread_threads = 128;           // threads of a spreading tile workgroup (128, 192 or 256)
    int build_blocks_per_cu = 32;
    int interp_blocks_per_cu = 32;
    int cu_count = 256;
    // learned surrogate
    Mlp mlp;
    // Lagrangian refinement: per-workgroup marker sums and offsets
    uint32_t *refine_scratch = nullptr;
    int64_t refine_cap = 0;
    // derivative shape functions: queue of (marker, staggering) pairs for the FP64 route
    uint32_t *grad_queue = nullptr;
    int64_t grad_queue_cap = 0;
    // time step
    unsigned long long *step_ctr = nullptr;
    int64_t step_sorted_n = -1;   // markers of the last exact step (its rows are in tile order)
    // per-kernel timing
    bool timing = false;
    bool capturing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;
    size_t ev_used = 0;
};

// Timing marks around a launch (no-ops unless timing is on and no graph is
// being captured).
struct TimedLaunch {
    Ctx &c;
    int id;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(Ctx &c_, int id_, hipStream_t s_);
    ~TimedLaunch();
};

// ---- launchers (enqueue only; return hipError_t) --------------------------

hipError_t launch_build_exact(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                              uint32_t *home, float *phi, uint8_t *route, hipStream_t s);
hipError_t launch_build_fast(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                             uint32_t *home, float *phi, uint8_t *route, hipStream_t s, bool trilinear_blend);
// fast-MLS fused with interpolation and forcing in spreading-tile order (uniform
// grids: one symmetric table, odd sub-node count); fast_fused_ok tells whether
// the context qualifies (tables built).
bool fast_fused_ok(const Ctx &c);
hipError_t launch_fast_interp(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                              uint32_t *home, float *phi, uint8_t *route, const float *u, const float *v,
                              const float *w, const float *vb, const float *area, float dt, float *U, float *F,
                              hipStream_t s, bool trilinear_blend);
// order: row p holds marker order[p] (the time step's tile order); NULL: row = marker.
// Outputs of the interpolation (eq. 6), direct forcing and c_l F_l (eq. 8)
// that the learned build computes from its rows in a time step: U and F by
// marker, c_l F_l by row (cf, cf_stride), tile maxima in tmax (tstride per
// component) keyed by tile_of_marker.  U == nullptr: no interpolation.
struct LearnedInterp {
    const float *u = nullptr, *v = nullptr, *w = nullptr, *vb = nullptr, *area = nullptr;
    float inv_dt = 0.0f;
    float *U = nullptr, *F = nullptr, *cf = nullptr;
    int64_t cf_stride = 0;
    const uint32_t *tile_of_marker = nullptr;
    uint32_t *tmax = nullptr;
    int64_t tstride = 0;
};
hipError_t launch_build_learned(Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                                uint32_t *home, float *phi, uint8_t *route, hipStream_t s, const uint32_t *order = nullptr,
                                const LearnedInterp *interp = nullptr);
// The interpolation arguments of a learned time step on the context's rows.
LearnedInterp learned_interp(const Ctx &c, const float *u, const float *v, const float *w, const float *vb,
                             const float *area, float dt, float *U, float *F);
hipError_t launch_table_build(const Ctx &c, hipStream_t s);
hipError_t launch_collide(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                          const int32_t *body, int32_t *coll, uint8_t *flags, hipStream_t s);
hipError_t launch_collide_clear(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                                int32_t *coll, hipStream_t s);
hipError_t launch_refine(Ctx &c, int64_t ntri, const int32_t *tri, int64_t nvert, const float *xv,
                         const float *yv, const float *zv, double ratio, int level, int64_t cap, float *x,
                         float *y, float *z, float *area, float *normal, int32_t *parent, uint8_t *tri_level,
                         int64_t *count, hipStream_t s);
hipError_t launch_build_grad(Ctx &c, int64_t n, const float *x, const float *y, const float *z, int stagger,
                             uint32_t *home, float *phi, float *dphi, hipStream_t s);
hipError_t launch_interp_grad(Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                              const float *u, const float *v, const float *w, const float *p, float *U, float *G,
                              float *P, float *GP, hipStream_t s);
hipError_t launch_interp(const Ctx &c, int64_t n, const uint32_t *home, const float *phi,
                         const float *u, const float *v, const float *w,
                         float *U, float *V, float *W, hipStream_t s);
hipError_t launch_spread(Ctx &c, int64_t n, const uint32_t *home, const float *phi,
                         const float *area, const float *Fx, const float *Fy, const float *Fz,
                         float *fx, float *fy, float *fz, hipStream_t s);

// The exact time step in spreading-tile order: markers are binned by the tile
// of their cell straight from their positions (entries = tile-sorted marker
// indices, markers without a valid support last), the fused build writes row
// p of home / phi for marker entries[p] together with U, F and per-block
// force maxima, and the tile kernels read the rows of a tile contiguously.
int build_blocks(const Ctx &c, int64_t n);   // workgroups of a build launch over n markers
// Bins the markers by spreading tile from their positions x, y, z; with jx
// non-NULL the positions are first jittered (amplitude jitter, the step's
// generator and device counter) into jx, jy, jz, and those are binned.
hipError_t launch_sort_positions(Ctx &c, int64_t n, const float *x, const float *y, const float *z, hipStream_t s,
                                 float *jx = nullptr, float *jy = nullptr, float *jz = nullptr, float jitter = 0.0f,
                                 uint64_t seed = 0);
int compact_nf(const Ctx &c);
mls_status reserve_compact(mls_ctx *ctx, int64_t n);
hipError_t launch_build_interp(const Ctx &c, int64_t n, const float *x, const float *y, const float *z,
                               uint32_t *home, float *phi, uint8_t *route, const float *u, const float *v,
                               const float *w, const float *vb, const float *area, float dt, float *U, float *F,
                               hipStream_t s);
hipError_t launch_spread_sorted(Ctx &c, int64_t n, const uint32_t *home, const float *phi, float *fx, float *fy,
                                float *fz, hipStream_t s);
// Dynamic LDS of a spreading tile workgroup: the int64 box of one component.
size_t spread_lds_bytes(const Ctx &c);

// Allocation-free spreading: its scratch is the library's fixed device array.
// noalloc_setup takes that array's address on the current device (once per
// device); noalloc_bytes is the scratch a call of n markers needs.
hipError_t noalloc_setup(int device);
size_t noalloc_bytes(const Ctx &c, int64_t n);
hipError_t launch_spread_noalloc(Ctx &c, int64_t n, const uint32_t *home, const float *phi, const float *area,
                                 const float *Fx, const float *Fy, const float *Fz, float *fx, float *fy, float *fz,
                                 hipStream_t s);

hipError_t launch_jitter(const Ctx &c, int64_t n, const float *x0, const float *y0, const float *z0,
                         float *x, float *y, float *z, float amp, uint64_t seed, hipStream_t s);
hipError_t launch_force(const Ctx &c, int64_t n, const float *vb, const float *U, float dt, float *F,
                        hipStream_t s);
hipError_t launch_step_advance(const Ctx &c, hipStream_t s);

FastTables fast_tables(const Ctx &c);

// (Re)cut the spreading tiles for edge `want` (see mls_ctx_create).
mls_status setup_tiles(Ctx &c, int want);

// learned surrogate (training and feature kernels)
hipError_t mlp_alloc(Ctx &c);
void mlp_free(Ctx &c);
hipError_t mlp_reserve(Ctx &c, int64_t batch);
hipError_t mlp_pack(Ctx &c, hipStream_t s);
hipError_t launch_features(const Ctx &c, int64_t n, const float *x, const float *y, const float *z, float *feat,
                           hipStream_t s);
hipError_t mlp_forward_batch(Ctx &c, int64_t m, const float *feat, int64_t rows, const int64_t *idx, float *y,
                             hipStream_t s);
hipError_t mlp_grad_batch(Ctx &c, int64_t m, const float *feat, const float *target, int64_t rows,
                          const int64_t *idx, float mu, float *grad, float *loss, hipStream_t s);
hipError_t mlp_adam(Ctx &c, float lr, hipStream_t s);

}  // namespace mls

// The opaque handle of the C ABI.
struct mls_ctx {
    mls::Ctx c;
};
