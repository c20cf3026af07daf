// internal.h -- shared definitions of the gfx950 pair-counting library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "fcfc.h"

namespace fcfc {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

#define FCFC_HIP(call)                                                              \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            ::fcfc::set_error("%s:%d: %s failed: %s", __FILE__, __LINE__, #call,    \
                              hipGetErrorString(e_));                               \
            return FCFC_EHIP;                                                       \
        }                                                                           \
    } while (0)

#define FCFC_TRY(expr)                       \
    do {                                     \
        fcfc_status s_ = (expr);             \
        if (s_ != FCFC_OK) return s_;        \
    } while (0)

// ---------------------------------------------------------------------------
// grid of cubic cells (Sect. 2.1): cell (cx,cy,cz) covers
// [lo + c*side, lo + (c+1)*side) per axis; linear key (cz*ny + cy)*nx + cx, so
// the cells of one row (fixed cy, cz) are consecutive and their points form a
// single contiguous range after sorting.
// ---------------------------------------------------------------------------
struct Grid {
    int nx = 0, ny = 0, nz = 0;
    double lo[3] = {0, 0, 0};
    double side = 0;      // cell side (FP64)
    double L = 0;         // > 0 periodic
    int k = 0;            // cells per prune radius used to size the grid
    int64_t ncell() const { return (int64_t)nx * ny * nz; }
};

// A work item: one A tile (consecutive sorted points of one row, spanning at
// most a few cells) against one contiguous piece of one B row.  32 bytes.
struct Item {
    uint32_t a_begin;   // first A point (sorted index)
    uint32_t b_begin;   // first B point
    uint32_t b_end;     // one past the last B point
    uint32_t b_rowcell; // linear index of cell (x = 0) of the B row
    uint32_t acnt_xb0;  // bits 0..15: A point count; bits 16..31: int16 unwrapped x of first B cell
    uint32_t meta;      // int8 dy | int8 dz << 8 | (sx+1) << 16 | (sy+1) << 18 | (sz+1) << 20 | flags << 24
    uint32_t cost;      // ordering key
    uint32_t tile;      // A tile index (features, batched catalogue lookup)
};
static_assert(sizeof(Item) == 32, "Item must be 32 bytes");

enum : uint32_t { ITEM_SAMEROW = 1u };

// ---------------------------------------------------------------------------
// FP32 look-up table over a squared quantity v (Sect. 3.2.3):
// entry j = (uint)(v * scale) covers [j/scale, (j+1)/scale).  Entries are
// int16: a clean entry holds the bin (>= 0) or LUT_NONE (-1, out of range); a
// hot entry holds -2 - k with k the first edge whose error band [lo_k, hi_k)
// meets the entry.
// ---------------------------------------------------------------------------
enum : int16_t { LUT_NONE = -1 };
inline int16_t lut_hot_code(int k) { return (int16_t)(-2 - k); }

struct Lut1D {
    int n = 0;                 // bins
    std::vector<double> E;     // n+1 squared edges (FP64)
    std::vector<float> lo, hi; // n+1 FP32 band ends: v < lo_k => V < E_k; v >= hi_k => V >= E_k
    std::vector<int16_t> tab;  // entries
    float scale = 1.f;         // power of two
    float vmax = 0.f;          // hi_n: v >= vmax is out of range
    double band_rel = 0;       // widest band half-width relative to its edge
};

// error model |Q32 - Q64| <= A*sqrt(Q) + B + C*Q for a squared quantity Q
struct ErrModel {
    double A = 0, B = 0, C = 0;
    double operator()(double Q) const { return A * __builtin_sqrt(Q > 0 ? Q : 0) + B + C * Q; }
};

struct Plan {
    int kind = 0, los = 0;
    int n1 = 0, n2 = 1, nbins = 0;
    std::vector<double> e1, e2;
    double L = 0;               // > 0 periodic
    double rprune = 0;          // prune radius (FP64)
    fcfc_tuning tune{};
    bool grid_set = false;
    Grid grid;
    double grid_ext[3] = {0, 0, 0};  // open box: extent of the bounds per axis
    double grid_hi[3] = {0, 0, 0};   // open box: upper bounds (inclusive)
    double obs_dist = 0;        // open box: distance from the origin to the box
    double coord_max = 0;       // largest |coordinate| inside the box
    // bands and tables, set by finalize_numerics() once the grid is known
    bool numerics_ready = false;
    double e_axis = 0;          // bound on the FP32 error of one displacement component
    Lut1D lut1, lut2;           // s (or s_perp) and pi tables
    Lut1D lut1b, lut2b;         // the same with twice the entries (has_big)
    Lut1D lutbin;               // first-axis table for binning given FP64 values (built on first use)
    Lut1D luttri;               // table for FP32 triangle sides (bands for luttri_e per axis)
    double luttri_e = 0;
    bool has_big = false;       // counts may use the larger tables where LDS allows
    float r2prune32 = 0;        // FP32 candidate threshold (>= every relevant value)
    float d2small = 0;          // pairs closer than this are always rechecked (mu)
    float mu_tolA = 0, mu_tolB = 0, mu_tolC = 0;  // mu band: n*(A*rs + B*rs^2 + C)
    bool mu_top_closed = true;
    uint64_t id = 0;            // unique plan id (cells remember it)
    // stats of the last count
    fcfc_stats stats{};
    void* stats_dev = nullptr; // device u64[4]: candidates, rechecks, items, in_range
    hipStream_t last_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool have_stats = false;
    int64_t* last_counts = nullptr;  // device histogram of the last count (for stats)
    int64_t last_counts_n = 0;       // its entries when not nbins (triangle counts)
    void* timing_dev = nullptr;      // last recorded per-item times (u32) followed by the items
    uint32_t timing_n = 0;
    int last_pts = 0;
    std::vector<char> host_stage;    // host copies of uploaded tables / kernel arguments
    std::vector<char> host_args;
    // learned cost model for FCFC_ORDER_LEARNED (not owned)
    struct Model* model = nullptr;
    // tree plans: the leaf extent the FP32 bands were built for (raised, and
    // the bands rebuilt, when a count meets larger leaves)
    double tree_side = 0;
};

struct Cells {
    uint64_t plan_id = 0;
    Grid grid;
    int64_t n = 0;
    bool weighted = false;
    bool has_abs = false;
    double wmin = 0, wmax = 0;  // smallest non-zero |w|, largest |w|
    float4* pos32 = nullptr;    // cell-local FP32 (x', y', z', cellx bits)
    float4* abs32 = nullptr;    // absolute FP32 (mid-point line of sight only)
    double* pos64 = nullptr;    // sorted FP64 xyz (AoS)
    double* w = nullptr;        // sorted weights
    uint32_t* cell_start = nullptr;  // ncell + 1
    // sorted keys: cell key << xbits | the point's x position within its cell
    // on 2^xbits steps, so that every row of cells is sorted by x
    uint32_t* xkey = nullptr;
    int xbits = 0;
    void* block = nullptr;      // single allocation holding everything
    // k-d tree of a tree plan: points in tree order, 2^tree_levels leaves
    // (cell_start then holds the leaf offsets), each leaf's points relative
    // to a lattice origin leaf_org * tree_q (tree_q a power of two, so that
    // the FP32 offset between two leaves is exact), and the FP64 bounding
    // box of every node in heap order (node h has children 2h+1, 2h+2)
    bool tree = false;
    int tree_levels = 0;
    int4* leaf_org = nullptr;
    double* node_box = nullptr;  // 6 per node: lo x, y, z, hi x, y, z
    double tree_q = 0;
    double tree_ext = 0;         // largest coordinate of a point relative to its leaf origin
};

// Sub-cell x bits of the sort key for a grid of ncells cells (catalogues x
// cells for a batched build): the key fills whole bytes up to 32 bits, with
// at least 8 sub-cell bits when the cell key leaves room for them.
int key_xbits(int64_t ncells);

// plan / numerics helpers (plan.cpp)
const char* last_error();
fcfc_status fcfc_set_bounds_internal(Plan* p, const double lo[3], const double hi[3]);
fcfc_status plan_finalize_grid(Plan* p);
fcfc_status plan_finalize_numerics(Plan* p);
int choose_k(const Plan* p, int64_t n_hint);
int stencil_rows(const Plan* p, bool half, std::vector<int4>& rows);
// Table over the first-axis squared edges for binning values given in FP64:
// its bands cover only the rounding of a value to FP32, so it depends on the
// edges alone (no grid); built on first use and kept by the plan.
fcfc_status plan_bin_table(Plan* p, const Lut1D** out);
// Table over the first-axis squared edges for squared lengths formed in FP32
// from components each within e_axis of their FP64 values (triangle sides);
// rebuilt when e_axis changes, kept by the plan.
fcfc_status plan_side_table(Plan* p, double e_axis, const Lut1D** out);

// Fixed-point scale 2^S of the exact weighted sums (plan.cpp): every non-zero
// product of nfactors (2: pairs, 3: triangles) weights is an integer below
// 2^62 once multiplied by 2^S.  wmin*: smallest non-zero |w| (0: none),
// wmax*: largest |w|.  FCFC_ERANGE when the smallest product underflows, 2^S
// overflows or the range is too wide.
fcfc_status weight_scale_rule(double wmin1, double wmax1, double wmin2, double wmax2, int nfactors, int* S);

// build (build.hip)
fcfc_status build_cells(Plan* p, const fcfc_catalog* cat, hipStream_t st, Cells** out);
// k-d tree build and dual-tree work list (tree.hip)
fcfc_status build_tree(Plan* p, const fcfc_catalog* cat, hipStream_t st, Cells** out);
// Work items of a tree count: every A leaf against the B ranges its
// traversal of the B tree keeps; item counts per A leaf into icount (count
// pass, items == nullptr) or the items at ioff (write pass).
void tree_items_enqueue(const Cells* ca, const Cells* cb, bool is_auto, double rprune, double coord_max, int bchunk,
                        const uint32_t* ioff, uint32_t* icount, Item* items, uint32_t items_cap, hipStream_t st);
uint32_t tree_leaves(const Cells* c);
// B tree level split among the work-list threads: tree_leaves(ca) << split slots
int tree_wl_split(const Cells* ca, const Cells* cb);
// validation flags of a build
enum : uint32_t { VF_NONFINITE = 1u, VF_BOX = 2u, VF_WNONFINITE = 4u };
// validation of a catalogue against the plan (finite, inside the box) and its
// weight range, with idx[i] = i (build.hip)
fcfc_status validate_points(Plan* p, const fcfc_catalog* cat, uint32_t* idx, uint32_t* keys, uint32_t* flags,
                            uint64_t* wst, hipStream_t st);
fcfc_status fit_bounds(Plan* p, const fcfc_catalog* cats, int ncat, hipStream_t st);
void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
void fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t st);
// relative error bound assumed for the hardware FP32 rsq and rcp (plan.cpp)
double trans_rel_bound();

// Per-launch statistics (weight range, bounding box) are gathered in
// STAT_SLOTS slots of one 128-byte line each, workgroup b updating slot
// b % STAT_SLOTS: one address taking an atomic from every workgroup
// serialised them (about 11 ns each).  Minima are kept as maxima of the
// complemented bits, so that a zero fill initialises every slot; the host
// reduces the slots after its read-back.
constexpr int STAT_SLOTS = 64;
constexpr int STAT_STRIDE = 16;  // u64 per slot
constexpr size_t STAT_BYTES = (size_t)STAT_SLOTS * STAT_STRIDE * 8;
// weight statistics of a build: bits of the smallest non-zero |w| (~0 when
// there is none) and of the largest |w|
void weight_stats_reduce(const uint64_t* slots, uint64_t* bmin, uint64_t* bmax);

// batched build (build.hip)
struct CatDesc {
    const double* xyz;
    const double* w;
    int64_t n;
    int64_t off;
};
size_t batch_build_scratch(int64_t ntot);
void batch_build_enqueue(const Plan* p, int xbits, const CatDesc* desc, const int64_t* offs, int ncat, int64_t ntot,
                         bool weighted, uint32_t** key, uint32_t** idx, uint32_t** tk, uint32_t** tv, void* sort_scr,
                         uint32_t* flags, uint64_t* wst, float4* pos32, float4* abs32, double* pos64, double* w,
                         uint32_t* cs, hipStream_t st);

// count (count.hip)
// Learned cost model (mlp.hip): predicted log2(1 + ticks) of n work items
// into pred[n]; feat is scratch of 4 n floats.
struct Model;
void model_item_costs(const Model* md, const Item* items, uint32_t n, float kcells, float* feat, float* pred,
                      hipStream_t st);
// A frozen copy of a model for a pipeline that outlives later training: the
// parameters are copied on `st` into `params` (model_param_bytes(), owned by
// the caller), the normalisation with them; free with model_snapshot_free
// (the host object only).
size_t model_param_bytes();
Model* model_snapshot(const Model* src, float* params, hipStream_t st);
void model_snapshot_free(Model* m);
// Predict-only count: with `predict` set, count_pairs builds the work list,
// scores it with the model and returns the predicted time (ms) without counting.
struct PredictReq {
    const Model* model = nullptr;
    double pred_ms = 0;
    int64_t items = 0;
};
// Caller-provided device scratch for a count that must not allocate: every
// scratch buffer of the count is carved out of [base, base + bytes)
// (256-byte aligned); FCFC_ERANGE when it does not fit.  Per-item timings
// are then not recorded, and launch statistics are kept only in a plan whose
// statistics buffer an earlier allocating count has already made.
struct Workspace {
    char* base = nullptr;
    size_t bytes = 0;
};
fcfc_status count_pairs(Plan* p, Cells* c1, Cells* c2, int64_t* d_counts, double* d_wcounts,
                        hipStream_t st, PredictReq* pr = nullptr, const Workspace* ws = nullptr);

struct BatchImpl;
// pairs: 2 * npairs catalogue indices (A, B), A == B for an auto count
fcfc_status batch_create_impl(Plan* p, const fcfc_catalog* cats, int ncat, const int32_t* pairs, int npairs,
                              hipStream_t st, BatchImpl** out);
fcfc_status batch_run_impl(BatchImpl* b, int64_t* d_counts, double* d_wcounts, bool use_graph, hipStream_t st);
fcfc_status batch_check_impl(BatchImpl* b, hipStream_t st, uint32_t* nitems, float* ms);
fcfc_status batch_stats_impl(BatchImpl* b, hipStream_t st, int64_t out[3]);
void batch_free_impl(BatchImpl* b);

int device_cu_count();

// Stream-ordered device memory from the library's pool (mem.cpp): dev_alloc
// returns FCFC_ENOMEM (with the error text set) on failure; dev_free returns
// the memory on stream `st`.
fcfc_status dev_alloc(void** ptr, size_t bytes, hipStream_t st);
void dev_free(void* ptr, hipStream_t st);

}  // namespace fcfc
