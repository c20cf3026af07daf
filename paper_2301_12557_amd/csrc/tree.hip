// tree.hip -- the k-d tree of Sect. 2.2 built on the GPU, and the work list
// of a dual-tree count (Sect. 3.1): every A leaf against the B node ranges
// its traversal of the B tree keeps.
//
// The tree is implicit and balanced over leaf units of `leaf` consecutive
// points (the last unit may be shorter): nl = ceil(n / leaf) units, depth
// L = ceil(log2 nl), node (l, k) holding the units [ub(l, k), ub(l, k + 1))
// with ub(l, k) = floor(k nl / 2^l).  A node's two children split its units
// at their middle, so every split is the median to within one leaf, and a
// node of the last level holds one unit or none.  Nodes are numbered in heap
// order: h = 2^l - 1 + k, children 2h + 1 and 2h + 2.
//
// Level by level, the points of each node are ordered along the axis of the
// longest extent of the node's region (the parent's region cut at the
// parent's split): one LSD radix sort of a 32-bit key, the node in the high
// bits and the coordinate on 2^(32 - l) steps across the node's region in the
// low ones.  The paper
// splits along the axis of largest variance; the region's extent needs no
// reduction over the points and gives the same tree on any device.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"
#include "worklist.h"

namespace fcfc {

__host__ __device__ inline uint32_t tunit_bound(int l, uint64_t k, uint64_t nl) { return (uint32_t)((k * nl) >> l); }
__device__ inline uint32_t tnode_of_unit(int l, uint64_t u, uint64_t nl) {
    return (uint32_t)((((u + 1) << l) - 1) / nl);
}

// axis of the longest extent of each node's region at level l (ties: lowest axis)
__global__ void k_tree_dims(int l, const double* __restrict__ region, int* __restrict__ dims) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (1u << l)) return;
    const double* r = region + 6 * ((size_t)(1u << l) - 1 + k);
    int d = 0;
    double best = r[3] - r[0];
    for (int a = 1; a < 3; a++) {
        const double ex = r[3 + a] - r[a];
        if (ex > best) {
            best = ex;
            d = a;
        }
    }
    dims[k] = d;
}

// Sort key of each element at level l: its node (the high l bits; nodes lie
// in position order, so sorting keeps every node's range) and its coordinate
// along the node's axis, placed on 2^(32 - l) steps across the node's region
// (the low bits).  Points on one step keep their order; any order of them is
// a valid split, since every box is formed from the points afterwards.
__global__ void k_tree_keys(int l, int64_t n, int leaf, uint64_t nl, const double* __restrict__ xyz,
                            const uint32_t* __restrict__ idx, const int* __restrict__ dims,
                            const double* __restrict__ region, uint32_t* __restrict__ key,
                            uint32_t* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = tnode_of_unit(l, (uint64_t)i / (uint64_t)leaf, nl);
    const int d = dims[k];
    const double* r = region + 6 * ((size_t)(1u << l) - 1 + k);
    const double lo = r[d], ext = r[3 + d] - r[d];
    const double x = xyz[3 * (size_t)idx[i] + d];
    const int b = 32 - l;
    const double steps = ldexp(1.0, b);
    double t = ext > 0.0 ? (x - lo) / ext * steps : 0.0;
    t = fmin(fmax(t, 0.0), steps - 1.0);
    const uint64_t q = (uint64_t)t;
    key[i] = (uint32_t)((b < 32 ? ((uint64_t)k << b) : 0ull) | q);
    val[i] = (uint32_t)i;
}

__global__ void k_tree_permute(int64_t n, const uint32_t* __restrict__ val, const uint32_t* __restrict__ in,
                               uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[val[i]];
}

// children's regions: the parent's, cut at the coordinate of the first point
// of the right child along the parent's axis
__global__ void k_tree_regions(int l, int leaf, uint64_t nl, const double* __restrict__ xyz,
                               const uint32_t* __restrict__ idx, const int* __restrict__ dims,
                               double* __restrict__ region) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (1u << l)) return;
    const size_t h = (size_t)(1u << l) - 1 + k;
    double r[6];
    for (int a = 0; a < 6; a++) r[a] = region[6 * h + a];
    double* left = region + 6 * (2 * h + 1);
    double* right = region + 6 * (2 * h + 2);
    for (int a = 0; a < 6; a++) {
        left[a] = r[a];
        right[a] = r[a];
    }
    const uint32_t u0 = tunit_bound(l, k, nl), u1 = tunit_bound(l, (uint64_t)k + 1, nl);
    if (u1 - u0 < 2) return;
    const uint32_t m = tunit_bound(l + 1, 2ull * k + 1, nl);
    const int d = dims[k];
    const double c = xyz[3 * (size_t)idx[(size_t)m * leaf] + d];
    left[3 + d] = c;
    right[d] = c;
}

__global__ void k_tree_gather(int64_t n, const double* __restrict__ xyz, const double* __restrict__ w,
                              const uint32_t* __restrict__ idx, double* __restrict__ pos64, double* __restrict__ wout,
                              float4* __restrict__ abs32) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const size_t i = idx[p];
    const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    pos64[3 * p] = x;
    pos64[3 * p + 1] = y;
    pos64[3 * p + 2] = z;
    if (wout) wout[p] = w[i];
    if (abs32) abs32[p] = make_float4((float)x, (float)y, (float)z, 0.f);
}

__global__ void k_box_empty(double* __restrict__ box, int64_t nodes) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= nodes) return;
    for (int a = 0; a < 3; a++) {
        box[6 * h + a] = INFINITY;
        box[6 * h + 3 + a] = -INFINITY;
    }
}

__device__ inline double wave_min(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// One wavefront per leaf unit: its bounding box (the node of the last level
// holding it), its lattice origin floor(lo / q) and the largest coordinate of
// its points relative to that origin (slots of ordered bits, one per unit mod
// STAT_SLOTS).
__global__ __launch_bounds__(256) void k_leaf_box(int64_t n, int leaf, uint64_t nl, int L,
                                                  const double* __restrict__ pos64, double q,
                                                  double* __restrict__ box, int4* __restrict__ org,
                                                  unsigned long long* __restrict__ slots) {
    const uint64_t u = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (u >= nl) return;
    const int64_t p0 = (int64_t)u * leaf, p1 = std::min<int64_t>(p0 + leaf, n);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t p = p0 + lane; p < p1; p += 64)
        for (int a = 0; a < 3; a++) {
            const double v = pos64[3 * p + a];
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
    for (int a = 0; a < 3; a++) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    if (lane != 0) return;
    const size_t h = ((size_t)1 << L) - 1 + tnode_of_unit(L, u, nl);
    int j[3] = {0, 0, 0};
    double ext = 0.0;
    if (p1 > p0) {
        for (int a = 0; a < 3; a++) {
            box[6 * h + a] = lo[a];
            box[6 * h + 3 + a] = hi[a];
            j[a] = (int)floor(lo[a] / q);
            ext = fmax(ext, hi[a] - (double)j[a] * q);
        }
    }
    org[u] = make_int4(j[0], j[1], j[2], 0);
    atomicMax(&slots[(u % STAT_SLOTS) * STAT_STRIDE], (unsigned long long)__double_as_longlong(ext));
}

// FP32 coordinates of every point relative to its leaf's lattice origin
__global__ void k_leaf_local(int64_t n, int leaf, const double* __restrict__ pos64, const int4* __restrict__ org,
                             double q, float4* __restrict__ pos32) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int4 j = org[p / leaf];
    pos32[p] = make_float4((float)(pos64[3 * p] - (double)j.x * q), (float)(pos64[3 * p + 1] - (double)j.y * q),
                           (float)(pos64[3 * p + 2] - (double)j.z * q), 0.f);
}

__global__ void k_box_up(int l, double* __restrict__ box) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (1u << l)) return;
    const size_t h = (size_t)(1u << l) - 1 + k;
    const double* a = box + 6 * (2 * h + 1);
    const double* b = box + 6 * (2 * h + 2);
    for (int i = 0; i < 3; i++) {
        box[6 * h + i] = fmin(a[i], b[i]);
        box[6 * h + 3 + i] = fmax(a[3 + i], b[3 + i]);
    }
}

static size_t al256t(size_t b) { return (b + 255) & ~(size_t)255; }
static unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

uint32_t tree_leaves(const Cells* c) {
    return c->n > 0 ? (uint32_t)((c->n + c->xbits - 1) / c->xbits) : 1u;
}

fcfc_status build_tree(Plan* p, const fcfc_catalog* cat, hipStream_t st, Cells** out) {
    const int64_t n = cat->n;
    const int leaf = p->tune.tree_leaf;
    const uint64_t nl = n > 0 ? (uint64_t)((n + leaf - 1) / leaf) : 1;
    int L = 0;
    while (((uint64_t)1 << L) < nl) L++;
    const int64_t nodes = ((int64_t)2 << L) - 1;
    const bool weighted = cat->w != nullptr;
    const bool need_abs = (p->los == FCFC_LOS_MIDPOINT && p->kind != FCFC_BIN_S);
    // lattice spacing: a power of two with every coordinate below 2^22 spacings
    int e = 0;
    frexp(std::max(p->coord_max, 1.0), &e);
    const double q = ldexp(1.0, e - 22);

    const int64_t PAD = 8;
    size_t o_pos32 = 0;
    size_t o_abs32 = o_pos32 + al256t((size_t)(n + PAD) * 16);
    size_t o_pos64 = o_abs32 + (need_abs ? al256t((size_t)std::max<int64_t>(n, 1) * 16) : 0);
    size_t o_w = o_pos64 + al256t((size_t)std::max<int64_t>(n, 1) * 24);
    size_t o_org = o_w + (weighted ? al256t((size_t)(n + PAD) * 8) : 0);
    size_t o_box = o_org + al256t((size_t)nl * 16);
    size_t total = o_box + al256t((size_t)nodes * 48);
    Cells* c = new (std::nothrow) Cells();
    if (!c) return FCFC_ENOMEM;
    char* blk = nullptr;
    if (dev_alloc((void**)&blk, total, st) != FCFC_OK) {
        delete c;
        set_error("build_cells: cannot allocate %zu bytes for the tree", total);
        return FCFC_ENOMEM;
    }
    c->block = blk;
    c->plan_id = p->id;
    c->grid = p->grid;
    c->n = n;
    c->weighted = weighted || n == 0;
    c->has_abs = need_abs;
    c->pos32 = (float4*)(blk + o_pos32);
    c->abs32 = need_abs ? (float4*)(blk + o_abs32) : nullptr;
    c->pos64 = (double*)(blk + o_pos64);
    c->w = weighted ? (double*)(blk + o_w) : nullptr;
    c->cell_start = nullptr;
    c->xkey = nullptr;
    c->xbits = leaf;  // points per leaf unit
    c->tree = true;
    c->tree_levels = L;
    c->leaf_org = (int4*)(blk + o_org);
    c->node_box = (double*)(blk + o_box);
    c->tree_q = q;

    // scratch: idx, key, val, tk, tv, idx2, dims, regions, flags + stats, ext slots, sort
    const size_t s_n = al256t((size_t)std::max<int64_t>(n, 1) * 4);
    const size_t s_dims = al256t(((size_t)1 << L) * 4);
    const size_t s_reg = al256t((size_t)nodes * 48);
    const size_t s_misc = 256 + STAT_BYTES;
    const size_t s_sort = al256t(radix_scratch_bytes(n));
    const size_t stotal = 6 * s_n + s_dims + s_reg + s_misc + STAT_BYTES + s_sort;
    char* scr = nullptr;
    if (dev_alloc((void**)&scr, stotal, st) != FCFC_OK) {
        dev_free(blk, st);
        delete c;
        set_error("build_cells: cannot allocate the tree build's scratch");
        return FCFC_ENOMEM;
    }
    uint32_t* idx = (uint32_t*)scr;
    uint32_t* key = (uint32_t*)(scr + s_n);
    uint32_t* val = (uint32_t*)(scr + 2 * s_n);
    uint32_t* tk = (uint32_t*)(scr + 3 * s_n);
    uint32_t* tv = (uint32_t*)(scr + 4 * s_n);
    uint32_t* idx2 = (uint32_t*)(scr + 5 * s_n);
    int* dims = (int*)(scr + 6 * s_n);
    double* region = (double*)(scr + 6 * s_n + s_dims);
    uint32_t* flags = (uint32_t*)(scr + 6 * s_n + s_dims + s_reg);
    uint64_t* wst = (uint64_t*)(scr + 6 * s_n + s_dims + s_reg + 256);
    unsigned long long* xslots = (unsigned long long*)(scr + 6 * s_n + s_dims + s_reg + s_misc);
    void* sort_scr = scr + 6 * s_n + s_dims + s_reg + s_misc + STAT_BYTES;
    auto fail = [&](fcfc_status s) {
        dev_free(scr, st);
        dev_free(blk, st);
        delete c;
        return s;
    };

    fill_u32((uint32_t*)(c->pos32 + n), 0u, PAD * 4, st);
    if (weighted) fill_u64((uint64_t*)(c->w + n), 0ull, PAD, st);
    fill_u64((uint64_t*)xslots, 0ull, STAT_SLOTS * STAT_STRIDE, st);
    // validation (finite, inside the plan bounds) and weight range; idx = identity
    fcfc_status vs = validate_points(p, cat, idx, key, flags, wst, st);
    if (vs != FCFC_OK) return fail(vs);
    // root region: the plan bounds
    const double root[6] = {p->grid.lo[0], p->grid.lo[1], p->grid.lo[2],
                            p->grid_hi[0], p->grid_hi[1], p->grid_hi[2]};
    if (hipMemcpyAsync(region, root, sizeof(root), hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("build_cells: HIP copy failed");
        return fail(FCFC_EHIP);
    }
    for (int l = 0; l < L; l++) {
        const unsigned nb = blocks_for((int64_t)1 << l);
        hipLaunchKernelGGL(k_tree_dims, dim3(nb), dim3(256), 0, st, l, region, dims);
        hipLaunchKernelGGL(k_tree_keys, dim3(blocks_for(n)), dim3(256), 0, st, l, n, leaf, nl, cat->xyz, idx, dims,
                           region, key, val);
        uint32_t *k0 = key, *v0 = val, *k1 = tk, *v1 = tv;
        radix_sort_pairs(&k0, &v0, &k1, &v1, n, 32, sort_scr, st);
        hipLaunchKernelGGL(k_tree_permute, dim3(blocks_for(n)), dim3(256), 0, st, n, v0, idx, idx2);
        std::swap(idx, idx2);
        hipLaunchKernelGGL(k_tree_regions, dim3(nb), dim3(256), 0, st, l, leaf, nl, cat->xyz, idx, dims, region);
    }
    hipLaunchKernelGGL(k_tree_gather, dim3(blocks_for(n)), dim3(256), 0, st, n, cat->xyz, cat->w, idx, c->pos64,
                       c->w, c->abs32);
    hipLaunchKernelGGL(k_box_empty, dim3(blocks_for(nodes)), dim3(256), 0, st, c->node_box, nodes);
    hipLaunchKernelGGL(k_leaf_box, dim3((unsigned)((nl + 3) / 4)), dim3(256), 0, st, n, leaf, nl, L, c->pos64, q,
                       c->node_box, c->leaf_org, xslots);
    hipLaunchKernelGGL(k_leaf_local, dim3(blocks_for(n)), dim3(256), 0, st, n, leaf, c->pos64, c->leaf_org, q,
                       c->pos32);
    for (int l = L - 1; l >= 0; l--)
        hipLaunchKernelGGL(k_box_up, dim3(blocks_for((int64_t)1 << l)), dim3(256), 0, st, l, c->node_box);
    std::vector<uint64_t> hws(STAT_SLOTS * STAT_STRIDE), hx(STAT_SLOTS * STAT_STRIDE);
    uint32_t fl = 0;
    hipError_t e1 = hipMemcpyAsync(&fl, flags, 4, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipMemcpyAsync(hws.data(), wst, STAT_BYTES, hipMemcpyDeviceToHost, st);
    hipError_t e3 = hipMemcpyAsync(hx.data(), xslots, STAT_BYTES, hipMemcpyDeviceToHost, st);
    hipError_t e4 = hipStreamSynchronize(st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
        set_error("build_cells: HIP error %s", hipGetErrorString(e4 != hipSuccess ? e4 : e1));
        return fail(FCFC_EHIP);
    }
    dev_free(scr, st);
    scr = nullptr;
    if (fl & (VF_NONFINITE | VF_WNONFINITE)) {
        set_error("build_cells: non-finite position or weight");
        dev_free(blk, st);
        delete c;
        return FCFC_ENONFINITE;
    }
    if (fl & VF_BOX) {
        set_error("build_cells: a point lies outside the plan bounds");
        dev_free(blk, st);
        delete c;
        return FCFC_EBOX;
    }
    uint64_t xb = 0;
    for (int sl = 0; sl < STAT_SLOTS; sl++) xb = std::max<uint64_t>(xb, hx[(size_t)sl * STAT_STRIDE]);
    double ext;
    memcpy(&ext, &xb, 8);
    c->tree_ext = ext;
    if (weighted) {
        uint64_t bmin = 0, bmax = 0;
        weight_stats_reduce(hws.data(), &bmin, &bmax);
        double a, b;
        memcpy(&a, &bmin, 8);
        memcpy(&b, &bmax, 8);
        c->wmin = (bmin == ~0ull) ? 0.0 : a;
        c->wmax = b;
    }
    *out = c;
    return FCFC_OK;
}

// ---------------------------------------------------------------------------
// dual-tree work list: one thread per A leaf and B subtree of level `split`
// (enough threads to fill the device) walks that subtree depth first
// (stackless: the tree is implicit), drops nodes whose bounding box lies
// farther than the prune radius from the leaf's, takes whole the node ranges
// of B leaves and of nodes lying wholly within reach, and merges consecutive
// ranges (tree order keeps a subtree's points contiguous).  Auto counts take
// B points at or after the A leaf only, the leaf itself with the j > i rule.
// ---------------------------------------------------------------------------
struct TreeWL {
    const double* boxA;
    const double* boxB;
    int LA, LB, leafA, leafB;
    uint64_t nlA, nlB;
    int64_t nA, nB;
    double rlim2, rin2;
    uint32_t bchunk;
    int is_auto;
    int split;  // each thread walks one B subtree of this level for its A leaf
};

__device__ inline void box_d2(const double* a, const double* b, double& mind2, double& maxd2) {
    mind2 = 0.0;
    maxd2 = 0.0;
    for (int i = 0; i < 3; i++) {
        const double g = fmax(0.0, fmax(b[i] - a[3 + i], a[i] - b[3 + i]));
        const double m = fmax(b[3 + i] - a[i], a[3 + i] - b[i]);
        mind2 += g * g;
        maxd2 += m * m;
    }
}

__global__ __launch_bounds__(256) void k_tree_items(TreeWL w, const uint32_t* __restrict__ ioff,
                                                    uint32_t* __restrict__ icount, Item* __restrict__ items,
                                                    uint32_t items_cap) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (w.nlA << w.split)) return;
    const uint64_t ua = tid >> w.split;
    const int l0 = w.split;
    const uint32_t a0 = (uint32_t)(ua * (uint64_t)w.leafA);
    const uint32_t a1 = (uint32_t)std::min<int64_t>((int64_t)a0 + w.leafA, w.nA);
    uint32_t cnt = 0;
    if (a1 <= a0) {
        if (!items) icount[tid] = 0;
        return;
    }
    const double* ab = w.boxA + 6 * (((size_t)1 << w.LA) - 1 + tnode_of_unit(w.LA, ua, w.nlA));
    double abox[6];
    for (int i = 0; i < 6; i++) abox[i] = ab[i];
    uint32_t base = items ? ioff[tid] : 0u;
    const uint32_t meta0 = (1u << 16) | (1u << 18) | (1u << 20);  // no periodic shift
    auto put = [&](uint32_t b0, uint32_t b1, bool same) {
        for (uint32_t s = b0; s < b1; s += w.bchunk) {
            const uint32_t e = min(b1, s + w.bchunk);
            if (items) {
                const uint32_t at = base + cnt;
                if (at < items_cap) {
                    Item it;
                    it.a_begin = a0;
                    it.b_begin = s;
                    it.b_end = e;
                    it.b_rowcell = s / (uint32_t)w.leafB;
                    it.acnt_xb0 = a1 - a0;
                    it.meta = meta0 | (same ? (ITEM_SAMEROW << 24) : 0u);
                    it.cost = (uint32_t)min<uint64_t>((uint64_t)(a1 - a0) * (e - s), 0xffffffffull);
                    it.tile = (uint32_t)ua;
                    items[at] = it;
                }
            }
            cnt++;
        }
    };
    uint32_t rb = 0, re = 0;
    bool open = false;
    auto flush = [&]() {
        if (open) put(rb, re, false);
        open = false;
    };
    auto emit = [&](uint32_t s, uint32_t e) {
        if (w.is_auto) {
            s = max(s, a0);
            if (s >= e) return;
            if (s < a1) {  // the range holds the A leaf itself (ranges are whole leaves)
                flush();
                put(a0, a1, true);
                s = a1;
                if (s >= e) return;
            }
        }
        if (open && s == re) {
            re = e;
        } else {
            flush();
            rb = s;
            re = e;
            open = true;
        }
    };
    int l = l0;
    uint64_t k = tid & ((1ull << l0) - 1);
    for (;;) {
        const uint32_t u0 = tunit_bound(l, k, w.nlB), u1 = tunit_bound(l, k + 1, w.nlB);
        const uint32_t p0 = (uint32_t)std::min<int64_t>((int64_t)u0 * w.leafB, w.nB);
        const uint32_t p1 = (uint32_t)std::min<int64_t>((int64_t)u1 * w.leafB, w.nB);
        bool down = false;
        if (p1 > p0 && !(w.is_auto && p1 <= a0)) {
            double mind2, maxd2;
            box_d2(abox, w.boxB + 6 * (((size_t)1 << l) - 1 + k), mind2, maxd2);
            if (mind2 < w.rlim2) {
                if (l == w.LB || maxd2 < w.rin2)
                    emit(p0, p1);
                else
                    down = true;
            }
        }
        if (down) {
            l++;
            k *= 2;
            continue;
        }
        while (l > l0 && (k & 1)) {
            l--;
            k >>= 1;
        }
        if (l == l0) break;
        k++;
    }
    flush();
    if (!items) icount[tid] = cnt;
}

// B tree level whose subtrees the work-list threads take: about 2^19 threads
// (each walks its subtree alone, so it takes many of them to cover the
// latency of the walk; on MI355X 2^16 left the full C3 DR work list at 100 ms,
// 2^19 at 55 ms)
int tree_wl_split(const Cells* ca, const Cells* cb) {
    const uint64_t nla = tree_leaves(ca);
    int s = 0;
    while (s < cb->tree_levels && (nla << s) < 524288) s++;
    return s;
}

void tree_items_enqueue(const Cells* ca, const Cells* cb, bool is_auto, double rprune, double coord_max, int bchunk,
                        const uint32_t* ioff, uint32_t* icount, Item* items, uint32_t items_cap, hipStream_t st) {
    TreeWL w;
    w.boxA = ca->node_box;
    w.boxB = cb->node_box;
    w.LA = ca->tree_levels;
    w.LB = cb->tree_levels;
    w.leafA = ca->xbits;
    w.leafB = cb->xbits;
    w.nlA = tree_leaves(ca);
    w.nlB = tree_leaves(cb);
    w.nA = ca->n;
    w.nB = cb->n;
    // a box pair is dropped only when its smallest distance exceeds the prune
    // radius by far more than the rounding of the FP64 box arithmetic
    const double lim = rprune * (1.0 + 1e-9) + 1e-9 * coord_max;
    w.rlim2 = lim * lim;
    w.rin2 = rprune * rprune;
    w.bchunk = (uint32_t)bchunk;
    w.is_auto = is_auto ? 1 : 0;
    w.split = tree_wl_split(ca, cb);
    hipLaunchKernelGGL(k_tree_items, dim3(blocks_for((int64_t)(w.nlA << w.split))), dim3(256), 0, st, w, ioff, icount,
                       items, items_cap);
}

}  // namespace fcfc
