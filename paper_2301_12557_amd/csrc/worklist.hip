// worklist.hip -- enumeration of work items on the GPU.
//
// A tile is a run of at most `tile` consecutive sorted points of one A row
// (fixed cy, cz) spanning at most `seg` consecutive cells.
// For each tile and each row offset (dy, dz) of the pruned stencil, the B
// cells that can hold a pair in range form the x range [x0 - kx, x1 + kx]
// of the B row; since cells of a row are consecutive in the sort order their
// points are one contiguous range.  A periodic box splits that range into at
// most three pieces (direct, wrapped left, wrapped right), each with its own
// image shift (the per-node-pair wrap offsets of Sect. 3.1).  Auto counts
// use the half stencil (each unordered row pair once, Sect. 3.1) and, in the
// A row itself, only B points after the A point (mask flag) plus the piece
// wrapped from the right.
// A batched build may list pairs of catalogues (auto or cross): the items of
// pair (a, b) are those of the tiles of catalogue a against the rows of
// catalogue b, and items come out grouped by pair.
#include <algorithm>

#include "internal.h"
#include "worklist.h"

namespace fcfc {

__device__ inline int floor_div(int a, int n) {
    int q = a / n;
    if ((a % n != 0) && ((a < 0) != (n < 0))) q--;
    return q;
}

// Tiles of one A row: runs of up to `tile` consecutive sorted points, cut
// early only where a run would reach into a cell `seg` cells past the cell
// of its first point.  Calls emit(first point, count, first cell, last cell)
// in order.
template <typename F>
__device__ inline void row_tiles(const uint32_t* __restrict__ csA, int64_t rowcell, const WLArgs& w, int seg, F emit) {
    const uint32_t p1 = csA[rowcell + w.nx];
    uint32_t a = csA[rowcell];
    int c = 0;
    while (a < p1) {
        while (csA[rowcell + c + 1] <= a) c++;  // cell holding point a
        const uint32_t lim = csA[rowcell + min(c + seg, w.nx)];
        const uint32_t e = min(min(a + (uint32_t)w.tile, lim), p1);
        int c2 = c;
        while (csA[rowcell + c2 + 1] <= e - 1) c2++;  // cell holding the last point
        emit(a, e - a, c, c2);
        a = e;
    }
}

__global__ void k_tile_count(const uint32_t* __restrict__ csA, WLArgs w, uint32_t* __restrict__ tcount) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nrow = (int64_t)w.ny * w.nz * w.ncat;
    if (r >= nrow) return;
    uint32_t n = 0;
    row_tiles(csA, r * w.nx, w, w.seg, [&](uint32_t, uint32_t, int, int) { n++; });
    tcount[r] = n;
}

__global__ void k_tile_write(const uint32_t* __restrict__ csA, const uint32_t* __restrict__ keyA, WLArgs w,
                             const uint32_t* __restrict__ toff, Tile* __restrict__ tiles) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nrow = (int64_t)w.ny * w.nz * w.ncat;
    if (r >= nrow) return;
    uint32_t t = toff[r];
    row_tiles(csA, r * w.nx, w, w.seg, [&](uint32_t a, uint32_t cnt, int cxa, int cxb) {
        Tile tl;
        tl.a_begin = a;
        tl.a_count = cnt;
        tl.row = (uint32_t)r;
        tl.x01 = (uint32_t)(cxa & 0xffff) | ((uint32_t)cxb << 16);
        tl.klo = keyA[a];
        tl.khi = keyA[a + cnt - 1];
        tiles[t++] = tl;
    });
}

// First index in [lo, hi) of a sorted key array whose key is >= v (> v when
// `upper`).
__device__ inline uint32_t key_search(const uint32_t* __restrict__ key, uint32_t lo, uint32_t hi, uint64_t v,
                                      bool upper) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        const uint64_t k = key[mid];
        if (upper ? (k <= v) : (k < v)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Enumerate the pieces of (tile, stencil row) against the B rows of
// catalogue bcat (< 0: the tile's own catalogue); emit(item) is called for
// every work item, in a fixed order.
template <typename F>
__device__ inline void tile_row_items(const Tile& tl, int4 srow, const uint32_t* __restrict__ csB,
                                      const WLArgs& w, uint32_t tile_id, int bcat, bool is_auto, F emit) {
    // rows of a batched build are (catalogue, z, y); wrapping stays within the catalogue
    int cy = (int)(tl.row % (uint32_t)w.ny);
    int czc = (int)(tl.row / (uint32_t)w.ny);
    int cat = czc / w.nz;
    int cz = czc - cat * w.nz;
    if (bcat < 0) bcat = cat;
    int dy = srow.x, dz = srow.y, kx = srow.z;
    // an auto count takes each unordered pair of rows once (half stencil)
    if (is_auto && w.full_rows && (dz < 0 || (dz == 0 && dy < 0))) return;
    int yu = cy + dy, zu = cz + dz;
    int sy = 0, sz = 0, yb = yu, zb = zu;
    if (w.periodic) {
        sy = floor_div(yu, w.ny);
        sz = floor_div(zu, w.nz);
        if (sy < -1 || sy > 1 || sz < -1 || sz > 1) return;
        yb = yu - sy * w.ny;
        zb = zu - sz * w.nz;
    } else if (yu < 0 || yu >= w.ny || zu < 0 || zu >= w.nz) {
        return;
    }
    bool same = is_auto && dy == 0 && dz == 0;
    int x0 = (int)(tl.x01 & 0xffff), x1 = (int)(tl.x01 >> 16);
    int xlo = x0 - kx, xhi = x1 + kx;
    uint32_t rowcell = (((uint32_t)bcat * (uint32_t)w.nz + (uint32_t)zb) * (uint32_t)w.ny + (uint32_t)yb) * (uint32_t)w.nx;
    // the tile's x extent in cells of its row, bounded by the sort keys of its
    // first and last point (the key holds the x position within the cell on
    // 2^xbits steps, rounded down)
    const double steps = (double)(1u << w.xbits);
    const uint32_t xmask = (1u << w.xbits) - 1u;
    const uint32_t rowcellA = tl.row * (uint32_t)w.nx;
    const double ua_lo = (double)((tl.klo >> w.xbits) - rowcellA) + (double)(tl.klo & xmask) / steps;
    const double ua_hi = (double)((tl.khi >> w.xbits) - rowcellA) + (double)((tl.khi & xmask) + 1u) / steps;
    // largest |dx| of a pair in range for this row, in cells, rounded up; the
    // extra 1e-6 cells covers the rounding of the keys' FP64 positions
    const double reach = (double)__int_as_float(srow.w) + 1e-6;
    // pieces: 0 = direct, 1 = wrapped from the left (sx = -1), 2 = wrapped from the right (sx = +1)
    for (int pc = 0; pc < 3; pc++) {
        int c0, c1, sx;
        if (pc == 0) {
            c0 = max(xlo, 0);
            c1 = min(xhi, w.nx - 1);
            sx = 0;
        } else if (pc == 1) {
            if (!w.periodic || same || xlo >= 0) continue;
            c0 = max(xlo, -w.nx) + w.nx;
            c1 = min(xhi, -1) + w.nx;
            sx = -1;
        } else {
            if (!w.periodic || xhi < w.nx) continue;
            c0 = max(xlo, w.nx) - w.nx;
            c1 = min(xhi, 2 * w.nx - 1) - w.nx;
            sx = 1;
        }
        if (c0 > c1) continue;
        uint32_t bb = csB[rowcell + (uint32_t)c0], be = csB[rowcell + (uint32_t)c1 + 1];
        uint32_t flags = 0;
        if (same && pc == 0) {
            flags |= ITEM_SAMEROW;
            bb = max(bb, tl.a_begin);
        }
        if (w.keyB) {
            // B points of this piece within reach of the tile, in the B row's
            // own cell units (the piece's image shift moves them by sx nx)
            const double lo = ua_lo - reach - (double)(sx * w.nx);
            const double hi = ua_hi + reach - (double)(sx * w.nx);
            const uint64_t base = (uint64_t)rowcell << w.xbits;
            if (hi < (double)c0) continue;  // the whole piece is out of reach
            if (lo > (double)c0) bb = key_search(w.keyB, bb, be, base + (uint64_t)floor(lo * steps), false);
            if (hi < (double)(c1 + 1)) be = key_search(w.keyB, bb, be, base + (uint64_t)floor(hi * steps), true);
        }
        if (bb >= be) continue;
        int xb0 = c0 + sx * w.nx;
        uint32_t meta = ((uint32_t)(uint8_t)(int8_t)dy) | ((uint32_t)(uint8_t)(int8_t)dz << 8) |
                        ((uint32_t)(sx + 1) << 16) | ((uint32_t)(sy + 1) << 18) | ((uint32_t)(sz + 1) << 20) |
                        (flags << 24);
        for (uint32_t b = bb; b < be; b += (uint32_t)w.bchunk) {
            Item it;
            it.a_begin = tl.a_begin;
            it.b_begin = b;
            it.b_end = min(be, b + (uint32_t)w.bchunk);
            it.b_rowcell = rowcell;
            // the kernel walks B cells from the cell of the item's first point
            const int xs = w.keyB ? (int)((w.keyB[b] >> w.xbits) - rowcell) + sx * w.nx : xb0;
            it.acnt_xb0 = (tl.a_count & 0xffffu) | ((uint32_t)(uint16_t)(int16_t)xs << 16);
            it.meta = meta;
            uint64_t pairs = (uint64_t)tl.a_count * (uint64_t)(it.b_end - it.b_begin);
            it.cost = (uint32_t)min<uint64_t>(pairs, 0xffffffffull);
            it.tile = tile_id;
            emit(it);
        }
    }
}

// Pair-tile pt of a pair-mode list -> pair and tile; false past the last one.
__device__ inline bool pair_tile(const WLArgs& w, int64_t pt, int& pr, uint32_t& ti) {
    if (pt >= (int64_t)w.ptile_off[w.npairs]) return false;
    int lo = 0, hi = w.npairs;  // ptile_off[lo] <= pt < ptile_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)w.ptile_off[mid] <= pt) lo = mid;
        else hi = mid;
    }
    pr = lo;
    ti = w.ptile_first[lo] + (uint32_t)(pt - (int64_t)w.ptile_off[lo]);
    return true;
}

// Items of index t = (tile or pair-tile) * nrows + stencil row.
template <typename F>
__device__ inline void index_items(const Tile* __restrict__ tiles, uint32_t ntiles, const int4* __restrict__ srows,
                                   const uint32_t* __restrict__ csB, const WLArgs& w, int64_t t, F emit) {
    const int64_t ti0 = t / w.nrows;
    const int r = (int)(t % w.nrows);
    if (w.npairs > 0) {
        int pr;
        uint32_t ti;
        if (!pair_tile(w, ti0, pr, ti)) return;
        const int ca = w.pairs[2 * pr], cb = w.pairs[2 * pr + 1];
        tile_row_items(tiles[ti], srows[r], csB, w, ti, cb, ca == cb, emit);
    } else if (ti0 < (int64_t)ntiles) {
        tile_row_items(tiles[ti0], srows[r], csB, w, (uint32_t)ti0, -1, w.is_auto != 0, emit);
    }
}

static __device__ inline int64_t index_total(const WLArgs& w) {
    return (int64_t)(w.npairs > 0 ? w.ptiles_cap : w.tiles_cap) * w.nrows;
}

__global__ void k_item_count(const Tile* __restrict__ tiles, const uint32_t* __restrict__ ntiles_dev,
                             const int4* __restrict__ srows, const uint32_t* __restrict__ csB, WLArgs w,
                             uint32_t* __restrict__ icount) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= index_total(w)) return;
    uint32_t c = 0;
    index_items(tiles, *ntiles_dev, srows, csB, w, t, [&](const Item&) { c++; });
    icount[t] = c;
}

__global__ void k_item_write(const Tile* __restrict__ tiles, const uint32_t* __restrict__ ntiles_dev,
                             const int4* __restrict__ srows, const uint32_t* __restrict__ csB, WLArgs w,
                             const uint32_t* __restrict__ ioff, Item* __restrict__ items,
                             uint32_t items_cap) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= index_total(w)) return;
    uint32_t o = ioff[t];
    index_items(tiles, *ntiles_dev, srows, csB, w, t, [&](const Item& it) {
        if (o < items_cap) items[o] = it;
        o++;
    });
}

// Pair-tile ranges: the tiles of catalogue c are those of its rows
// [c ny nz, (c+1) ny nz), consecutive in the tile list.  One thread (a few
// hundred pairs at most).
__global__ void k_pair_tiles(const uint32_t* __restrict__ toff, const uint32_t* __restrict__ ntiles_dev, WLArgs w,
                             uint32_t* __restrict__ ptile_off, uint32_t* __restrict__ ptile_first) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int64_t rows = (int64_t)w.ny * w.nz;
    const uint32_t ntiles = *ntiles_dev;
    uint32_t acc = 0;
    for (int p = 0; p < w.npairs; p++) {
        const int c = w.pairs[2 * p];
        const uint32_t t0 = toff[(int64_t)c * rows];
        const uint32_t t1 = (c + 1 < w.ncat) ? toff[(int64_t)(c + 1) * rows] : ntiles;
        ptile_first[p] = t0;
        ptile_off[p] = acc;
        acc += t1 - t0;
    }
    ptile_off[w.npairs] = acc;
}

// First work item of each pair (items come out grouped by pair), clamped to
// the item count so that a clamped list never sends a reader past it.
__global__ void k_pair_items(const uint32_t* __restrict__ ioff, const uint32_t* __restrict__ nitems_dev, WLArgs w,
                             uint32_t* __restrict__ pair_items) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > w.npairs) return;
    const uint32_t n = *nitems_dev;
    const int64_t idx = (int64_t)w.ptile_off[p] * w.nrows;
    const uint32_t v = (p < w.npairs && idx < index_total(w)) ? ioff[idx] : n;
    pair_items[p] = v < n ? v : n;
}

// Chunks of `chunk_items` items per catalogue, catalogues in the given order
// (longest first); prefix[o] is the first chunk of the o-th catalogue.
__global__ void k_chunk_prefix(const uint32_t* __restrict__ cat_items, const uint32_t* __restrict__ cat_order,
                               int ncat, int chunk_items, uint32_t* __restrict__ prefix, uint32_t* __restrict__ nchunks) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int o = 0; o < ncat; o++) {
        uint32_t c = cat_order[o];
        uint32_t n = cat_items[c + 1] - cat_items[c];
        prefix[o] = acc;
        acc += (n + (uint32_t)chunk_items - 1) / (uint32_t)chunk_items;
    }
    prefix[ncat] = acc;
    *nchunks = acc;
}

// Longest-first key: the cost rounded to a power of sqrt(2) (bucket 0..63),
// reversed so that an ascending stable sort puts the largest first while
// items of one bucket keep their enumeration order (A tiles and B rows stay
// close together in memory).
__device__ inline uint32_t cost_key(uint32_t c) {
    uint32_t lg = c ? 31u - (uint32_t)__clz(c) : 0u;  // floor(log2 c)
    uint32_t half = (lg >= 1 && ((c >> (lg - 1)) & 1u)) ? 1u : 0u;
    return 63u - min(63u, 2u * lg + half);
}

__global__ void k_item_keys(const Item* __restrict__ items, const uint32_t* __restrict__ nitems_dev,
                            uint32_t cap, uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    uint32_t n = *nitems_dev;
    key[i] = (i < n) ? cost_key(items[i].cost) : 255u;
    val[i] = i;
}

// The same key within each pair of a pair-mode list: (pair << 6) | cost key,
// so that a stable sort keeps the pairs where they are (items are grouped by
// pair) and puts each pair's largest items first.  Items past the end get
// `last`, above every other key.
__global__ void k_pair_item_keys(const Item* __restrict__ items, const uint32_t* __restrict__ nitems_dev,
                                 uint32_t cap, const uint32_t* __restrict__ pair_items, int npairs, uint32_t last,
                                 uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    uint32_t k = last;
    if (i < *nitems_dev) {
        int lo = 0, hi = npairs;  // pair_items[lo] <= i < pair_items[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pair_items[mid] <= i) lo = mid;
            else hi = mid;
        }
        k = ((uint32_t)lo << 6) | cost_key(items[i].cost);
    }
    key[i] = k;
    val[i] = i;
}

// The same with the learned key: half-octave buckets of the predicted time
// (log2 of ticks), longest first; the cost key for every item if any
// prediction was not finite (*bad).
__global__ void k_pair_pred_keys(const Item* __restrict__ items, const uint32_t* __restrict__ nitems_dev,
                                 uint32_t cap, const uint32_t* __restrict__ pair_items, int npairs, uint32_t last,
                                 const float* __restrict__ pred, const unsigned long long* __restrict__ bad,
                                 uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    uint32_t k = last;
    if (i < *nitems_dev) {
        int lo = 0, hi = npairs;  // pair_items[lo] <= i < pair_items[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pair_items[mid] <= i) lo = mid;
            else hi = mid;
        }
        uint32_t c;
        if (*bad) {
            c = cost_key(items[i].cost);
        } else {
            const float b = fminf(fmaxf(2.f * pred[i], 0.f), 63.f);
            c = 63u - (uint32_t)b;
        }
        k = ((uint32_t)lo << 6) | c;
    }
    key[i] = k;
    val[i] = i;
}

__global__ void k_item_permute(const Item* __restrict__ in, const uint32_t* __restrict__ perm,
                               const uint32_t* __restrict__ nitems_dev, uint32_t cap, Item* __restrict__ out) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    if (i < *nitems_dev) out[i] = in[perm[i]];
}

}  // namespace fcfc
