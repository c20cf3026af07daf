// worklist.h -- work-list enumeration kernels (A tiles x pruned B row pieces).
#pragma once

#include "internal.h"

namespace fcfc {

struct Tile {
    uint32_t a_begin;  // first A point
    uint32_t a_count;  // points in the tile
    uint32_t row;      // A row index cz*ny + cy
    uint32_t x01;      // first (bits 0..15) and last (bits 16..31) cell x spanned
    uint32_t klo, khi; // sort keys of the first and last point (x-ordered within the row)
};

struct WLArgs {
    int nx, ny, nz;
    int seg;        // most cells a tile may span
    int tile;       // points per tile
    int bchunk;     // B points per item
    int nrows;      // stencil rows (x: dy, y: dz, z: kx, w: float bits of the x reach in cells)
    // sorted keys of the B points (cell key << xbits | sub-cell x): B ranges
    // are trimmed to the points within reach of the tile's x extent
    const uint32_t* keyB;
    int xbits;
    int periodic;
    int is_auto;
    uint32_t tiles_cap;
    int ncat;       // catalogues stacked along z (batched build); 1 otherwise
    int full_rows;  // the stencil table holds every row (auto pairs then skip the lower half)
    // pair mode (batched build, npairs > 0): items of every (A catalogue, B
    // catalogue) pair; pair-tile t of pair p is tile ptile_first[p] + t -
    // ptile_off[p], and index ranges of k_item_count / k_item_write run over
    // pair-tiles (ptiles_cap of them) instead of tiles
    const int32_t* pairs;         // 2 per pair: A catalogue, B catalogue (equal: auto count)
    const uint32_t* ptile_off;    // npairs + 1
    const uint32_t* ptile_first;  // npairs
    int npairs;
    uint32_t ptiles_cap;
};

__global__ void k_tile_count(const uint32_t* __restrict__ csA, WLArgs w, uint32_t* __restrict__ tcount);
__global__ void k_tile_write(const uint32_t* __restrict__ csA, const uint32_t* __restrict__ keyA, WLArgs w,
                             const uint32_t* __restrict__ toff, Tile* __restrict__ tiles);
__global__ void k_item_count(const Tile* __restrict__ tiles, const uint32_t* __restrict__ ntiles_dev,
                             const int4* __restrict__ srows, const uint32_t* __restrict__ csB, WLArgs w,
                             uint32_t* __restrict__ icount);
__global__ void k_item_write(const Tile* __restrict__ tiles, const uint32_t* __restrict__ ntiles_dev,
                             const int4* __restrict__ srows, const uint32_t* __restrict__ csB, WLArgs w,
                             const uint32_t* __restrict__ ioff, Item* __restrict__ items, uint32_t items_cap);
__global__ void k_pair_tiles(const uint32_t* __restrict__ toff, const uint32_t* __restrict__ ntiles_dev, WLArgs w,
                             uint32_t* __restrict__ ptile_off, uint32_t* __restrict__ ptile_first);
__global__ void k_pair_items(const uint32_t* __restrict__ ioff, const uint32_t* __restrict__ nitems_dev, WLArgs w,
                             uint32_t* __restrict__ pair_items);
__global__ void k_chunk_prefix(const uint32_t* __restrict__ cat_items, const uint32_t* __restrict__ cat_order,
                               int ncat, int chunk_items, uint32_t* __restrict__ prefix, uint32_t* __restrict__ nchunks);
__global__ void k_item_keys(const Item* __restrict__ items, const uint32_t* __restrict__ nitems_dev,
                            uint32_t cap, uint32_t* __restrict__ key, uint32_t* __restrict__ val);
__global__ void k_pair_item_keys(const Item* __restrict__ items, const uint32_t* __restrict__ nitems_dev,
                                 uint32_t cap, const uint32_t* __restrict__ pair_items, int npairs, uint32_t last,
                                 uint32_t* __restrict__ key, uint32_t* __restrict__ val);
__global__ void k_pair_pred_keys(const Item* __restrict__ items, const uint32_t* __restrict__ nitems_dev,
                                 uint32_t cap, const uint32_t* __restrict__ pair_items, int npairs, uint32_t last,
                                 const float* __restrict__ pred, const unsigned long long* __restrict__ bad,
                                 uint32_t* __restrict__ key, uint32_t* __restrict__ val);
__global__ void k_item_permute(const Item* __restrict__ in, const uint32_t* __restrict__ perm,
                               const uint32_t* __restrict__ nitems_dev, uint32_t cap, Item* __restrict__ out);

size_t scan_scratch_bytes(int64_t n);
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, void* scratch,
                        hipStream_t st);
size_t radix_scratch_bytes(int64_t n);
void radix_sort_pairs(uint32_t** k, uint32_t** v, uint32_t** tk, uint32_t** tv, int64_t n, int key_bits,
                      void* scratch, hipStream_t st);

}  // namespace fcfc
