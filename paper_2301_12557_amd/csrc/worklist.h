// worklist.h -- work-list enumeration kernels (A tiles x pruned B row pieces).
#pragma once

#include "internal.h"

namespace fcfc {

struct Tile {
    uint32_t a_begin;  // first A point
    uint32_t a_count;  // points in the tile
    uint32_t row;      // A row index cz*ny + cy
    uint32_t x01;      // first (bits 0..15) and last (bits 16..31) cell x spanned
};

struct WLArgs {
    int nx, ny, nz;
    int seg;        // most cells a tile may span
    int tile;       // points per tile
    int bchunk;     // B points per item
    int nrows;      // stencil rows
    int periodic;
    int is_auto;
    uint32_t tiles_cap;
    int ncat;       // catalogues stacked along z (batched build); 1 otherwise
};

__global__ void k_tile_count(const uint32_t* __restrict__ csA, WLArgs w, uint32_t* __restrict__ tcount);
__global__ void k_tile_write(const uint32_t* __restrict__ csA, const float4* __restrict__ posA, WLArgs w,
                             const uint32_t* __restrict__ toff, Tile* __restrict__ tiles);
__global__ void k_item_count(const Tile* __restrict__ tiles, const uint32_t* __restrict__ ntiles_dev,
                             const int4* __restrict__ srows, const uint32_t* __restrict__ csB, WLArgs w,
                             uint32_t* __restrict__ icount);
__global__ void k_item_write(const Tile* __restrict__ tiles, const uint32_t* __restrict__ ntiles_dev,
                             const int4* __restrict__ srows, const uint32_t* __restrict__ csB, WLArgs w,
                             const uint32_t* __restrict__ ioff, Item* __restrict__ items, uint32_t items_cap);
__global__ void k_cat_items(const uint32_t* __restrict__ toff, const uint32_t* __restrict__ ioff,
                            const uint32_t* __restrict__ nitems_dev, WLArgs w, uint32_t* __restrict__ cat_items);
__global__ void k_chunk_prefix(const uint32_t* __restrict__ cat_items, const uint32_t* __restrict__ cat_order,
                               int ncat, int chunk_items, uint32_t* __restrict__ prefix, uint32_t* __restrict__ nchunks);
__global__ void k_item_keys(const Item* __restrict__ items, const uint32_t* __restrict__ nitems_dev,
                            uint32_t cap, uint32_t* __restrict__ key, uint32_t* __restrict__ val);
__global__ void k_item_permute(const Item* __restrict__ in, const uint32_t* __restrict__ perm,
                               const uint32_t* __restrict__ nitems_dev, uint32_t cap, Item* __restrict__ out);

size_t scan_scratch_bytes(int64_t n);
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, void* scratch,
                        hipStream_t st);
size_t radix_scratch_bytes(int64_t n);
void radix_sort_pairs(uint32_t** k, uint32_t** v, uint32_t** tk, uint32_t** tv, int64_t n, int key_bits,
                      void* scratch, hipStream_t st);

}  // namespace fcfc
