// binlut.h -- binning one FP64 squared separation with a look-up table over
// the squared edges (Sect. 3.2.3): FP32 table entry, FP32 band ends around
// every edge, FP64 binary search for a value inside a band.  The tables come
// from plan_bin_table (bands that cover the rounding of a value to FP32) and
// are laid out in LDS as [int16 entries][(lo, hi) float pairs, nb + 2][FP64
// squared edges, nb + 1].
#pragma once

#include <math.h>
#include <string.h>

#include <vector>

#include "internal.h"

namespace fcfc {

// Edges certainly at or below v, walking forward from the first edge k0 whose
// band meets the table entry (edges before it lie wholly below the entry);
// band[k] = (lo_k, hi_k).  Returns the bin, -1 (no bin) or -2 (v inside an
// edge's band).
__device__ inline int bin_hot(const float2* __restrict__ band, int nb, int k0, float v) {
    int k = k0;
    for (; k <= nb; k++) {
        const float2 b = band[k];
        if (v >= b.y) continue;  // at or above E_k for certain
        if (v >= b.x) return -2;  // inside E_k's band
        break;                    // below E_k for certain
    }
    return (k >= 1 && k <= nb) ? k - 1 : -1;
}

// FP64 definition: the number c of squared edges at or below x, by binary
// search; bin c - 1 when 1 <= c <= nb.
__device__ inline int bin_exact(const double* __restrict__ E, int nb, double x) {
    int lo = 0, hi = nb + 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (E[mid] <= x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo >= 1 && lo <= nb) ? lo - 1 : -1;
}

struct BinTable {
    const int16_t* lut;
    const float2* band;  // (lo_k, hi_k) for k = 0..nb, then (+inf, +inf)
    const double* E;
    float scale, vmax;
    int nb;
};

// Table entry of x: the bin (>= 0), -1 (no bin) or a hot entry (<= -2).
__device__ __attribute__((always_inline)) inline int bin_entry(const BinTable& s, double x, float& v) {
    v = (float)x;
    // NaN and negative values (-0.0 compares equal to 0) and values at or
    // above the top band end (at or above E_n) land in no bin
    const bool ok = (x >= 0.0) && (v < s.vmax);
    const int e = s.lut[ok ? (uint32_t)(v * s.scale) : 0u];
    return ok ? e : -1;
}

// Rare path: walk the bands from k0; a value inside a band takes the FP64
// definition.
__device__ __attribute__((noinline)) inline int bin_resolve(const BinTable& s, int k0, float v, double x,
                                                            uint32_t& rechk) {
    int b = bin_hot(s.band, s.nb, k0, v);
    if (b == -2) {
        rechk++;
        b = bin_exact(s.E, s.nb, x);
    }
    return b;
}

// Place v against band k0 and the start of band k0+1: the bin, or -2 when
// that does not decide (inside a band, or several edges in one entry).  Bin
// nb (k0 = nb) means at or above the top edge.
__device__ __attribute__((always_inline)) inline int bin_near(const BinTable& s, int k0, float v) {
    const float2 b0 = s.band[k0];
    const float lo1 = s.band[k0 + 1].x;
    return v < b0.x ? k0 - 1 : ((v >= b0.y && v < lo1) ? k0 : -2);
}

// Bin of one value: 0..nb-1, or -1.
__device__ __attribute__((always_inline)) inline int bin_value(const BinTable& s, double x, uint32_t& rechk) {
    float v;
    int e = bin_entry(s, x, v);
    if (e < -1) {
        const int k0 = -2 - e;
        e = bin_near(s, k0, v);
        if (e == -2) e = bin_resolve(s, k0, v, x, rechk);
        if (e >= s.nb) e = -1;
    }
    return e;
}

// bin_value for a value known to be finite and non-negative (a squared
// separation of finite points): the FP64 sign and NaN test is not needed.
__device__ __attribute__((always_inline)) inline int bin_value_nonneg(const BinTable& s, double x, uint32_t& rechk) {
    const float v = (float)x;
    const bool ok = v < s.vmax;
    int e = s.lut[ok ? (uint32_t)(v * s.scale) : 0u];
    e = ok ? e : -1;
    if (e < -1) {
        const int k0 = -2 - e;
        e = bin_near(s, k0, v);
        if (e == -2) e = bin_resolve(s, k0, v, x, rechk);
        if (e >= s.nb) e = -1;
    }
    return e;
}

static inline int bin_al16(int b) { return (b + 15) & ~15; }

// Host: the tables blob in the LDS layout; offsets of the bands and edges and
// the blob size (a multiple of 16 bytes).
struct BinBlob {
    int nt = 0, nb = 0, off_band = 0, off_e = 0, bytes = 0;
    float scale = 1.f, vmax = 0.f;
};
inline BinBlob bin_blob(const Lut1D& T, std::vector<char>& h) {
    BinBlob b;
    b.nt = (int)T.tab.size();
    b.nb = T.n;
    b.off_band = bin_al16(b.nt * 2);
    b.off_e = b.off_band + bin_al16((b.nb + 2) * 8);
    b.bytes = b.off_e + bin_al16((b.nb + 1) * 8);
    b.scale = T.scale;
    b.vmax = T.vmax;
    h.assign((size_t)b.bytes, 0);
    memcpy(h.data(), T.tab.data(), (size_t)b.nt * 2);
    float* band = (float*)(h.data() + b.off_band);
    for (int k = 0; k <= b.nb; k++) {
        band[2 * k] = T.lo[k];
        band[2 * k + 1] = T.hi[k];
    }
    band[2 * (b.nb + 1)] = INFINITY;  // sentinel: no edge above the top one
    band[2 * (b.nb + 1) + 1] = INFINITY;
    memcpy(h.data() + b.off_e, T.E.data(), (size_t)(b.nb + 1) * 8);
    return b;
}

}  // namespace fcfc
