// triplets.hip -- exact triangle counts by side lengths, the three-point
// extension of the pair counts (Sect. 6 lists three-point statistics as
// future work): every set of three distinct points is counted once when its
// three sides s = |x_b - x_a| (Sect. 2.5; minimum image in a periodic box)
// lie in [e_0, e_n), into the bin of its sorted side bins (a <= b <= c).
//
// Each wave takes primaries i in sorted order, a few at a time from a global
// cursor.  It gathers the points after i (in the order of their coordinates,
// z first) whose side to i is in range from the cells around i's cell into an
// LDS list (ballot compaction; the list is the scan order of the cells), then
// bins every pair (p, q) of the list by its third side.  A triangle is found
// exactly once, from its first vertex in that order.
// Lists longer than the LDS region are taken in chunks: chunk A against itself
// and against every later chunk B, each chunk rebuilt by rescanning the cells.
//
// Sides are formed in FP32 from displacements relative to the primary and
// binned with a banded look-up table (binlut.h) whose bands cover the FP32
// error; a side inside an edge's band is formed again in FP64, in the same
// operation order as the pair definition, and binned exactly, so the counts
// equal those of the FP64 definition.
//
// Weighted counts: a triangle weighs fl(fl(a b) c) for its three point
// weights sorted by value, a <= b <= c (independent of the point order); a
// bin's weighted count is the exact sum of those products rounded once.  Each
// product times 2^S is an integer below 2^62 in magnitude; the workgroup sums
// it in three LDS limbs (bits 0-23, 24-47 and the signed rest), which cannot
// overflow before 2^40 additions, and merges them into 128-bit accumulators.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "binlut.h"
#include "internal.h"

namespace fcfc {

constexpr int TRI_CAP = 128;       // list entries per LDS region (two regions per wave)
// pairs of a list taken by column q in groups (p, q), (p + 1, q), p even; a
// full list has TRI_CAP^2 / 4 groups
constexpr int TRI_GROUPS = TRI_CAP / 2 * ((TRI_CAP + 1) / 2);
constexpr int TRI_ORDERED_MAX_BINS = 16;  // ordered counters (nb^3 of them) up to this many bins
constexpr int TRI_MAX_WAVES = 16;
constexpr int TRI_MAX_BINS = 32;   // sorted bin triples: C(34, 3) = 5984 u64 counters

struct TriArgs {
    const double* pos;        // sorted FP64 xyz
    const uint32_t* cs;       // cell_start, ncell + 1
    const uint32_t* xkey;     // sorted keys: cell << xbits | sub-cell x
    int xbits;
    const int4* stencil;      // rows of cells: (dy, dz, first dx, last dx)
    int nst;
    int nx, ny, nz;
    double L, halfL;          // L > 0: periodic
    double inner;             // > 0: a primary farther than this from every face has no wrapped neighbour
    int exact_pairs;          // 1: two neighbours may differ by more than L/2 per axis (L < 4 r): FP64 sides
    int64_t n;
    const double* w;          // sorted weights (weighted counts)
    double wscale;            // 2^S
    unsigned long long* out_w;  // 2 per counter: low, high 64 bits of a signed 128-bit sum
    int off_wl;               // LDS: three u64 limbs per counter
    const uint4* tab;         // table blob for FP32 squared sides (binlut.h layout)
    int tab_words;
    int off_band, off_e, off_hist, off_t3, off_ptab, off_lists;
    int lists_words;          // 16-byte words of the list regions
    int nb;
    float scale, vmax;
    float top;                // index of the table's last entry (out of range), as a float
    int nhist;                // counters: sorted bin triples, or nb^3 ordered ones
    unsigned long long* out;  // nhist counters (accumulated)
    uint32_t* cursor;
    uint32_t claim;           // primaries taken per claim of the cursor
    unsigned long long* stats;  // [0] side evaluations, [1] FP64 rechecks
};

// Squared separation of (bx, by, bz) - (ax, ay, az), the definition: per-axis
// minimum image in a periodic box, then (dx dx + dy dy) + dz dz, no fused
// operations.
__device__ __attribute__((always_inline)) inline double side2(double ax, double ay, double az, double bx, double by,
                                                              double bz, double L, double h) {
    double dx = bx - ax, dy = by - ay, dz = bz - az;
    if (L > 0.0) {
        dx = dx > h ? dx - L : (dx < -h ? dx + L : dx);
        dy = dy > h ? dy - L : (dy < -h ? dy + L : dy);
        dz = dz > h ? dz - L : (dz < -h ? dz + L : dz);
    }
    return (dx * dx + dy * dy) + dz * dz;  // built with -ffp-contract=off
}

// Bin of a squared side v >= 0 formed in FP32 (table bands cover its error):
// the bin, -1 (out of range) or -2 (inside an edge's band: the FP64 side
// decides).  The index is clamped to the table's last entry, which lies above
// the top band and holds "out of range".
__device__ __attribute__((always_inline)) inline int bin32(const BinTable& T, float top, float v) {
    int e = T.lut[(uint32_t)fminf(v * T.scale, top)];
    if (e < -1) {
        const int k0 = -2 - e;
        e = bin_near(T, k0, v);
        if (e == -2)
            e = bin_hot(T.band, T.nb, k0, v);
        else if (e >= T.nb)
            e = -1;
    }
    return e;
}

// Counter of the sorted bin triple a <= b <= c: C(c+2, 3) + C(b+1, 2) + a,
// with C(c+2, 3) from a table in LDS (t3[c]) and the full-rate 24-bit
// multiply for C(b+1, 2).
__device__ __attribute__((always_inline)) inline int tri_slot(const int* t3, int b1, int b2, int b3) {
    const int lo = min(b1, min(b2, b3));
    const int hi = max(b1, max(b2, b3));
    const int mid = b1 + b2 + b3 - lo - hi;
    return t3[hi] + (int)(__umul24((uint32_t)mid, (uint32_t)mid + 1u) >> 1) + lo;
}

// Counter of the ordered bin triple (b1, b2, b3): (b1 nb + b2) nb + b3.  A list
// entry of bin b holds the code b nb^2 | (b nb) << 16, so the counter of the
// triangle (primary, p, q) with third side in bin s is
// (code_p & 0xffff) + (code_q >> 16) + s.  The six orders of a triple are
// summed into its sorted bin after the count.
__device__ __attribute__((always_inline)) inline uint32_t tri_code(uint32_t bin, uint32_t nb) {
    const uint32_t c1 = __umul24(bin, nb);
    return __umul24(c1, nb) | (c1 << 16);
}

// A list of neighbours of the primary: each entry's displacement from the
// primary in FP32 with the bin of its side to the primary, or that bin's code
// for ordered counters (bits of .w), its sorted index and, for weighted
// counts, its weight.
struct TriList {
    float4* d;
    uint32_t* idx;
    double* w;
};

// weight of a triangle: the three weights sorted by value, fl(fl(a b) c)
__device__ __attribute__((always_inline)) inline double tri_weight(double a, double b, double c) {
    const double lo = fmin(a, fmin(b, c)), hi = fmax(a, fmax(b, c));
    const double mid = (a <= b) ? ((b <= c) ? b : fmax(a, c)) : ((a <= c) ? a : fmax(b, c));
    return (lo * mid) * hi;
}

// add q = (weight) 2^S, an integer below 2^62 in magnitude, to counter k
__device__ __attribute__((always_inline)) inline void tri_add_weight(unsigned long long* wl, int nhist, int k,
                                                                    double q) {
    const long long t = (long long)q;
    atomicAdd(&wl[k], (unsigned long long)(t & 0xffffffll));
    atomicAdd(&wl[nhist + k], (unsigned long long)((t >> 24) & 0xffffffll));
    atomicAdd(&wl[2 * nhist + k], (unsigned long long)(t >> 48));
}

__device__ inline void wave_sync_lds_tri() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline uint32_t lane_prefix_tri(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One candidate neighbour j of the primary: the FP64 displacement of the
// definition (minimum image when Lw > 0), rounded to FP32, with the bin of its
// squared length (from the FP32 square; inside an edge's band from the FP64
// one) or -1.
template <bool U>
__device__ __attribute__((always_inline)) inline int tri_point(const TriArgs& a, const BinTable& T, double dx,
                                                              double dy, double dz, double Lw, float4& e,
                                                              uint32_t& rechk) {
    if (Lw > 0.0) {
        const double h = a.halfL;
        dx = dx > h ? dx - Lw : (dx < -h ? dx + Lw : dx);
        dy = dy > h ? dy - Lw : (dy < -h ? dy + Lw : dy);
        dz = dz > h ? dz - Lw : (dz < -h ? dz + Lw : dz);
    }
    e = make_float4((float)dx, (float)dy, (float)dz, 0.f);
    int bin = bin32(T, a.top, __builtin_fmaf(e.z, e.z, __builtin_fmaf(e.y, e.y, e.x * e.x)));
    if (bin == -2) {
        rechk++;
        bin = bin_exact(T.E, T.nb, (dx * dx + dy * dy) + dz * dz);
    }
    e.w = __uint_as_float(U ? tri_code((uint32_t)bin, (uint32_t)a.nb) : (uint32_t)bin);
    return bin;
}

// Scan the cells around primary i (cell cx, cy, cz) and keep the neighbours
// after i with side ij in range whose position in the scan order lies in
// [lo, lo + TRI_CAP), into R.  Returns the number found up to the point the
// scan stopped (all of them when `whole`).  nside (wave-uniform) counts the
// points scanned.
//
// "After" is the order of the stored coordinates (z, then y, then x, then the
// sorted index): a triangle is found once, from its first vertex in that
// order.  A plane through the primary splits its neighbourhood in halves, so
// the lists are about equally long (an order by cell splits it at cell faces,
// and the pairs of the longer lists cost more than the shorter ones save).
// Rows of a higher z cell lie wholly after i and rows of a lower one wholly
// before it (the cell of a coordinate never decreases as it grows); rows of
// i's own z cell are tested point by point.
//
// The scan order is the stencil's rows in turn, each row's one or two index
// ranges (a periodic run of cells wraps once at most), and the points of a
// range by index.  The ranges of up to 32 rows are fetched at once, one per
// lane, and their concatenation is then taken 128 positions at a time, two
// per lane, so that the loads of a step do not wait on one another.
template <bool W, bool U>
__device__ uint32_t tri_gather(const TriArgs& a, const BinTable& T, int64_t i, double xi, double yi, double zi,
                               uint32_t icell, int cx, int cy, int cz, double Lw, uint32_t lo, bool whole,
                               const TriList& R, int lane, unsigned long long& nside, uint32_t& rechk) {
    uint32_t running = 0;
    const uint32_t hi = lo + TRI_CAP;
    for (int s0 = 0; s0 < a.nst; s0 += 32) {
        // lane l: range (l & 1) of row s0 + l / 2; mixed: a row of i's z cell
        uint32_t b0 = 0, b1 = 0;
        bool mixed = false;
        const int s = s0 + (lane >> 1);
        if (s < a.nst) {
            const int4 o = a.stencil[s];
            int y = cy + o.x, z = cz + o.y, xa = cx + o.z, xb = cx + o.w;
            int pa1 = 1, pb1 = 0;
            bool inside_grid = true;
            if (a.L > 0.0) {
                y += y < 0 ? a.ny : (y >= a.ny ? -a.ny : 0);
                z += z < 0 ? a.nz : (z >= a.nz ? -a.nz : 0);
                if (xa < 0) {
                    pa1 = 0;
                    pb1 = xb;
                    xa += a.nx;
                    xb = a.nx - 1;
                } else if (xb >= a.nx) {
                    pa1 = 0;
                    pb1 = xb - a.nx;
                    xb = a.nx - 1;
                }
            } else {
                inside_grid = y >= 0 && y < a.ny && z >= 0 && z < a.nz;
                xa = max(xa, 0);
                xb = min(xb, a.nx - 1);
            }
            const int x0 = (lane & 1) ? pa1 : xa, x1 = (lane & 1) ? pb1 : xb;
            if (inside_grid && x0 <= x1 && z >= cz) {
                const uint32_t row = ((uint32_t)z * (uint32_t)a.ny + (uint32_t)y) * (uint32_t)a.nx;
                b0 = a.cs[row + (uint32_t)x0];
                b1 = a.cs[row + (uint32_t)x1 + 1u];
                mixed = z == cz;
            }
        }
        const uint32_t cnt = b1 - b0;
        uint32_t incl = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t v = (uint32_t)__shfl_up((int)incl, d, 64);
            if (lane >= d) incl += v;
        }
        const uint32_t excl = incl - cnt;
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        // ranges not yet used up, in scan order (wave-uniform); ranges of i's z cell
        uint64_t open = __ballot(cnt > 0);
        const uint64_t mixm = __ballot(mixed);
        bool stop = false;
        for (uint32_t c0 = 0; c0 < total && !stop; c0 += 128) {
            const uint32_t g0 = c0 + (uint32_t)lane, g1 = g0 + 64u;
            uint32_t j0 = 0, j1 = 0;
            bool t0 = false, t1 = false;  // the point lies in i's z cell: test its order
            while (open) {
                const int L = __builtin_ctzll(open);
                const uint32_t se = (uint32_t)__builtin_amdgcn_readlane((int)excl, L);
                const uint32_t sc = (uint32_t)__builtin_amdgcn_readlane((int)cnt, L);
                const uint32_t sb = (uint32_t)__builtin_amdgcn_readlane((int)b0, L);
                const bool mx = (mixm >> L) & 1ull;
                if (se >= c0 + 128u) break;
                if (g0 - se < sc) {
                    j0 = sb + (g0 - se);
                    t0 = mx;
                }
                if (g1 - se < sc) {
                    j1 = sb + (g1 - se);
                    t1 = mx;
                }
                if (se + sc > c0 + 128u) break;  // the range goes on into the next step
                open &= open - 1;
            }
            const bool v0 = g0 < total, v1 = g1 < total;
            double p0x = 0, p0y = 0, p0z = 0, p1x = 0, p1y = 0, p1z = 0;
            if (v0) {
                p0x = a.pos[3 * (size_t)j0];
                p0y = a.pos[3 * (size_t)j0 + 1];
                p0z = a.pos[3 * (size_t)j0 + 2];
            }
            if (v1) {
                p1x = a.pos[3 * (size_t)j1];
                p1y = a.pos[3 * (size_t)j1 + 1];
                p1z = a.pos[3 * (size_t)j1 + 2];
            }
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const uint32_t j = h ? j1 : j0;
                const double px = h ? p1x : p0x, py = h ? p1y : p0y, pz = h ? p1z : p0z;
                const bool after = !(h ? t1 : t0) ||
                                   (pz > zi || (pz == zi && (py > yi || (py == yi && (px > xi || (px == xi && j > i))))));
                const bool v = (h ? v1 : v0) && after;
                float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
                int bin = -1;
                if (v) bin = tri_point<U>(a, T, px - xi, py - yi, pz - zi, Lw, e, rechk);
                const bool ok = bin >= 0;
                const uint64_t m = __ballot(ok);
                if (ok) {
                    const uint32_t seq = running + lane_prefix_tri(m);
                    if (seq >= lo && seq < hi) {
                        const uint32_t k = seq - lo;
                        R.d[k] = e;
                        R.idx[k] = j;
                        if (W) R.w[k] = a.w[j];
                    }
                }
                running += (uint32_t)__popcll(m);
            }
            nside += min(total - c0, 128u);
            stop = !whole && running >= hi;
        }
        if (stop) break;
    }
    wave_sync_lds_tri();
    return running;
}

// The side between list entries p and q: FP32 from the two displacements
// (both within reach of the primary, so their difference is the minimum image
// with no wrap), binned; inside a band, the FP64 side of the definition from
// the sorted positions.
// EXACT: the box is too small for that (L < 4 r): every side is the FP64 one.
// `live` false: a padding pair whose result is discarded (not counted as a
// recheck); its entries are valid, so the recheck's reads stay in bounds.
template <bool EXACT>
__device__ __attribute__((always_inline)) inline int tri_side_bin(const TriArgs& a, const BinTable& T, float4 ep,
                                                                 float4 eq, const uint32_t* pidx, int p,
                                                                 const uint32_t* qidx, int q, bool live,
                                                                 uint32_t& rechk) {
    const float ex = eq.x - ep.x, ey = eq.y - ep.y, ez = eq.z - ep.z;
    int b = EXACT ? -2 : bin32(T, a.top, __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex)));
    if (b == -2) {
        rechk += live ? 1u : 0u;
        const double* pp = a.pos + 3 * (size_t)pidx[p];
        const double* pq = a.pos + 3 * (size_t)qidx[q];
        b = bin_exact(T.E, T.nb, side2(pp[0], pp[1], pp[2], pq[0], pq[1], pq[2], a.L, a.halfL));
    }
    return b;
}

// Counter of the triangle whose two sides to the primary are list entries with
// .w bits wp and wq and whose third side is in bin s.
template <bool U>
__device__ __attribute__((always_inline)) inline int tri_counter(const int* t3, uint32_t wp, uint32_t wq, int s) {
    if (U) return (int)((wp & 0xffffu) + (wq >> 16)) + s;
    return tri_slot(t3, (int)wp, (int)wq, s);
}

// Every pair p < q of one list.  Each lane takes groups (p, q), (p + 1, q)
// from the group table (p | q << 8, by column q, so the first G(m) groups are
// those of a list of m entries), reading the entry of q once for both pairs,
// two groups per step (g and g + 64) so that their reads overlap.  When
// p + 1 = q the group has one pair; a second group past the list repeats the
// first.  Such pairs are formed on valid entries and discarded.
template <bool W, bool U, bool EXACT>
__device__ void tri_self(const TriArgs& a, const BinTable& T, const TriList& R, int m, double wi, const int* t3,
                         const uint16_t* gtab, unsigned long long* hist, unsigned long long* wl, int lane,
                         unsigned long long& nside, uint32_t& rechk) {
    nside += (unsigned long long)(m * (m - 1) / 2);
    const int ng = (m / 2) * ((m + 1) / 2);
    for (int g = lane; g < ng; g += 128) {
        const bool second = g + 64 < ng;
        const uint32_t wA = gtab[g], wB = gtab[second ? g + 64 : g];
        int p[4], q[4];
        bool live[4];
        p[0] = wA & 255;
        q[0] = wA >> 8;
        p[1] = p[0] + 1;
        q[1] = q[0];
        p[2] = wB & 255;
        q[2] = wB >> 8;
        p[3] = p[2] + 1;
        q[3] = q[2];
        live[0] = true;
        live[1] = p[1] < q[1];
        live[2] = second;
        live[3] = second && p[3] < q[3];
        const float4 eqA = R.d[q[0]], eqB = R.d[q[2]];
        float4 ep[4];
#pragma unroll
        for (int u = 0; u < 4; u++) ep[u] = R.d[p[u]];
        int sb[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            sb[u] = tri_side_bin<EXACT>(a, T, ep[u], u < 2 ? eqA : eqB, R.idx, p[u], R.idx, q[u], live[u], rechk);
            sb[u] = live[u] ? sb[u] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint32_t cq = __float_as_uint(u < 2 ? eqA.w : eqB.w);
            const int k = tri_counter<U>(t3, __float_as_uint(ep[u].w), cq, max(sb[u], 0));
            if (W) {
                if (sb[u] >= 0) {
                    atomicAdd(&hist[k], 1ull);
                    tri_add_weight(wl, a.nhist, k, tri_weight(wi, R.w[p[u]], R.w[q[u]]) * a.wscale);
                }
            } else {
                // a pair out of range adds to this lane's dump counter (no branch)
                atomicAdd(&hist[sb[u] >= 0 ? k : a.nhist + lane], 1ull);
            }
        }
    }
}

// Every pair of an earlier list P (m1 entries) and a later list Q (m2), two
// entries of Q per lane per step.
template <bool W, bool U, bool EXACT>
__device__ void tri_cross(const TriArgs& a, const BinTable& T, const TriList& P, int m1, const TriList& Q, int m2,
                          double wi, const int* t3, unsigned long long* hist, unsigned long long* wl, int lane,
                          unsigned long long& nside, uint32_t& rechk) {
    nside += (unsigned long long)m1 * (unsigned long long)m2;
    for (int p = 0; p < m1; p++) {
        const float4 ep = P.d[p];
        const uint32_t pb = __float_as_uint(ep.w);
        const double pw = W ? P.w[p] : 0.0;
        for (int q = lane; q < m2; q += 128) {
            const bool two = q + 64 < m2;
            const int q1 = two ? q + 64 : q;
            const float4 e0 = Q.d[q], e1 = Q.d[q1];
            const int s0 = tri_side_bin<EXACT>(a, T, ep, e0, P.idx, p, Q.idx, q, true, rechk);
            int s1 = tri_side_bin<EXACT>(a, T, ep, e1, P.idx, p, Q.idx, q1, two, rechk);
            s1 = two ? s1 : -1;
            if (s0 >= 0) {
                const int k = tri_counter<U>(t3, pb, __float_as_uint(e0.w), s0);
                atomicAdd(&hist[k], 1ull);
                if (W) tri_add_weight(wl, a.nhist, k, tri_weight(wi, pw, Q.w[q]) * a.wscale);
            }
            if (s1 >= 0) {
                const int k = tri_counter<U>(t3, pb, __float_as_uint(e1.w), s1);
                atomicAdd(&hist[k], 1ull);
                if (W) tri_add_weight(wl, a.nhist, k, tri_weight(wi, pw, Q.w[q1]) * a.wscale);
            }
        }
    }
}

// LDS bytes of one list region: displacement + bin (16), index (4), weight (8)
template <bool W>
constexpr int tri_region_bytes() {
    return TRI_CAP * (W ? 28 : 20);
}

// U: ordered counters (nb^3 of them, unweighted counts with few bins);
// otherwise sorted-triple counters.
template <bool W, bool U>
__global__ __launch_bounds__(TRI_MAX_WAVES * 64) void k_triplets(TriArgs a) {
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    {
        uint4* dst = (uint4*)smem;
        for (int k = tid; k < a.tab_words; k += nthr) dst[k] = a.tab[k];
        unsigned long long* h = (unsigned long long*)(smem + a.off_hist);
        for (int k = tid; k < a.nhist; k += nthr) h[k] = 0ull;
        int* t3w = (int*)(smem + a.off_t3);
        for (int k = tid; k <= TRI_MAX_BINS; k += nthr) t3w[k] = k * (k + 1) * (k + 2) / 6;
        uint16_t* gt = (uint16_t*)(smem + a.off_ptab);
        for (int g = tid; g < TRI_GROUPS; g += nthr) {
            // column q holds ceil(q / 2) groups; the columns before q hold G(q)
            int q = (int)(2.0f * __builtin_amdgcn_sqrtf((float)g));
            while (q > 1 && (q / 2) * ((q + 1) / 2) > g) q--;
            while (((q + 1) / 2) * ((q + 2) / 2) <= g) q++;
            const int p = 2 * (g - (q / 2) * ((q + 1) / 2));
            gt[g] = (uint16_t)(p | (q << 8));
        }
        if (W) {
            unsigned long long* z = (unsigned long long*)(smem + a.off_wl);
            for (int k = tid; k < 3 * a.nhist; k += nthr) z[k] = 0ull;
        }
        // list regions start zeroed: a padding pair reads valid indices
        uint4* lz = (uint4*)(smem + a.off_lists);
        for (int k = tid; k < a.lists_words; k += nthr) lz[k] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    BinTable T;
    T.lut = (const int16_t*)smem;
    T.band = (const float2*)(smem + a.off_band);
    T.E = (const double*)(smem + a.off_e);
    T.scale = a.scale;
    T.vmax = a.vmax;
    T.nb = a.nb;
    unsigned long long* hist = (unsigned long long*)(smem + a.off_hist);
    const int* t3 = (const int*)(smem + a.off_t3);
    const uint16_t* ptab = (const uint16_t*)(smem + a.off_ptab);
    unsigned long long* wl = W ? (unsigned long long*)(smem + a.off_wl) : nullptr;
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int RB = tri_region_bytes<W>();
    char* base = smem + a.off_lists + (size_t)wave * 2 * RB;
    TriList R1, R2;
    R1.d = (float4*)base;
    R1.idx = (uint32_t*)(R1.d + TRI_CAP);
    R1.w = (double*)(R1.idx + TRI_CAP);
    R2.d = (float4*)(base + RB);
    R2.idx = (uint32_t*)(R2.d + TRI_CAP);
    R2.w = (double*)(R2.idx + TRI_CAP);
    unsigned long long nside = 0;
    uint32_t rechk = 0;
    // Primaries are claimed `claim` at a time: one atomic per primary on the
    // one cursor serialised the whole grid (about 11 ns per claim).
    uint32_t next = 0, last = 0;
    for (;;) {
        if (next >= last) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(a.cursor, a.claim);
            base = __builtin_amdgcn_readfirstlane(base);
            if ((int64_t)base >= a.n) break;
            next = base;
            last = (uint32_t)std::min<int64_t>((int64_t)base + a.claim, a.n);
        }
        const int64_t i = next++;
        const double xi = a.pos[3 * (size_t)i], yi = a.pos[3 * (size_t)i + 1], zi = a.pos[3 * (size_t)i + 2];
        const double wi = W ? a.w[i] : 0.0;
        const uint32_t cell = a.xkey[i] >> a.xbits;
        const int cx = (int)(cell % (uint32_t)a.nx);
        const int cy = (int)((cell / (uint32_t)a.nx) % (uint32_t)a.ny);
        const int cz = (int)(cell / ((uint32_t)a.nx * (uint32_t)a.ny));
        // a primary this far inside the box has no neighbour across a face:
        // its sides need no minimum image
        const bool inside = a.inner > 0.0 && xi > a.inner && xi < a.L - a.inner && yi > a.inner &&
                            yi < a.L - a.inner && zi > a.inner && zi < a.L - a.inner;
        const double Lw = inside ? 0.0 : a.L;
        const uint32_t m = tri_gather<W, U>(a, T, i, xi, yi, zi, cell, cx, cy, cz, Lw, 0, true, R1, lane, nside, rechk);
        if (m < 2) continue;
        const uint32_t nch = (m + TRI_CAP - 1) / TRI_CAP;
        for (uint32_t A = 0; A < nch; A++) {
            if (A > 0) {
                wave_sync_lds_tri();
                tri_gather<W, U>(a, T, i, xi, yi, zi, cell, cx, cy, cz, Lw, A * TRI_CAP, false, R1, lane, nside, rechk);
            }
            const int mA = (int)std::min<uint32_t>(TRI_CAP, m - A * TRI_CAP);
            if (a.exact_pairs)
                tri_self<W, U, true>(a, T, R1, mA, wi, t3, ptab, hist, wl, lane, nside, rechk);
            else
                tri_self<W, U, false>(a, T, R1, mA, wi, t3, ptab, hist, wl, lane, nside, rechk);
            for (uint32_t B = A + 1; B < nch; B++) {
                wave_sync_lds_tri();
                tri_gather<W, U>(a, T, i, xi, yi, zi, cell, cx, cy, cz, Lw, B * TRI_CAP, false, R2, lane, nside, rechk);
                const int mB = (int)std::min<uint32_t>(TRI_CAP, m - B * TRI_CAP);
                if (a.exact_pairs)
                    tri_cross<W, U, true>(a, T, R1, mA, R2, mB, wi, t3, hist, wl, lane, nside, rechk);
                else
                    tri_cross<W, U, false>(a, T, R1, mA, R2, mB, wi, t3, hist, wl, lane, nside, rechk);
            }
        }
        wave_sync_lds_tri();
    }
    __syncthreads();
    for (int k = tid; k < a.nhist; k += nthr) {
        const unsigned long long v = hist[k];
        if (v) atomicAdd(&a.out[k], v);
        if (W) {
            // limbs -> one signed 128-bit value, added with the carry
            const unsigned long long l0 = wl[k], l1 = wl[a.nhist + k], l2 = wl[2 * a.nhist + k];
            if (l0 | l1 | l2) {
                const __int128 s128 = ((__int128)(long long)l2 << 48) + ((__int128)l1 << 24) + (__int128)l0;
                const unsigned long long vlo = (unsigned long long)s128;
                unsigned long long vhi = (unsigned long long)(s128 >> 64);
                const unsigned long long o = atomicAdd(&a.out_w[2 * k], vlo);
                if (o + vlo < o) vhi += 1ull;
                if (vhi) atomicAdd(&a.out_w[2 * k + 1], vhi);
            }
        }
    }
    // statistics: one atomic per wave (nside is the same in every lane)
    for (int o = 32; o >= 1; o >>= 1) rechk += __shfl_xor(rechk, o, 64);
    if (lane == 0) {
        atomicAdd(&a.stats[0], nside);
        if (rechk) atomicAdd(&a.stats[1], (unsigned long long)rechk);
    }
}

// compact sorted-triple counters -> the row-major [nb][nb][nb] histogram
__global__ void k_tri_expand(const unsigned long long* __restrict__ c, int nb, int64_t* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nb * nb * nb) return;
    const int a = f / (nb * nb), b = (f / nb) % nb, cc = f % nb;
    out[f] = (a <= b && b <= cc) ? (int64_t)c[cc * (cc + 1) * (cc + 2) / 6 + b * (b + 1) / 2 + a] : 0;
}

// ordered-triple counters -> the row-major [nb][nb][nb] histogram: bin
// (a, b, c), a <= b <= c, sums the counters of the distinct orders of its bins
__global__ void k_tri_fold(const unsigned long long* __restrict__ c, int nb, int64_t* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nb * nb * nb) return;
    const int a = f / (nb * nb), b = (f / nb) % nb, cc = f % nb;
    if (!(a <= b && b <= cc)) {
        out[f] = 0;
        return;
    }
    const int v[3] = {a, b, cc};
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    unsigned long long sum = 0;
    int seen[6];
    int ns = 0;
    for (int k = 0; k < 6; k++) {
        const int idx = (v[perm[k][0]] * nb + v[perm[k][1]]) * nb + v[perm[k][2]];
        bool dup = false;
        for (int u = 0; u < ns; u++) dup = dup || seen[u] == idx;
        if (dup) continue;
        seen[ns++] = idx;
        sum += c[idx];
    }
    out[f] = (int64_t)sum;
}

// signed 128-bit fixed point (lo, hi) times 2^-S, rounded once to nearest even
__device__ inline double tri_fixed_to_double(unsigned long long lo, unsigned long long hi, int S) {
    const __int128 v = (__int128)(((unsigned __int128)hi << 64) | (unsigned __int128)lo);
    const bool neg = v < 0;
    const unsigned __int128 m = neg ? (unsigned __int128)(-(v + 1)) + 1u : (unsigned __int128)v;
    if (m == 0) return 0.0;
    const unsigned long long mh = (unsigned long long)(m >> 64), ml = (unsigned long long)m;
    const int nbits = mh ? 128 - __clzll(mh) : 64 - __clzll(ml);
    double r;
    if (nbits <= 53) {
        r = ldexp((double)ml, -S);
    } else {
        const int sh = nbits - 53;
        unsigned __int128 top = m >> sh;
        const unsigned __int128 rem = m - (top << sh);
        const unsigned __int128 half = (unsigned __int128)1 << (sh - 1);
        if (rem > half || (rem == half && (top & 1u))) top += 1u;
        r = ldexp((double)(unsigned long long)top, sh - S);
    }
    return neg ? -r : r;
}

__global__ void k_tri_expand_w(const unsigned long long* __restrict__ acc, int nb, int S, double* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nb * nb * nb) return;
    const int a = f / (nb * nb), b = (f / nb) % nb, cc = f % nb;
    if (a <= b && b <= cc) {
        const int k = cc * (cc + 1) * (cc + 2) / 6 + b * (b + 1) / 2 + a;
        out[f] = tri_fixed_to_double(acc[2 * k], acc[2 * k + 1], S);
    } else {
        out[f] = 0.0;
    }
}

// cell offsets whose nearest points can be within reff of each other; a
// periodic axis with fewer than 2K + 1 cells takes each of its cells once
static void tri_stencil(const Grid& g, double rprune, std::vector<int4>& st) {
    const double s = g.side;
    const double reff = rprune * (1.0 + 1e-7) + 1e-9 * s;
    const int K = (int)ceil(reff / s) + 1;
    const int n[3] = {g.nx, g.ny, g.nz};
    std::vector<int> off[3];
    std::vector<bool> prune[3];
    for (int ax = 0; ax < 3; ax++) {
        if (g.L > 0 && n[ax] < 2 * K + 1) {
            for (int d = 0; d < n[ax]; d++) {
                off[ax].push_back(d);
                prune[ax].push_back(false);
            }
        } else {
            for (int d = -K; d <= K; d++) {
                off[ax].push_back(d);
                prune[ax].push_back(true);
            }
        }
    }
    st.clear();
    for (size_t iz = 0; iz < off[2].size(); iz++)
        for (size_t iy = 0; iy < off[1].size(); iy++)
            for (size_t ix = 0; ix < off[0].size(); ix++) {
                double t2 = 0;
                const int d[3] = {off[0][ix], off[1][iy], off[2][iz]};
                const bool pr[3] = {prune[0][ix], prune[1][iy], prune[2][iz]};
                for (int ax = 0; ax < 3; ax++) {
                    if (!pr[ax]) continue;
                    const double gap = std::max(std::abs(d[ax]) - 1, 0) * s;
                    t2 += gap * gap;
                }
                if (t2 < reff * reff) st.push_back(make_int4(d[0], d[1], d[2], 0));
            }
}

// The stencil as rows: the cells of one (dy, dz) form one run of x offsets
// (the prune keeps |dx| up to a bound, or a whole short periodic axis), stored
// as (dy, dz, first dx, last dx).
static void tri_rows(std::vector<int4>& st) {
    std::vector<int4> rows;
    for (const int4& c : st) {
        bool found = false;
        for (int4& r : rows)
            if (r.x == c.y && r.y == c.z) {
                r.z = std::min(r.z, c.x);
                r.w = std::max(r.w, c.x);
                found = true;
                break;
            }
        if (!found) rows.push_back(make_int4(c.y, c.z, c.x, c.x));
    }
    st.swap(rows);
}

}  // namespace fcfc

using namespace fcfc;

extern "C" fcfc_status fcfc_count_triplets(fcfc_plan_t plan, fcfc_cells_t cells, int64_t* d_counts,
                                           double* d_wcounts, void* stream) {
    clear_error();
    Plan* p = (Plan*)plan;
    Cells* c = (Cells*)cells;
    if (!p) {
        set_error("count_triplets: null plan");
        return FCFC_EINVAL;
    }
    if (p->kind != FCFC_BIN_S) {
        set_error("count_triplets: needs an s plan");
        return FCFC_EINVAL;
    }
    const int nb = p->n1;
    if (nb > TRI_MAX_BINS) {
        set_error("count_triplets: at most %d bins", TRI_MAX_BINS);
        return FCFC_ERANGE;
    }
    if (!c || !d_counts) {
        set_error("count_triplets: null cells or output");
        return FCFC_EINVAL;
    }
    if (c->tree) {
        set_error("count_triplets: takes the cells of a grid plan");
        return FCFC_EINVAL;
    }
    if (c->plan_id != p->id) {
        set_error("count_triplets: the cell set was built on a different plan");
        return FCFC_EGRID;
    }
    const bool weighted = d_wcounts != nullptr;
    if (weighted && !c->weighted) {
        set_error("count_triplets: weighted counts need a cell set built with weights");
        return FCFC_EINVAL;
    }
    // every product fl(fl(a b) c) is a multiple of 2^-S; its magnitude lies
    // between those of the smallest and the largest non-zero weights cubed
    int S = 0;
    if (weighted) FCFC_TRY(weight_scale_rule(c->wmin, c->wmax, c->wmin, c->wmax, 3, &S));
    hipStream_t st = (hipStream_t)stream;
    const Grid& g = c->grid;
    const double Lbox = g.L > 0 ? g.L : 0.0;
    // neighbours lie within r' (r plus room for rounding) of the primary
    const double rr = p->rprune * (1.0 + 1e-6) + 1e-9 * Lbox;
    // FP32 sides: a displacement from the primary is the FP64 one rounded to
    // FP32 (u r' per axis); the side between two neighbours is the rounded
    // difference of two of them (u 2 r' more), and the FP64 sides of the
    // definition carry a few ulps of the coordinates; twice that for margin
    const double U = 5.9604644775390625e-08;
    const double e_axis = 2.0 * (4.0 * U * rr + 4.0 * 2.220446049250313e-16 * (Lbox + rr));
    const Lut1D* Tp = nullptr;
    FCFC_TRY(plan_side_table(p, e_axis, &Tp));
    std::vector<int4> sten;
    tri_stencil(g, p->rprune, sten);
    tri_rows(sten);

    TriArgs a{};
    std::vector<char> blob_h;
    const BinBlob B = bin_blob(*Tp, blob_h);
    // unweighted counts with few bins use nb^3 ordered counters (no sort of
    // the three bins per triangle), folded into sorted bins afterwards
    const bool ordered = !weighted && nb <= TRI_ORDERED_MAX_BINS;
    a.nhist = ordered ? nb * nb * nb : (nb + 2) * (nb + 1) * nb / 6;
    a.off_band = B.off_band;
    a.off_e = B.off_e;
    a.off_hist = B.bytes;
    a.off_t3 = a.off_hist + bin_al16((a.nhist + 64) * 8);  // counters, then 64 dump counters
    a.off_ptab = a.off_t3 + bin_al16((TRI_MAX_BINS + 1) * 4);
    a.off_wl = a.off_ptab + bin_al16(TRI_GROUPS * 2);
    a.off_lists = a.off_wl + (weighted ? bin_al16(a.nhist * 24) : 0);
    const int per_wave = 2 * (weighted ? tri_region_bytes<true>() : tri_region_bytes<false>());
    int dev = 0, maxlds = 65536;
    FCFC_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) maxlds = 65536;
    int waves = TRI_MAX_WAVES;
    while (waves > 1 && a.off_lists + waves * per_wave > maxlds) waves--;
    if (a.off_lists + waves * per_wave > maxlds) {
        set_error("count_triplets: the tables and histogram of %d bins do not fit the LDS%s", nb,
                  weighted ? " with weighted sums" : "");
        return FCFC_ERANGE;
    }
    const int lds = a.off_lists + waves * per_wave;
    a.lists_words = waves * per_wave / 16;
    const int variant = weighted ? 2 : (ordered ? 1 : 0);
    const void* kern = weighted  ? (const void*)k_triplets<true, false>
                       : ordered ? (const void*)k_triplets<false, true>
                                 : (const void*)k_triplets<false, false>;

    // device block: tables, stencil, counters, weighted sums, cursor
    const size_t sz_tab = (size_t)B.bytes, sz_st = sten.size() * sizeof(int4), sz_out = (size_t)a.nhist * 8,
                 sz_w = weighted ? (size_t)a.nhist * 16 : 0;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_st = sz_tab, o_out = o_st + up(sz_st), o_w = o_out + up(sz_out), o_cur = o_w + up(sz_w),
                 total = o_cur + 256;
    std::vector<char>& h = p->host_stage;
    h.assign(o_out, 0);
    memcpy(h.data(), blob_h.data(), sz_tab);
    memcpy(h.data() + o_st, sten.data(), sz_st);
    char* blk = nullptr;
    FCFC_TRY(dev_alloc((void**)&blk, total, st));
    fcfc_status s = FCFC_OK;
    if (hipMemcpyAsync(blk, h.data(), o_out, hipMemcpyHostToDevice, st) != hipSuccess) s = FCFC_EHIP;
    if (s == FCFC_OK && !p->stats_dev) {
        if (hipMalloc(&p->stats_dev, 64) != hipSuccess || hipEventCreate(&p->ev0) != hipSuccess ||
            hipEventCreate(&p->ev1) != hipSuccess)
            s = FCFC_EHIP;
    }
    if (s == FCFC_OK) {
        fill_u64((uint64_t*)(blk + o_out), 0ull, a.nhist, st);
        if (weighted) fill_u64((uint64_t*)(blk + o_w), 0ull, 2 * (int64_t)a.nhist, st);
        fill_u32((uint32_t*)(blk + o_cur), 0u, 1, st);
        fill_u64((uint64_t*)p->stats_dev, 0ull, 8, st);
        a.pos = c->pos64;
        a.w = weighted ? c->w : nullptr;
        a.wscale = ldexp(1.0, S);
        a.out_w = weighted ? (unsigned long long*)(blk + o_w) : nullptr;
        a.cs = c->cell_start;
        a.xkey = c->xkey;
        a.xbits = c->xbits;
        a.stencil = (const int4*)(blk + o_st);
        a.nst = (int)sten.size();
        a.nx = g.nx;
        a.ny = g.ny;
        a.nz = g.nz;
        a.L = g.L > 0 ? g.L : 0.0;
        a.halfL = a.L * 0.5;
        // two neighbours differ by less than 2 r' per axis: with 2 r' <= L / 2
        // that difference is their minimum image
        a.inner = (a.L > 0 && 4.0 * rr <= a.L) ? rr : 0.0;
        a.exact_pairs = (a.L > 0 && 4.0 * rr > a.L) ? 1 : 0;
        a.n = c->n;
        a.tab = (const uint4*)blk;
        a.tab_words = B.bytes / 16;
        a.nb = nb;
        a.scale = B.scale;
        a.vmax = B.vmax;
        a.top = (float)(B.nt - 1);
        a.out = (unsigned long long*)(blk + o_out);
        a.cursor = (uint32_t*)(blk + o_cur);
        a.stats = (unsigned long long*)p->stats_dev;
        static bool attr_set[3][64] = {};
        if (dev >= 64 || !attr_set[variant][dev]) {
            if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds) != hipSuccess)
                s = FCFC_EHIP;
            else if (dev < 64)
                attr_set[variant][dev] = true;
        }
        int occ = 0;
        if (s == FCFC_OK && hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, waves * 64, lds) != hipSuccess)
            s = FCFC_EHIP;
        if (s == FCFC_OK) {
            int64_t nblk = (int64_t)device_cu_count() * std::max(1, occ);
            const int64_t need = std::max<int64_t>(1, (c->n + waves - 1) / waves);
            nblk = std::min(nblk, need);
            // about eight claims per wave, at most 32 primaries each
            a.claim = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(32, c->n / (nblk * waves * 8)));
            if (hipEventRecord(p->ev0, st) != hipSuccess) s = FCFC_EHIP;
            if (s == FCFC_OK) {
                if (weighted)
                    hipLaunchKernelGGL((k_triplets<true, false>), dim3((unsigned)nblk), dim3(waves * 64), (size_t)lds,
                                       st, a);
                else if (ordered)
                    hipLaunchKernelGGL((k_triplets<false, true>), dim3((unsigned)nblk), dim3(waves * 64), (size_t)lds,
                                       st, a);
                else
                    hipLaunchKernelGGL((k_triplets<false, false>), dim3((unsigned)nblk), dim3(waves * 64), (size_t)lds,
                                       st, a);
                if (hipGetLastError() != hipSuccess || hipEventRecord(p->ev1, st) != hipSuccess) s = FCFC_EHIP;
            }
            if (s == FCFC_OK) {
                const int nf = nb * nb * nb;
                if (ordered)
                    hipLaunchKernelGGL(k_tri_fold, dim3((nf + 255) / 256), dim3(256), 0, st,
                                       (const unsigned long long*)(blk + o_out), nb, d_counts);
                else
                    hipLaunchKernelGGL(k_tri_expand, dim3((nf + 255) / 256), dim3(256), 0, st,
                                       (const unsigned long long*)(blk + o_out), nb, d_counts);
                if (weighted)
                    hipLaunchKernelGGL(k_tri_expand_w, dim3((nf + 255) / 256), dim3(256), 0, st,
                                       (const unsigned long long*)(blk + o_w), nb, S, d_wcounts);
                if (hipGetLastError() != hipSuccess) s = FCFC_EHIP;
            }
        }
    }
    dev_free(blk, st);
    if (s != FCFC_OK) {
        set_error("count_triplets: HIP failure");
        return s;
    }
    p->last_stream = st;
    p->last_counts = d_counts;
    p->last_counts_n = (int64_t)nb * nb * nb;
    p->have_stats = true;
    p->stats.items = c->n;
    p->stats.lut_entries = (int32_t)Tp->tab.size();
    p->stats.group_waves = waves;
    return FCFC_OK;
}
