// count.hip -- the persistent pair-counting kernel and its host driver.
//
// Each wavefront pulls work items (A tile x B row piece) from a global
// cursor.  Its lanes hold up to P A points in registers (cell-local FP32);
// B points are wave-uniform and stream through scalar loads cell by cell.
// Per pair: FP32 displacement and squared separation on the vector ALUs,
// prune test, bin via the squared-separation look-up table in LDS
// (Sect. 3.2.3; hot entries resolve by comparison against the FP32 band ends,
// the reverse traversal of Sect. 3.2.1), mu from the hardware reciprocal
// square root, and an LDS atomic into the workgroup's private histogram
// (Sect. 4.1.2: private histograms instead of conflicting scatters).  Pairs
// inside an error band are queued per wave in LDS and re-evaluated 64 at a
// time with the FP64 definition from the sorted FP64 coordinates.  The
// workgroup histograms are merged into the global int64 (and exact 128-bit
// weighted) accumulators with global atomics.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "worklist.h"

namespace fcfc {

// Wave-uniform reads (items, B points, B cell offsets, B weights) go through
// the constant address space so that they become scalar loads; those arrays
// are never written while the kernel runs.
#if defined(__HIP_DEVICE_COMPILE__)
#define FCFC_CONST __attribute__((address_space(4)))
#else
#define FCFC_CONST
#endif
__device__ inline float4 ldc_f4(const float4* p, uint32_t i) {
    const float FCFC_CONST* q = (const float FCFC_CONST*)p + 4 * (size_t)i;
    return make_float4(q[0], q[1], q[2], q[3]);
}
__device__ inline double ldc_f64(const double* p, uint32_t i) { return ((const double FCFC_CONST*)p)[i]; }
__device__ inline uint32_t ldc_u32(const uint32_t* p, uint32_t i) { return ((const uint32_t FCFC_CONST*)p)[i]; }
__device__ inline int4 ldc_i4(const int4* p, uint32_t i) {
    const int FCFC_CONST* q = (const int FCFC_CONST*)p + 4 * (size_t)i;
    return make_int4(q[0], q[1], q[2], q[3]);
}
__device__ inline Item ldc_item(const Item* p, uint32_t i) {
    const uint32_t FCFC_CONST* q = (const uint32_t FCFC_CONST*)p + 8 * (size_t)i;
    Item it;
    it.a_begin = q[0];
    it.b_begin = q[1];
    it.b_end = q[2];
    it.b_rowcell = q[3];
    it.acnt_xb0 = q[4];
    it.meta = q[5];
    it.cost = q[6];
    it.tile = q[7];
    return it;
}

enum { COUNT_SINGLE = 0, COUNT_BATCH = 1, COUNT_TREE = 2 };
constexpr int CT_MAX = 1024;        // threads per workgroup (16 waves: 4 per SIMD, one workgroup per CU)
constexpr int QCAP = 192;           // compaction queue entries per wave (63 + 64 P), plus one dump entry
constexpr int QCAP_MID = 127;       // mid-point queues (16-byte entries) drain after each A point: 63 + 64
// recheck entries per wave: RB_FLUSH - 1 waiting plus the up to 64 of one
// binning pass (rechecks are rare; a small buffer leaves LDS for more waves)
constexpr int RB_FLUSH = 32;
constexpr int RB_CAP = RB_FLUSH + 64;
constexpr int ASTAGE = 128;         // staged A points per wave (mid-point line of sight)

// queue entry size in floats: (v1, v2, ids), or (dx, dy, dz, ids) for the
// mid-point line of sight
template <int KIND, int LOS>
struct QStride {
    static constexpr int value = (LOS == FCFC_LOS_MIDPOINT && KIND != FCFC_BIN_S) ? 4 : 3;
};
// A wavefront empties the LDS histograms into the outputs after claiming
// 2^26 candidate pairs since it last did (fcfc_tuning.flush_log2 lowers it).
constexpr int FLUSH_LOG2_MAX = 26;

struct CountArgs {
    const float4* posA;
    const float4* absA;
    const double* p64A;
    const double* wA;
    const float4* posB;
    const double* p64B;
    const double* wB;
    const uint32_t* csB;
    const Item* items;
    const uint32_t* nitems_dev;
    uint32_t* cursor;
    const int16_t* lut1;
    const int16_t* lut2;
    const float2* band1;  // (lo_k, hi_k) for k = 0..n1, then (+inf, +inf)
    const float2* band2;
    const double* E1;    // FP64 squared edges
    const double* E2;
    unsigned long long* out_counts;
    unsigned long long* out_w;  // 2 per bin: low, high 64 bits of a signed 128-bit sum
    unsigned long long* stats;  // [0] candidates [1] rechecks [5] bad prediction [6] early merges
    uint32_t* times;            // per item duration (wall clock ticks) or null
    int nlut1, nlut2;
    float scale1, scale2, vmax1, vmax2;
    int n1, n2, nbins;
    int nx;
    float side32;
    // tree counts: lattice origins of the A and B leaves (units of tree_q),
    // points per leaf, B leaves and B points
    const int4* leaf_orgA;
    const int4* leaf_orgB;
    float tree_q;
    uint32_t tree_leaf, tree_nleafB, nB;
    double L, halfL;
    float r2prune, d2small;
    float mu_n, tolA, tolB, tolC;
    int mu_top_closed;
    double wscale;  // 2^(S - 32): pair weight -> the high limb of the exact sum's fixed point
    int copies;
    unsigned long long flush_pairs;     // a wave merges after claiming this many pairs
    uint32_t grab_single;               // single claims below this list position
    unsigned long long grab_gap;        // then claims of up to 8 positions at least this many ticks apart
    uint32_t shard_count, shard_index;  // this launch takes items shard_index, + shard_count, ...
    // batched mode: chunks of items per output histogram (one per catalogue pair)
    const uint32_t* nchunks_dev;
    uint32_t* chunk_cursor;
    const uint32_t* chunk_prefix;  // ncat + 1, in histogram order
    const uint32_t* cat_order;     // histogram index at each order position
    const uint32_t* cat_items;     // ncat + 1: items of histogram c are [cat_items[c], cat_items[c+1])
    int ncat;                      // histograms
    int chunk_items;
    // LDS layout (bytes)
    int off_lut1, off_lut2, off_band1, off_band2, off_hist, off_whist, off_q, off_rb, off_astage,
        off_misc, lds_bytes;
};

// The arguments live in device memory and are read through the constant
// address space (scalar loads); a by-value kernel argument would be copied to
// scratch as soon as a helper takes its address.
typedef const CountArgs FCFC_CONST& ArgsRef;

struct Smem {
    const int16_t* lut1;
    const int16_t* lut2;
    const float2* band1;
    const float2* band2;
    uint32_t* hist;
    unsigned long long* wl;  // exact weighted limbs, [bin][2]: low 32 bits, high part (signed)
    float* qf;        // this wave's compaction queue (entries of QStride floats)
    const float* qf_lane;  // qf + lane * QStride: this lane's entry when binning from entry 0
    uint32_t* rb;     // this wave's recheck entries (a, b, item)
    float4* astage;   // this wave's A points in absolute FP32 (mid-point line of sight)
    unsigned long long* misc;
};

// ---------------------------------------------------------------------------
// FP64 definition (independent of the FP32 path): bins of one pair from the
// sorted FP64 coordinates.  Contraction is disabled for the whole library, so
// each product and sum below rounds separately, in the order written.
// Returns the flat bin or -1.  For a periodic box the item's image shift must
// be the minimum image of b as seen from a, otherwise the pair belongs to
// another item and -1 is returned.
// ---------------------------------------------------------------------------
__device__ inline int upper_edge_count(const double* __restrict__ E, int n, double v) {
    // number of edges E[0..n] with E[k] <= v (binary search)
    int lo = 0, hi = n + 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (E[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int KIND, int LOS>
__device__ int exact_bin(ArgsRef a, double ax, double ay, double az, double bx, double by, double bz,
                         int sx, int sy, int sz) {
    double dx = bx - ax;
    double dy = by - ay;
    double dz = bz - az;
    if (a.L > 0.0) {
        int cx = 0, cy = 0, cz = 0;
        if (dx > a.halfL) { dx -= a.L; cx = -1; } else if (dx < -a.halfL) { dx += a.L; cx = 1; }
        if (dy > a.halfL) { dy -= a.L; cy = -1; } else if (dy < -a.halfL) { dy += a.L; cy = 1; }
        if (dz > a.halfL) { dz -= a.L; cz = -1; } else if (dz < -a.halfL) { dz += a.L; cz = 1; }
        if (cx != sx || cy != sy || cz != sz) return -1;
    }
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double d2 = (xx + yy) + zz;
    double pi2 = 0.0;
    if (KIND != FCFC_BIN_S) {
        if (LOS == FCFC_LOS_Z) {
            pi2 = zz;
        } else {
            double lx = ax + bx;
            double ly = ay + by;
            double lz = az + bz;
            double t1 = dx * lx;
            double t2 = dy * ly;
            double t3 = dz * lz;
            double dot = (t1 + t2) + t3;
            double q1 = lx * lx;
            double q2 = ly * ly;
            double q3 = lz * lz;
            double ll = (q1 + q2) + q3;
            double dd = dot * dot;
            pi2 = (ll > 0.0) ? dd / ll : 0.0;
        }
    }
    if (KIND == FCFC_BIN_S || KIND == FCFC_BIN_S_MU) {
        int c = upper_edge_count(a.E1, a.n1, d2);
        if (c < 1 || c > a.n1) return -1;
        int k = c - 1;
        if (KIND == FCFC_BIN_S) return k;
        int j;
        if (d2 == 0.0) {
            j = 0;  // mu = 0; the first mu edge is 0
        } else {
            // largest j in [0, n2] with (j/n2)^2 * d2 <= pi2
            int lo = 0, hi = a.n2 + 1;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                double m = (double)mid / (double)a.n2;
                double M = m * m;
                if (M * d2 <= pi2) lo = mid + 1;
                else hi = mid;
            }
            j = lo - 1;  // >= 0 since M_0 = 0
            if (j == a.n2) {
                if (!a.mu_top_closed) return -1;
                j = a.n2 - 1;
            }
        }
        return k * a.n2 + j;
    }
    double sp2;
    if (LOS == FCFC_LOS_Z) {
        sp2 = xx + yy;
    } else {
        sp2 = d2 - pi2;
        if (sp2 < 0.0) sp2 = 0.0;
    }
    int c1 = upper_edge_count(a.E1, a.n1, sp2);
    if (c1 < 1 || c1 > a.n1) return -1;
    int c2 = upper_edge_count(a.E2, a.n2, pi2);
    if (c2 < 1 || c2 > a.n2) return -1;
    return (c1 - 1) * a.n2 + (c2 - 1);
}

// ---------------------------------------------------------------------------
// FP32 look-up with bands: returns bin (>= 0), -1 (out of range) or sets amb.
// ---------------------------------------------------------------------------
__device__ inline int lut_entry(const int16_t* __restrict__ lut, float scale, float v) {
    return (int)lut[(uint32_t)(v * scale)];
}
// A clean entry (>= -1) is the bin itself, -1 meaning out of range.  A hot
// entry (<= -2) holds -2 - k, k the first edge whose band meets the entry (the
// edges below k lie wholly below the entry).  Most hot entries meet one band:
// v is then placed by band k and the start of band k + 1, read together; when
// v reaches band k + 1 (several edges in one entry) the walk goes on over the
// next bands.  band[k] = (lo_k, hi_k), band[n + 1] = (+inf, +inf).  Returns the
// bin, -1 (out of range) or -2 (v inside a band: the pair needs the FP64
// recheck).
__device__ inline int lut_hot_bin(const float2* __restrict__ band, int n, int e, float v) {
    int k = -2 - e;
    const float2 b0 = band[k];
    const float lo1 = band[k + 1].x;
    if (v < b0.x) return k - 1;
    if (v < b0.y) return -2;
    if (v < lo1) return k < n ? k : -1;
    for (k = k + 1; k <= n; k++) {
        const float2 b = band[k];
        if (v >= b.y) continue;
        if (v >= b.x) return -2;
        break;
    }
    return (k >= 1 && k <= n) ? k - 1 : -1;
}

// Kernel constants kept in registers.
struct KConst {
    float scale1, scale2, vmax1, vmax2, r2prune, d2small, mu_n, mu_nm1, tolA, tolB, tolC, side32;
    float tolC_v;  // tolC held in a vector register (an fma takes one scalar operand)
    int n1, n2, nbins, nx, copies;
    double wscale;
};

// t: the pair weight times 2^(S - 32), where the weight times 2^S is an
// integer q below 2^62 in magnitude.  The limbs of q are hi = floor(t), the
// floor of q / 2^32, and lo = (t - hi) 2^32 in [0, 2^32), so q = hi 2^32 + lo;
// every step is exact in FP64 (t has at most 30 integer bits and its
// fraction holds the 32 low bits of q).
__device__ inline void add_weight(const Smem& s, int flat, double t) {
    const double hi = floor(t);
    const uint32_t lo = (uint32_t)((t - hi) * 4294967296.0);
    const int hi32 = (int)hi;
    unsigned long long* wb = s.wl + 2 * flat;
    atomicAdd(wb, (unsigned long long)lo);
    atomicAdd(wb + 1, (unsigned long long)(long long)hi32);
}

// Re-evaluate `cnt` queued pairs (entries base .. base+cnt-1) in FP64.
template <int KIND, int LOS, bool W>
__device__ __attribute__((always_inline)) inline void process_rechecks(ArgsRef a, const Smem& s, int base, int cnt, int lane,
                                 unsigned long long& nrechk) {
    if (lane < cnt) {
        const uint32_t* e = s.rb + (size_t)(base + lane) * 3;
        uint32_t ia = e[0], ib = e[1], it = e[2];
        uint32_t meta = a.items[it].meta;
        int sx = (int)((meta >> 16) & 3u) - 1;
        int sy = (int)((meta >> 18) & 3u) - 1;
        int sz = (int)((meta >> 20) & 3u) - 1;
        const double* pa = a.p64A + 3 * (size_t)ia;
        const double* pb = a.p64B + 3 * (size_t)ib;
        int flat = exact_bin<KIND, LOS>(a, pa[0], pa[1], pa[2], pb[0], pb[1], pb[2], sx, sy, sz);
        if (flat >= 0) {
            atomicAdd(&s.hist[flat], 1u);
            if (W) {
                double p = a.wA[ia] * a.wB[ib];
                add_weight(s, flat, p * a.wscale);
            }
        }
    }
    nrechk += (unsigned long long)cnt;
}

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Third word of a raw buffer resource on gfx9-family devices (32-bit data format).
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;

// 16 bytes at byte offset voff + soff of a buffer (zeros past its end).
__device__ inline float4 load_b(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
}

__device__ inline uint32_t lane_prefix(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Per-wave context of the current work item.
struct WaveCtx {
    uint32_t a_begin, b_begin, it;
    int rcount;
    unsigned long long nrechk;
};

// Bin `cnt` queued in-range pairs (entries base .. base+cnt-1), one per lane.
// Entry: (v1, v2, ids) with ids = (b - b_begin) << 10 | a_slot << 3, and
//   s:              v1 = d2
//   (s,mu), z:      v1 = d2, v2 = dz
//   (sp,pi), z:     v1 = sp2, v2 = pi2
//   mid-point:      (dx, dy, dz, ids) (line of sight from the staged A point)
// ids holds the byte offsets of the pair's weights from the item's first A
// and B weights: a_slot * 8 = ids & 0x3f8 and (b - b_begin) * 8 = (ids >> 7)
// with the low three bits cleared.
// The common path is branch-free; hot table entries and rechecks take
// wave-uniform branches that are rarely entered.
template <int KIND, int LOS, bool W>
__device__ __attribute__((always_inline)) inline void bin_queue(ArgsRef a, const KConst& k, const Smem& s,
                                                                uint32_t* hist_l, int base, int cnt, int lane,
                                                                WaveCtx& c) {
    const bool valid = lane < cnt;
    // entry (v1, v2, ids) or, mid-point, (dx, dy, dz, ids)
    constexpr bool MIDQ = (LOS == FCFC_LOS_MIDPOINT && KIND != FCFC_BIN_S);
    constexpr int QS = QStride<KIND, LOS>::value;
    float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t ids = 0;
    if (valid) {
        // the scalar byte offset of the first entry, kept opaque so that it is
        // added once instead of being re-associated with negative constants
        int boff = base * QS * 4;
        __asm__ volatile("" : "+s"(boff));
        const float* qe = (const float*)((const char*)s.qf_lane + boff);
        if (MIDQ) {
            e = *(const float4*)qe;
            ids = __float_as_uint(e.w);
        } else {
            e.x = qe[0];
            e.y = qe[1];
            ids = __float_as_uint(qe[2]);
        }
    }
    // the weights of the pair, fetched early (product formed only for pairs in range)
    double wa = 0.0, wb = 0.0;
    if (W && valid) {
        wb = *(const double*)((const char*)(a.wB + c.b_begin) + ((ids >> 7) & ~7u));
        wa = *(const double*)((const char*)(a.wA + c.a_begin) + (ids & 0x3f8u));
    }
    // Wave masks, each built from ballots of single compares (a ballot of a
    // compare is that compare's lane mask, so no per-lane boolean is formed):
    //   rm: pairs within an FP32 band of an edge (FP64 recheck),
    //   um: pairs binned here (in range, not rechecked).
    const uint64_t vmask = cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
    uint64_t rm, um;
    int flat;
    if (KIND == FCFC_BIN_S) {
        const float d2 = e.x;
        int sb = lut_entry(s.lut1, k.scale1, d2);
        const bool hot = sb < -1;
        if (__builtin_amdgcn_ballot_w64(hot)) {
            if (hot) sb = lut_hot_bin(s.band1, k.n1, sb, d2);
        }
        rm = __builtin_amdgcn_ballot_w64(sb == -2) & vmask;
        um = __builtin_amdgcn_ballot_w64(sb >= 0) & vmask;
        flat = sb;
    } else if (KIND == FCFC_BIN_S_MU) {
        float d2, proj_n;  // proj_n: |projection on the line of sight| * n_mu / |l|
        if (LOS == FCFC_LOS_Z) {
            d2 = e.x;
            proj_n = fabsf(e.y) * k.mu_n;
        } else {
            const float dxx = e.x, dyy = e.y, dzz = e.z;
            d2 = __builtin_fmaf(dzz, dzz, __builtin_fmaf(dyy, dyy, dxx * dxx));
            const float4 q = *(const float4*)((const char*)s.astage + ((ids & 0x3f8u) << 1));
            const float lx = q.x + dxx, ly = q.y + dyy, lz = q.z + dzz;
            const float dot = __builtin_fmaf(dzz, lz, __builtin_fmaf(dyy, ly, dxx * lx));
            const float ll = __builtin_fmaf(lz, lz, __builtin_fmaf(ly, ly, lx * lx));
            proj_n = fabsf(dot) * (__builtin_amdgcn_rsqf(ll) * k.mu_n);
        }
        int sb = lut_entry(s.lut1, k.scale1, d2);
        const bool hot = sb < -1;
        if (__builtin_amdgcn_ballot_w64(hot)) {
            if (hot) sb = lut_hot_bin(s.band1, k.n1, sb, d2);
        }
        const float rs = __builtin_amdgcn_rsqf(d2);
        const float mun = proj_n * rs;
        const int mb = min((int)mun, k.n2 - 1);
        // distance to the nearest interior mu edge (edges 0 and n need no
        // recheck: mu >= 0 always, and mu = 1 belongs to the last bin)
        const float cr = __builtin_amdgcn_fmed3f(rintf(mun), 1.0f, k.mu_nm1);
        const float tol = __builtin_fmaf(k.tolA, rs, k.tolC_v);
        rm = (__builtin_amdgcn_ballot_w64(sb == -2) | __builtin_amdgcn_ballot_w64(fabsf(mun - cr) < tol) |
              __builtin_amdgcn_ballot_w64(d2 < k.d2small)) &
             vmask;
        um = __builtin_amdgcn_ballot_w64(sb >= 0) & vmask & ~rm;
        flat = (int)__umul24((uint32_t)sb, (uint32_t)k.n2) + mb;
    } else {
        float sp2, pi2;
        if (LOS == FCFC_LOS_Z) {
            sp2 = e.x;
            pi2 = e.y;
        } else {
            const float dxx = e.x, dyy = e.y, dzz = e.z;
            const float d2 = __builtin_fmaf(dzz, dzz, __builtin_fmaf(dyy, dyy, dxx * dxx));
            const float4 q = *(const float4*)((const char*)s.astage + ((ids & 0x3f8u) << 1));
            const float lx = q.x + dxx, ly = q.y + dyy, lz = q.z + dzz;
            const float dot = __builtin_fmaf(dzz, lz, __builtin_fmaf(dyy, ly, dxx * lx));
            const float ll = __builtin_fmaf(lz, lz, __builtin_fmaf(ly, ly, lx * lx));
            pi2 = (dot * dot) * __builtin_amdgcn_rcpf(ll);
            sp2 = fmaxf(d2 - pi2, 0.0f);
        }
        // beyond a table's top band end the pair is certainly out of range
        const uint64_t inm =
            __builtin_amdgcn_ballot_w64(sp2 < k.vmax1) & __builtin_amdgcn_ballot_w64(pi2 < k.vmax2) & vmask;
        const bool inr = __builtin_amdgcn_inverse_ballot_w64(inm);
        const float sp2c = inr ? sp2 : 0.0f;
        const float pi2c = inr ? pi2 : 0.0f;
        int b1 = lut_entry(s.lut1, k.scale1, sp2c);
        int b2 = lut_entry(s.lut2, k.scale2, pi2c);
        const bool hot1 = b1 < -1, hot2 = b2 < -1;
        if (__builtin_amdgcn_ballot_w64(hot1 | hot2)) {
            if (hot1) b1 = lut_hot_bin(s.band1, k.n1, b1, sp2c);
            if (hot2) b2 = lut_hot_bin(s.band2, k.n2, b2, pi2c);
        }
        rm = (__builtin_amdgcn_ballot_w64(b1 == -2) | __builtin_amdgcn_ballot_w64(b2 == -2)) & inm;
        um = __builtin_amdgcn_ballot_w64(b1 >= 0) & __builtin_amdgcn_ballot_w64(b2 >= 0) & inm & ~rm;
        flat = (int)__umul24((uint32_t)b1, (uint32_t)k.n2) + b2;
    }
    if (__builtin_amdgcn_inverse_ballot_w64(um)) {
        atomicAdd(&hist_l[flat], 1u);
        if (W) {
            // fl(wa * wb) * 2^(S - 32) is exact: the scale only moves the exponent, and
            // the host chose S so that every scaled product lies in [2^20, 2^30)
            add_weight(s, flat, (wa * wb) * k.wscale);
        }
    }
    const uint64_t m = rm;
    if (m) {
        const int pos = c.rcount + (int)lane_prefix(m);
        if (__builtin_amdgcn_inverse_ballot_w64(m)) {
            uint32_t* r = s.rb + (size_t)pos * 3;
            r[0] = c.a_begin + ((ids >> 3) & 127u);
            r[1] = c.b_begin + (ids >> 10);
            r[2] = c.it;
        }
        c.rcount += (int)__popcll(m);
        if (c.rcount >= RB_FLUSH) {
            const int n = c.rcount < 64 ? c.rcount : 64;
            wave_sync_lds();
            process_rechecks<KIND, LOS, W>(a, s, c.rcount - n, n, lane, c.nrechk);
            wave_sync_lds();
            c.rcount -= n;
        }
    }
}

// Unweighted (s_perp, pi) counts along a fixed axis run two 12-wave
// workgroups per CU, six waves per SIMD, which leaves each lane 80 VGPRs (512
// per SIMD, allocated 8 at a time): one register more drops a wave from every
// SIMD (on MI355X the batched 200-mock pipeline ran 156 ms per 50 mocks at 79
// VGPRs, 199 ms at 81, when it ran at six waves).
// Unweighted s and (s, mu) counts are held to 64 VGPRs, eight waves per SIMD
// in two 16-wave workgroups (on MI355X: C5 4.21 -> 4.01 ms, C2 unweighted
// 4.46 -> 4.32 ms, the 200-mock batch 8 % faster; the spills this costs sit
// in the per-item code, outside the loop over B points).  Weighted and mid-point counts are held to 16 waves per
// CU by their LDS tables and queues, so they keep the registers (capping the
// mid-point ones at 80 only added spills).
// MODE: COUNT_SINGLE (one grid count), COUNT_BATCH (a stacked build's pair
// list) or COUNT_TREE (a count over k-d tree leaves).
template <int KIND, int LOS, bool AUTO, bool W, int P, int MODE>
__global__ __launch_bounds__(CT_MAX) __attribute__((amdgpu_waves_per_eu((W || LOS || MODE == COUNT_TREE) ? 4 : (KIND != FCFC_BIN_SPERP_PI ? 8 : 6))))
void k_count(const CountArgs* argp) {
    constexpr bool BATCH = MODE == COUNT_BATCH;
    constexpr bool TREE = MODE == COUNT_TREE;
    ArgsRef a = *(const CountArgs FCFC_CONST*)argp;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    Smem s;
    s.lut1 = (const int16_t*)(smem + a.off_lut1);
    s.lut2 = (const int16_t*)(smem + a.off_lut2);
    s.band1 = (const float2*)(smem + a.off_band1);
    s.band2 = (const float2*)(smem + a.off_band2);
    s.hist = (uint32_t*)(smem + a.off_hist);
    s.wl = (unsigned long long*)(smem + a.off_whist);
    constexpr int QS = QStride<KIND, LOS>::value;
    s.qf = (float*)(smem + a.off_q) + (size_t)wave * ((QS == 4 ? QCAP_MID : QCAP) + 1) * QS;
    s.qf_lane = s.qf + lane * QS;
    s.rb = (uint32_t*)(smem + a.off_rb) + (size_t)wave * RB_CAP * 3;
    s.astage = (float4*)(smem + a.off_astage) + (size_t)wave * ASTAGE;
    s.misc = (unsigned long long*)(smem + a.off_misc);

    // stage tables, clear histograms
    {
        uint32_t* d = (uint32_t*)(smem + a.off_lut1);
        const uint32_t* src = (const uint32_t*)a.lut1;
        for (int i = tid; i < (a.nlut1 + 1) / 2; i += nthr) d[i] = src[i];
        if (KIND == FCFC_BIN_SPERP_PI) {
            d = (uint32_t*)(smem + a.off_lut2);
            src = (const uint32_t*)a.lut2;
            for (int i = tid; i < (a.nlut2 + 1) / 2; i += nthr) d[i] = src[i];
        }
        float2* b1 = (float2*)(smem + a.off_band1);
        for (int i = tid; i < a.n1 + 2; i += nthr) b1[i] = a.band1[i];
        if (KIND == FCFC_BIN_SPERP_PI) {
            float2* b2 = (float2*)(smem + a.off_band2);
            for (int i = tid; i < a.n2 + 2; i += nthr) b2[i] = a.band2[i];
        }
        for (int i = tid; i < a.nbins * a.copies; i += nthr) s.hist[i] = 0u;
        if (W)
            for (int i = tid; i < 2 * a.nbins; i += nthr) s.wl[i] = 0ull;
        if (tid < 4) s.misc[tid] = 0ull;
    }
    __syncthreads();

    KConst k;
    k.scale1 = a.scale1;
    k.scale2 = a.scale2;
    k.vmax1 = a.vmax1;
    k.vmax2 = a.vmax2;
    k.r2prune = a.r2prune;
    k.d2small = a.d2small;
    k.mu_n = a.mu_n;
    k.mu_nm1 = a.mu_n - 1.0f;
    // one mu bin has no interior edge: nothing is near one
    k.tolA = a.n2 > 1 ? a.tolA : 0.0f;
    k.tolB = a.tolB;
    k.tolC = a.n2 > 1 ? a.tolC : 0.0f;
    k.tolC_v = k.tolC;
    __asm__ volatile("" : "+v"(k.tolC_v));
    k.side32 = a.side32;
    k.n1 = a.n1;
    k.n2 = a.n2;
    k.nbins = a.nbins;
    k.nx = a.nx;
    k.copies = a.copies;
    k.wscale = a.wscale;
    uint32_t* hist_l = s.hist + (size_t)(lane % k.copies) * k.nbins;
    WaveCtx c;
    c.rcount = 0;
    c.nrechk = 0;
    unsigned long long ncand = 0;
    const float far = 1.0e18f;

    // Items are pulled dynamically; the index of the item after next and the
    // inputs (item record, A points, B cell offsets) of the next item are
    // fetched while the current one is processed.
    struct ItemIn {
        Item item;
        float4 av[P];
        float4 aabs[P];
        uint32_t csv;  // lane t: start of B cell xw0 + t of the item's row
        // tree: the A leaf origin, and in lane t the FP32 offset of B leaf
        // b_rowcell + t from it
        int4 ja;
        float tox, toy, toz;
    };
    auto load_in = [&](uint32_t itx, ItemIn& in) __attribute__((always_inline)) {
        in.item = ldc_item(a.items, itx);
        const uint32_t a_begin = in.item.a_begin;
        const uint32_t acnt = in.item.acnt_xb0 & 0xffffu;
#pragma unroll
        for (int p = 0; p < P; p++) {
            const uint32_t i = (uint32_t)(lane + 64 * p);
            in.av[p] = make_float4(far, far, far, __int_as_float(0));
            if (i < acnt) in.av[p] = a.posA[a_begin + i];
            if (LOS == FCFC_LOS_MIDPOINT && KIND != FCFC_BIN_S) {
                in.aabs[p] = make_float4(far, far, far, 0.f);
                if (i < acnt) in.aabs[p] = a.absA[a_begin + i];
            }
        }
        if (TREE) {
            in.ja = ldc_i4(a.leaf_orgA, in.item.tile);
            const int4 jb = a.leaf_orgB[min(in.item.b_rowcell + (uint32_t)lane, a.tree_nleafB - 1u)];
            in.tox = (float)(jb.x - in.ja.x) * a.tree_q;
            in.toy = (float)(jb.y - in.ja.y) * a.tree_q;
            in.toz = (float)(jb.z - in.ja.z) * a.tree_q;
        } else {
            const int xb0 = (int)(int16_t)(in.item.acnt_xb0 >> 16);
            const int sxi = (int)((in.item.meta >> 16) & 3u) - 1;
            const int xw0 = xb0 - sxi * a.nx;
            const int cx = min(xw0 + lane, a.nx);
            in.csv = a.csB[in.item.b_rowcell + (uint32_t)cx];
        }
    };

    unsigned long long wave_pairs = 0;  // pairs claimed since this wave last emptied the histogram
    unsigned long long nflush = 0;      // merges made by this wave before the end
    const unsigned long long flush_pairs = a.flush_pairs;
    uint32_t out_off = 0;               // first bin of the current catalogue in the outputs
    // u32 overflow guard of the LDS histogram: every wave empties it (atomic
    // exchange) after claiming flush_pairs <= 2^26 pairs, so it never holds
    // more than 16 (2^26 + 128 x 2^19) = 2^31 increments (items hold at most
    // 128 x b_chunk pairs, b_chunk <= 2^19)
    auto exchange_out = [&]() __attribute__((always_inline)) {
        nflush++;
        for (int b = lane; b < k.nbins * k.copies; b += 64) {
            uint32_t v = atomicExch(&s.hist[b], 0u);
            if (v) atomicAdd(&a.out_counts[out_off + b % k.nbins], (unsigned long long)v);
        }
        if (W) {
            for (int b = lane; b < k.nbins; b += 64) {
                unsigned long long lo = atomicExch(&s.wl[2 * b], 0ull);
                unsigned long long hi = atomicExch(&s.wl[2 * b + 1], 0ull);
                __int128 v = ((__int128)(long long)hi << 32) + (__int128)lo;
                unsigned long long vlo = (unsigned long long)v;
                unsigned long long vhi = (unsigned long long)(v >> 64);
                unsigned long long o = atomicAdd(&a.out_w[2 * ((size_t)out_off + b)], vlo);
                if (o + vlo < o) vhi += 1ull;
                if (vhi) atomicAdd(&a.out_w[2 * ((size_t)out_off + b) + 1], vhi);
            }
        }
    };
    // workgroup-wide merge of the LDS histograms into the outputs, then clear
    auto merge_out = [&]() __attribute__((always_inline)) {
        for (int b = tid; b < k.nbins; b += nthr) {
            uint32_t cnt = 0;
            for (int r = 0; r < k.copies; r++) {
                cnt += s.hist[r * k.nbins + b];
                s.hist[r * k.nbins + b] = 0u;
            }
            if (cnt) atomicAdd(&a.out_counts[out_off + b], (unsigned long long)cnt);
            if (W) {
                unsigned long long lo = s.wl[2 * b], hi = s.wl[2 * b + 1];
                s.wl[2 * b] = 0ull;
                s.wl[2 * b + 1] = 0ull;
                if (lo | hi) {
                    __int128 v = ((__int128)(long long)hi << 32) + (__int128)lo;
                    unsigned long long vlo = (unsigned long long)v;
                    unsigned long long vhi = (unsigned long long)(v >> 64);
                    unsigned long long o = atomicAdd(&a.out_w[2 * ((size_t)out_off + b)], vlo);
                    if (o + vlo < o) vhi += 1ull;
                    if (vhi) atomicAdd(&a.out_w[2 * ((size_t)out_off + b) + 1], vhi);
                }
            }
        }
    };
    auto drain_rechecks = [&]() __attribute__((always_inline)) {
        while (c.rcount > 0) {
            const int n = c.rcount < 64 ? c.rcount : 64;
            wave_sync_lds();
            process_rechecks<KIND, LOS, W>(a, s, c.rcount - n, n, lane, c.nrechk);
            wave_sync_lds();
            c.rcount -= n;
        }
    };
    // Process items handed out by grab() (an index, or ~0u when there are no more).
    auto process_items = [&](auto grab) __attribute__((always_inline)) {
    uint32_t cur_it = grab();
    uint32_t nxt_it = grab();
    ItemIn cur, nxt;
    if (cur_it != ~0u) load_in(cur_it, cur);
    // timing: an item's time runs from its start to the next item's start on
    // this wave (fetch and loop overhead included), the last one to the end
    unsigned long long t_prev = 0;
    uint32_t prev_it = ~0u;
    while (cur_it != ~0u) {
        const uint32_t it = cur_it;
        if (a.times && lane == 0) {
            const unsigned long long t = wall_clock64();
            if (prev_it != ~0u) a.times[prev_it] = (uint32_t)min<unsigned long long>(t - t_prev, 0xffffffffull);
            t_prev = t;
            prev_it = it;
        }
        const uint32_t nn = grab();
        if (nxt_it != ~0u) load_in(nxt_it, nxt);
        const Item& item = cur.item;
        const uint32_t a_begin = item.a_begin;
        const uint32_t acnt = item.acnt_xb0 & 0xffffu;
        const int xb0 = (int)(int16_t)(item.acnt_xb0 >> 16);
        const int idy = (int)(int8_t)(item.meta & 0xffu);
        const int idz = (int)(int8_t)((item.meta >> 8) & 0xffu);
        const int sxi = (int)((item.meta >> 16) & 3u) - 1;
        const bool samerow = AUTO && ((item.meta >> 24) & ITEM_SAMEROW);
        const uint32_t b_begin = item.b_begin;
        const uint32_t b_end = item.b_end;
        c.a_begin = a_begin;
        c.b_begin = b_begin;
        c.it = it;

        const uint64_t pairs = (uint64_t)acnt * (uint64_t)(b_end - b_begin);
        ncand += pairs;
        wave_pairs += pairs;
        if (wave_pairs >= flush_pairs) {
            wave_pairs = 0;
            exchange_out();
        }
        const float Dy = (float)idy * k.side32;
        const float Dz = (float)idz * k.side32;
        float ax[P], ay[P], az[P];
        // tree: the A points relative to their leaf origin (offset per B leaf)
        float ayr[P], azr[P];
        int acx[P];
        uint32_t aidx[P], ids_lane[P];
#pragma unroll
        for (int p = 0; p < P; p++) {
            const uint32_t i = (uint32_t)(lane + 64 * p);
            aidx[p] = a_begin + i;
            ids_lane[p] = i << 3;
            const float4 v = cur.av[p];
            ax[p] = v.x;
            ay[p] = v.y - Dy;
            az[p] = v.z - Dz;
            ayr[p] = v.y;
            azr[p] = v.z;
            acx[p] = __float_as_int(v.w);
            if (LOS == FCFC_LOS_MIDPOINT && KIND != FCFC_BIN_S) {
                const float4 q = cur.aabs[p];
                s.astage[i] = make_float4(2.0f * q.x, 2.0f * q.y, 2.0f * q.z, 0.f);
            }
        }
        int qn = 0;
        int xu = xb0;
        int xw = xb0 - sxi * a.nx;
        int t = 0;
        uint32_t j = b_begin;
        // The current B cell: points up to cell_end, A x positions relative to it.
        uint32_t cell_end = 0;
        float axx[P];
        // Advance to the next cell of the row piece that holds points at or after
        // j (cells are consecutive in the sorted points); false when none is left.
        auto next_cell = [&]() __attribute__((always_inline)) -> bool {
            if (j >= b_end) return false;  // the item's B points are done
            if (TREE) {
                // the next B leaf that holds points at or after j: its end, and
                // the A points moved into its frame (leaf origins lie on a
                // lattice of power-of-two spacing, so the offset is exact)
                uint32_t leaf = item.b_rowcell + (uint32_t)t;
                while (leaf < a.tree_nleafB) {
                    uint32_t ce = min((leaf + 1u) * a.tree_leaf, a.nB);
                    ce = ce < b_end ? ce : b_end;
                    float ox, oy, oz;
                    if (t < 64) {  // prefetched with the item
                        ox = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cur.tox), t));
                        oy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cur.toy), t));
                        oz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cur.toz), t));
                    } else {
                        const int4 jb = ldc_i4(a.leaf_orgB, leaf);
                        ox = (float)(jb.x - cur.ja.x) * a.tree_q;
                        oy = (float)(jb.y - cur.ja.y) * a.tree_q;
                        oz = (float)(jb.z - cur.ja.z) * a.tree_q;
                    }
                    leaf++;
                    t++;
                    if (ce > j) {
                        cell_end = ce;
#pragma unroll
                        for (int p = 0; p < P; p++) {
                            axx[p] = ax[p] - ox;
                            ay[p] = ayr[p] - oy;
                            az[p] = azr[p] - oz;
                        }
                        return true;
                    }
                }
                return false;
            }
            while (xw < a.nx) {
                uint32_t ce = (t + 1 < 64) ? __builtin_amdgcn_readlane(cur.csv, t + 1)
                                           : ldc_u32(a.csB, item.b_rowcell + (uint32_t)xw + 1u);
                ce = ce < b_end ? ce : b_end;
                const int xc = xu;
                xw++;
                xu++;
                t++;
                if (ce > j) {
                    cell_end = ce;
#pragma unroll
                    for (int p = 0; p < P; p++) axx[p] = ax[p] - (float)(xc - acx[p]) * k.side32;
                    return true;
                }
            }
            return false;
        };
        bool have = j < b_end && next_cell();
        // B points arrive 64 at a time, one per lane, by buffer loads issued a
        // whole batch ahead, and each step takes its point from the batch with
        // v_readlane.  (Fetching one point per step left every step waiting on
        // a load issued only a step or two before.)  Even batches live in bx,
        // odd ones in by, and each register set is reloaded in place once it is
        // used up, so no batch is copied.  The buffer covers the item's B range;
        // offsets past it read zeros.
        const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(a.posB + b_begin), (short)0, (int)((b_end - b_begin) * 16u), BUFFER_RSRC_WORD3);
        const uint32_t lane16 = (uint32_t)lane * 16u;
        float4 bx = load_b(rB, lane16, 0u);
        float4 by = load_b(rB, lane16, 1024u);
        uint32_t bstart = b_begin;  // first point of the batch being counted
        // Count the points of the batch in `buf` (from j to the batch's end).
        auto run_batch = [&](const float4& buf, auto mask_tag) __attribute__((always_inline)) {
            constexpr bool MASK = decltype(mask_tag)::value;
            const uint32_t bend = min(bstart + 64u, b_end);
            while (have && j < bend) {
                const uint32_t stop = min(cell_end, bend);
                uint32_t jbits = (j - b_begin) << 10;
                for (; j < stop; j++, jbits += 1024u) {
                    const int tl = (int)(j - bstart);  // the lane holding point j
                    const float3 b = make_float3(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(buf.x), tl)),
                                                 __int_as_float(__builtin_amdgcn_readlane(__float_as_int(buf.y), tl)),
                                                 __int_as_float(__builtin_amdgcn_readlane(__float_as_int(buf.z), tl)));
#pragma unroll
                    for (int p = 0; p < P; p++) {
                        const float dx = b.x - axx[p];
                        const float dy = b.y - ay[p];
                        const float dz = b.z - az[p];
                        bool in;
                        float v1, v2, v3 = 0.f;
                        if (KIND == FCFC_BIN_SPERP_PI && LOS == FCFC_LOS_Z) {
                            v1 = __builtin_fmaf(dy, dy, dx * dx);
                            v2 = dz * dz;
                            in = (v1 < k.vmax1) & (v2 < k.vmax2);
                        } else {
                            const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                            in = d2 < k.r2prune;
                            if (LOS == FCFC_LOS_MIDPOINT && KIND != FCFC_BIN_S) {
                                v1 = dx;
                                v2 = dy;
                                v3 = dz;
                            } else {
                                v1 = d2;
                                v2 = dz;
                            }
                        }
                        if (MASK) in = in & (j > aidx[p]);
                        const uint64_t m = __builtin_amdgcn_ballot_w64(in);
                        // lanes in range append at qn + (lanes below in the mask);
                        // the others store nothing
                        float* qb = s.qf + qn * QS;
                        if (in) {
                            const uint32_t pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                            const float idf = __uint_as_float(jbits | ids_lane[p]);
                            float* qe = qb + pre * QS;
                            if (QS == 4) {
                                *(float4*)qe = make_float4(v1, v2, v3, idf);
                            } else {
                                qe[0] = v1;
                                qe[1] = v2;
                                qe[2] = idf;
                            }
                        }
                        qn += (int)__popcll(m);
                        if (QS == 4 && qn >= 64) {
                            // 16-byte entries: drain after each A point, so the
                            // queue holds at most 63 + 64 entries
                            wave_sync_lds();
                            bin_queue<KIND, LOS, W>(a, k, s, hist_l, qn - 64, 64, lane, c);
                            wave_sync_lds();
                            qn -= 64;
                        }
                    }
                    while (QS != 4 && qn >= 64) {
                        wave_sync_lds();
                        bin_queue<KIND, LOS, W>(a, k, s, hist_l, qn - 64, 64, lane, c);
                        wave_sync_lds();
                        qn -= 64;
                    }
                }
                if (j == cell_end) have = next_cell();
            }
        };
        auto run_item = [&](auto mask_tag) __attribute__((always_inline)) {
            for (;;) {
                run_batch(bx, mask_tag);
                if (!have || j >= b_end) break;
                bstart += 64u;
                bx = load_b(rB, lane16, (bstart + 64u - b_begin) * 16u);
                run_batch(by, mask_tag);
                if (!have || j >= b_end) break;
                bstart += 64u;
                by = load_b(rB, lane16, (bstart + 64u - b_begin) * 16u);
            }
        };
        if (samerow)
            run_item(std::integral_constant<bool, true>());
        else
            run_item(std::integral_constant<bool, false>());
        if (qn > 0) {
            wave_sync_lds();
            bin_queue<KIND, LOS, W>(a, k, s, hist_l, 0, qn, lane, c);
            wave_sync_lds();
        }
        cur = nxt;
        cur_it = nxt_it;
        nxt_it = nn;
    }
    if (a.times && lane == 0 && prev_it != ~0u)
        a.times[prev_it] = (uint32_t)min<unsigned long long>(wall_clock64() - t_prev, 0xffffffffull);
    };
    if (!BATCH) {
        const uint32_t nitems = __builtin_amdgcn_readfirstlane(*a.nitems_dev);
        const uint32_t sc = a.shard_count, si = a.shard_index;
        // Every wave of the device claims work on one cursor; at one claim per
        // item those atomics serialise (about 12 ns each on MI355X) into the
        // bound of a launch of short items.  Past the first grab_single positions
        // (the largest items of the longest-first list, claimed one at a time so
        // that they spread over the waves) a wave claims as many positions (up
        // to 8) as keep its claims grab_gap wall-clock ticks apart, judged by
        // the time its last claim took to count.
        const uint32_t gsingle = a.grab_single;
        const uint64_t ggap = a.grab_gap;
        uint32_t chunk_pos = 0, chunk_left = 0, claimed = 0;
        uint64_t t_claim = 0;
        process_items([&]() -> uint32_t {
            if (chunk_left == 0) {
                uint32_t want = 1u;
                if (chunk_pos >= gsingle) {
                    const uint64_t now = wall_clock64();
                    if (claimed > 0) {
                        const uint64_t per = (now - t_claim) / claimed;
                        want = per == 0 ? 8u : (uint32_t)min<uint64_t>(8u, max<uint64_t>(1u, (ggap + per - 1) / per));
                    }
                    t_claim = now;
                }
                uint32_t v = 0;
                if (lane == 0) v = atomicAdd(a.cursor, want);
                chunk_pos = __builtin_amdgcn_readfirstlane(v);
                chunk_left = want;
                claimed = want;
            }
            const uint32_t v = chunk_pos++;
            chunk_left--;
            // one shard of the ordered list: items si, si + sc, si + 2 sc, ...
            const uint64_t idx = (uint64_t)v * sc + si;
            return idx < nitems ? (uint32_t)idx : ~0u;
        });
        drain_rechecks();
        __syncthreads();
        merge_out();
    } else {
        // Workgroup-synchronous chunks of items of one catalogue at a time: the
        // LDS histograms always belong to the workgroup's current catalogue.
        uint32_t* sm32 = (uint32_t*)(s.misc + 1);  // [0] chunk, [1] cursor within the chunk
        const uint32_t nchunks = __builtin_amdgcn_readfirstlane(*a.nchunks_dev);
        uint32_t cur_cat = ~0u;
        for (;;) {
            if (tid == 0) {
                sm32[0] = atomicAdd(a.chunk_cursor, 1u);
                sm32[1] = 0u;
            }
            __syncthreads();
            const uint32_t chunk = __builtin_amdgcn_readfirstlane(sm32[0]);
            if (chunk >= nchunks) break;
            // chunk -> position in the catalogue order (binary search on the chunk prefix)
            int lo = 0, hi = a.ncat;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (ldc_u32(a.chunk_prefix, (uint32_t)mid) <= chunk) lo = mid;
                else hi = mid;
            }
            const uint32_t cat = ldc_u32(a.cat_order, (uint32_t)lo);
            const uint32_t local = chunk - ldc_u32(a.chunk_prefix, (uint32_t)lo);
            const uint32_t ib = ldc_u32(a.cat_items, cat) + local * (uint32_t)a.chunk_items;
            const uint32_t ie_cat = ldc_u32(a.cat_items, cat + 1u);
            const uint32_t ie = min(ib + (uint32_t)a.chunk_items, ie_cat);
            if (cat != cur_cat) {
                if (cur_cat != ~0u) merge_out();
                __syncthreads();
                cur_cat = cat;
                out_off = cat * (uint32_t)k.nbins;
            }
            process_items([&]() -> uint32_t {
                uint32_t v = 0;
                if (lane == 0) v = atomicAdd(&sm32[1], 1u);
                v = __builtin_amdgcn_readfirstlane(v) + ib;
                return v < ie ? v : ~0u;
            });
            drain_rechecks();
            __syncthreads();
        }
        if (cur_cat != ~0u) merge_out();
    }
    if (lane == 0 && a.stats) {
        atomicAdd(&a.stats[0], ncand);
        atomicAdd(&a.stats[1], c.nrechk);
        if (nflush) atomicAdd(&a.stats[6], nflush);
    }
}

// 128-bit fixed-point sums -> FP64, rounded to nearest even, times 2^-S
__global__ void k_finalize_w(const unsigned long long* __restrict__ acc, int nbins, int S, double* __restrict__ out) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    unsigned long long lo = acc[2 * b], hi = acc[2 * b + 1];
    __int128 v = (__int128)(((unsigned __int128)hi << 64) | (unsigned __int128)lo);
    bool neg = v < 0;
    unsigned __int128 m = neg ? (unsigned __int128)(-(v + 1)) + 1u : (unsigned __int128)v;
    double r;
    if (m == 0) {
        r = 0.0;
    } else {
        unsigned long long mh = (unsigned long long)(m >> 64), ml = (unsigned long long)m;
        int nb = mh ? 128 - __clzll(mh) : 64 - __clzll(ml);
        if (nb <= 53) {
            r = ldexp((double)ml, -S);
        } else {
            int sh = nb - 53;
            unsigned __int128 top = m >> sh;
            unsigned __int128 rem = m - (top << sh);
            unsigned __int128 half = (unsigned __int128)1 << (sh - 1);
            if (rem > half || (rem == half && (top & 1u))) top += 1u;
            r = ldexp((double)(unsigned long long)top, sh - S);
        }
    }
    out[b] = neg ? -r : r;
}

// ---------------------------------------------------------------------------
// kernel table
// ---------------------------------------------------------------------------
typedef void (*CountKernel)(const CountArgs*);

template <int KIND, int LOS, bool AUTO, bool W, int MODE>
static CountKernel pick_p(int P) {
    if (P == 1) return k_count<KIND, LOS, AUTO, W, 1, MODE>;
    return k_count<KIND, LOS, AUTO, W, 2, MODE>;
}
template <int KIND, int LOS>
static CountKernel pick_aw(bool is_auto, bool w, int P) {
    if (is_auto)
        return w ? pick_p<KIND, LOS, true, true, COUNT_SINGLE>(P) : pick_p<KIND, LOS, true, false, COUNT_SINGLE>(P);
    return w ? pick_p<KIND, LOS, false, true, COUNT_SINGLE>(P) : pick_p<KIND, LOS, false, false, COUNT_SINGLE>(P);
}
// tree counts: tiles of 128 points (a leaf holds at most 128)
template <int KIND, int LOS>
static CountKernel pick_tw(bool is_auto, bool w) {
    if (is_auto) return w ? k_count<KIND, LOS, true, true, 2, COUNT_TREE> : k_count<KIND, LOS, true, false, 2, COUNT_TREE>;
    return w ? k_count<KIND, LOS, false, true, 2, COUNT_TREE> : k_count<KIND, LOS, false, false, 2, COUNT_TREE>;
}
static CountKernel pick_tree_kernel(int kind, int los, bool is_auto, bool w) {
    if (kind == FCFC_BIN_S) return pick_tw<FCFC_BIN_S, FCFC_LOS_Z>(is_auto, w);
    if (kind == FCFC_BIN_S_MU)
        return los == FCFC_LOS_Z ? pick_tw<FCFC_BIN_S_MU, FCFC_LOS_Z>(is_auto, w)
                                 : pick_tw<FCFC_BIN_S_MU, FCFC_LOS_MIDPOINT>(is_auto, w);
    return los == FCFC_LOS_Z ? pick_tw<FCFC_BIN_SPERP_PI, FCFC_LOS_Z>(is_auto, w)
                             : pick_tw<FCFC_BIN_SPERP_PI, FCFC_LOS_MIDPOINT>(is_auto, w);
}
static CountKernel pick_kernel(int kind, int los, bool is_auto, bool w, int P) {
    if (kind == FCFC_BIN_S) return pick_aw<FCFC_BIN_S, FCFC_LOS_Z>(is_auto, w, P);
    if (kind == FCFC_BIN_S_MU)
        return los == FCFC_LOS_Z ? pick_aw<FCFC_BIN_S_MU, FCFC_LOS_Z>(is_auto, w, P)
                                 : pick_aw<FCFC_BIN_S_MU, FCFC_LOS_MIDPOINT>(is_auto, w, P);
    return los == FCFC_LOS_Z ? pick_aw<FCFC_BIN_SPERP_PI, FCFC_LOS_Z>(is_auto, w, P)
                             : pick_aw<FCFC_BIN_SPERP_PI, FCFC_LOS_MIDPOINT>(is_auto, w, P);
}
// batched counts (auto and cross pairs of a stacked build): the auto
// instantiation serves both, since only items of an auto pair carry the
// same-row flag
template <int KIND, int LOS>
static CountKernel pick_bw(bool w, int P) {
    return w ? pick_p<KIND, LOS, true, true, COUNT_BATCH>(P) : pick_p<KIND, LOS, true, false, COUNT_BATCH>(P);
}
static CountKernel pick_batch_kernel(int kind, int los, bool w, int P) {
    if (kind == FCFC_BIN_S) return pick_bw<FCFC_BIN_S, FCFC_LOS_Z>(w, P);
    if (kind == FCFC_BIN_S_MU)
        return los == FCFC_LOS_Z ? pick_bw<FCFC_BIN_S_MU, FCFC_LOS_Z>(w, P)
                                 : pick_bw<FCFC_BIN_S_MU, FCFC_LOS_MIDPOINT>(w, P);
    return los == FCFC_LOS_Z ? pick_bw<FCFC_BIN_SPERP_PI, FCFC_LOS_Z>(w, P)
                             : pick_bw<FCFC_BIN_SPERP_PI, FCFC_LOS_MIDPOINT>(w, P);
}

static int al16(int b) { return (b + 15) & ~15; }
static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// host-side preparation shared by the single and batched drivers
// ---------------------------------------------------------------------------
struct LaunchSetup {
    CountArgs a;  // LDS layout and numeric constants (device pointers bound later)
    int waves = 16, P = 2, T = 128, seg = 1, bchunk = 16384, copies = 1;
    std::vector<int4> rows;
    int nrows = 0;
    std::vector<char> htab;  // tables blob: lut1, lut2, band1, band2, E1, E2, stencil rows
    int lut_entries = 0;     // entries of the look-up table used for s (or s_perp)
    size_t tb_l1 = 0, tb_l2 = 0, tb_b1 = 0, tb_b2 = 0, tb_e1 = 0, tb_e2 = 0, tb_rows = 0, tb_total = 0;
    CountKernel kern = nullptr;
};

// Common fixed-point scale 2^S making every weight product an integer.
static fcfc_status weight_scale(double wmin1, double wmax1, double wmin2, double wmax2, int* S) {
    return weight_scale_rule(wmin1, wmax1, wmin2, wmax2, 2, S);
}

// Most cells a tile may span, unless tuned: 32, so that tiles are cut by
// their point count and fill every lane.  B ranges are trimmed to the tile's
// actual x extent, so a wide tile costs only its extent (measured on MI355X:
// C5 7.0 -> 5.6 ms, C2 8.5 -> 8.3 ms against the earlier density-based span).
static int tile_seg(const Plan* p) { return p->tune.seg_cells > 0 ? std::min(32, p->tune.seg_cells) : 32; }

static fcfc_status setup_launch(Plan* p, bool is_auto, bool weighted, bool batch, int S, LaunchSetup& L) {
    const Grid& g = p->grid;
    const bool tree = p->tune.tree_leaf > 0 && !batch;
    L.T = (tree || p->tune.tile_points != 64) ? 128 : 64;
    L.P = L.T / 64;
    L.seg = tile_seg(p);
    // B points per item: tree ranges (whole subtrees) are cut finer than the
    // grid's row pieces, which are short by themselves
    L.bchunk = p->tune.b_chunk >= 256 ? p->tune.b_chunk : (tree ? 2048 : 16384);
    L.copies = (p->tune.hist_copies == 2 || p->tune.hist_copies == 4) ? p->tune.hist_copies : 1;
    L.nrows = stencil_rows(p, is_auto, L.rows);
    const bool two = (p->kind == FCFC_BIN_SPERP_PI);
    const bool mid = (p->los == FCFC_LOS_MIDPOINT && p->kind != FCFC_BIN_S);
    const int qbytes = mid ? (QCAP_MID + 1) * 16 : (QCAP + 1) * 12;
    const int per_wave = qbytes + RB_CAP * 12 + (mid ? ASTAGE * 16 : 0);
    int dev = 0, maxlds = 65536;
    FCFC_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) maxlds = 65536;
    L.kern = tree    ? pick_tree_kernel(p->kind, p->los, is_auto, weighted)
             : batch ? pick_batch_kernel(p->kind, p->los, weighted, L.P)
                     : pick_kernel(p->kind, p->los, is_auto, weighted, L.P);
    FCFC_HIP(hipFuncSetAttribute((const void*)L.kern, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds));
    // LDS shared by the workgroup's waves for tables of n1t and n2t entries
    auto shared_for = [&](int n1t, int n2t) {
        return al16(n1t * 2 + 4) + al16(n2t * 2 + 4) + al16((p->n1 + 2) * 8) +
               al16(two ? (p->n2 + 2) * 8 : 0) + al16(p->nbins * 4 * L.copies) +
               (weighted ? al16(p->nbins * 16) : 0);
    };
    // Workgroup size for a given shared part, and the waves resident per CU.
    // Default, from timings on MI355X: two 16-wave workgroups per CU when
    // the registers and the LDS allow it, else two 12-wave workgroups (three
    // waves per SIMD each) when they fit, else one workgroup of the largest
    // even wave count that fits (odd counts leave the SIMDs unevenly loaded
    // and ran measurably slower).
    auto choose_waves = [&](int shared, int& waves, int& resident) {
        auto lds_for = [&](int w) { return shared + w * per_wave + 64; };
        if (p->tune.group_waves >= 1 && p->tune.group_waves <= 16) {
            waves = p->tune.group_waves;
            while (waves > 1 && lds_for(waves) > maxlds) waves--;
        } else {
            waves = 16;
            while (waves > 1 && lds_for(waves) > maxlds) waves--;
            int occ16 = 0, occ12 = 0;
            if (waves == 16 &&
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ16, (const void*)L.kern, 16 * 64, lds_for(16)) ==
                    hipSuccess &&
                occ16 >= 2)
                waves = 16;
            else if (lds_for(12) <= maxlds &&
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ12, (const void*)L.kern, 12 * 64, lds_for(12)) ==
                    hipSuccess &&
                occ12 >= 2)
                waves = 12;
            else if (waves > 2)
                waves &= ~1;
        }
        int occ = 0;
        if (lds_for(waves) > maxlds ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)L.kern, waves * 64, lds_for(waves)) !=
                hipSuccess)
            occ = 0;
        resident = waves * occ;
        return lds_for(waves) <= maxlds;
    };
    // The larger look-up tables (fewer entries that meet a band) are used
    // whenever they keep as many waves resident: on MI355X they ran C1 0.34
    // -> 0.26 ms and unweighted C2 5.6 -> 5.3 ms, while costing the weighted
    // C2 kernel two of its 16 waves (7.5 -> 7.8 ms) where they are not used.
    const Lut1D* T1 = &p->lut1;
    const Lut1D* T2 = &p->lut2;
    int shared_bytes = shared_for((int)T1->tab.size(), two ? (int)T2->tab.size() : 0);
    int waves = 1, resident = 0;
    const bool fits = choose_waves(shared_bytes, waves, resident);
    if (p->has_big) {
        const int sb = shared_for((int)p->lut1b.tab.size(), two ? (int)p->lut2b.tab.size() : 0);
        int wb = 1, rb = 0;
        if (choose_waves(sb, wb, rb) && rb >= resident && rb > 0) {
            T1 = &p->lut1b;
            T2 = &p->lut2b;
            shared_bytes = sb;
            waves = wb;
        }
    }
    if (!fits && T1 == &p->lut1) {
        set_error("count: %d bytes of LDS needed (tables + histogram), device allows %d", shared_bytes + per_wave + 64,
                  maxlds);
        return FCFC_ERANGE;
    }
    L.waves = waves;
    L.lut_entries = (int)T1->tab.size();
    CountArgs& a = L.a;
    memset(&a, 0, sizeof(a));
    a.nlut1 = (int)T1->tab.size();
    a.nlut2 = two ? (int)T2->tab.size() : 0;
    a.copies = L.copies;
    int off = 0;
    a.off_lut1 = off;
    off += al16(a.nlut1 * 2 + 4);
    a.off_lut2 = off;
    off += al16(a.nlut2 * 2 + 4);
    a.off_band1 = off;
    off += al16((p->n1 + 2) * 8);
    a.off_band2 = off;
    off += al16(two ? (p->n2 + 2) * 8 : 0);
    a.off_hist = off;
    off += al16(p->nbins * 4 * L.copies);
    a.off_whist = off;
    off += weighted ? al16(p->nbins * 16) : 0;
    a.off_q = off;
    off += L.waves * qbytes;
    a.off_rb = off;
    off += L.waves * RB_CAP * 12;
    a.off_astage = off;
    off += mid ? L.waves * ASTAGE * 16 : 0;
    a.off_misc = off;
    off += 64;
    a.lds_bytes = off;
    // tables blob
    L.tb_l1 = (size_t)al16(a.nlut1 * 2 + 4);
    L.tb_l2 = (size_t)al16(a.nlut2 * 2 + 4);
    L.tb_b1 = (size_t)al16((p->n1 + 2) * 8);
    L.tb_b2 = (size_t)al16((p->n2 + 2) * 8);
    L.tb_e1 = (size_t)al16((p->n1 + 1) * 8);
    L.tb_e2 = (size_t)al16((p->n2 + 1) * 8);
    L.tb_rows = (size_t)al16(std::max(1, L.nrows) * 16);
    L.tb_total = L.tb_l1 + L.tb_l2 + L.tb_b1 + L.tb_b2 + L.tb_e1 + L.tb_e2 + L.tb_rows;
    L.htab.assign(L.tb_total, 0);
    {
        size_t o = 0;
        memcpy(&L.htab[o], T1->tab.data(), T1->tab.size() * 2);
        o += L.tb_l1;
        if (two) memcpy(&L.htab[o], T2->tab.data(), T2->tab.size() * 2);
        o += L.tb_l2;
        // bands as (lo, hi) pairs, then a sentinel pair above the top edge
        auto put_bands = [&](size_t at, const Lut1D* T, int n) {
            float* b = (float*)&L.htab[at];
            for (int k = 0; k <= n; k++) {
                b[2 * k] = T->lo[k];
                b[2 * k + 1] = T->hi[k];
            }
            b[2 * (n + 1)] = INFINITY;
            b[2 * (n + 1) + 1] = INFINITY;
        };
        put_bands(o, T1, p->n1);
        o += L.tb_b1;
        if (two) put_bands(o, T2, p->n2);
        o += L.tb_b2;
        memcpy(&L.htab[o], T1->E.data(), (p->n1 + 1) * 8);
        o += L.tb_e1;
        if (two) memcpy(&L.htab[o], T2->E.data(), (p->n2 + 1) * 8);
        o += L.tb_e2;
        if (L.nrows) memcpy(&L.htab[o], L.rows.data(), L.nrows * 16);
    }
    // numeric constants
    a.scale1 = T1->scale;
    a.scale2 = two ? T2->scale : 1.f;
    a.vmax1 = T1->vmax;
    a.vmax2 = two ? T2->vmax : 0.f;
    a.n1 = p->n1;
    a.n2 = p->n2;
    a.nbins = p->nbins;
    a.nx = g.nx;
    a.side32 = (float)g.side;
    a.L = g.L;
    a.halfL = g.L * 0.5;
    a.r2prune = p->r2prune32;
    a.d2small = p->d2small;
    a.mu_n = (float)p->n2;
    a.tolA = p->mu_tolA;
    a.tolB = p->mu_tolB;
    a.tolC = p->mu_tolC;
    a.mu_top_closed = 1;
    a.wscale = ldexp(1.0, S - 32);
    a.ncat = 1;
    a.flush_pairs = 1ull << (p->tune.flush_log2 >= 1 && p->tune.flush_log2 <= FLUSH_LOG2_MAX ? p->tune.flush_log2
                                                                                              : FLUSH_LOG2_MAX);
    a.shard_count = (p->tune.shard_count >= 1) ? (uint32_t)p->tune.shard_count : 1u;
    a.shard_index = (p->tune.shard_count >= 1) ? (uint32_t)p->tune.shard_index : 0u;
    FCFC_HIP(hipFuncSetAttribute((const void*)L.kern, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes));
    return FCFC_OK;
}

// Point the table pointers of the arguments into the uploaded blob; returns the stencil rows.
static int4* bind_tables(const LaunchSetup& L, char* tab, CountArgs& a) {
    char* o = tab;
    a.lut1 = (const int16_t*)o;
    o += L.tb_l1;
    a.lut2 = (const int16_t*)o;
    o += L.tb_l2;
    a.band1 = (const float2*)o;
    o += L.tb_b1;
    a.band2 = (const float2*)o;
    o += L.tb_b2;
    a.E1 = (const double*)o;
    o += L.tb_e1;
    a.E2 = (const double*)o;
    o += L.tb_e2;
    return (int4*)o;
}

static WLArgs make_wl(const Plan* p, const LaunchSetup& L, bool is_auto, int ncat, int64_t npoints_a) {
    const Grid& g = p->grid;
    WLArgs w{};
    w.nx = g.nx;
    w.ny = g.ny;
    w.nz = g.nz;
    w.seg = L.seg;
    w.tile = L.T;
    w.bchunk = L.bchunk;
    w.nrows = std::max(1, L.nrows);
    w.periodic = g.L > 0;
    w.is_auto = is_auto;
    w.full_rows = !is_auto;  // stencil_rows keeps the half stencil for auto counts
    w.ncat = ncat;
    // tiles end at `tile` points, at a span of `seg` cells, or at a row end
    const int64_t nrow = (int64_t)g.ny * g.nz * ncat;
    w.tiles_cap = (uint32_t)std::min<int64_t>(nrow * ((g.nx + L.seg - 1) / L.seg + 1) + npoints_a / L.T + 1,
                                              0xffffffffLL);
    return w;
}

// Claims on the work cursor: the first four rounds of positions (one per
// wave each) one at a time; after that each wave spaces its claims so that
// all waves together make at most one claim per 24 ns, about half of what
// one cursor sustains (measured on MI355X: C5 5.4 -> 4.4 ms once claims were
// grouped; grouping the largest items as well slowed counts of few items,
// and grouping large items slowed C3 DR).
static void set_grab(CountArgs& a, uint32_t nitems, int64_t waves) {
    (void)nitems;
    const int64_t w = std::max<int64_t>(1, waves);
    a.grab_single = (uint32_t)std::min<int64_t>(4 * w, 0xffffffffLL);
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;
    a.grab_gap = (unsigned long long)((double)w * 24e-9 * (double)khz * 1e3);
}

static int grid_blocks(const LaunchSetup& L, uint32_t nitems, int* occ_out = nullptr) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)L.kern, L.waves * 64, L.a.lds_bytes) !=
            hipSuccess ||
        occ < 1)
        occ = 1;
    if (occ_out) *occ_out = occ;
    int64_t nblk = (int64_t)device_cu_count() * occ;
    int64_t need = ((int64_t)nitems + L.waves - 1) / L.waves;
    if (nblk > need) nblk = std::max<int64_t>(1, need);
    return (int)nblk;
}

// sum and maximum over i of 2^pred[i] - 1 (predicted ticks): out[0] += sum;
// out[1] = max, as the bits of a non-negative double (ordered like integers)
__global__ __launch_bounds__(256) void k_sum_exp2m1(const float* __restrict__ pred, uint32_t n, double* out) {
    __shared__ double part[4], pmax[4];
    double acc = 0, mx = 0;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float v = pred[i];
        const double t = (double)exp2f(fminf(fmaxf(v, 0.f), 40.f)) - 1.0;
        acc += t;
        mx = fmax(mx, t);
    }
    for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o);
        mx = fmax(mx, __shfl_xor(mx, o));
    }
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6] = acc;
        pmax[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
        const double m = fmax(fmax(pmax[0], pmax[1]), fmax(pmax[2], pmax[3]));
        atomicMax((unsigned long long*)(out + 1), (unsigned long long)__double_as_longlong(m));
    }
}

__global__ __launch_bounds__(256) void k_pred_check(const float* __restrict__ pred, uint32_t n,
                                                    unsigned long long* bad) {
    bool b = false;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) b |= !isfinite(pred[i]);
    if (__any(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1ull);
}

// k_pred_check over the first *n_dev predictions (a batched list sized on the device)
__global__ __launch_bounds__(256) void k_pred_check_dev(const float* __restrict__ pred, const uint32_t* n_dev,
                                                        unsigned long long* bad) {
    const uint32_t n = *n_dev;
    bool b = false;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) b |= !isfinite(pred[i]);
    if (__any(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1ull);
}

// learned sort key: half-octave buckets of the predicted time, longest first;
// the heuristic key (cost = A points x B points) if any prediction was bad
__global__ void k_pred_keys(const Item* __restrict__ items, const float* __restrict__ pred,
                            const unsigned long long* __restrict__ bad, uint32_t n, uint32_t* __restrict__ key,
                            uint32_t* __restrict__ val) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t k;
    if (*bad) {
        const uint32_t c = items[i].cost;
        const uint32_t lg = c ? 31u - (uint32_t)__clz(c) : 0u;
        const uint32_t half = (lg >= 1 && ((c >> (lg - 1)) & 1u)) ? 1u : 0u;
        k = 63u - min(63u, 2u * lg + half);
    } else {
        const float b = fminf(fmaxf(2.f * pred[i], 0.f), 63.f);
        k = 63u - (uint32_t)b;
    }
    key[i] = k;
    val[i] = i;
}

// ---------------------------------------------------------------------------
// single count
// ---------------------------------------------------------------------------
fcfc_status count_pairs(Plan* p, Cells* c1, Cells* c2, int64_t* d_counts, double* d_wcounts, hipStream_t st,
                        PredictReq* pr, const Workspace* ws) {
    const bool is_auto = (c2 == nullptr);
    Cells* cb = is_auto ? c1 : c2;
    const bool weighted = d_wcounts != nullptr;
    const Grid& g = p->grid;
    const bool tree = c1->tree;
    if (tree != cb->tree || tree != (p->tune.tree_leaf > 0)) {
        set_error("count_pairs: cell sets and plan disagree on grid or tree");
        return FCFC_EGRID;
    }
    if (tree) {
        if (pr) {
            set_error("count_pairs: predictions take grid plans only");
            return FCFC_EINVAL;
        }
        // FP32 bands for leaf-local coordinates: rebuilt when these trees hold
        // points farther from their leaf origins than the bands assume
        const double ext = std::max(c1->tree_ext, cb->tree_ext);
        if (ext > p->tree_side) {
            p->tree_side = ext * (1.0 + 1e-9);
            FCFC_TRY(plan_finalize_numerics(p));
        }
    }
    int S = 0;
    if (weighted) {
        if (!c1->weighted || !cb->weighted) {
            set_error("count_pairs: weighted counts need weights in both cell sets");
            return FCFC_EINVAL;
        }
        FCFC_TRY(weight_scale(c1->wmin, c1->wmax, cb->wmin, cb->wmax, &S));
    }
    LaunchSetup L;
    FCFC_TRY(setup_launch(p, is_auto, weighted, false, S, L));
    CountArgs& a = L.a;
    const bool sorted = !pr && p->tune.order != FCFC_ORDER_BUILT;
    const Model* model =
        pr ? pr->model : ((p->tune.order == FCFC_ORDER_LEARNED && !tree) ? p->model : nullptr);
    WLArgs w = make_wl(p, L, is_auto, 1, c1->n);
    w.keyB = cb->xkey;
    w.xbits = cb->xbits;
    // grid: A rows and tiles x stencil rows; tree: A leaves
    const int64_t nseg = tree ? 1 : (int64_t)g.ny * g.nz;
    const int64_t tiles_cap = tree ? 1 : w.tiles_cap;
    if (tiles_cap >= 0xffffffffLL / std::max(1, L.nrows)) {
        set_error("count_pairs: work list too large");
        return FCFC_ERANGE;
    }
    const int64_t npair_tr = tree ? ((int64_t)tree_leaves(c1) << tree_wl_split(c1, cb)) : tiles_cap * w.nrows;

    // scratch 1: tables, tiles, tile counts/offsets, item counts/offsets, counters, arguments
    size_t s_tab = al256(L.tb_total);
    size_t s_tc = al256((size_t)nseg * 4);
    size_t s_tiles = al256((size_t)tiles_cap * sizeof(Tile));
    size_t s_ic = al256((size_t)npair_tr * 4);
    size_t s_scan = al256(std::max(scan_scratch_bytes(nseg), scan_scratch_bytes(npair_tr)));
    size_t s_ctr = 256;
    size_t s_args = al256(sizeof(CountArgs));
    size_t s_acc = weighted ? al256((size_t)p->nbins * 16) : 0;
    size_t s1 = s_tab + 2 * s_tc + s_tiles + 2 * s_ic + s_scan + s_ctr + s_args + s_acc;
    char* scr = nullptr;
    if (ws) {
        // the caller's workspace: nothing is allocated
        if (s1 > ws->bytes) {
            set_error("count_pairs: %zu bytes of scratch needed before the work list, the workspace holds %zu", s1,
                      ws->bytes);
            return FCFC_ERANGE;
        }
        scr = ws->base;
    } else if (dev_alloc((void**)&scr, s1, st) != FCFC_OK) {
        set_error("count_pairs: cannot allocate %zu bytes of scratch", s1);
        return FCFC_ENOMEM;
    }
    auto release = [&](char* ptr) {
        if (!ws) dev_free(ptr, st);
    };
    char* q = scr;
    char* tab = q;
    q += s_tab;
    uint32_t* tcount = (uint32_t*)q;
    q += s_tc;
    uint32_t* toff = (uint32_t*)q;
    q += s_tc;
    Tile* tiles = (Tile*)q;
    q += s_tiles;
    uint32_t* icount = (uint32_t*)q;
    q += s_ic;
    uint32_t* ioff = (uint32_t*)q;
    q += s_ic;
    void* scan_scr = q;
    q += s_scan;
    uint32_t* ctr = (uint32_t*)q;  // [0] ntiles [1] nitems [2] cursor
    q += s_ctr;
    CountArgs* args_dev = (CountArgs*)q;
    q += s_args;
    unsigned long long* wacc = (unsigned long long*)q;

    p->host_stage.swap(L.htab);
    FCFC_HIP(hipMemcpyAsync(tab, p->host_stage.data(), L.tb_total, hipMemcpyHostToDevice, st));
    int4* srows = bind_tables(L, tab, a);
    fill_u32(ctr, 0u, 64, st);
    if (tree) {
        tree_items_enqueue(c1, cb, is_auto, p->rprune, p->coord_max, L.bchunk, nullptr, icount, nullptr, 0, st);
    } else {
        hipLaunchKernelGGL(k_tile_count, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st, c1->cell_start, w,
                           tcount);
        scan_exclusive_u32(tcount, toff, nseg, &ctr[0], scan_scr, st);
        hipLaunchKernelGGL(k_tile_write, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st, c1->cell_start,
                           c1->xkey, w, toff, tiles);
        hipLaunchKernelGGL(k_item_count, dim3((unsigned)((npair_tr + 255) / 256)), dim3(256), 0, st, tiles, &ctr[0],
                           srows, cb->cell_start, w, icount);
    }
    scan_exclusive_u32(icount, ioff, npair_tr, &ctr[1], scan_scr, st);
    uint32_t hctr[2] = {0, 0};
    FCFC_HIP(hipMemcpyAsync(hctr, ctr, 8, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipStreamSynchronize(st));
    uint32_t nitems = hctr[1];
    size_t s_items = al256((size_t)std::max<uint32_t>(nitems, 1) * sizeof(Item));
    size_t s_sort = sorted ? al256((size_t)std::max<uint32_t>(nitems, 1) * 4) : 0;
    size_t s_rs = sorted ? al256(radix_scratch_bytes(nitems)) : 0;
    size_t s_times = (p->tune.record_timing && !pr && !ws) ? al256((size_t)std::max<uint32_t>(nitems, 1) * 4) : 0;
    size_t s_pred = model ? al256((size_t)std::max<uint32_t>(nitems, 1) * 20) : 0;
    size_t s2 = 2 * s_items + 4 * s_sort + s_rs + s_times + s_pred;
    char* scr2 = nullptr;
    if (ws) {
        // s1 is a sum of 256-byte multiples, so the second part stays aligned
        if (s1 + s2 > ws->bytes) {
            set_error("count_pairs: %u work items need %zu bytes of scratch, the workspace holds %zu", nitems, s1 + s2,
                      ws->bytes);
            return FCFC_ERANGE;
        }
        scr2 = ws->base + s1;
    } else if (dev_alloc((void**)&scr2, s2, st) != FCFC_OK) {
        dev_free(scr, st);
        set_error("count_pairs: cannot allocate %zu bytes for %u work items", s2, nitems);
        return FCFC_ENOMEM;
    }
    Item* items = (Item*)scr2;
    Item* items2 = (Item*)(scr2 + s_items);
    if (tree)
        tree_items_enqueue(c1, cb, is_auto, p->rprune, p->coord_max, L.bchunk, ioff, nullptr, items, nitems, st);
    else
        hipLaunchKernelGGL(k_item_write, dim3((unsigned)((npair_tr + 255) / 256)), dim3(256), 0, st, tiles, &ctr[0],
                           srows, cb->cell_start, w, ioff, items, nitems);
    Item* run_items = items;
    float* pred = model ? (float*)(scr2 + 2 * s_items + 4 * s_sort + s_rs + s_times) : nullptr;
    const float kcells = (float)(p->rprune / g.side);
    if (pr) {
        // predict-only: score the work list and stop
        const int nblk = grid_blocks(L, nitems);
        double tk[2] = {0, 0};  // predicted ticks: sum, largest item
        if (nitems > 0) {
            model_item_costs(model, items, nitems, kcells, pred + nitems, pred, st);
            double* dsum = (double*)&ctr[8];
            fill_u64((uint64_t*)dsum, 0ull, 2, st);
            hipLaunchKernelGGL(k_sum_exp2m1, dim3(std::min<uint32_t>((nitems + 255) / 256, 1024)), dim3(256), 0, st,
                               pred, nitems, dsum);
            FCFC_HIP(hipMemcpyAsync(tk, dsum, 16, hipMemcpyDeviceToHost, st));
        }
        FCFC_HIP(hipStreamSynchronize(st));
        release(scr2);
        release(scr);
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, 0) != hipSuccess || khz <= 0) khz = 100000;
        pr->items = nitems;
        // the schedule can finish no earlier than the mean load of a wave or the largest item
        pr->pred_ms = std::max(tk[0] / ((double)nblk * L.waves), tk[1]) / (double)khz;
        return FCFC_OK;
    }
    // launch statistics: the plan's buffer and events, made by the first
    // allocating count (a count into a workspace keeps none without them)
    if (!p->stats_dev && !ws) {
        FCFC_HIP(hipMalloc(&p->stats_dev, 64));
        FCFC_HIP(hipEventCreate(&p->ev0));
        FCFC_HIP(hipEventCreate(&p->ev1));
    }
    const bool keep_stats = p->stats_dev != nullptr;
    if (keep_stats) fill_u64((uint64_t*)p->stats_dev, 0ull, 8, st);
    if (sorted && nitems > 1) {
        uint32_t* k0 = (uint32_t*)(scr2 + 2 * s_items);
        uint32_t* v0 = (uint32_t*)(scr2 + 2 * s_items + s_sort);
        uint32_t* k1 = (uint32_t*)(scr2 + 2 * s_items + 2 * s_sort);
        uint32_t* v1 = (uint32_t*)(scr2 + 2 * s_items + 3 * s_sort);
        void* rs = scr2 + 2 * s_items + 4 * s_sort;
        if (model) {
            // learned order: longest predicted first; any non-finite prediction
            // sends the whole list back to the heuristic key (flag in stats[5])
            model_item_costs(model, items, nitems, kcells, pred + nitems, pred, st);
            // (ctr[8..9] were zeroed with the other counters)
            unsigned long long* bad = keep_stats ? (unsigned long long*)p->stats_dev + 5 : (unsigned long long*)&ctr[8];
            hipLaunchKernelGGL(k_pred_check, dim3(std::min<uint32_t>((nitems + 255) / 256, 1024)), dim3(256), 0, st,
                               pred, nitems, bad);
            hipLaunchKernelGGL(k_pred_keys, dim3((nitems + 255) / 256), dim3(256), 0, st, items, pred, bad, nitems, k0,
                               v0);
        } else {
            hipLaunchKernelGGL(k_item_keys, dim3((nitems + 255) / 256), dim3(256), 0, st, items, &ctr[1], nitems, k0,
                               v0);
        }
        radix_sort_pairs(&k0, &v0, &k1, &v1, nitems, 8, rs, st);
        hipLaunchKernelGGL(k_item_permute, dim3((nitems + 255) / 256), dim3(256), 0, st, items, v0, &ctr[1], nitems,
                           items2);
        run_items = items2;
    }
    uint32_t* times = p->tune.record_timing ? (uint32_t*)(scr2 + 2 * s_items + 4 * s_sort + s_rs) : nullptr;

    fill_u64((uint64_t*)d_counts, 0ull, p->nbins, st);
    if (weighted) fill_u64((uint64_t*)wacc, 0ull, 2 * (int64_t)p->nbins, st);

    a.posA = c1->pos32;
    a.absA = c1->abs32;
    a.p64A = c1->pos64;
    a.wA = c1->w;
    a.posB = cb->pos32;
    a.p64B = cb->pos64;
    a.wB = cb->w;
    a.csB = cb->cell_start;
    if (tree) {
        a.leaf_orgA = c1->leaf_org;
        a.leaf_orgB = cb->leaf_org;
        a.tree_q = (float)c1->tree_q;
        a.tree_leaf = (uint32_t)cb->xbits;
        a.tree_nleafB = tree_leaves(cb);
        a.nB = (uint32_t)cb->n;
    }
    a.items = run_items;
    a.nitems_dev = &ctr[1];
    a.cursor = &ctr[2];
    a.out_counts = (unsigned long long*)d_counts;
    a.out_w = weighted ? wacc : nullptr;
    a.stats = keep_stats ? (unsigned long long*)p->stats_dev : nullptr;
    a.times = times;

    int occ = 1;
    const int nblk = grid_blocks(L, nitems, &occ);
    set_grab(a, nitems, (int64_t)nblk * L.waves);
    if (keep_stats) FCFC_HIP(hipEventRecord(p->ev0, st));
    p->host_args.resize(sizeof(CountArgs));
    memcpy(p->host_args.data(), &a, sizeof(CountArgs));
    FCFC_HIP(hipMemcpyAsync(args_dev, p->host_args.data(), sizeof(CountArgs), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(L.kern, dim3((unsigned)nblk), dim3(L.waves * 64), (size_t)a.lds_bytes, st,
                       (const CountArgs*)args_dev);
    FCFC_HIP(hipGetLastError());
    if (keep_stats) FCFC_HIP(hipEventRecord(p->ev1, st));
    if (weighted)
        hipLaunchKernelGGL(k_finalize_w, dim3((p->nbins + 255) / 256), dim3(256), 0, st, wacc, p->nbins, S, d_wcounts);
    if (times) {
        // keep the per-item times and items for the scheduler (plan-owned)
        if (p->timing_dev) (void)hipFree(p->timing_dev);
        p->timing_dev = nullptr;
        p->timing_n = 0;
        size_t tb = (size_t)nitems * (4 + sizeof(Item));
        if (hipMalloc(&p->timing_dev, std::max<size_t>(tb, 256)) == hipSuccess) {
            FCFC_HIP(hipMemcpyAsync(p->timing_dev, times, (size_t)nitems * 4, hipMemcpyDeviceToDevice, st));
            FCFC_HIP(hipMemcpyAsync((char*)p->timing_dev + (size_t)nitems * 4, run_items, (size_t)nitems * sizeof(Item),
                                    hipMemcpyDeviceToDevice, st));
            p->timing_n = nitems;
        }
    }
    release(scr2);
    release(scr);
    p->last_stream = st;
    p->have_stats = keep_stats;
    p->stats.items = nitems;
    p->stats.cells = tree ? (int64_t)tree_leaves(c1) : g.ncell();
    p->stats.grid[0] = g.nx;
    p->stats.grid[1] = g.ny;
    p->stats.grid[2] = g.nz;
    p->stats.cells_per_rmax = g.k;
    p->stats.cell_side = g.side;
    p->stats.wg_per_cu = occ;
    p->stats.group_waves = L.waves;
    p->stats.lut_entries = L.lut_entries;
    p->stats.order_used = model ? FCFC_ORDER_LEARNED : (sorted ? FCFC_ORDER_HEURISTIC : FCFC_ORDER_BUILT);
    p->last_pts = L.P;
    return FCFC_OK;
}

// ---------------------------------------------------------------------------
// batched auto counts of many periodic catalogues
// ---------------------------------------------------------------------------
__global__ void k_clamp_items(uint32_t* ctr, uint32_t cap) {
    if (ctr[1] > cap) {
        ctr[1] = cap;
        ctr[5] = 1u;  // overflow flag
    }
}

struct BatchImpl {
    Plan* plan = nullptr;
    int ncat = 0;
    int npairs = 0;  // histograms written: one per (A, B) catalogue pair
    int xbits = 0;   // sub-cell x bits of the sort keys
    int64_t ntot = 0;
    bool weighted = false;
    int S = 0;
    LaunchSetup L;
    WLArgs wl;
    int64_t nseg = 0, npair_tr = 0;
    uint32_t items_cap = 0;
    int nblk = 1;
    // device
    CatDesc* desc = nullptr;
    int64_t* offs = nullptr;
    uint32_t *key = nullptr, *idx = nullptr, *tk = nullptr, *tv = nullptr;
    uint32_t *key_s = nullptr, *idx_s = nullptr;  // sorted arrays (after ping-pong)
    void* sort_scr = nullptr;
    uint32_t* flags = nullptr;
    uint64_t* wst = nullptr;
    float4* pos32 = nullptr;
    float4* abs32 = nullptr;  // absolute FP32 positions (mid-point line of sight only)
    double* pos64 = nullptr;
    double* w = nullptr;
    uint32_t* cs = nullptr;
    int32_t* pairs = nullptr;  // 2 per pair
    uint32_t *ptile_off = nullptr, *ptile_first = nullptr;
    // largest-first order within each pair: keys, values, sort scratch, sorted items
    uint32_t *sk0 = nullptr, *sv0 = nullptr, *sk1 = nullptr, *sv1 = nullptr;
    // learned order (plan order FCFC_ORDER_LEARNED with a model attached): a
    // frozen copy of the model, item features, predictions, non-finite flag
    Model* msnap = nullptr;
    float* mparams = nullptr;
    float *feat = nullptr, *pred = nullptr;
    unsigned long long* bad = nullptr;
    float kcells = 1.f;
    void* isort_scr = nullptr;
    Item* items2 = nullptr;
    int sort_bits = 8;
    uint32_t key_last = 0;
    uint32_t *tcount = nullptr, *toff = nullptr, *icount = nullptr, *ioff = nullptr;
    void* scan_scr = nullptr;
    Tile* tiles = nullptr;
    Item* items = nullptr;
    uint32_t* ctr = nullptr;  // [0] ntiles [1] nitems [2] cursor [3] nchunks [4] chunk cursor [5] overflow
    unsigned long long* kstats = nullptr;  // counting launch: [0] candidates [1] rechecks [6] early merges
    // pair_items: npairs + 1 item offsets; pair_order: pairs by decreasing estimated cost
    uint32_t *pair_items = nullptr, *pair_order = nullptr, *chunk_prefix = nullptr;
    unsigned long long* counts = nullptr;
    unsigned long long* wacc = nullptr;
    double* wout = nullptr;
    char* tab = nullptr;
    CountArgs* args_dev = nullptr;
    std::vector<void*> allocs;
    std::vector<char> host_args;
    std::vector<uint32_t> host_order;
    std::vector<int32_t> host_pairs;
    std::vector<CatDesc> host_desc;
    std::vector<int64_t> host_offs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t cap = nullptr;  // capture stream (the caller's may be the legacy default stream)
};

static fcfc_status balloc(BatchImpl* b, void** p, size_t bytes) {
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) {
        set_error("batch: cannot allocate %zu bytes", bytes);
        return FCFC_ENOMEM;
    }
    b->allocs.push_back(*p);
    return FCFC_OK;
}

void batch_free_impl(BatchImpl* b) {
    if (!b) return;
    model_snapshot_free(b->msnap);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    (void)hipDeviceSynchronize();
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (void* p : b->allocs) (void)hipFree(p);
    delete b;
}

// Enqueue the build and the work list (up to the item counts).
static void batch_enqueue_front(BatchImpl* b, hipStream_t st) {
    Plan* p = b->plan;
    uint32_t *k = b->key, *v = b->idx, *tk = b->tk, *tv = b->tv;
    batch_build_enqueue(p, b->xbits, b->desc, b->offs, b->ncat, b->ntot, b->weighted, &k, &v, &tk, &tv, b->sort_scr,
                        b->flags, b->wst, b->pos32, b->abs32, b->pos64, b->w, b->cs, st);
    b->key_s = k;
    b->idx_s = v;
    // the sorted keys trim the B ranges (the ping-pong buffer that holds them
    // is the same on every run: the pass count is fixed)
    b->wl.keyB = k;
    b->wl.xbits = b->xbits;
    int4* srows = (int4*)(b->tab + (b->L.tb_total - b->L.tb_rows));
    fill_u32(b->ctr, 0u, 64, st);
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)((b->nseg + 255) / 256)), dim3(256), 0, st, b->cs, b->wl, b->tcount);
    scan_exclusive_u32(b->tcount, b->toff, b->nseg, &b->ctr[0], b->scan_scr, st);
    hipLaunchKernelGGL(k_tile_write, dim3((unsigned)((b->nseg + 255) / 256)), dim3(256), 0, st, b->cs, k, b->wl,
                       b->toff, b->tiles);
    hipLaunchKernelGGL(k_pair_tiles, dim3(1), dim3(1), 0, st, b->toff, &b->ctr[0], b->wl, b->ptile_off, b->ptile_first);
    hipLaunchKernelGGL(k_item_count, dim3((unsigned)((b->npair_tr + 255) / 256)), dim3(256), 0, st, b->tiles, &b->ctr[0],
                       srows, b->cs, b->wl, b->icount);
    scan_exclusive_u32(b->icount, b->ioff, b->npair_tr, &b->ctr[1], b->scan_scr, st);
}

// Enqueue the rest: items, catalogue ranges, chunks, counting kernel, merge.
static void batch_enqueue_back(BatchImpl* b, hipStream_t st) {
    Plan* p = b->plan;
    int4* srows = (int4*)(b->tab + (b->L.tb_total - b->L.tb_rows));
    hipLaunchKernelGGL(k_clamp_items, dim3(1), dim3(1), 0, st, b->ctr, b->items_cap);
    hipLaunchKernelGGL(k_item_write, dim3((unsigned)((b->npair_tr + 255) / 256)), dim3(256), 0, st, b->tiles, &b->ctr[0],
                       srows, b->cs, b->wl, b->ioff, b->items, b->items_cap);
    hipLaunchKernelGGL(k_pair_items, dim3((b->npairs + 1 + 255) / 256), dim3(256), 0, st, b->ioff, &b->ctr[1], b->wl,
                       b->pair_items);
    // each pair's items largest first (pairs stay in place)
    {
        const unsigned nb = (b->items_cap + 255) / 256;
        uint32_t *k0 = b->sk0, *v0 = b->sv0, *k1 = b->sk1, *v1 = b->sv1;
        if (b->msnap) {
            model_item_costs(b->msnap, b->items, b->items_cap, b->kcells, b->feat, b->pred, st);
            fill_u64((uint64_t*)b->bad, 0ull, 1, st);
            hipLaunchKernelGGL(k_pred_check_dev, dim3(std::min<uint32_t>(nb, 1024)), dim3(256), 0, st, b->pred,
                               &b->ctr[1], b->bad);
            hipLaunchKernelGGL(k_pair_pred_keys, dim3(nb), dim3(256), 0, st, b->items, &b->ctr[1], b->items_cap,
                               b->pair_items, b->npairs, b->key_last, b->pred, b->bad, k0, v0);
        } else {
            hipLaunchKernelGGL(k_pair_item_keys, dim3(nb), dim3(256), 0, st, b->items, &b->ctr[1], b->items_cap,
                               b->pair_items, b->npairs, b->key_last, k0, v0);
        }
        radix_sort_pairs(&k0, &v0, &k1, &v1, b->items_cap, b->sort_bits, b->isort_scr, st);
        hipLaunchKernelGGL(k_item_permute, dim3(nb), dim3(256), 0, st, b->items, v0, &b->ctr[1], b->items_cap,
                           b->items2);
    }
    hipLaunchKernelGGL(k_chunk_prefix, dim3(1), dim3(1), 0, st, b->pair_items, b->pair_order, b->npairs,
                       b->L.a.chunk_items, b->chunk_prefix, &b->ctr[3]);
    fill_u64((uint64_t*)b->counts, 0ull, (int64_t)b->npairs * p->nbins, st);
    if (b->weighted) fill_u64((uint64_t*)b->wacc, 0ull, 2 * (int64_t)b->npairs * p->nbins, st);
    fill_u64((uint64_t*)b->kstats, 0ull, 8, st);
    hipLaunchKernelGGL(b->L.kern, dim3((unsigned)b->nblk), dim3(b->L.waves * 64), (size_t)b->L.a.lds_bytes, st,
                       (const CountArgs*)b->args_dev);
    if (b->weighted)
        hipLaunchKernelGGL(k_finalize_w, dim3((b->npairs * p->nbins + 255) / 256), dim3(256), 0, st, b->wacc,
                           b->npairs * p->nbins, b->S, b->wout);
}

fcfc_status batch_create_impl(Plan* p, const fcfc_catalog* cats, int ncat, const int32_t* pairs, int npairs,
                              hipStream_t st, BatchImpl** out) {
    if (p->tune.tree_leaf > 0) {
        set_error("batch_create: batches take grid plans (tree_leaf = 0)");
        return FCFC_EINVAL;
    }
    if (p->L <= 0 && !p->grid_set) {
        set_error("batch_create: an open-box plan needs fcfc_plan_fit_bounds or fcfc_plan_set_bounds first");
        return FCFC_ESTATE;
    }
    BatchImpl* b = new (std::nothrow) BatchImpl();
    if (!b) return FCFC_ENOMEM;
    b->plan = p;
    b->ncat = ncat;
    b->npairs = npairs;
    // weighted when any catalogue has weights; an empty catalogue has no weights to give
    b->weighted = false;
    for (int c = 0; c < ncat; c++) b->weighted = b->weighted || cats[c].w != nullptr;
    b->host_desc.resize(ncat);
    b->host_offs.resize(ncat + 1);
    b->host_pairs.assign(pairs, pairs + 2 * (size_t)npairs);
    int64_t tot = 0;
    for (int c = 0; c < ncat; c++) {
        if (cats[c].n > 0 && (cats[c].w != nullptr) != b->weighted) {
            delete b;
            set_error("batch_create: either every catalogue has weights or none");
            return FCFC_EINVAL;
        }
        b->host_desc[c] = CatDesc{cats[c].xyz, cats[c].w, cats[c].n, tot};
        b->host_offs[c] = tot;
        tot += cats[c].n;
    }
    b->host_offs[ncat] = tot;
    b->ntot = tot;
    if (tot >= ((int64_t)1 << 31)) {
        delete b;
        set_error("batch_create: more than 2^31 points in the batch");
        return FCFC_ERANGE;
    }
    const Grid& g = p->grid;
    if ((int64_t)ncat * g.ncell() >= ((int64_t)1 << 31)) {
        delete b;
        set_error("batch_create: catalogues x cells exceeds 2^31");
        return FCFC_ERANGE;
    }
    bool all_auto = true;
    for (int q = 0; q < npairs; q++) all_auto = all_auto && (pairs[2 * q] == pairs[2 * q + 1]);
    // pair order: largest estimated cost first (n^2 / 2 for an auto count, n_a n_b for a cross count)
    std::vector<double> cost(npairs);
    for (int q = 0; q < npairs; q++) {
        const double na = (double)cats[pairs[2 * q]].n, nb = (double)cats[pairs[2 * q + 1]].n;
        cost[q] = (pairs[2 * q] == pairs[2 * q + 1]) ? 0.5 * na * na : na * nb;
    }
    b->host_order.resize(npairs);
    for (int q = 0; q < npairs; q++) b->host_order[q] = (uint32_t)q;
    std::stable_sort(b->host_order.begin(), b->host_order.end(),
                     [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
    fcfc_status s = setup_launch(p, all_auto, b->weighted, true, 0, b->L);
    if (s != FCFC_OK) {
        delete b;
        return s;
    }
    b->wl = make_wl(p, b->L, all_auto, ncat, tot);
    b->xbits = key_xbits((int64_t)ncat * g.ncell());
    b->nseg = (int64_t)g.ny * g.nz * ncat;  // A rows
    // pair-tiles: every pair takes the tiles of its A catalogue (each bounded as in make_wl)
    std::vector<int64_t> cat_tiles(ncat);
    int64_t tiles = 0;
    for (int c = 0; c < ncat; c++) {
        cat_tiles[c] = (int64_t)g.ny * g.nz * ((g.nx + b->L.seg - 1) / b->L.seg + 1) + cats[c].n / b->L.T + 1;
        tiles += cat_tiles[c];
    }
    int64_t ptiles = 0;
    for (int q = 0; q < npairs; q++) ptiles += cat_tiles[pairs[2 * q]];
    b->npair_tr = ptiles * b->wl.nrows;
    if (tiles >= 0xffffffffLL || b->npair_tr >= 0xffffffffLL) {
        delete b;
        set_error("batch_create: work list too large");
        return FCFC_ERANGE;
    }
    b->wl.npairs = npairs;
    b->wl.ptiles_cap = (uint32_t)ptiles;
    b->wl.tiles_cap = (uint32_t)tiles;
    const int nb = p->nbins;
    const bool need_abs = (p->los == FCFC_LOS_MIDPOINT && p->kind != FCFC_BIN_S);
#define BA(ptr, bytes)                                                         \
    do {                                                                       \
        fcfc_status s_ = balloc(b, (void**)&(ptr), (bytes));                   \
        if (s_ != FCFC_OK) {                                                   \
            batch_free_impl(b);                                                \
            return s_;                                                         \
        }                                                                      \
    } while (0)
    BA(b->desc, sizeof(CatDesc) * ncat);
    BA(b->offs, sizeof(int64_t) * (ncat + 1));
    BA(b->key, 4 * (size_t)tot);
    BA(b->idx, 4 * (size_t)tot);
    BA(b->tk, 4 * (size_t)tot);
    BA(b->tv, 4 * (size_t)tot);
    BA(b->sort_scr, batch_build_scratch(tot));
    BA(b->flags, 64);
    BA(b->wst, STAT_BYTES);
    BA(b->pos32, 16 * (size_t)(tot + 8));
    if (need_abs) BA(b->abs32, 16 * (size_t)(tot + 8));
    BA(b->pos64, 24 * (size_t)tot);
    if (b->weighted) BA(b->w, 8 * (size_t)(tot + 8));
    BA(b->cs, 4 * (size_t)(g.ncell() * ncat + 1));
    BA(b->tcount, 4 * (size_t)b->nseg);
    BA(b->toff, 4 * (size_t)b->nseg);
    BA(b->icount, 4 * (size_t)b->npair_tr);
    BA(b->ioff, 4 * (size_t)b->npair_tr);
    BA(b->scan_scr, std::max(scan_scratch_bytes(b->nseg), scan_scratch_bytes(b->npair_tr)));
    BA(b->tiles, sizeof(Tile) * (size_t)b->wl.tiles_cap);
    BA(b->ctr, 256);
    BA(b->kstats, 64);
    BA(b->pairs, 8 * (size_t)npairs);
    BA(b->ptile_off, 4 * (size_t)(npairs + 1));
    BA(b->ptile_first, 4 * (size_t)npairs);
    BA(b->pair_items, 4 * (size_t)(npairs + 1));
    BA(b->pair_order, 4 * (size_t)npairs);
    BA(b->chunk_prefix, 4 * (size_t)(npairs + 1));
    BA(b->counts, 8 * (size_t)npairs * nb);
    if (b->weighted) {
        BA(b->wacc, 16 * (size_t)npairs * nb);
        BA(b->wout, 8 * (size_t)npairs * nb);
    }
    BA(b->tab, b->L.tb_total);
    BA(b->args_dev, sizeof(CountArgs));
    b->wl.pairs = b->pairs;
    b->wl.ptile_off = b->ptile_off;
    b->wl.ptile_first = b->ptile_first;
    FCFC_HIP(hipMemcpy(b->desc, b->host_desc.data(), sizeof(CatDesc) * ncat, hipMemcpyHostToDevice));
    FCFC_HIP(hipMemcpy(b->offs, b->host_offs.data(), sizeof(int64_t) * (ncat + 1), hipMemcpyHostToDevice));
    FCFC_HIP(hipMemcpy(b->pairs, b->host_pairs.data(), 8 * (size_t)npairs, hipMemcpyHostToDevice));
    FCFC_HIP(hipMemcpy(b->pair_order, b->host_order.data(), 4 * (size_t)npairs, hipMemcpyHostToDevice));
    FCFC_HIP(hipMemcpy(b->tab, b->L.htab.data(), b->L.tb_total, hipMemcpyHostToDevice));
    FCFC_HIP(hipEventCreate(&b->ev0));
    FCFC_HIP(hipEventCreate(&b->ev1));
    // one eager pass of the front half sizes the work list and validates the data
    batch_enqueue_front(b, st);
    uint32_t hctr[2] = {0, 0};
    uint64_t hw[2] = {0, 0};
    std::vector<uint64_t> hws(STAT_SLOTS * STAT_STRIDE);
    uint32_t hflags = 0;
    FCFC_HIP(hipMemcpyAsync(hctr, b->ctr, 8, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipMemcpyAsync(hws.data(), b->wst, STAT_BYTES, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipMemcpyAsync(&hflags, b->flags, 4, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipStreamSynchronize(st));
    if (hflags & 5u) {
        batch_free_impl(b);
        set_error("batch_create: non-finite position or weight");
        return FCFC_ENONFINITE;
    }
    if (hflags & 2u) {
        batch_free_impl(b);
        set_error(p->L > 0 ? "batch_create: a point lies outside [0, L)"
                           : "batch_create: a point lies outside the plan bounds");
        return FCFC_EBOX;
    }
    if (b->weighted) {
        weight_stats_reduce(hws.data(), &hw[0], &hw[1]);
        double wmin = 0, wmax = 0;
        if (hw[0] != ~0ull) memcpy(&wmin, &hw[0], 8);
        memcpy(&wmax, &hw[1], 8);
        fcfc_status ws = weight_scale(wmin, wmax, wmin, wmax, &b->S);
        if (ws != FCFC_OK) {
            batch_free_impl(b);
            return ws;
        }
    }
    b->items_cap = std::max<uint32_t>(hctr[1], 1);
    BA(b->items, sizeof(Item) * (size_t)b->items_cap);
    BA(b->items2, sizeof(Item) * (size_t)b->items_cap);
    BA(b->sk0, 4 * (size_t)b->items_cap);
    BA(b->sv0, 4 * (size_t)b->items_cap);
    BA(b->sk1, 4 * (size_t)b->items_cap);
    BA(b->sv1, 4 * (size_t)b->items_cap);
    BA(b->isort_scr, radix_scratch_bytes(b->items_cap));
    if (p->tune.order == FCFC_ORDER_LEARNED && p->model) {
        BA(b->mparams, model_param_bytes());
        BA(b->feat, 16 * (size_t)b->items_cap);
        BA(b->pred, 4 * (size_t)b->items_cap);
        BA(b->bad, 64);
        b->msnap = model_snapshot(p->model, b->mparams, st);
        if (!b->msnap) {
            batch_free_impl(b);
            set_error("batch_create: cannot copy the cost model");
            return FCFC_EHIP;
        }
        b->kcells = (float)(p->rprune / g.side);
        FCFC_HIP(hipStreamSynchronize(st));
    }
#undef BA
    // pair keys (pair << 6 | cost key) sort in whole bytes; the end key is above them all
    b->sort_bits = 8;
    while (((uint64_t)npairs << 6) >= ((uint64_t)1 << b->sort_bits)) b->sort_bits += 8;
    b->key_last = (uint32_t)(((uint64_t)1 << b->sort_bits) - 1);
    CountArgs& a = b->L.a;
    (void)bind_tables(b->L, b->tab, a);
    a.posA = b->pos32;
    a.absA = b->abs32;
    a.p64A = b->pos64;
    a.wA = b->weighted ? b->w : nullptr;
    a.posB = b->pos32;
    a.p64B = b->pos64;
    a.wB = a.wA;
    a.csB = b->cs;
    a.items = b->items2;
    a.nitems_dev = &b->ctr[1];
    a.cursor = &b->ctr[2];
    a.out_counts = b->counts;
    a.out_w = b->weighted ? b->wacc : nullptr;
    a.stats = b->kstats;
    a.times = nullptr;
    a.wscale = ldexp(1.0, b->S - 32);
    a.nchunks_dev = &b->ctr[3];
    a.chunk_cursor = &b->ctr[4];
    a.chunk_prefix = b->chunk_prefix;
    a.cat_order = b->pair_order;
    a.cat_items = b->pair_items;
    a.ncat = npairs;
    // A workgroup takes chunks of 32 items per wavefront and waits for its
    // slowest wave at the end of each; measured on MI355X, 8 lost 6 % to those
    // waits and 128 or more left long tails (few chunks per pair).
    const int per_wave = (p->tune.batch_chunk >= 1 && p->tune.batch_chunk <= 1024) ? p->tune.batch_chunk : 32;
    a.chunk_items = std::max(16, b->L.waves * per_wave);
    b->host_args.resize(sizeof(CountArgs));
    memcpy(b->host_args.data(), &a, sizeof(CountArgs));
    FCFC_HIP(hipMemcpy(b->args_dev, b->host_args.data(), sizeof(CountArgs), hipMemcpyHostToDevice));
    b->nblk = grid_blocks(b->L, b->items_cap);
    *out = b;
    return FCFC_OK;
}

fcfc_status batch_run_impl(BatchImpl* b, int64_t* d_counts, double* d_wcounts, bool use_graph, hipStream_t st) {
    Plan* p = b->plan;
    if (d_wcounts && !b->weighted) {
        set_error("batch_run: weighted counts requested but the catalogues have no weights");
        return FCFC_EINVAL;
    }
    if (use_graph) {
        if (!b->gexec) {
            if (!b->cap) FCFC_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
            FCFC_HIP(hipStreamSynchronize(st));
            FCFC_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
            batch_enqueue_front(b, b->cap);
            batch_enqueue_back(b, b->cap);
            hipGraph_t g = nullptr;
            FCFC_HIP(hipStreamEndCapture(b->cap, &g));
            b->graph = g;
            FCFC_HIP(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
        }
        FCFC_HIP(hipEventRecord(b->ev0, st));
        FCFC_HIP(hipGraphLaunch(b->gexec, st));
        FCFC_HIP(hipEventRecord(b->ev1, st));
    } else {
        FCFC_HIP(hipEventRecord(b->ev0, st));
        batch_enqueue_front(b, st);
        batch_enqueue_back(b, st);
        FCFC_HIP(hipEventRecord(b->ev1, st));
    }
    const size_t nbytes = (size_t)b->npairs * p->nbins * 8;
    FCFC_HIP(hipMemcpyAsync(d_counts, b->counts, nbytes, hipMemcpyDeviceToDevice, st));
    if (d_wcounts) FCFC_HIP(hipMemcpyAsync(d_wcounts, b->wout, nbytes, hipMemcpyDeviceToDevice, st));
    return FCFC_OK;
}

fcfc_status batch_check_impl(BatchImpl* b, hipStream_t st, uint32_t* nitems, float* ms) {
    uint32_t h[6];
    FCFC_HIP(hipMemcpyAsync(h, b->ctr, 24, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipStreamSynchronize(st));
    if (nitems) *nitems = h[1];
    if (ms && hipEventElapsedTime(ms, b->ev0, b->ev1) != hipSuccess) *ms = -1.f;
    if (h[5]) {
        set_error("batch: the work list outgrew the capacity sized at creation (catalogue contents changed)");
        return FCFC_ERANGE;
    }
    return FCFC_OK;
}

fcfc_status batch_stats_impl(BatchImpl* b, hipStream_t st, int64_t out[3]) {
    unsigned long long h[8];
    FCFC_HIP(hipMemcpyAsync(h, b->kstats, 64, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipStreamSynchronize(st));
    out[0] = (int64_t)h[0];
    out[1] = (int64_t)h[1];
    out[2] = (int64_t)h[6];
    return FCFC_OK;
}

}  // namespace fcfc
