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

constexpr int CT_MAX = 1024;        // threads per workgroup (16 waves: 4 per SIMD, one workgroup per CU)
constexpr int QCAP = 192;           // compaction queue entries per wave (63 + 64 P), plus one dump entry
constexpr int RB_CAP = 128;         // recheck entries per wave
constexpr int ASTAGE = 128;         // staged A points per wave (mid-point line of sight)
constexpr uint64_t FLUSH_PAIRS = 1ull << 26;  // per wave

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
    const uint16_t* lut1;
    const uint16_t* lut2;
    const float* band1;  // lo[0..n1], hi[0..n1]
    const float* band2;
    const double* E1;    // FP64 squared edges
    const double* E2;
    unsigned long long* out_counts;
    unsigned long long* out_w;  // 2 per bin: low, high 64 bits of a signed 128-bit sum
    unsigned long long* stats;  // [0] candidates [1] rechecks [2] in range
    uint32_t* times;            // per item duration (wall clock ticks) or null
    int nlut1, nlut2;
    float scale1, scale2, vmax1, vmax2;
    int n1, n2, nbins;
    int nx;
    float side32;
    double L, halfL;
    float r2prune, d2small;
    float mu_n, tolA, tolB, tolC;
    int mu_top_closed;
    double wscale;
    int copies;
    // LDS layout (bytes)
    int off_lut1, off_lut2, off_band1, off_band2, off_hist, off_whist, off_q, off_qw, off_rb, off_astage,
        off_misc, lds_bytes;
};

// The arguments live in device memory and are read through the constant
// address space (scalar loads); a by-value kernel argument would be copied to
// scratch as soon as a helper takes its address.
typedef const CountArgs FCFC_CONST& ArgsRef;

struct Smem {
    const uint16_t* lut1;
    const uint16_t* lut2;
    const float* band1;
    const float* band2;
    uint32_t* hist;
    unsigned long long* wlo;
    unsigned long long* whi;
    float4* q;        // this wave's compaction queue
    double* qw;       // this wave's queued weight products
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
__device__ inline uint32_t lut_entry(const uint16_t* __restrict__ lut, float scale, float v) {
    return lut[(uint32_t)(v * scale)];
}
// A clean entry holds the bin, or 0x7fff for "out of range".
__device__ inline int lut_clean_bin(uint32_t e) { return (e == 0x7fffu) ? -1 : (int)e; }
// A hot entry (bit 15) holds the first edge whose band meets the entry: count the
// edges certainly <= v (reverse-free forward traversal over the few banded
// edges) and flag v inside a band as ambiguous.
__device__ inline int lut_hot_bin(const float* __restrict__ band, int n, uint32_t e, float v, bool& amb) {
    int k = (int)(e & 0x7fffu);
    int c = k;
    for (; k <= n; k++) {
        if (v >= band[n + 1 + k]) {
            c = k + 1;
        } else {
            if (v >= band[k]) amb = true;
            break;
        }
    }
    return (c >= 1 && c <= n) ? c - 1 : -1;
}

// Kernel constants kept in registers.
struct KConst {
    float scale1, scale2, vmax1, vmax2, r2prune, d2small, mu_n, mu_nm1, tolA, tolB, tolC, side32;
    int n1, n2, nbins, nx, copies;
    double wscale;
};

__device__ inline void add_weight(const Smem& s, int flat, double p, double wscale) {
    long long t = (long long)(p * wscale);
    unsigned long long lo = (unsigned long long)(uint32_t)(t & 0xffffffffll);
    unsigned long long hi = (unsigned long long)(t >> 32);
    atomicAdd(&s.wlo[flat], lo);
    atomicAdd(&s.whi[flat], hi);
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
                add_weight(s, flat, p, a.wscale);
            }
        }
    }
    nrechk += (unsigned long long)cnt;
}

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
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
// Entry: (v1, v2, v3, ids) with ids = (b - b_begin) << 7 | a_slot, and
//   s:              v1 = d2
//   (s,mu), z:      v1 = d2, v2 = dz
//   (sp,pi), z:     v1 = sp2, v2 = pi2
//   mid-point:      v1, v2, v3 = dx, dy, dz (line of sight from the staged A point)
// The common path is branch-free; hot table entries and rechecks take
// wave-uniform branches that are rarely entered.
template <int KIND, int LOS, bool W>
__device__ __attribute__((always_inline)) inline void bin_queue(ArgsRef a, const KConst& k, const Smem& s,
                                                                uint32_t* hist_l, int base, int cnt, int lane,
                                                                WaveCtx& c) {
    const bool valid = lane < cnt;
    float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) e = s.q[base + lane];
    const uint32_t ids = __float_as_uint(e.w);
    bool amb = false;
    int flat;
    if (KIND == FCFC_BIN_S) {
        const float d2 = e.x;
        const uint32_t ent = lut_entry(s.lut1, k.scale1, d2);
        int sb = lut_clean_bin(ent);
        const bool hot = (ent & 0x8000u) != 0u;
        if (__builtin_amdgcn_ballot_w64(hot)) {
            if (hot) sb = lut_hot_bin(s.band1, k.n1, ent, d2, amb);
        }
        flat = sb;
    } else if (KIND == FCFC_BIN_S_MU) {
        float d2, proj_n;  // proj_n: |projection on the line of sight| * n_mu / |l|
        if (LOS == FCFC_LOS_Z) {
            d2 = e.x;
            proj_n = fabsf(e.y) * k.mu_n;
        } else {
            const float dxx = e.x, dyy = e.y, dzz = e.z;
            d2 = __builtin_fmaf(dzz, dzz, __builtin_fmaf(dyy, dyy, dxx * dxx));
            const float4 q = s.astage[ids & 127u];
            const float lx = q.x + dxx, ly = q.y + dyy, lz = q.z + dzz;
            const float dot = __builtin_fmaf(dzz, lz, __builtin_fmaf(dyy, ly, dxx * lx));
            const float ll = __builtin_fmaf(lz, lz, __builtin_fmaf(ly, ly, lx * lx));
            proj_n = fabsf(dot) * (__builtin_amdgcn_rsqf(ll) * k.mu_n);
        }
        const uint32_t ent = lut_entry(s.lut1, k.scale1, d2);
        int sb = lut_clean_bin(ent);
        const bool hot = (ent & 0x8000u) != 0u;
        if (__builtin_amdgcn_ballot_w64(hot)) {
            if (hot) sb = lut_hot_bin(s.band1, k.n1, ent, d2, amb);
        }
        const float rs = __builtin_amdgcn_rsqf(d2);
        const float mun = proj_n * rs;
        const int mb = min((int)mun, k.n2 - 1);
        const float cr = rintf(mun);
        const float dist = fabsf(mun - cr);
        const float tol = __builtin_fmaf(__builtin_fmaf(k.tolB, rs, k.tolA), rs, k.tolC);
        const bool near_edge = (dist < tol) & (cr >= 1.0f) & (cr <= k.mu_nm1);
        amb = amb | near_edge | (d2 < k.d2small);
        flat = (sb >= 0) ? (int)__umul24((uint32_t)sb, (uint32_t)k.n2) + mb : -1;
    } else {
        float sp2, pi2;
        if (LOS == FCFC_LOS_Z) {
            sp2 = e.x;
            pi2 = e.y;
        } else {
            const float dxx = e.x, dyy = e.y, dzz = e.z;
            const float d2 = __builtin_fmaf(dzz, dzz, __builtin_fmaf(dyy, dyy, dxx * dxx));
            const float4 q = s.astage[ids & 127u];
            const float lx = q.x + dxx, ly = q.y + dyy, lz = q.z + dzz;
            const float dot = __builtin_fmaf(dzz, lz, __builtin_fmaf(dyy, ly, dxx * lx));
            const float ll = __builtin_fmaf(lz, lz, __builtin_fmaf(ly, ly, lx * lx));
            pi2 = (dot * dot) * __builtin_amdgcn_rcpf(ll);
            sp2 = fmaxf(d2 - pi2, 0.0f);
        }
        // beyond a table's top band end the pair is certainly out of range
        const bool inr = (sp2 < k.vmax1) & (pi2 < k.vmax2);
        const float sp2c = inr ? sp2 : 0.0f;
        const float pi2c = inr ? pi2 : 0.0f;
        const uint32_t e1 = lut_entry(s.lut1, k.scale1, sp2c);
        const uint32_t e2 = lut_entry(s.lut2, k.scale2, pi2c);
        int b1 = lut_clean_bin(e1), b2 = lut_clean_bin(e2);
        const bool hot1 = (e1 & 0x8000u) != 0u, hot2 = (e2 & 0x8000u) != 0u;
        if (__builtin_amdgcn_ballot_w64(hot1 | hot2)) {
            if (hot1) b1 = lut_hot_bin(s.band1, k.n1, e1, sp2c, amb);
            if (hot2) b2 = lut_hot_bin(s.band2, k.n2, e2, pi2c, amb);
        }
        amb = amb & inr;
        flat = (inr & (b1 >= 0) & (b2 >= 0)) ? (int)__umul24((uint32_t)b1, (uint32_t)k.n2) + b2 : -1;
    }
    amb = amb & valid;
    if (valid & !amb & (flat >= 0)) {
        atomicAdd(&hist_l[flat], 1u);
        if (W) add_weight(s, flat, s.qw[base + lane], k.wscale);
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(amb);
    if (m) {
        const int pos = c.rcount + (int)lane_prefix(m);
        if (amb) {
            uint32_t* r = s.rb + (size_t)pos * 3;
            r[0] = c.a_begin + (ids & 127u);
            r[1] = c.b_begin + (ids >> 7);
            r[2] = c.it;
        }
        c.rcount += (int)__popcll(m);
        if (c.rcount >= 64) {
            wave_sync_lds();
            process_rechecks<KIND, LOS, W>(a, s, c.rcount - 64, 64, lane, c.nrechk);
            wave_sync_lds();
            c.rcount -= 64;
        }
    }
}

template <int KIND, int LOS, bool AUTO, bool W, int P>
__global__ __launch_bounds__(CT_MAX) void k_count(const CountArgs* argp) {
    ArgsRef a = *(const CountArgs FCFC_CONST*)argp;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    Smem s;
    s.lut1 = (const uint16_t*)(smem + a.off_lut1);
    s.lut2 = (const uint16_t*)(smem + a.off_lut2);
    s.band1 = (const float*)(smem + a.off_band1);
    s.band2 = (const float*)(smem + a.off_band2);
    s.hist = (uint32_t*)(smem + a.off_hist);
    s.wlo = (unsigned long long*)(smem + a.off_whist);
    s.whi = s.wlo + a.nbins;
    s.q = (float4*)(smem + a.off_q) + (size_t)wave * (QCAP + 1);
    s.qw = (double*)(smem + a.off_qw) + (size_t)wave * (QCAP + 1);
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
        float* b1 = (float*)(smem + a.off_band1);
        for (int i = tid; i < 2 * (a.n1 + 1); i += nthr) b1[i] = a.band1[i];
        if (KIND == FCFC_BIN_SPERP_PI) {
            float* b2 = (float*)(smem + a.off_band2);
            for (int i = tid; i < 2 * (a.n2 + 1); i += nthr) b2[i] = a.band2[i];
        }
        for (int i = tid; i < a.nbins * a.copies; i += nthr) s.hist[i] = 0u;
        if (W)
            for (int i = tid; i < 2 * a.nbins; i += nthr) s.wlo[i] = 0ull;
        if (tid == 0) s.misc[0] = 0ull;
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
    k.tolA = a.tolA;
    k.tolB = a.tolB;
    k.tolC = a.tolC;
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
    const uint32_t nitems = __builtin_amdgcn_readfirstlane(*a.nitems_dev);
    const float far = 1.0e18f;

    // Items are pulled dynamically; the index of the item after next and the
    // inputs (item record, A points, B cell offsets) of the next item are
    // fetched while the current one is processed.
    struct ItemIn {
        Item item;
        float4 av[P];
        float4 aabs[P];
        double aw[P];
        uint32_t csv;  // lane t: start of B cell xw0 + t of the item's row
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
            if (W) in.aw[p] = (i < acnt) ? a.wA[a_begin + i] : 0.0;
        }
        const int xb0 = (int)(int16_t)(in.item.acnt_xb0 >> 16);
        const int sxi = (int)((in.item.meta >> 16) & 3u) - 1;
        const int xw0 = xb0 - sxi * a.nx;
        const int cx = min(xw0 + lane, a.nx);
        in.csv = a.csB[in.item.b_rowcell + (uint32_t)cx];
    };

    unsigned long long wave_pairs = 0;  // pairs claimed since this wave last emptied the histogram
    uint32_t cur_it = 0, nxt_it = 0;
    if (lane == 0) {
        cur_it = atomicAdd(a.cursor, 1u);
        nxt_it = atomicAdd(a.cursor, 1u);
    }
    cur_it = __builtin_amdgcn_readfirstlane(cur_it);
    nxt_it = __builtin_amdgcn_readfirstlane(nxt_it);
    ItemIn cur, nxt;
    if (cur_it < nitems) load_in(cur_it, cur);
    while (cur_it < nitems) {
        uint32_t nn = 0;
        if (lane == 0) nn = atomicAdd(a.cursor, 1u);
        if (nxt_it < nitems) load_in(nxt_it, nxt);
        const uint32_t it = cur_it;
        unsigned long long t0 = 0;
        if (a.times && lane == 0) t0 = wall_clock64();
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
        // u32 overflow guard of the LDS histogram: every wave empties it (atomic
        // exchange) after claiming 2^26 pairs, so it never holds 16 * (2^26 + item)
        // < 2^31 increments
        wave_pairs += pairs;
        if (wave_pairs >= FLUSH_PAIRS) {
            wave_pairs = 0;
            for (int b = lane; b < a.nbins * a.copies; b += 64) {
                uint32_t v = atomicExch(&s.hist[b], 0u);
                if (v) atomicAdd(&a.out_counts[b % a.nbins], (unsigned long long)v);
            }
            if (W) {
                for (int b = lane; b < a.nbins; b += 64) {
                    unsigned long long lo = atomicExch(&s.wlo[b], 0ull);
                    unsigned long long hi = atomicExch(&s.whi[b], 0ull);
                    __int128 v = ((__int128)(long long)hi << 32) + (__int128)lo;
                    unsigned long long vlo = (unsigned long long)v;
                    unsigned long long vhi = (unsigned long long)(v >> 64);
                    unsigned long long o = atomicAdd(&a.out_w[2 * b], vlo);
                    if (o + vlo < o) vhi += 1ull;
                    if (vhi) atomicAdd(&a.out_w[2 * b + 1], vhi);
                }
            }
        }
        const float Dy = (float)idy * k.side32;
        const float Dz = (float)idz * k.side32;
        float ax[P], ay[P], az[P];
        double wa[P];
        int acx[P];
        uint32_t aidx[P], ids_lane[P];
#pragma unroll
        for (int p = 0; p < P; p++) {
            const uint32_t i = (uint32_t)(lane + 64 * p);
            aidx[p] = a_begin + i;
            ids_lane[p] = i;
            const float4 v = cur.av[p];
            ax[p] = v.x;
            ay[p] = v.y - Dy;
            az[p] = v.z - Dz;
            acx[p] = __float_as_int(v.w);
            if (LOS == FCFC_LOS_MIDPOINT && KIND != FCFC_BIN_S) {
                const float4 q = cur.aabs[p];
                s.astage[i] = make_float4(2.0f * q.x, 2.0f * q.y, 2.0f * q.z, 0.f);
            }
            if (W) wa[p] = cur.aw[p];
        }
        int qn = 0;
        int xu = xb0;
        int xw = xb0 - sxi * a.nx;
        int t = 0;
        uint32_t j = b_begin;
        while (j < b_end && xw < a.nx) {
            uint32_t cell_end = (t + 1 < 64) ? __builtin_amdgcn_readlane(cur.csv, t + 1)
                                             : ldc_u32(a.csB, item.b_rowcell + (uint32_t)xw + 1u);
            cell_end = cell_end < b_end ? cell_end : b_end;
            if (cell_end > j) {
                float axx[P];
#pragma unroll
                for (int p = 0; p < P; p++) axx[p] = ax[p] - (float)(xu - acx[p]) * k.side32;
                auto cell_loop = [&](auto mask_tag) __attribute__((always_inline)) {
                    constexpr bool MASK = decltype(mask_tag)::value;
                    float4 nb = ldc_f4(a.posB, j);
                    double nw = W ? ldc_f64(a.wB, j) : 0.0;
                    for (; j < cell_end; j++) {
                        const float4 b = nb;
                        const double wb = nw;
                        const uint32_t jbits = (j - b_begin) << 7;
                        // prefetch the next B point (arrays carry padding past the last point)
                        nb = ldc_f4(a.posB, j + 1);
                        if (W) nw = ldc_f64(a.wB, j + 1);
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
                            // every lane writes; lanes out of range write the dump entry QCAP
                            const int slot = in ? qn + (int)lane_prefix(m) : QCAP;
                            s.q[slot] = make_float4(v1, v2, v3, __uint_as_float(jbits | ids_lane[p]));
                            if (W) s.qw[slot] = wa[p] * wb;
                            qn += (int)__popcll(m);
                        }
                        while (qn >= 64) {
                            wave_sync_lds();
                            bin_queue<KIND, LOS, W>(a, k, s, hist_l, qn - 64, 64, lane, c);
                            wave_sync_lds();
                            qn -= 64;
                        }
                    }
                };
                if (samerow)
                    cell_loop(std::integral_constant<bool, true>());
                else
                    cell_loop(std::integral_constant<bool, false>());
                j = cell_end;
            }
            xw++;
            xu++;
            t++;
        }
        if (qn > 0) {
            wave_sync_lds();
            bin_queue<KIND, LOS, W>(a, k, s, hist_l, 0, qn, lane, c);
            wave_sync_lds();
        }
        if (a.times && lane == 0) {
            unsigned long long t1 = wall_clock64();
            a.times[it] = (uint32_t)min<unsigned long long>(t1 - t0, 0xffffffffull);
        }
        cur = nxt;
        cur_it = nxt_it;
        nxt_it = __builtin_amdgcn_readfirstlane(nn);
    }
    if (c.rcount > 0) {
        wave_sync_lds();
        process_rechecks<KIND, LOS, W>(a, s, 0, c.rcount, lane, c.nrechk);
    }
    if (lane == 0 && a.stats) {
        atomicAdd(&a.stats[0], ncand);
        atomicAdd(&a.stats[1], c.nrechk);
    }
    __syncthreads();
    for (int b = tid; b < a.nbins; b += nthr) {
        uint32_t cnt = 0;
        for (int r = 0; r < a.copies; r++) cnt += s.hist[r * a.nbins + b];
        if (cnt) atomicAdd(&a.out_counts[b], (unsigned long long)cnt);
        if (W) {
            unsigned long long lo = s.wlo[b], hi = s.whi[b];
            if (lo | hi) {
                __int128 v = ((__int128)(long long)hi << 32) + (__int128)lo;
                unsigned long long vlo = (unsigned long long)v;
                unsigned long long vhi = (unsigned long long)(v >> 64);
                unsigned long long o = atomicAdd(&a.out_w[2 * b], vlo);
                if (o + vlo < o) vhi += 1ull;
                if (vhi) atomicAdd(&a.out_w[2 * b + 1], vhi);
            }
        }
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

template <int KIND, int LOS, bool AUTO, bool W>
static CountKernel pick_p(int P) {
    if (P == 1) return k_count<KIND, LOS, AUTO, W, 1>;
    return k_count<KIND, LOS, AUTO, W, 2>;
}
template <int KIND, int LOS>
static CountKernel pick_aw(bool is_auto, bool w, int P) {
    if (is_auto) return w ? pick_p<KIND, LOS, true, true>(P) : pick_p<KIND, LOS, true, false>(P);
    return w ? pick_p<KIND, LOS, false, true>(P) : pick_p<KIND, LOS, false, false>(P);
}
static CountKernel pick_kernel(int kind, int los, bool is_auto, bool w, int P) {
    if (kind == FCFC_BIN_S) return pick_aw<FCFC_BIN_S, FCFC_LOS_Z>(is_auto, w, P);
    if (kind == FCFC_BIN_S_MU)
        return los == FCFC_LOS_Z ? pick_aw<FCFC_BIN_S_MU, FCFC_LOS_Z>(is_auto, w, P)
                                 : pick_aw<FCFC_BIN_S_MU, FCFC_LOS_MIDPOINT>(is_auto, w, P);
    return los == FCFC_LOS_Z ? pick_aw<FCFC_BIN_SPERP_PI, FCFC_LOS_Z>(is_auto, w, P)
                             : pick_aw<FCFC_BIN_SPERP_PI, FCFC_LOS_MIDPOINT>(is_auto, w, P);
}

static int al16(int b) { return (b + 15) & ~15; }

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct DevTables {
    char* base = nullptr;
    uint16_t* lut1;
    uint16_t* lut2;
    float* band1;
    float* band2;
    double* E1;
    double* E2;
    int4* srows;
};

fcfc_status count_pairs(Plan* p, Cells* c1, Cells* c2, int64_t* d_counts, double* d_wcounts, hipStream_t st) {
    const bool is_auto = (c2 == nullptr);
    Cells* cb = is_auto ? c1 : c2;
    const bool weighted = d_wcounts != nullptr;
    const Grid& g = p->grid;
    // ---- weights: common fixed-point scale 2^S making every product an integer
    int S = 0;
    if (weighted) {
        if (!c1->weighted || !cb->weighted) {
            set_error("count_pairs: weighted counts need weights in both cell sets");
            return FCFC_EINVAL;
        }
        double wmin = std::min(c1->wmin, cb->wmin), wmax = std::max(c1->wmax, cb->wmax);
        (void)wmin;
        if (c1->wmin > 0 && cb->wmin > 0) {
            double pmin = c1->wmin * cb->wmin;
            int e;
            frexp(pmin, &e);
            S = 53 - e;
            double pmax = c1->wmax * cb->wmax;
            if (!(ldexp(pmax, S) < ldexp(1.0, 62))) {
                set_error("count_pairs: weight dynamic range too wide for exact accumulation "
                          "(max/min pair weight %.3g)", pmax / pmin);
                return FCFC_ERANGE;
            }
        }
        (void)wmax;
    }
    // ---- tuning
    int T = p->tune.tile_points == 64 ? 64 : 128;
    int P = T / 64;
    int seg = p->tune.seg_cells > 0 ? std::min(32, p->tune.seg_cells) : 0;
    if (seg == 0) {
        double ppc = (double)c1->n / std::max<int64_t>(1, g.ncell());
        seg = (int)std::max(1.0, std::min(16.0, floor((double)T / std::max(ppc, 1e-9))));
        if (ppc >= T / 2) seg = 1;
    }
    int bchunk = p->tune.b_chunk >= 256 ? p->tune.b_chunk : 16384;
    int copies = (p->tune.hist_copies == 2 || p->tune.hist_copies == 4) ? p->tune.hist_copies : 1;
    int order = p->tune.order;

    std::vector<int4> rows;
    int nrows = stencil_rows(p, is_auto, rows);
    const Lut1D& L1 = p->lut1;
    const Lut1D& L2 = p->lut2;
    const bool two = (p->kind == FCFC_BIN_SPERP_PI);

    // ---- LDS layout
    CountArgs a;
    memset(&a, 0, sizeof(a));
    a.nlut1 = (int)L1.tab.size();
    a.nlut2 = two ? (int)L2.tab.size() : 0;
    a.copies = copies;
    int off = 0;
    a.off_lut1 = off;
    off += al16(a.nlut1 * 2 + 4);
    a.off_lut2 = off;
    off += al16(a.nlut2 * 2 + 4);
    a.off_band1 = off;
    off += al16(2 * (p->n1 + 1) * 4);
    a.off_band2 = off;
    off += al16(two ? 2 * (p->n2 + 1) * 4 : 0);
    a.off_hist = off;
    off += al16(p->nbins * 4 * copies);
    a.off_whist = off;
    off += weighted ? al16(p->nbins * 16) : 0;
    const int shared_bytes = off;
    const bool mid = (p->los == FCFC_LOS_MIDPOINT && p->kind != FCFC_BIN_S);
    const int per_wave = (QCAP + 1) * 16 + (weighted ? (QCAP + 1) * 8 : 0) + RB_CAP * 12 + (mid ? ASTAGE * 16 : 0);
    int dev = 0, maxlds = 65536;
    FCFC_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) maxlds = 65536;
    // as many waves per workgroup (up to 16, one workgroup per CU) as the LDS allows
    int waves = 16;
    while (waves > 1 && shared_bytes + waves * per_wave + 16 > maxlds) waves--;
    if (shared_bytes + waves * per_wave + 16 > maxlds) {
        set_error("count_pairs: %d bytes of LDS needed (tables + histogram), device allows %d",
                  shared_bytes + per_wave + 16, maxlds);
        return FCFC_ERANGE;
    }
    const int CT = waves * 64;
    a.off_q = off;
    off += waves * (QCAP + 1) * 16;
    a.off_qw = off;
    off += weighted ? waves * (QCAP + 1) * 8 : 0;
    a.off_rb = off;
    off += waves * RB_CAP * 12;
    a.off_astage = off;
    off += mid ? waves * ASTAGE * 16 : 0;
    a.off_misc = off;
    off += 16;
    a.lds_bytes = off;

    // ---- small tables to the device (one block)
    size_t tb_l1 = (size_t)al16(a.nlut1 * 2 + 4), tb_l2 = (size_t)al16(a.nlut2 * 2 + 4);
    size_t tb_b1 = (size_t)al16(2 * (p->n1 + 1) * 4), tb_b2 = (size_t)al16(2 * (p->n2 + 1) * 4);
    size_t tb_e1 = (size_t)al16((p->n1 + 1) * 8), tb_e2 = (size_t)al16((p->n2 + 1) * 8);
    size_t tb_rows = (size_t)al16(std::max(1, nrows) * 16);
    size_t tb_total = tb_l1 + tb_l2 + tb_b1 + tb_b2 + tb_e1 + tb_e2 + tb_rows;
    std::vector<char> htab(tb_total, 0);
    {
        size_t o = 0;
        memcpy(&htab[o], L1.tab.data(), L1.tab.size() * 2);
        o += tb_l1;
        if (two) memcpy(&htab[o], L2.tab.data(), L2.tab.size() * 2);
        o += tb_l2;
        memcpy(&htab[o], L1.lo.data(), (p->n1 + 1) * 4);
        memcpy(&htab[o + (p->n1 + 1) * 4], L1.hi.data(), (p->n1 + 1) * 4);
        o += tb_b1;
        if (two) {
            memcpy(&htab[o], L2.lo.data(), (p->n2 + 1) * 4);
            memcpy(&htab[o + (p->n2 + 1) * 4], L2.hi.data(), (p->n2 + 1) * 4);
        }
        o += tb_b2;
        memcpy(&htab[o], L1.E.data(), (p->n1 + 1) * 8);
        o += tb_e1;
        if (two) memcpy(&htab[o], L2.E.data(), (p->n2 + 1) * 8);
        o += tb_e2;
        if (nrows) memcpy(&htab[o], rows.data(), nrows * 16);
    }

    // ---- work-list sizes
    WLArgs w;
    w.nx = g.nx;
    w.ny = g.ny;
    w.nz = g.nz;
    w.seg = seg;
    w.tile = T;
    w.bchunk = bchunk;
    w.nrows = std::max(1, nrows);
    w.periodic = g.L > 0;
    w.is_auto = is_auto;
    int64_t nseg = (int64_t)((g.nx + seg - 1) / seg) * g.ny * g.nz;
    int64_t tiles_cap = nseg + c1->n / T + 1;
    if (tiles_cap > 0xffffffffLL / std::max(1, nrows)) {
        set_error("count_pairs: work list too large");
        return FCFC_ERANGE;
    }
    w.tiles_cap = (uint32_t)tiles_cap;
    int64_t npair_tr = tiles_cap * w.nrows;

    // scratch 1: tables, tiles, tile counts/offsets, item counts/offsets, counters
    size_t s_tab = (tb_total + 255) & ~(size_t)255;
    size_t s_tc = ((size_t)nseg * 4 + 255) & ~(size_t)255;
    size_t s_tiles = ((size_t)tiles_cap * sizeof(Tile) + 255) & ~(size_t)255;
    size_t s_ic = ((size_t)npair_tr * 4 + 255) & ~(size_t)255;
    size_t s_scan = (std::max(scan_scratch_bytes(nseg), scan_scratch_bytes(npair_tr)) + 255) & ~(size_t)255;
    size_t s_ctr = 256;
    size_t s_args = (sizeof(CountArgs) + 255) & ~(size_t)255;
    size_t s_acc = weighted ? (((size_t)p->nbins * 16 + 255) & ~(size_t)255) : 0;
    size_t s1 = s_tab + 2 * s_tc + s_tiles + 2 * s_ic + s_scan + s_ctr + s_args + s_acc;
    char* scr = nullptr;
    if (hipMallocAsync((void**)&scr, s1, st) != hipSuccess) {
        set_error("count_pairs: cannot allocate %zu bytes of scratch", s1);
        return FCFC_ENOMEM;
    }
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

    p->host_stage.swap(htab);
    FCFC_HIP(hipMemcpyAsync(tab, p->host_stage.data(), tb_total, hipMemcpyHostToDevice, st));
    DevTables dt;
    {
        char* o = tab;
        dt.lut1 = (uint16_t*)o;
        o += tb_l1;
        dt.lut2 = (uint16_t*)o;
        o += tb_l2;
        dt.band1 = (float*)o;
        o += tb_b1;
        dt.band2 = (float*)o;
        o += tb_b2;
        dt.E1 = (double*)o;
        o += tb_e1;
        dt.E2 = (double*)o;
        o += tb_e2;
        dt.srows = (int4*)o;
    }
    fill_u32(ctr, 0u, 64, st);
    // tiles
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st, c1->cell_start, w, tcount);
    scan_exclusive_u32(tcount, toff, nseg, &ctr[0], scan_scr, st);
    hipLaunchKernelGGL(k_tile_write, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st, c1->cell_start, c1->pos32,
                       w, toff, tiles);
    // items: count, scan, size on the host
    hipLaunchKernelGGL(k_item_count, dim3((unsigned)((npair_tr + 255) / 256)), dim3(256), 0, st, tiles, &ctr[0],
                       dt.srows, cb->cell_start, w, icount);
    scan_exclusive_u32(icount, ioff, npair_tr, &ctr[1], scan_scr, st);
    uint32_t hctr[2] = {0, 0};
    FCFC_HIP(hipMemcpyAsync(hctr, ctr, 8, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipStreamSynchronize(st));
    uint32_t nitems = hctr[1];
    size_t s_items = ((size_t)std::max<uint32_t>(nitems, 1) * sizeof(Item) + 255) & ~(size_t)255;
    size_t s_sort = order ? (((size_t)std::max<uint32_t>(nitems, 1) * 4 + 255) & ~(size_t)255) : 0;
    size_t s_rs = order ? ((radix_scratch_bytes(nitems) + 255) & ~(size_t)255) : 0;
    size_t s_times = p->tune.record_timing ? (((size_t)std::max<uint32_t>(nitems, 1) * 4 + 255) & ~(size_t)255) : 0;
    size_t s2 = 2 * s_items + 4 * s_sort + s_rs + s_times;
    char* scr2 = nullptr;
    if (hipMallocAsync((void**)&scr2, s2, st) != hipSuccess) {
        (void)hipFreeAsync(scr, st);
        set_error("count_pairs: cannot allocate %zu bytes for %u work items", s2, nitems);
        return FCFC_ENOMEM;
    }
    Item* items = (Item*)scr2;
    Item* items2 = (Item*)(scr2 + s_items);
    hipLaunchKernelGGL(k_item_write, dim3((unsigned)((npair_tr + 255) / 256)), dim3(256), 0, st, tiles, &ctr[0],
                       dt.srows, cb->cell_start, w, ioff, items, nitems);
    Item* run_items = items;
    if (order && nitems > 1) {
        uint32_t* k0 = (uint32_t*)(scr2 + 2 * s_items);
        uint32_t* v0 = (uint32_t*)(scr2 + 2 * s_items + s_sort);
        uint32_t* k1 = (uint32_t*)(scr2 + 2 * s_items + 2 * s_sort);
        uint32_t* v1 = (uint32_t*)(scr2 + 2 * s_items + 3 * s_sort);
        void* rs = scr2 + 2 * s_items + 4 * s_sort;
        hipLaunchKernelGGL(k_item_keys, dim3((nitems + 255) / 256), dim3(256), 0, st, items, &ctr[1], nitems, k0, v0);
        radix_sort_pairs(&k0, &v0, &k1, &v1, nitems, 8, rs, st);
        hipLaunchKernelGGL(k_item_permute, dim3((nitems + 255) / 256), dim3(256), 0, st, items, v0, &ctr[1], nitems,
                           items2);
        run_items = items2;
    }
    uint32_t* times = p->tune.record_timing ? (uint32_t*)(scr2 + 2 * s_items + 4 * s_sort + s_rs) : nullptr;

    // outputs
    fill_u64((uint64_t*)d_counts, 0ull, p->nbins, st);
    if (weighted) fill_u64((uint64_t*)wacc, 0ull, 2 * (int64_t)p->nbins, st);
    if (!p->stats_dev) {
        FCFC_HIP(hipMalloc(&p->stats_dev, 64));
        FCFC_HIP(hipEventCreate(&p->ev0));
        FCFC_HIP(hipEventCreate(&p->ev1));
    }
    fill_u64((uint64_t*)p->stats_dev, 0ull, 8, st);

    a.posA = c1->pos32;
    a.absA = c1->abs32;
    a.p64A = c1->pos64;
    a.wA = c1->w;
    a.posB = cb->pos32;
    a.p64B = cb->pos64;
    a.wB = cb->w;
    a.csB = cb->cell_start;
    a.items = run_items;
    a.nitems_dev = &ctr[1];
    a.cursor = &ctr[2];
    a.lut1 = dt.lut1;
    a.lut2 = dt.lut2;
    a.band1 = dt.band1;
    a.band2 = dt.band2;
    a.E1 = dt.E1;
    a.E2 = dt.E2;
    a.out_counts = (unsigned long long*)d_counts;
    a.out_w = weighted ? wacc : nullptr;
    a.stats = (unsigned long long*)p->stats_dev;
    a.times = times;
    a.scale1 = L1.scale;
    a.scale2 = two ? L2.scale : 1.f;
    a.vmax1 = L1.vmax;
    a.vmax2 = two ? L2.vmax : 0.f;
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
    a.wscale = ldexp(1.0, S);

    CountKernel kern = pick_kernel(p->kind, p->los, is_auto, weighted, P);
    FCFC_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes));
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, CT, a.lds_bytes) != hipSuccess || occ < 1)
        occ = 1;
    int cus = device_cu_count();
    int64_t nblk = (int64_t)cus * occ;
    int64_t need = ((int64_t)nitems + waves - 1) / waves;
    if (nblk > need) nblk = std::max<int64_t>(1, need);
    FCFC_HIP(hipEventRecord(p->ev0, st));
    p->host_args.resize(sizeof(CountArgs));
    memcpy(p->host_args.data(), &a, sizeof(CountArgs));
    FCFC_HIP(hipMemcpyAsync(args_dev, p->host_args.data(), sizeof(CountArgs), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(CT), (size_t)a.lds_bytes, st, (const CountArgs*)args_dev);
    FCFC_HIP(hipGetLastError());
    FCFC_HIP(hipEventRecord(p->ev1, st));
    if (weighted)
        hipLaunchKernelGGL(k_finalize_w, dim3((p->nbins + 255) / 256), dim3(256), 0, st, wacc, p->nbins, S, d_wcounts);
    if (times) {
        // keep the per-item times and features for the scheduler: copy to plan-owned buffer
        if (p->timing_dev) (void)hipFree(p->timing_dev);
        p->timing_dev = nullptr;
        size_t tb = (size_t)nitems * (4 + sizeof(Item));
        if (hipMalloc(&p->timing_dev, std::max<size_t>(tb, 256)) == hipSuccess) {
            FCFC_HIP(hipMemcpyAsync(p->timing_dev, times, (size_t)nitems * 4, hipMemcpyDeviceToDevice, st));
            FCFC_HIP(hipMemcpyAsync((char*)p->timing_dev + (size_t)nitems * 4, run_items, (size_t)nitems * sizeof(Item),
                                    hipMemcpyDeviceToDevice, st));
            p->timing_n = nitems;
        }
    }
    (void)hipFreeAsync(scr2, st);
    (void)hipFreeAsync(scr, st);
    p->last_stream = st;
    p->have_stats = true;
    p->stats.items = nitems;
    p->stats.cells = g.ncell();
    p->stats.grid[0] = g.nx;
    p->stats.grid[1] = g.ny;
    p->stats.grid[2] = g.nz;
    p->stats.cells_per_rmax = g.k;
    p->stats.cell_side = g.side;
    p->stats.wg_per_cu = occ;
    p->last_pts = (int)P;
    return FCFC_OK;
}

}  // namespace fcfc
