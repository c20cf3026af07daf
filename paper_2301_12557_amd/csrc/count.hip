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

constexpr int CT = 256;             // threads per workgroup
constexpr int CWAVES = CT / 64;
constexpr int RB_CAP = 128;         // recheck entries per wave
constexpr uint64_t FLUSH_PAIRS = 1ull << 30;
constexpr int BG = 4;               // B points per scalar load group (arrays are padded by BG-1)

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
    int off_lut1, off_lut2, off_band1, off_band2, off_hist, off_whist, off_rb, off_misc, lds_bytes;
};

struct Smem {
    const uint16_t* lut1;
    const uint16_t* lut2;
    const float* band1;
    const float* band2;
    uint32_t* hist;
    unsigned long long* wlo;
    unsigned long long* whi;
    uint32_t* rb;
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
__device__ int exact_bin(const CountArgs& a, const double* pa, const double* pb, int sx, int sy, int sz) {
    double ax = pa[0], ay = pa[1], az = pa[2];
    double bx = pb[0], by = pb[1], bz = pb[2];
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
__device__ inline int lut_bin(const uint16_t* __restrict__ lut, const float* __restrict__ band, int n,
                              float scale, float v, bool& amb) {
    uint32_t e = lut[(uint32_t)(v * scale)];
    if (!(e & 0x8000u)) return (e == 0x7fffu) ? -1 : (int)e;
    // hot entry: count edges certainly <= v starting at the first banded edge
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

__device__ inline void add_weight(const Smem& s, int flat, double p, double wscale) {
    long long t = (long long)(p * wscale);
    unsigned long long lo = (unsigned long long)(uint32_t)(t & 0xffffffffll);
    unsigned long long hi = (unsigned long long)(t >> 32);
    atomicAdd(&s.wlo[flat], lo);
    atomicAdd(&s.whi[flat], hi);
}

// Re-evaluate `cnt` queued pairs (entries base .. base+cnt-1) in FP64.
template <int KIND, int LOS, bool W>
__device__ void process_rechecks(const CountArgs& a, const Smem& s, int base, int cnt, int lane,
                                 unsigned long long& nrechk) {
    if (lane < cnt) {
        const uint32_t* e = s.rb + (size_t)(base + lane) * 3;
        uint32_t ia = e[0], ib = e[1], it = e[2];
        uint32_t meta = a.items[it].meta;
        int sx = (int)((meta >> 16) & 3u) - 1;
        int sy = (int)((meta >> 18) & 3u) - 1;
        int sz = (int)((meta >> 20) & 3u) - 1;
        double pa[3] = {a.p64A[3 * (size_t)ia], a.p64A[3 * (size_t)ia + 1], a.p64A[3 * (size_t)ia + 2]};
        double pb[3] = {a.p64B[3 * (size_t)ib], a.p64B[3 * (size_t)ib + 1], a.p64B[3 * (size_t)ib + 2]};
        int flat = exact_bin<KIND, LOS>(a, pa, pb, sx, sy, sz);
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

template <int KIND, int LOS, bool AUTO, bool W, int P>
__global__ __launch_bounds__(CT) void k_count(const CountArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    Smem s;
    s.lut1 = (const uint16_t*)(smem + a.off_lut1);
    s.lut2 = (const uint16_t*)(smem + a.off_lut2);
    s.band1 = (const float*)(smem + a.off_band1);
    s.band2 = (const float*)(smem + a.off_band2);
    s.hist = (uint32_t*)(smem + a.off_hist);
    s.wlo = (unsigned long long*)(smem + a.off_whist);
    s.whi = s.wlo + a.nbins;
    s.rb = (uint32_t*)(smem + a.off_rb);
    s.misc = (unsigned long long*)(smem + a.off_misc);

    const int tid = threadIdx.x;
    // stage tables, clear histograms
    {
        uint32_t* d = (uint32_t*)(smem + a.off_lut1);
        const uint32_t* src = (const uint32_t*)a.lut1;
        for (int i = tid; i < (a.nlut1 + 1) / 2; i += CT) d[i] = src[i];
        if (KIND == FCFC_BIN_SPERP_PI) {
            d = (uint32_t*)(smem + a.off_lut2);
            src = (const uint32_t*)a.lut2;
            for (int i = tid; i < (a.nlut2 + 1) / 2; i += CT) d[i] = src[i];
        }
        float* b1 = (float*)(smem + a.off_band1);
        for (int i = tid; i < 2 * (a.n1 + 1); i += CT) b1[i] = a.band1[i];
        if (KIND == FCFC_BIN_SPERP_PI) {
            float* b2 = (float*)(smem + a.off_band2);
            for (int i = tid; i < 2 * (a.n2 + 1); i += CT) b2[i] = a.band2[i];
        }
        for (int i = tid; i < a.nbins * a.copies; i += CT) s.hist[i] = 0u;
        if (W)
            for (int i = tid; i < 2 * a.nbins; i += CT) s.wlo[i] = 0ull;
        if (tid == 0) s.misc[0] = 0ull;
    }
    __syncthreads();

    const int lane = tid & 63;
    const int wave = tid >> 6;
    const uint64_t lanemask_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    Smem sw = s;
    sw.rb = s.rb + (size_t)wave * RB_CAP * 3;
    uint32_t* hist_l = s.hist + (size_t)(lane % a.copies) * a.nbins;
    int rcount = 0;
    unsigned long long ncand = 0, nrechk = 0;
    const uint32_t nitems = __builtin_amdgcn_readfirstlane(*a.nitems_dev);
    const float far = 1.0e18f;

    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(a.cursor, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= nitems) break;
        unsigned long long t0 = 0;
        if (a.times && lane == 0) t0 = wall_clock64();
        const Item item = ldc_item(a.items, it);
        const uint32_t a_begin = item.a_begin;
        const uint32_t acnt = item.acnt_xb0 & 0xffffu;
        const int xb0 = (int)(int16_t)(item.acnt_xb0 >> 16);
        const int idy = (int)(int8_t)(item.meta & 0xffu);
        const int idz = (int)(int8_t)((item.meta >> 8) & 0xffu);
        const int sxi = (int)((item.meta >> 16) & 3u) - 1;
        const bool samerow = AUTO && ((item.meta >> 24) & ITEM_SAMEROW);
        const uint32_t b_end = item.b_end;
        const uint64_t pairs = (uint64_t)acnt * (uint64_t)(b_end - item.b_begin);
        ncand += pairs;
        // u32 overflow guard of the LDS histogram: exchange it out every 2^30 claimed pairs
        {
            unsigned long long old = 0;
            if (lane == 0) old = atomicAdd(&s.misc[0], (unsigned long long)pairs);
            old = __shfl(old, 0);
            if ((old / FLUSH_PAIRS) != ((old + pairs) / FLUSH_PAIRS)) {
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
        }
        const float Dy = (float)idy * a.side32;
        const float Dz = (float)idz * a.side32;
        float ax[P], ay[P], az[P], lx2[P], ly2[P], lz2[P];
        double wa[P];
        int acx[P];
        uint32_t aidx[P];
#pragma unroll
        for (int p = 0; p < P; p++) {
            uint32_t i = (uint32_t)(lane + 64 * p);
            aidx[p] = a_begin + i;
            float4 v = make_float4(far, far, far, __int_as_float(0));
            if (i < acnt) v = a.posA[a_begin + i];
            ax[p] = v.x;
            ay[p] = v.y - Dy;
            az[p] = v.z - Dz;
            acx[p] = __float_as_int(v.w);
            if (LOS == FCFC_LOS_MIDPOINT && KIND != FCFC_BIN_S) {
                float4 q = make_float4(far, far, far, 0.f);
                if (i < acnt) q = a.absA[a_begin + i];
                lx2[p] = 2.0f * q.x;
                ly2[p] = 2.0f * q.y;
                lz2[p] = 2.0f * q.z;
            }
            if (W) wa[p] = (i < acnt) ? a.wA[a_begin + i] : 0.0;
        }
        int xu = xb0;
        int xw = xb0 - sxi * a.nx;
        uint32_t j = item.b_begin;
        const uint32_t rowcell = item.b_rowcell;
        while (j < b_end && xw < a.nx) {
            uint32_t cell_end = ldc_u32(a.csB, rowcell + (uint32_t)xw + 1u);
            cell_end = cell_end < b_end ? cell_end : b_end;
            if (cell_end > j) {
                float axx[P];
#pragma unroll
                for (int p = 0; p < P; p++) axx[p] = ax[p] - (float)(xu - acx[p]) * a.side32;
                for (; j < cell_end; j += BG) {
                    // a group of BG B points in one scalar load (arrays carry BG-1 points of padding)
                    float4 bg[BG];
                    double wg[BG];
#pragma unroll
                    for (int q = 0; q < BG; q++) {
                        bg[q] = ldc_f4(a.posB, j + q);
                        if (W) wg[q] = ldc_f64(a.wB, j + q);
                    }
#pragma unroll
                    for (int q = 0; q < BG; q++) {
                    if (q == 0 || j + q < cell_end) {
                    const uint32_t jb = j + q;
                    const float4 b = bg[q];
                    const double wb = W ? wg[q] : 0.0;
#pragma unroll
                    for (int p = 0; p < P; p++) {
                        const float dx = b.x - axx[p];
                        const float dy = b.y - ay[p];
                        const float dz = b.z - az[p];
                        bool amb = false;
                        int flat = -1;
                        bool in;
                        float d2 = 0.f, sp2 = 0.f, pi2 = 0.f;
                        if (KIND == FCFC_BIN_SPERP_PI && LOS == FCFC_LOS_Z) {
                            sp2 = __builtin_fmaf(dy, dy, dx * dx);
                            pi2 = dz * dz;
                            in = (sp2 < a.vmax1) && (pi2 < a.vmax2);
                        } else {
                            d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                            in = d2 < a.r2prune;
                        }
                        if (samerow) in = in && (jb > aidx[p]);
                        if (in) {
                            if (KIND == FCFC_BIN_S) {
                                flat = lut_bin(s.lut1, s.band1, a.n1, a.scale1, d2, amb);
                            } else if (KIND == FCFC_BIN_S_MU) {
                                int sb = lut_bin(s.lut1, s.band1, a.n1, a.scale1, d2, amb);
                                const float rs = __builtin_amdgcn_rsqf(d2);
                                float mun;
                                if (LOS == FCFC_LOS_Z) {
                                    mun = fabsf(dz) * (rs * a.mu_n);
                                } else {
                                    const float lx = lx2[p] + dx, ly = ly2[p] + dy, lz = lz2[p] + dz;
                                    const float dot = __builtin_fmaf(dz, lz, __builtin_fmaf(dy, ly, dx * lx));
                                    const float ll = __builtin_fmaf(lz, lz, __builtin_fmaf(ly, ly, lx * lx));
                                    mun = fabsf(dot) * (__builtin_amdgcn_rsqf(ll) * (rs * a.mu_n));
                                }
                                int mb = (int)mun;
                                mb = mb < a.n2 - 1 ? mb : a.n2 - 1;
                                const float cr = rintf(mun);
                                const float dist = fabsf(mun - cr);
                                const float tol = __builtin_fmaf(__builtin_fmaf(a.tolB, rs, a.tolA), rs, a.tolC);
                                amb = amb || ((dist < tol) && (cr >= 1.0f) && (cr <= a.mu_n - 1.0f)) ||
                                      (d2 < a.d2small);
                                flat = (sb >= 0) ? sb * a.n2 + mb : -1;
                            } else {
                                if (LOS == FCFC_LOS_MIDPOINT) {
                                    const float lx = lx2[p] + dx, ly = ly2[p] + dy, lz = lz2[p] + dz;
                                    const float dot = __builtin_fmaf(dz, lz, __builtin_fmaf(dy, ly, dx * lx));
                                    const float ll = __builtin_fmaf(lz, lz, __builtin_fmaf(ly, ly, lx * lx));
                                    pi2 = (dot * dot) * __builtin_amdgcn_rcpf(ll);
                                    sp2 = fmaxf(d2 - pi2, 0.0f);
                                }
                                // beyond a table's top band end the pair is certainly out of range
                                if (sp2 < a.vmax1 && pi2 < a.vmax2) {
                                    int b1 = lut_bin(s.lut1, s.band1, a.n1, a.scale1, sp2, amb);
                                    int b2 = lut_bin(s.lut2, s.band2, a.n2, a.scale2, pi2, amb);
                                    flat = (b1 >= 0 && b2 >= 0) ? b1 * a.n2 + b2 : -1;
                                }
                            }
                            if (!amb && flat >= 0) {
                                atomicAdd(&hist_l[flat], 1u);
                                if (W) add_weight(s, flat, wa[p] * wb, a.wscale);
                            }
                        }
                        // queue ambiguous pairs (wave-uniform bookkeeping)
                        const uint64_t m = __ballot(amb);
                        if (m) {
                            const int pos = rcount + (int)__popcll(m & lanemask_lt);
                            if (amb) {
                                uint32_t* e = sw.rb + (size_t)pos * 3;
                                e[0] = aidx[p];
                                e[1] = jb;
                                e[2] = it;
                            }
                            rcount += (int)__popcll(m);
                            if (rcount >= 64) {
                                wave_sync_lds();
                                process_rechecks<KIND, LOS, W>(a, sw, rcount - 64, 64, lane, nrechk);
                                wave_sync_lds();
                                rcount -= 64;
                            }
                        }
                    }
                    }
                    }
                }
                j = cell_end;
            }
            xw++;
            xu++;
        }
        if (a.times && lane == 0) {
            unsigned long long t1 = wall_clock64();
            a.times[it] = (uint32_t)min<unsigned long long>(t1 - t0, 0xffffffffull);
        }
    }
    if (rcount > 0) {
        wave_sync_lds();
        process_rechecks<KIND, LOS, W>(a, sw, 0, rcount, lane, nrechk);
    }
    if (lane == 0 && a.stats) {
        atomicAdd(&a.stats[0], ncand);
        atomicAdd(&a.stats[1], nrechk);
    }
    __syncthreads();
    unsigned long long tot = 0;
    for (int b = tid; b < a.nbins; b += CT) {
        uint32_t c = 0;
        for (int r = 0; r < a.copies; r++) c += s.hist[r * a.nbins + b];
        if (c) {
            atomicAdd(&a.out_counts[b], (unsigned long long)c);
            tot += c;
        }
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
    if (a.stats && tot) atomicAdd(&a.stats[2], tot);
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
typedef void (*CountKernel)(CountArgs);

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
    int seg = p->tune.seg_cells > 0 ? std::min(64, p->tune.seg_cells) : 0;
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
    a.off_rb = off;
    off += CWAVES * RB_CAP * 12;
    a.off_misc = off;
    off += 16;
    a.lds_bytes = off;
    int dev = 0, maxlds = 65536;
    FCFC_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) maxlds = 65536;
    if (a.lds_bytes > maxlds) {
        set_error("count_pairs: %d bytes of LDS needed (tables + histogram), device allows %d", a.lds_bytes, maxlds);
        return FCFC_ERANGE;
    }

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
    size_t s_acc = weighted ? (((size_t)p->nbins * 16 + 255) & ~(size_t)255) : 0;
    size_t s1 = s_tab + 2 * s_tc + s_tiles + 2 * s_ic + s_scan + s_ctr + s_acc;
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
    unsigned long long* wacc = (unsigned long long*)q;

    FCFC_HIP(hipMemcpyAsync(tab, htab.data(), tb_total, hipMemcpyHostToDevice, st));
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
        radix_sort_pairs(&k0, &v0, &k1, &v1, nitems, 32, rs, st);
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
    int64_t need = ((int64_t)nitems + CWAVES - 1) / CWAVES;
    if (nblk > need) nblk = std::max<int64_t>(1, need);
    FCFC_HIP(hipEventRecord(p->ev0, st));
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(CT), (size_t)a.lds_bytes, st, a);
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
