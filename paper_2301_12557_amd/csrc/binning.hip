// binning.hip -- the histogram update routine on its own (Sect. 3.2): squared
// separations handed over in FP64 are binned, one at a time, into int64
// counts with a look-up table over the squared edges (Sect. 3.2.3), FP32
// band ends around every edge and the FP64 squared edges.
//
// The bin of a value v is the i with E_i <= v < E_{i+1}; NaN, negative values
// and values at or above the top edge land in no bin.  Per value: one FP32
// conversion and the table entry from LDS.  An entry that meets an edge's
// band holds that edge k; the value is then placed against band k and the
// start of band k+1, read as one 16-byte LDS access, without a branch.  A
// value inside a band (or in an entry spanning several edges) takes the FP64
// binary search over the squared edges.  The bands cover the rounding of the
// value to FP32, so every decision taken in FP32 is the FP64 decision.
//
// The input is streamed once with 16-byte loads by a grid of one
// 1024-thread workgroup per CU.  Each workgroup counts into as many LDS
// histogram copies as fit (up to one per thread), laid out [bin][copy]: with
// 64 or more copies the 64 lanes of a wave never share an address.  At the
// end it merges them into the int64 counts with one global atomic per bin.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "binlut.h"
#include "internal.h"

namespace fcfc {

constexpr int BIN_THREADS = 1024;
// 16-byte loads per thread per step; with the two register sets of the
// pipelined loop, twice that many are in flight.  Measured on MI355X over
// 6.4e9 values (20 linear bins): 1 -> 7.7 ms, 2 -> 7.9, 3 -> 8.3, 4 -> 8.6,
// 8 -> 10.4; non-temporal loads 8.6 ms against 9.3 with plain loads (4).
constexpr int BIN_UNROLL = 1;
constexpr int64_t BIN_PER_GROUP = 1ll << 31;  // values per workgroup, so u32 counters cannot wrap

typedef double dbl2 __attribute__((ext_vector_type(2)));

struct BinArgs {
    const double* v;          // values
    int64_t n;
    int64_t head;             // values before the first 16-byte aligned pair (0 or 1)
    int64_t npair;            // aligned pairs after the head
    const uint4* tab;         // tables blob, laid out as the LDS prefix
    int tab_words;            // 16-byte words of the blob
    int nt, nb;               // table entries, bins
    int off_band, off_e, off_hist, off_tot, off_misc;
    float scale, vmax;
    int hbits;                // LDS histogram copies per workgroup: 1 << hbits
    unsigned long long* out;  // int64 counts, accumulated
    unsigned long long* stats;  // [0] values, [1] FP64 rechecks
};

struct BinSmem : BinTable {
    uint32_t* hist;
};

// Bin 2U values: every table read is issued before the first is used.  Hot
// entries (edge k0) are placed against (lo, hi) of band k0 and lo of band
// k0+1 for every lane at once; what that cannot decide (rare) is resolved
// under one branch.  Values in no bin go to the dump row nb, so the LDS adds
// need no branch.
template <int U>
__device__ __attribute__((always_inline)) inline void bin_values(const BinSmem& s, const double* x, uint32_t copy,
                                                                 int hbits, uint32_t& rechk) {
    float v[2 * U];
    int e[2 * U];
#pragma unroll
    for (int k = 0; k < 2 * U; k++) e[k] = bin_entry(s, x[k], v[k]);
    bool hot = false;
#pragma unroll
    for (int k = 0; k < 2 * U; k++) hot |= e[k] < -1;
    if (hot) {
        int k0[2 * U];
        bool slow = false;
#pragma unroll
        for (int k = 0; k < 2 * U; k++) {
            const bool h = e[k] < -1;
            k0[k] = h ? -2 - e[k] : 0;
            // below band k0: k0 edges at or below v; between bands k0 and
            // k0+1: k0+1 edges (bin k0, the dump row when k0 = nb)
            const int r = bin_near(s, k0[k], v[k]);
            if (h) e[k] = r;
            slow |= h && r == -2;
        }
        if (slow) {
#pragma unroll
            for (int k = 0; k < 2 * U; k++)
                if (e[k] == -2) e[k] = bin_resolve(s, k0[k], v[k], x[k], rechk);
        }
    }
#pragma unroll
    for (int k = 0; k < 2 * U; k++) {
        const uint32_t b = (uint32_t)e[k] < (uint32_t)s.nb ? (uint32_t)e[k] : (uint32_t)s.nb;
        atomicAdd(&s.hist[(b << hbits) + copy], 1u);
    }
}

__global__ __launch_bounds__(BIN_THREADS) void k_bin_squared(BinArgs a) {
    extern __shared__ __align__(16) char smem[];
    const uint32_t tid = threadIdx.x;
    // tables into LDS; histogram copies (with the dump row) and totals to zero
    {
        uint4* dst = (uint4*)smem;
        for (int i = tid; i < a.tab_words; i += BIN_THREADS) dst[i] = a.tab[i];
        uint32_t* z = (uint32_t*)(smem + a.off_hist);
        const int nz = (a.off_misc + 16 - a.off_hist) / 4;
        for (int i = tid; i < nz; i += BIN_THREADS) z[i] = 0u;
    }
    __syncthreads();
    BinSmem s;
    s.lut = (const int16_t*)smem;
    s.band = (const float2*)(smem + a.off_band);
    s.E = (const double*)(smem + a.off_e);
    s.hist = (uint32_t*)(smem + a.off_hist);
    s.scale = a.scale;
    s.vmax = a.vmax;
    s.nb = a.nb;
    const int hbits = a.hbits;
    const uint32_t copy = tid & ((1u << hbits) - 1u);
    uint32_t rechk = 0;

    const dbl2* __restrict__ v2 = (const dbl2*)(a.v + a.head);
    const int64_t stride = (int64_t)gridDim.x * BIN_THREADS;
    int64_t i = (int64_t)blockIdx.x * BIN_THREADS + tid;
    constexpr int U = BIN_UNROLL;
    if (i + (U - 1) * stride < a.npair) {
        // software pipelined over two register sets: one step's loads are in
        // flight while the other's values are binned (loads past the end are
        // clamped to the last pair and their values unused)
        const int64_t last = a.npair - 1;
        dbl2 q[U], r[U];
#pragma unroll
        for (int u = 0; u < U; u++) q[u] = __builtin_nontemporal_load(v2 + i + u * stride);
        for (;;) {
            int64_t nx = i + U * stride;
            bool more = nx + (U - 1) * stride < a.npair;
#pragma unroll
            for (int u = 0; u < U; u++) r[u] = __builtin_nontemporal_load(v2 + std::min(nx + u * stride, last));
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the binning
            {
                double x[2 * U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    x[2 * u] = q[u].x;
                    x[2 * u + 1] = q[u].y;
                }
                bin_values<U>(s, x, copy, hbits, rechk);
            }
            i = nx;
            if (!more) break;
            nx = i + U * stride;
            more = nx + (U - 1) * stride < a.npair;
#pragma unroll
            for (int u = 0; u < U; u++) q[u] = __builtin_nontemporal_load(v2 + std::min(nx + u * stride, last));
            __builtin_amdgcn_sched_barrier(0);
            {
                double x[2 * U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    x[2 * u] = r[u].x;
                    x[2 * u + 1] = r[u].y;
                }
                bin_values<U>(s, x, copy, hbits, rechk);
            }
            i = nx;
            if (!more) break;
        }
    }
    for (; i < a.npair; i += stride) {
        const dbl2 q = v2[i];
        const double x[2] = {q.x, q.y};
        bin_values<1>(s, x, copy, hbits, rechk);
    }
    // the unaligned head value and an odd tail value
    if (blockIdx.x == 0 && tid < 2) {
        const int64_t j = (tid == 0) ? (a.head ? 0 : -1) : (((a.n - a.head) & 1) ? a.n - 1 : -1);
        if (j >= 0) {
            float v;
            int e = bin_entry(s, a.v[j], v);
            if (e < -1) e = bin_resolve(s, -2 - e, v, a.v[j], rechk);
            if (e >= 0) atomicAdd(&s.hist[((uint32_t)e << hbits) + copy], 1u);
        }
    }
    if (rechk) atomicAdd((uint32_t*)(smem + a.off_misc), rechk);
    __syncthreads();

    // merge the copies: a wave sums 64 copies of one bin (hbits >= 6), or a
    // thread sums all copies of its bin
    uint32_t* tot = (uint32_t*)(smem + a.off_tot);
    const int H = 1 << hbits;
    if (hbits >= 6) {
        const int lane = tid & 63, wave = tid >> 6;
        const int chunks = a.nb << (hbits - 6);
        for (int c = wave; c < chunks; c += BIN_THREADS / 64) {
            uint32_t x = s.hist[c * 64 + lane];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
            if (lane == 0 && x) atomicAdd(&tot[c >> (hbits - 6)], x);
        }
    } else {
        for (int b = tid; b < a.nb; b += BIN_THREADS) {
            uint32_t x = 0;
            for (int k = 0; k < H; k++) x += s.hist[(b << hbits) + k];
            tot[b] = x;
        }
    }
    __syncthreads();
    for (int b = tid; b < a.nb; b += BIN_THREADS)
        if (tot[b]) atomicAdd(&a.out[b], (unsigned long long)tot[b]);
    if (tid == 0) {
        const uint32_t r = *(volatile uint32_t*)(smem + a.off_misc);
        if (r) atomicAdd(&a.stats[1], (unsigned long long)r);
        if (blockIdx.x == 0) atomicAdd(&a.stats[0], (unsigned long long)a.n);
    }
}

static int al16(int b) { return (b + 15) & ~15; }

}  // namespace fcfc

using namespace fcfc;

extern "C" fcfc_status fcfc_bin_squared(fcfc_plan_t plan, const double* d_s2, int64_t n, int64_t* d_counts,
                                        void* stream) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || !d_counts || n < 0 || (n > 0 && !d_s2)) {
        set_error("bin_squared: null plan, values or counts, or a negative size");
        return FCFC_EINVAL;
    }
    if (n > (1ll << 61)) {
        set_error("bin_squared: at most 2^61 values per call");
        return FCFC_EINVAL;
    }
    if (((uintptr_t)d_s2 & 7) != 0) {
        set_error("bin_squared: values must be 8-byte aligned");
        return FCFC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const Lut1D* Tp = nullptr;
    FCFC_TRY(plan_bin_table(p, &Tp));
    const Lut1D& T = *Tp;
    const int nb = p->n1, nt = (int)T.tab.size();

    BinArgs a{};
    std::vector<char>& h = p->host_stage;
    const BinBlob L = bin_blob(T, h);
    a.nt = nt;
    a.nb = nb;
    a.off_band = L.off_band;
    a.off_e = L.off_e;
    a.off_hist = L.bytes;
    const int tab_bytes = a.off_hist;
    int dev = 0, maxlds = 65536;
    FCFC_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) maxlds = 65536;
    // as many histogram copies as fit, up to one per thread
    int hbits = 10;
    auto lds_for = [&](int hb) { return tab_bytes + al16(((nb + 1) << hb) * 4) + al16(nb * 4) + 16; };
    while (hbits > 0 && lds_for(hbits) > maxlds) hbits--;
    if (lds_for(hbits) > maxlds) {
        set_error("bin_squared: %d bins and a %d-entry table do not fit the LDS", nb, nt);
        return FCFC_ERANGE;
    }
    a.hbits = hbits;
    a.off_tot = a.off_hist + al16(((nb + 1) << hbits) * 4);
    a.off_misc = a.off_tot + al16(nb * 4);
    const int lds = a.off_misc + 16;
    a.tab_words = tab_bytes / 16;
    a.scale = T.scale;
    a.vmax = T.vmax;

    void* blob = nullptr;
    FCFC_TRY(dev_alloc(&blob, (size_t)tab_bytes, st));
    fcfc_status s = FCFC_OK;
    if (hipMemcpyAsync(blob, h.data(), (size_t)tab_bytes, hipMemcpyHostToDevice, st) != hipSuccess) s = FCFC_EHIP;

    if (s == FCFC_OK && !p->stats_dev) {
        if (hipMalloc(&p->stats_dev, 64) != hipSuccess || hipEventCreate(&p->ev0) != hipSuccess ||
            hipEventCreate(&p->ev1) != hipSuccess)
            s = FCFC_EHIP;
    }
    if (s == FCFC_OK) {
        fill_u64((uint64_t*)p->stats_dev, 0ull, 8, st);
        fill_u64((uint64_t*)d_counts, 0ull, nb, st);
        a.v = d_s2;
        a.n = n;
        a.head = (n > 0 && ((uintptr_t)d_s2 & 15) != 0) ? 1 : 0;
        a.npair = (n - a.head) / 2;
        a.tab = (const uint4*)blob;
        a.out = (unsigned long long*)d_counts;
        a.stats = (unsigned long long*)p->stats_dev;
        static bool attr_set[64] = {};
        if (dev < 64 && !attr_set[dev]) {
            if (hipFuncSetAttribute((const void*)k_bin_squared, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds) !=
                hipSuccess)
                s = FCFC_EHIP;
            else
                attr_set[dev] = true;
        }
        int occ = 0;
        if (s == FCFC_OK &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_bin_squared, BIN_THREADS, lds) !=
                hipSuccess)
            s = FCFC_EHIP;
        if (s == FCFC_OK) {
            int64_t nblk = (int64_t)device_cu_count() * std::max(1, occ);
            const int64_t need = std::max<int64_t>(1, (a.npair + BIN_THREADS - 1) / BIN_THREADS);
            nblk = std::min(nblk, need);
            nblk = std::max(nblk, (n + BIN_PER_GROUP - 1) / BIN_PER_GROUP);
            if (hipEventRecord(p->ev0, st) != hipSuccess) s = FCFC_EHIP;
            if (s == FCFC_OK) {
                hipLaunchKernelGGL(k_bin_squared, dim3((unsigned)nblk), dim3(BIN_THREADS), (size_t)lds, st, a);
                if (hipGetLastError() != hipSuccess || hipEventRecord(p->ev1, st) != hipSuccess) s = FCFC_EHIP;
            }
        }
    }
    dev_free(blob, st);
    if (s != FCFC_OK) {
        set_error("bin_squared: HIP failure");
        return s;
    }
    p->last_stream = st;
    p->last_counts = d_counts;
    p->last_counts_n = 0;
    p->have_stats = true;
    p->stats.items = 0;
    p->stats.lut_entries = nt;
    return FCFC_OK;
}
