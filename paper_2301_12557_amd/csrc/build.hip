// build.hip -- GPU cell-list construction (Sect. 2.1): bounding box, cell key
// per point with validation, stable LSD radix sort of (key, index), gather
// into cell-local FP32 / FP64 arrays, and cell offsets.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace fcfc {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

int key_xbits(int64_t ncells) {
    int cb = 0;
    while (cb < 31 && ((int64_t)1 << cb) < ncells) cb++;
    const int total = std::min(32, (cb + 8 + 7) / 8 * 8);
    return total - cb;
}

void weight_stats_reduce(const uint64_t* slots, uint64_t* bmin, uint64_t* bmax) {
    uint64_t m = 0, x = 0;
    for (int sl = 0; sl < STAT_SLOTS; sl++) {
        m = std::max(m, slots[(size_t)sl * STAT_STRIDE]);
        x = std::max(x, slots[(size_t)sl * STAT_STRIDE + 1]);
    }
    *bmin = ~m;  // ~0 when no slot saw a non-zero weight
    *bmax = x;
}

static int grid_for(int64_t n, int block = 256, int cap = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
}
void fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
}

int device_cu_count() {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return cu > 0 ? cu : 256;
}

// order-preserving map of a double to uint64 (for atomic min/max)
__device__ inline uint64_t ord_bits(double x) {
    uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
static double ord_value(uint64_t b) {
    uint64_t r = (b >> 63) ? (b & 0x7FFFFFFFFFFFFFFFull) : ~b;
    double x;
    memcpy(&x, &r, 8);
    return x;
}

// ---------------------------------------------------------------------------
// exclusive scan of uint32 (2048 elements per block, recursive on block sums)
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_TILE = SCAN_T * SCAN_I;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
    // sh: SCAN_T entries
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        uint32_t a = (t >= off) ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    uint32_t incl = sh[t];
    *total = sh[SCAN_T - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_block(const uint32_t* __restrict__ in,
                                                       uint32_t* __restrict__ out, int64_t n,
                                                       uint32_t* __restrict__ bsum) {
    __shared__ uint32_t sh[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
    uint32_t v[SCAN_I];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_I; i++) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, sh, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_I; i++) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0 && bsum) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_add(uint32_t* __restrict__ out, int64_t n, const uint32_t* __restrict__ boff) {
    int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    uint32_t a = boff[blockIdx.x];
    for (int r = 0; r < SCAN_I; r++, i += SCAN_T)
        if (i < n) out[i] += a;
}

__global__ void k_scan_total(const uint32_t* in, const uint32_t* out, int64_t n, uint32_t* total) {
    *total = (n > 0) ? out[n - 1] + in[n - 1] : 0u;
}

size_t scan_scratch_bytes(int64_t n) {
    size_t b = 0;
    int64_t m = n;
    while (m > SCAN_TILE) {
        m = (m + SCAN_TILE - 1) / SCAN_TILE;
        b += 2 * ((size_t)m * 4 + 256);
    }
    return b + 256;
}

// out may alias in only when n <= SCAN_TILE
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev,
                        void* scratch, hipStream_t st) {
    if (n <= 0) {
        if (total_dev) fill_u32(total_dev, 0u, 1, st);
        return;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(SCAN_T), 0, st, in, out, n, (uint32_t*)nullptr);
    } else {
        uint32_t* bs = (uint32_t*)scratch;
        uint32_t* bo = bs + ((nb * 4 + 256) / 4);
        void* rest = (void*)(bo + ((nb * 4 + 256) / 4));
        hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SCAN_T), 0, st, in, out, n, bs);
        scan_exclusive_u32(bs, bo, nb, nullptr, rest, st);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_T), 0, st, out, n, bo);
    }
    if (total_dev) hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, in, out, n, total_dev);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (key, value) pairs, 8-bit digits
// ---------------------------------------------------------------------------
constexpr int RS_T = 256, RS_I = 8, RS_TILE = RS_T * RS_I, RS_WAVES = RS_T / 64;

__global__ __launch_bounds__(RS_T) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                  uint32_t* __restrict__ hist, int nblk) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_I; r++) {
        int64_t i = base + r * RS_T + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(RS_T) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                     const uint32_t* __restrict__ vin,
                                                     uint32_t* __restrict__ kout,
                                                     uint32_t* __restrict__ vout, int64_t n, int shift,
                                                     const uint32_t* __restrict__ offs, int nblk) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[RS_WAVES][256];
    int t = threadIdx.x;
    int lane = t & 63, w = t >> 6;
    run[t] = offs[(int64_t)t * nblk + blockIdx.x];
    for (int q = 0; q < RS_WAVES; q++) wcnt[q][t] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_I; r++) {
        int64_t i = base + r * RS_T + t;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u;
        uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int q = 0; q < w; q++) pos += wcnt[q][d];
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int q = 0; q < RS_WAVES; q++) {
            add += wcnt[q][t];
            wcnt[q][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

size_t radix_scratch_bytes(int64_t n) {
    int64_t nblk = std::max<int64_t>(1, (n + RS_TILE - 1) / RS_TILE);
    size_t h = (size_t)nblk * 256 * 4 + 256;
    return 2 * h + scan_scratch_bytes(nblk * 256);
}

// Sorts by the low key_bits bits.  Ping-pongs between (k,v) and (tk,tv); on
// return k/v point at the sorted arrays (pointers may be swapped).
void radix_sort_pairs(uint32_t** k, uint32_t** v, uint32_t** tk, uint32_t** tv, int64_t n, int key_bits,
                      void* scratch, hipStream_t st) {
    if (n <= 1) return;
    int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
    uint32_t* hist = (uint32_t*)scratch;
    uint32_t* offs = hist + (((size_t)nblk * 256 * 4 + 256) / 4);
    void* sscr = (void*)(offs + (((size_t)nblk * 256 * 4 + 256) / 4));
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(RS_T), 0, st, *k, n, shift, hist, nblk);
        scan_exclusive_u32(hist, offs, (int64_t)nblk * 256, nullptr, sscr, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(RS_T), 0, st, *k, *v, *tk, *tv, n, shift, offs, nblk);
        std::swap(*k, *tk);
        std::swap(*v, *tv);
    }
}

// ---------------------------------------------------------------------------
// bounding box over catalogues
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_aabb(const double* __restrict__ xyz, int64_t n,
                                              uint64_t* __restrict__ mm /*slots: ~lo[3], hi[3] ord bits*/,
                                              uint32_t* __restrict__ flags) {
    __shared__ uint64_t smin[3][256], smax[3][256];
    __shared__ uint32_t sflag;
    if (threadIdx.x == 0) sflag = 0;
    uint64_t lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0, 0, 0};
    uint32_t f = 0;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        for (int a = 0; a < 3; a++) {
            double x = xyz[3 * i + a];
            if (!isfinite(x)) {
                f |= 1u;
                continue;
            }
            uint64_t b = ord_bits(x);
            lo[a] = b < lo[a] ? b : lo[a];
            hi[a] = b > hi[a] ? b : hi[a];
        }
    }
    for (int a = 0; a < 3; a++) {
        smin[a][threadIdx.x] = lo[a];
        smax[a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    if (f) atomicOr(&sflag, f);
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int a = 0; a < 3; a++) {
                uint64_t x = smin[a][threadIdx.x + off], y = smax[a][threadIdx.x + off];
                if (x < smin[a][threadIdx.x]) smin[a][threadIdx.x] = x;
                if (y > smax[a][threadIdx.x]) smax[a][threadIdx.x] = y;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long* slot = (unsigned long long*)mm + (size_t)(blockIdx.x % STAT_SLOTS) * STAT_STRIDE;
        for (int a = 0; a < 3; a++) {
            atomicMax(&slot[a], ~(unsigned long long)smin[a][0]);
            atomicMax(&slot[3 + a], (unsigned long long)smax[a][0]);
        }
        if (sflag) atomicOr(flags, sflag);
    }
}

fcfc_status fit_bounds(Plan* p, const fcfc_catalog* cats, int ncat, hipStream_t st) {
    uint64_t* d = nullptr;
    FCFC_TRY(dev_alloc((void**)&d, STAT_BYTES + 64, st));
    uint32_t* flags = (uint32_t*)(d + STAT_SLOTS * STAT_STRIDE);
    int64_t total = 0;
    fill_u64(d, 0ull, STAT_SLOTS * STAT_STRIDE + 8, st);
    for (int c = 0; c < ncat; c++) {
        if (cats[c].n <= 0) continue;
        total += cats[c].n;
        int g = grid_for(cats[c].n, 256, 4096);
        hipLaunchKernelGGL(k_aabb, dim3(g), dim3(256), 0, st, cats[c].xyz, cats[c].n, d, flags);
    }
    std::vector<uint64_t> h(STAT_SLOTS * STAT_STRIDE + 8);
    hipError_t e1 = hipMemcpyAsync(h.data(), d, STAT_BYTES + 64, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    dev_free(d, st);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        set_error("fit_bounds: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return FCFC_EHIP;
    }
    if (h[STAT_SLOTS * STAT_STRIDE] & 1u) {
        set_error("fit_bounds: non-finite coordinate");
        return FCFC_ENONFINITE;
    }
    double lo[3], hi[3];
    if (total == 0) {
        for (int a = 0; a < 3; a++) {
            lo[a] = 0;
            hi[a] = 1;
        }
    } else {
        for (int a = 0; a < 3; a++) {
            uint64_t l = 0, u = 0;  // max of ~lo bits, max of hi bits
            for (int sl = 0; sl < STAT_SLOTS; sl++) {
                l = std::max(l, h[(size_t)sl * STAT_STRIDE + a]);
                u = std::max(u, h[(size_t)sl * STAT_STRIDE + 3 + a]);
            }
            lo[a] = ord_value(~l);
            hi[a] = ord_value(u);
        }
    }
    return fcfc_set_bounds_internal(p, lo, hi);
}

// ---------------------------------------------------------------------------
// cell keys + validation
// ---------------------------------------------------------------------------
struct GridArgs {
    int nx, ny, nz;
    double lox, loy, loz;
    double hix, hiy, hiz;  // open box upper bounds (inclusive)
    double side;
    double L;
};


// Weight statistics of a workgroup: smallest non-zero and largest |w| as
// ordered bits.  Each wave reduces its lanes with shuffles and one lane
// updates the workgroup's LDS words (all 256 lanes contending for one LDS
// word made the key pass four times slower).
__device__ inline void wave_weight_stats(unsigned long long bmin, unsigned long long bmax, unsigned long long* swmin,
                                         unsigned long long* swmax) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long a = __shfl_xor(bmin, o), b = __shfl_xor(bmax, o);
        bmin = a < bmin ? a : bmin;
        bmax = b > bmax ? b : bmax;
    }
    if ((threadIdx.x & 63) == 0) {
        if (bmin != ~0ull) atomicMin(swmin, bmin);
        if (bmax) atomicMax(swmax, bmax);
    }
}

__device__ inline int cell_of(double x, double lo, double side, int n) {
    double f = floor((x - lo) / side);
    int c = (f < 0.0) ? 0 : ((f > (double)(n - 1)) ? n - 1 : (int)f);
    return c;
}
// position of x within cell c on 2^xbits steps, clamped to the cell
__device__ inline uint32_t subcell_of(double x, double lo, double side, int c, int xbits) {
    const double f = ((x - lo) / side - (double)c) * (double)(1u << xbits);
    const double top = (double)((1u << xbits) - 1u);
    return (uint32_t)((f < 0.0) ? 0.0 : ((f > top) ? top : floor(f)));
}

__global__ __launch_bounds__(256) void k_keys(const double* __restrict__ xyz, const double* __restrict__ w,
                                              int64_t n, GridArgs g, int xbits, uint32_t* __restrict__ key,
                                              uint32_t* __restrict__ idx, uint32_t* __restrict__ flags,
                                              uint64_t* __restrict__ wst /*slots: ~min nonzero |w|, max |w| bits*/) {
    __shared__ uint32_t sflag;
    __shared__ uint64_t swmin, swmax;
    if (threadIdx.x == 0) {
        sflag = 0;
        swmin = ~0ull;
        swmax = 0;
    }
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t f = 0;
    unsigned long long bmin = ~0ull, bmax = 0ull;
    if (i < n) {
        double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
            f |= VF_NONFINITE;
        } else if (g.L > 0) {
            if (!(x >= 0.0 && x < g.L && y >= 0.0 && y < g.L && z >= 0.0 && z < g.L)) f |= VF_BOX;
        } else {
            if (!(x >= g.lox && x <= g.hix && y >= g.loy && y <= g.hiy && z >= g.loz && z <= g.hiz)) f |= VF_BOX;
        }
        uint32_t cx = 0, cy = 0, cz = 0, q = 0;
        if (!f) {
            cx = cell_of(x, g.lox, g.side, g.nx);
            cy = cell_of(y, g.loy, g.side, g.ny);
            cz = cell_of(z, g.loz, g.side, g.nz);
            q = subcell_of(x, g.lox, g.side, (int)cx, xbits);
        }
        key[i] = (((cz * (uint32_t)g.ny + cy) * (uint32_t)g.nx + cx) << xbits) | q;
        idx[i] = (uint32_t)i;
        if (w) {
            double wv = w[i];
            if (!isfinite(wv)) {
                f |= VF_WNONFINITE;
            } else {
                double a = fabs(wv);
                unsigned long long b = (unsigned long long)__double_as_longlong(a);  // positive: bits are ordered
                if (a > 0.0) bmin = b;
                bmax = b;
            }
        }
        if (f) atomicOr(&sflag, f);
    }
    if (w) wave_weight_stats(bmin, bmax, (unsigned long long*)&swmin, (unsigned long long*)&swmax);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sflag) atomicOr(flags, sflag);
        if (w) {
            unsigned long long* slot = (unsigned long long*)wst + (size_t)(blockIdx.x % STAT_SLOTS) * STAT_STRIDE;
            if (swmin != ~0ull) atomicMax(&slot[0], ~(unsigned long long)swmin);
            if (swmax) atomicMax(&slot[1], (unsigned long long)swmax);
        }
    }
}

// ---------------------------------------------------------------------------
// gather sorted points into cell-local FP32, absolute FP32, FP64, weights
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ xyz, const double* __restrict__ w,
                                                const uint32_t* __restrict__ skey,
                                                const uint32_t* __restrict__ sidx, int64_t n, GridArgs g, int xbits,
                                                float4* __restrict__ pos32, float4* __restrict__ abs32,
                                                double* __restrict__ pos64, double* __restrict__ wout) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t i = sidx[p];
    uint32_t key = skey[p] >> xbits;
    uint32_t cx = key % (uint32_t)g.nx;
    uint32_t cy = (key / (uint32_t)g.nx) % (uint32_t)g.ny;
    uint32_t cz = key / ((uint32_t)g.nx * (uint32_t)g.ny);
    double x = xyz[3 * (int64_t)i], y = xyz[3 * (int64_t)i + 1], z = xyz[3 * (int64_t)i + 2];
    double ox = g.lox + (double)cx * g.side;
    double oy = g.loy + (double)cy * g.side;
    double oz = g.loz + (double)cz * g.side;
    pos32[p] = make_float4((float)(x - ox), (float)(y - oy), (float)(z - oz), __int_as_float((int)cx));
    if (abs32) abs32[p] = make_float4((float)x, (float)y, (float)z, 0.f);
    pos64[3 * p] = x;
    pos64[3 * p + 1] = y;
    pos64[3 * p + 2] = z;
    if (wout) wout[p] = w[i];
}

__global__ void k_cell_start(const uint32_t* __restrict__ skey, int64_t n, int64_t ncell, int xbits,
                             uint32_t* __restrict__ cs) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n) return;
    int64_t kprev = (p == 0) ? -1 : (int64_t)(skey[p - 1] >> xbits);
    int64_t kcur = (p == n) ? ncell : (int64_t)(skey[p] >> xbits);
    for (int64_t c = kprev + 1; c <= kcur; c++) cs[c] = (uint32_t)p;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static GridArgs make_grid_args(const Plan* p) {
    const Grid& gr = p->grid;
    GridArgs g;
    g.nx = gr.nx;
    g.ny = gr.ny;
    g.nz = gr.nz;
    g.lox = gr.lo[0];
    g.loy = gr.lo[1];
    g.loz = gr.lo[2];
    g.hix = p->grid_hi[0];
    g.hiy = p->grid_hi[1];
    g.hiz = p->grid_hi[2];
    g.side = gr.side;
    g.L = gr.L;
    return g;
}

fcfc_status validate_points(Plan* p, const fcfc_catalog* cat, uint32_t* idx, uint32_t* keys, uint32_t* flags,
                            uint64_t* wst, hipStream_t st) {
    GridArgs g = make_grid_args(p);
    fill_u32(flags, 0u, 1, st);
    fill_u64(wst, 0ull, STAT_SLOTS * STAT_STRIDE, st);
    if (cat->n > 0)
        hipLaunchKernelGGL(k_keys, dim3((unsigned)((cat->n + 255) / 256)), dim3(256), 0, st, cat->xyz, cat->w, cat->n,
                           g, key_xbits(p->grid.ncell()), keys, idx, flags, wst);
    FCFC_HIP(hipGetLastError());
    return FCFC_OK;
}

fcfc_status build_cells(Plan* p, const fcfc_catalog* cat, hipStream_t st, Cells** out) {
    if (p->tune.tree_leaf > 0) return build_tree(p, cat, st, out);
    int64_t n = cat->n;
    const Grid& gr = p->grid;
    int64_t ncell = gr.ncell();
    bool weighted = cat->w != nullptr;
    bool need_abs = (p->los == FCFC_LOS_MIDPOINT && p->kind != FCFC_BIN_S);
    // device block owned by the cell set
    // pos32 and w carry PAD trailing entries so that grouped scalar loads never leave the block
    const int64_t PAD = 8;
    size_t o_pos32 = 0;
    size_t o_abs32 = o_pos32 + align256((size_t)(n + PAD) * 16);
    size_t o_pos64 = o_abs32 + (need_abs ? align256((size_t)n * 16) : 0);
    size_t o_w = o_pos64 + align256((size_t)n * 24);
    size_t o_cs = o_w + (weighted ? align256((size_t)(n + PAD) * 8) : 0);
    size_t o_key = o_cs + align256((size_t)(ncell + 1) * 4);
    size_t total = o_key + align256((size_t)std::max<int64_t>(n, 1) * 4);
    Cells* c = new (std::nothrow) Cells();
    if (!c) return FCFC_ENOMEM;
    char* blk = nullptr;
    if (dev_alloc((void**)&blk, total, st) != FCFC_OK) {
        delete c;
        set_error("build_cells: cannot allocate %zu bytes", total);
        return FCFC_ENOMEM;
    }
    c->block = blk;
    c->plan_id = p->id;
    c->grid = gr;
    c->n = n;
    c->weighted = weighted || n == 0;  // an empty set takes part in weighted counts (it adds nothing)
    c->has_abs = need_abs;
    c->pos32 = (float4*)(blk + o_pos32);
    c->abs32 = need_abs ? (float4*)(blk + o_abs32) : nullptr;
    c->pos64 = (double*)(blk + o_pos64);
    c->w = weighted ? (double*)(blk + o_w) : nullptr;
    c->cell_start = (uint32_t*)(blk + o_cs);
    c->xkey = (uint32_t*)(blk + o_key);
    c->xbits = key_xbits(ncell);

    // scratch: keys, idx, tmp keys, tmp idx, flags + weight stats, sort scratch
    size_t s_keys = align256((size_t)std::max<int64_t>(n, 1) * 4);
    size_t s_misc = 256 + STAT_BYTES;
    size_t s_sort = align256(radix_scratch_bytes(n));
    size_t stotal = 4 * s_keys + s_misc + s_sort;
    char* scr = nullptr;
    if (dev_alloc((void**)&scr, stotal, st) != FCFC_OK) {
        dev_free(blk, st);
        delete c;
        set_error("build_cells: cannot allocate scratch");
        return FCFC_ENOMEM;
    }
    uint32_t* key = (uint32_t*)scr;
    uint32_t* idx = (uint32_t*)(scr + s_keys);
    uint32_t* tk = (uint32_t*)(scr + 2 * s_keys);
    uint32_t* tv = (uint32_t*)(scr + 3 * s_keys);
    uint32_t* flags = (uint32_t*)(scr + 4 * s_keys);
    uint64_t* wst = (uint64_t*)(scr + 4 * s_keys + 256);
    void* sort_scr = scr + 4 * s_keys + s_misc;

    GridArgs g = make_grid_args(p);
    fill_u32((uint32_t*)(c->pos32 + n), 0u, PAD * 4, st);
    if (weighted) fill_u64((uint64_t*)(c->w + n), 0ull, PAD, st);
    fill_u32(flags, 0u, 1, st);
    fill_u64(wst, 0ull, STAT_SLOTS * STAT_STRIDE, st);
    if (n > 0) {
        hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cat->xyz, cat->w, n, g,
                           c->xbits, key, idx, flags, wst);
        int bits = 0;
        while (bits < 32 && ((int64_t)1 << bits) < ncell) bits++;
        bits = std::min(32, bits + c->xbits);
        radix_sort_pairs(&key, &idx, &tk, &tv, n, bits, sort_scr, st);
        hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cat->xyz, cat->w, key,
                           idx, n, g, c->xbits, c->pos32, c->abs32, c->pos64, c->w);
        if (hipMemcpyAsync(c->xkey, key, (size_t)n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            dev_free(scr, st);
            dev_free(blk, st);
            delete c;
            set_error("build_cells: HIP copy failed");
            return FCFC_EHIP;
        }
    }
    hipLaunchKernelGGL(k_cell_start, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, key, n, ncell, c->xbits,
                       c->cell_start);
    uint64_t h[3] = {0, 0, 0};
    std::vector<uint64_t> hws(STAT_SLOTS * STAT_STRIDE);
    hipError_t e1 = hipMemcpyAsync(h, flags, 8, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipMemcpyAsync(hws.data(), wst, STAT_BYTES, hipMemcpyDeviceToHost, st);
    hipError_t e3 = hipStreamSynchronize(st);
    dev_free(scr, st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        dev_free(blk, st);
        delete c;
        set_error("build_cells: HIP error %s", hipGetErrorString(e3 != hipSuccess ? e3 : (e2 != hipSuccess ? e2 : e1)));
        return FCFC_EHIP;
    }
    uint32_t fl = (uint32_t)h[0];
    fcfc_status s = FCFC_OK;
    if (fl & (VF_NONFINITE | VF_WNONFINITE)) {
        set_error("build_cells: non-finite position or weight");
        s = FCFC_ENONFINITE;
    } else if (fl & VF_BOX) {
        set_error(p->L > 0 ? "build_cells: a point lies outside [0, L)" : "build_cells: a point lies outside the plan bounds");
        s = FCFC_EBOX;
    }
    if (s != FCFC_OK) {
        dev_free(blk, st);
        delete c;
        return s;
    }
    if (weighted) {
        weight_stats_reduce(hws.data(), &h[1], &h[2]);
        double a, b;
        memcpy(&a, &h[1], 8);
        memcpy(&b, &h[2], 8);
        c->wmin = (h[1] == ~0ull) ? 0.0 : a;
        c->wmax = b;
    }
    *out = c;
    return FCFC_OK;
}

// ---------------------------------------------------------------------------
// batched build: many catalogues on one grid (periodic, or an open box
// inside the plan bounds), sorted by the combined key (catalogue * ncell +
// cell) so that catalogue c occupies the cells [c * ncell, (c+1) * ncell) of
// one stacked grid
// ---------------------------------------------------------------------------
__device__ inline int find_cat(const int64_t* __restrict__ offs, int ncat, int64_t i) {
    int lo = 0, hi = ncat;  // offs[lo] <= i < offs[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (offs[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_bkeys(const CatDesc* __restrict__ cats, const int64_t* __restrict__ offs,
                                               int ncat, int64_t ntot, GridArgs g, int xbits, uint32_t* __restrict__ key,
                                               uint32_t* __restrict__ idx, uint32_t* __restrict__ flags,
                                               uint64_t* __restrict__ wst) {
    __shared__ uint32_t sflag;
    __shared__ uint64_t swmin, swmax;
    if (threadIdx.x == 0) {
        sflag = 0;
        swmin = ~0ull;
        swmax = 0;
    }
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long bmin = ~0ull, bmax = 0ull;
    if (i < ntot) {
        const int c = find_cat(offs, ncat, i);
        const CatDesc d = cats[c];
        const int64_t li = i - offs[c];
        double x = d.xyz[3 * li], y = d.xyz[3 * li + 1], z = d.xyz[3 * li + 2];
        uint32_t f = 0;
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
            f |= VF_NONFINITE;
        } else if (g.L > 0) {
            if (!(x >= 0.0 && x < g.L && y >= 0.0 && y < g.L && z >= 0.0 && z < g.L)) f |= VF_BOX;
        } else {
            if (!(x >= g.lox && x <= g.hix && y >= g.loy && y <= g.hiy && z >= g.loz && z <= g.hiz)) f |= VF_BOX;
        }
        uint32_t cx = 0, cy = 0, cz = 0, q = 0;
        if (!f) {
            cx = cell_of(x, g.lox, g.side, g.nx);
            cy = cell_of(y, g.loy, g.side, g.ny);
            cz = cell_of(z, g.loz, g.side, g.nz);
            q = subcell_of(x, g.lox, g.side, (int)cx, xbits);
        }
        key[i] = (((((uint32_t)c * (uint32_t)g.nz + cz) * (uint32_t)g.ny + cy) * (uint32_t)g.nx + cx) << xbits) | q;
        idx[i] = (uint32_t)i;
        if (d.w) {
            double wv = d.w[li];
            if (!isfinite(wv)) {
                f |= VF_WNONFINITE;
            } else {
                double a = fabs(wv);
                unsigned long long b = (unsigned long long)__double_as_longlong(a);
                if (a > 0.0) bmin = b;
                bmax = b;
            }
        }
        if (f) atomicOr(&sflag, f);
    }
    wave_weight_stats(bmin, bmax, (unsigned long long*)&swmin, (unsigned long long*)&swmax);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sflag) atomicOr(flags, sflag);
        unsigned long long* slot = (unsigned long long*)wst + (size_t)(blockIdx.x % STAT_SLOTS) * STAT_STRIDE;
        if (swmin != ~0ull) atomicMax(&slot[0], ~(unsigned long long)swmin);
        if (swmax) atomicMax(&slot[1], (unsigned long long)swmax);
    }
}

__global__ __launch_bounds__(256) void k_bgather(const CatDesc* __restrict__ cats, const int64_t* __restrict__ offs,
                                                 int ncat, const uint32_t* __restrict__ skey,
                                                 const uint32_t* __restrict__ sidx, int64_t n, GridArgs g, int xbits,
                                                 float4* __restrict__ pos32, float4* __restrict__ abs32,
                                                 double* __restrict__ pos64, double* __restrict__ wout) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t i = sidx[p];
    const int c = find_cat(offs, ncat, i);
    const CatDesc d = cats[c];
    const int64_t li = (int64_t)i - offs[c];
    uint32_t key = skey[p] >> xbits;
    uint32_t cx = key % (uint32_t)g.nx;
    uint32_t cy = (key / (uint32_t)g.nx) % (uint32_t)g.ny;
    uint32_t cz = (key / ((uint32_t)g.nx * (uint32_t)g.ny)) % (uint32_t)g.nz;
    double x = d.xyz[3 * li], y = d.xyz[3 * li + 1], z = d.xyz[3 * li + 2];
    const double ox = g.lox + (double)cx * g.side;
    const double oy = g.loy + (double)cy * g.side;
    const double oz = g.loz + (double)cz * g.side;
    pos32[p] = make_float4((float)(x - ox), (float)(y - oy), (float)(z - oz), __int_as_float((int)cx));
    if (abs32) abs32[p] = make_float4((float)x, (float)y, (float)z, 0.f);
    pos64[3 * p] = x;
    pos64[3 * p + 1] = y;
    pos64[3 * p + 2] = z;
    if (wout) wout[p] = d.w ? d.w[li] : 0.0;
}

size_t batch_build_scratch(int64_t ntot) { return radix_scratch_bytes(ntot); }

// Enqueue the batched build (no host synchronisation: capturable).
void batch_build_enqueue(const Plan* p, int xbits, const CatDesc* desc, const int64_t* offs, int ncat, int64_t ntot,
                         bool weighted, uint32_t** key, uint32_t** idx, uint32_t** tk, uint32_t** tv, void* sort_scr,
                         uint32_t* flags, uint64_t* wst, float4* pos32, float4* abs32, double* pos64, double* w,
                         uint32_t* cs, hipStream_t st) {
    GridArgs g = make_grid_args(p);
    const int64_t ncell_all = p->grid.ncell() * (int64_t)ncat;
    fill_u32((uint32_t*)(pos32 + ntot), 0u, 8 * 4, st);
    if (weighted) fill_u64((uint64_t*)(w + ntot), 0ull, 8, st);
    fill_u32(flags, 0u, 1, st);
    fill_u64(wst, 0ull, STAT_SLOTS * STAT_STRIDE, st);
    if (ntot > 0) {
        hipLaunchKernelGGL(k_bkeys, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, st, desc, offs, ncat, ntot, g,
                           xbits, *key, *idx, flags, wst);
        int bits = 0;
        while (bits < 32 && ((int64_t)1 << bits) < ncell_all) bits++;
        bits = std::min(32, bits + xbits);
        radix_sort_pairs(key, idx, tk, tv, ntot, bits, sort_scr, st);
        hipLaunchKernelGGL(k_bgather, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, st, desc, offs, ncat, *key,
                           *idx, ntot, g, xbits, pos32, abs32, pos64, weighted ? w : nullptr);
    }
    hipLaunchKernelGGL(k_cell_start, dim3((unsigned)((ntot + 1 + 255) / 256)), dim3(256), 0, st, *key, ntot, ncell_all,
                       xbits, cs);
}

}  // namespace fcfc
