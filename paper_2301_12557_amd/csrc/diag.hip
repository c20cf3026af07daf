// diag.hip -- measured accuracy of the hardware FP32 reciprocal and reciprocal
// square root that the counting kernel uses for mu and the mid-point pi.  The
// FP32 error bands assume a relative error bound for both; this entry point
// measures the true maximum over every FP32 input the kernel can meet.
#include <math.h>
#include <string.h>

#include "internal.h"

namespace fcfc {

// Largest relative error of rsq and rcp over FP32 inputs with bit patterns
// [lo, hi), each against the FP64 value of the exact function.
__global__ __launch_bounds__(256) void k_trans_err(uint32_t lo, uint32_t hi, unsigned long long* out) {
    double ers = 0, erc = 0;
    const uint32_t stride = gridDim.x * 256u;
    // hi + stride stays below 2^32 for the ranges used, so b never wraps
    for (uint32_t b = lo + blockIdx.x * 256u + threadIdx.x; b < hi; b += stride) {
        const float x = __uint_as_float(b);
        const double xd = (double)x;
        const double rs = (double)__builtin_amdgcn_rsqf(x);
        const double rc = (double)__builtin_amdgcn_rcpf(x);
        const double ts = 1.0 / sqrt(xd);
        const double tc = 1.0 / xd;
        ers = fmax(ers, fabs(rs - ts) / ts);
        erc = fmax(erc, fabs(rc - tc) / tc);
    }
    for (int o = 32; o > 0; o >>= 1) {
        ers = fmax(ers, __shfl_xor(ers, o));
        erc = fmax(erc, __shfl_xor(erc, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(ers));
        atomicMax(&out[1], (unsigned long long)__double_as_longlong(erc));
    }
}

}  // namespace fcfc

using namespace fcfc;

extern "C" fcfc_status fcfc_diag_transcendental(double* rsq_max_rel, double* rcp_max_rel, double* assumed,
                                                void* stream) {
    clear_error();
    if (!rsq_max_rel || !rcp_max_rel) return FCFC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long* d = nullptr;
    FCFC_HIP(hipMalloc((void**)&d, 16));
    fill_u64((uint64_t*)d, 0ull, 2, st);
    // every FP32 value in [2^-64, 2^64): squared separations, |l|^2 and their
    // products with the bin counts all lie far inside this range
    const uint32_t lo = (uint32_t)(127 - 64) << 23, hi = (uint32_t)(127 + 64) << 23;
    hipLaunchKernelGGL(k_trans_err, dim3(8192), dim3(256), 0, st, lo, hi, d);
    unsigned long long h[2] = {0, 0};
    fcfc_status s = FCFC_OK;
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(h, d, 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("diag_transcendental: HIP failure");
        s = FCFC_EHIP;
    }
    (void)hipFree(d);
    double a, b;
    memcpy(&a, &h[0], 8);
    memcpy(&b, &h[1], 8);
    *rsq_max_rel = a;
    *rcp_max_rel = b;
    if (assumed) *assumed = trans_rel_bound();
    return s;
}

// ---------------------------------------------------------------------------
// Roofline microbenchmarks: the rates the counting kernel is measured against.
// ---------------------------------------------------------------------------
namespace fcfc {

constexpr int MB_ITERS = 2048;

// 8 independent FP32 FMA chains per thread (2 flops per FMA)
__global__ __launch_bounds__(256) void k_peak_fma(float* out, float a, float b) {
    float x0 = threadIdx.x * 1e-3f, x1 = x0 + 1.f, x2 = x0 + 2.f, x3 = x0 + 3.f;
    float x4 = x0 + 4.f, x5 = x0 + 5.f, x6 = x0 + 6.f, x7 = x0 + 7.f;
    for (int i = 0; i < MB_ITERS; i++) {
#pragma unroll
        for (int r = 0; r < 8; r++) {
            x0 = __builtin_fmaf(x0, a, b);
            x1 = __builtin_fmaf(x1, a, b);
            x2 = __builtin_fmaf(x2, a, b);
            x3 = __builtin_fmaf(x3, a, b);
            x4 = __builtin_fmaf(x4, a, b);
            x5 = __builtin_fmaf(x5, a, b);
            x6 = __builtin_fmaf(x6, a, b);
            x7 = __builtin_fmaf(x7, a, b);
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

// conflict-free LDS atomics: lane l of a wave always hits word (wave * 64 + l)
template <typename T>
__global__ __launch_bounds__(256) void k_peak_lds_add(T* out, T inc) {
    __shared__ T h[256];
    h[threadIdx.x] = (T)0;
    __syncthreads();
    T* p = &h[threadIdx.x];
    for (int i = 0; i < MB_ITERS; i++) {
#pragma unroll
        for (int r = 0; r < 8; r++) atomicAdd(p, inc);
    }
    __syncthreads();
    out[blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

}  // namespace fcfc

extern "C" fcfc_status fcfc_diag_peaks(double* fma_tflops, double* lds_u32_per_s, double* lds_u64_per_s,
                                       double* copy_gbps, void* stream) {
    clear_error();
    hipStream_t st = (hipStream_t)stream;
    const int cus = device_cu_count();
    const int blocks = cus * 8;
    const size_t nout = (size_t)blocks * 256;
    const size_t copy_bytes = (size_t)1 << 30;
    char* buf = nullptr;
    if (hipMalloc((void**)&buf, nout * 8 + 2 * copy_bytes) != hipSuccess) {
        set_error("diag_peaks: cannot allocate %zu bytes", nout * 8 + 2 * copy_bytes);
        return FCFC_ENOMEM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    fcfc_status s = FCFC_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) s = FCFC_EHIP;
    auto timed = [&](auto launch) -> double {
        if (s != FCFC_OK) return 0.0;
        launch();  // warm-up
        float ms = 0.f;
        if (hipEventRecord(e0, st) != hipSuccess) s = FCFC_EHIP;
        launch();
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess)
            s = FCFC_EHIP;
        return (double)ms * 1e-3;
    };
    const double work = (double)nout * MB_ITERS * 8;  // operations per launch
    double t = timed([&] {
        hipLaunchKernelGGL(k_peak_fma, dim3(blocks), dim3(256), 0, st, (float*)buf, 0.999f, 1e-4f);
    });
    if (fma_tflops && t > 0) *fma_tflops = 8.0 * work * 2.0 / t / 1e12;
    t = timed([&] {
        hipLaunchKernelGGL(k_peak_lds_add<uint32_t>, dim3(blocks), dim3(256), 0, st, (uint32_t*)buf, 1u);
    });
    if (lds_u32_per_s && t > 0) *lds_u32_per_s = work / t;
    t = timed([&] {
        hipLaunchKernelGGL(k_peak_lds_add<unsigned long long>, dim3(blocks), dim3(256), 0, st,
                           (unsigned long long*)buf, 1ull);
    });
    if (lds_u64_per_s && t > 0) *lds_u64_per_s = work / t;
    char* src = buf + nout * 8;
    char* dst = src + copy_bytes;
    t = timed([&] {
        if (hipMemcpyAsync(dst, src, copy_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) s = FCFC_EHIP;
    });
    if (copy_gbps && t > 0) *copy_gbps = 2.0 * (double)copy_bytes / t / 1e9;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (s != FCFC_OK) set_error("diag_peaks: HIP failure");
    return s;
}
