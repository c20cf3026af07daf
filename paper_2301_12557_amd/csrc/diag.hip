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
