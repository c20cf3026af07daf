// noalloc.hip -- fcfc_count_pairs_noalloc: the pair count with every scratch
// buffer (work list, counters, sort space, kernel arguments, exact weighted
// accumulators) taken from one file-scope device array instead of the
// library's pool, for callers that cannot allocate device memory.
//
// The array lives in this source file.  Host code never passes its name to a
// kernel or a copy: in host code the name is a host-side stand-in, not the
// device address.  The device address is fetched once per device with
// hipGetSymbolAddress (the device made current by the caller) and kept per
// device; only that pointer is handed to the counting path.
#include <mutex>

#include "internal.h"

namespace fcfc {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;  // 64 MiB per device

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mutex;
static char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of this device's copy of `scratch`, fetched on the first call
// on the device (with that device current).
static fcfc_status scratch_for_current_device(char** out) {
    int dev = 0;
    FCFC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("count_pairs_noalloc: device %d beyond the %d devices supported", dev, NOALLOC_MAX_DEVICES);
        return FCFC_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("count_pairs_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return FCFC_EHIP;
        }
        g_scratch_ptr[dev] = (char*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return FCFC_OK;
}

}  // namespace fcfc

using namespace fcfc;

extern "C" int64_t fcfc_noalloc_scratch_bytes(void) { return (int64_t)NOALLOC_SCRATCH_BYTES; }

extern "C" fcfc_status fcfc_count_pairs_noalloc(fcfc_plan_t plan, fcfc_cells_t c1, fcfc_cells_t c2,
                                                int64_t* d_counts, double* d_wcounts, void* stream) {
    clear_error();
    Plan* p = (Plan*)plan;
    Cells* a = (Cells*)c1;
    Cells* b = (Cells*)c2;
    if (!p || !a || !d_counts) {
        set_error("count_pairs_noalloc: null plan, cells or output");
        return FCFC_EINVAL;
    }
    if (a->plan_id != p->id || (b && b->plan_id != p->id)) {
        set_error("count_pairs_noalloc: cell sets were built on a different plan");
        return FCFC_EGRID;
    }
    Workspace ws;
    FCFC_TRY(scratch_for_current_device(&ws.base));
    ws.bytes = NOALLOC_SCRATCH_BYTES;
    fcfc_status s = count_pairs(p, a, b, d_counts, d_wcounts, (hipStream_t)stream, nullptr, &ws);
    if (s == FCFC_OK) {
        p->last_counts = d_counts;
        p->last_counts_n = 0;
    }
    return s;
}
