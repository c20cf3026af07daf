// mem.cpp -- device memory for cell sets and per-call scratch.
//
// Every cell set and every count takes and returns device memory.  Going to
// the driver each time (hipMalloc / hipFree, or stream-ordered allocation
// from the device's default pool, which hands freed memory back at every
// synchronisation) costs hundreds of microseconds per call once the memory
// has been touched.  The library therefore keeps one stream-ordered pool
// per device that retains up to RETAIN bytes of freed memory for reuse.
#include <mutex>

#include "internal.h"

namespace fcfc {

static constexpr uint64_t RETAIN = 1ull << 30;  // freed bytes a pool keeps for reuse
static constexpr int MAX_DEV = 64;

static std::mutex g_mu;
static hipMemPool_t g_pool[MAX_DEV];
static bool g_tried[MAX_DEV];

// The library's pool for the current device, or null if none could be made
// (then the device's default pool serves).
static hipMemPool_t current_pool() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_tried[dev]) {
        g_tried[dev] = true;
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p = nullptr;
        if (hipMemPoolCreate(&p, &props) == hipSuccess) {
            uint64_t thr = RETAIN;
            if (hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &thr) == hipSuccess) {
                g_pool[dev] = p;
            } else {
                (void)hipMemPoolDestroy(p);
            }
        }
    }
    return g_pool[dev];
}

fcfc_status dev_alloc(void** ptr, size_t bytes, hipStream_t st) {
    *ptr = nullptr;
    hipMemPool_t pool = current_pool();
    const hipError_t e = pool ? hipMallocFromPoolAsync(ptr, bytes, pool, st) : hipMallocAsync(ptr, bytes, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        set_error("cannot allocate %zu bytes of device memory", bytes);
        return FCFC_ENOMEM;
    }
    return FCFC_OK;
}

void dev_free(void* ptr, hipStream_t st) {
    if (ptr) (void)hipFreeAsync(ptr, st);
}

}  // namespace fcfc
