// batch.hip -- C ABI of the batched pipeline (many catalogues, one cell
// build, one work list and one counting launch for a list of catalogue pairs).
#include <vector>

#include "internal.h"

using namespace fcfc;

static fcfc_status batch_create(fcfc_plan_t plan, const fcfc_catalog* cats, int32_t ncat, const int32_t* pairs,
                                int32_t npairs, void* stream, fcfc_batch_t* out) {
    Plan* p = (Plan*)plan;
    if (!p || !cats || ncat < 1 || !out || !pairs || npairs < 1) {
        set_error("batch_create: null plan, catalogues, pairs or output, or no catalogue / pair");
        return FCFC_EINVAL;
    }
    for (int c = 0; c < ncat; c++) {
        if (cats[c].n < 0 || (cats[c].n > 0 && !cats[c].xyz)) {
            set_error("batch_create: catalogue %d invalid", c);
            return FCFC_EINVAL;
        }
    }
    for (int q = 0; q < npairs; q++) {
        if (pairs[2 * q] < 0 || pairs[2 * q] >= ncat || pairs[2 * q + 1] < 0 || pairs[2 * q + 1] >= ncat) {
            set_error("batch_create: pair %d names a catalogue outside [0, %d)", q, ncat);
            return FCFC_EINVAL;
        }
    }
    BatchImpl* b = nullptr;
    fcfc_status s = batch_create_impl(p, cats, ncat, pairs, npairs, (hipStream_t)stream, &b);
    if (s == FCFC_OK) *out = (fcfc_batch_t)b;
    return s;
}

extern "C" fcfc_status fcfc_batch_create(fcfc_plan_t plan, const fcfc_catalog* cats, int32_t ncat, void* stream,
                                         fcfc_batch_t* out) {
    clear_error();
    if (ncat < 1 || ncat > (1 << 20)) {
        set_error("batch_create: need 1 .. 2^20 catalogues");
        return FCFC_EINVAL;
    }
    std::vector<int32_t> pairs(2 * (size_t)ncat);
    for (int c = 0; c < ncat; c++) pairs[2 * c] = pairs[2 * c + 1] = c;  // the auto count of every catalogue
    return batch_create(plan, cats, ncat, pairs.data(), ncat, stream, out);
}

extern "C" fcfc_status fcfc_batch_create_pairs(fcfc_plan_t plan, const fcfc_catalog* cats, int32_t ncat,
                                               const int32_t* pairs, int32_t npairs, void* stream,
                                               fcfc_batch_t* out) {
    clear_error();
    if (npairs > (1 << 20)) {
        set_error("batch_create_pairs: at most 2^20 pairs");
        return FCFC_EINVAL;
    }
    return batch_create(plan, cats, ncat, pairs, npairs, stream, out);
}

extern "C" fcfc_status fcfc_batch_run(fcfc_batch_t batch, int64_t* d_counts, double* d_wcounts, int32_t use_graph,
                                      void* stream) {
    clear_error();
    if (!batch || !d_counts) {
        set_error("batch_run: null batch or output");
        return FCFC_EINVAL;
    }
    return batch_run_impl((BatchImpl*)batch, d_counts, d_wcounts, use_graph != 0, (hipStream_t)stream);
}

extern "C" fcfc_status fcfc_batch_check(fcfc_batch_t batch, void* stream, uint32_t* n_items, float* ms) {
    clear_error();
    if (!batch) return FCFC_EINVAL;
    return batch_check_impl((BatchImpl*)batch, (hipStream_t)stream, n_items, ms);
}

extern "C" fcfc_status fcfc_batch_stats(fcfc_batch_t batch, void* stream, int64_t out[3]) {
    clear_error();
    if (!batch || !out) {
        set_error("batch_stats: null batch or output");
        return FCFC_EINVAL;
    }
    return batch_stats_impl((BatchImpl*)batch, (hipStream_t)stream, out);
}

extern "C" void fcfc_batch_free(fcfc_batch_t batch) { batch_free_impl((BatchImpl*)batch); }
