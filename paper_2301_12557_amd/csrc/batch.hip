// batch.hip -- C ABI of the batched pipeline (many periodic catalogues).
#include "internal.h"

using namespace fcfc;

extern "C" fcfc_status fcfc_batch_create(fcfc_plan_t plan, const fcfc_catalog* cats, int32_t ncat, void* stream,
                                         fcfc_batch_t* out) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || !cats || ncat < 1 || !out) {
        set_error("batch_create: null plan, catalogues or output, or ncat < 1");
        return FCFC_EINVAL;
    }
    for (int c = 0; c < ncat; c++) {
        if (cats[c].n < 0 || (cats[c].n > 0 && !cats[c].xyz)) {
            set_error("batch_create: catalogue %d invalid", c);
            return FCFC_EINVAL;
        }
    }
    BatchImpl* b = nullptr;
    fcfc_status s = batch_create_impl(p, cats, ncat, (hipStream_t)stream, &b);
    if (s == FCFC_OK) *out = (fcfc_batch_t)b;
    return s;
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

extern "C" void fcfc_batch_free(fcfc_batch_t batch) { batch_free_impl((BatchImpl*)batch); }
