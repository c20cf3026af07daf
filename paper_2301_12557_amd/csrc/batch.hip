// batch.hip -- auto counts of many periodic catalogues in one pipeline.
#include "internal.h"

using namespace fcfc;

extern "C" fcfc_status fcfc_batch_create(fcfc_plan_t plan, const fcfc_catalog* cats, int32_t ncat, void* stream,
                                         fcfc_batch_t* out) {
    (void)plan; (void)cats; (void)ncat; (void)stream; (void)out;
    set_error("batch_create: not available in this build");
    return FCFC_ESTATE;
}
extern "C" fcfc_status fcfc_batch_run(fcfc_batch_t batch, int64_t* d_counts, double* d_wcounts, int32_t use_graph,
                                      void* stream) {
    (void)batch; (void)d_counts; (void)d_wcounts; (void)use_graph; (void)stream;
    set_error("batch_run: not available in this build");
    return FCFC_ESTATE;
}
extern "C" void fcfc_batch_free(fcfc_batch_t batch) { (void)batch; }
