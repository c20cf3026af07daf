// api.cpp -- C ABI entry points (validation and dispatch).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

using namespace fcfc;

static bool valid_catalog(const fcfc_catalog* c) {
    if (!c || c->n < 0 || c->n > ((int64_t)1 << 31)) return false;
    if (c->n > 0 && !c->xyz) return false;
    return true;
}

extern "C" fcfc_status fcfc_plan_fit_bounds(fcfc_plan_t plan, const fcfc_catalog* cats, int32_t ncat, void* stream) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || !cats || ncat < 1) {
        set_error("fit_bounds: null plan or no catalogues");
        return FCFC_EINVAL;
    }
    if (p->L > 0 || p->grid_set) {
        set_error("fit_bounds: periodic plan or grid already fixed");
        return FCFC_ESTATE;
    }
    for (int i = 0; i < ncat; i++)
        if (!valid_catalog(&cats[i])) {
            set_error("fit_bounds: catalogue %d invalid", i);
            return FCFC_EINVAL;
        }
    return fit_bounds(p, cats, ncat, (hipStream_t)stream);
}

extern "C" fcfc_status fcfc_build_cells(fcfc_plan_t plan, const fcfc_catalog* cat, void* stream, fcfc_cells_t* out) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || !out || !valid_catalog(cat)) {
        set_error("build_cells: null plan/output or invalid catalogue (n must be in [0, 2^31])");
        return FCFC_EINVAL;
    }
    if (!p->grid_set) {
        set_error("build_cells: open-box plan needs fcfc_plan_fit_bounds or fcfc_plan_set_bounds first");
        return FCFC_ESTATE;
    }
    Cells* c = nullptr;
    fcfc_status s = build_cells(p, cat, (hipStream_t)stream, &c);
    if (s == FCFC_OK) *out = (fcfc_cells_t)c;
    return s;
}

extern "C" fcfc_status fcfc_count_pairs(fcfc_plan_t plan, fcfc_cells_t c1, fcfc_cells_t c2, int64_t* d_counts,
                                        double* d_wcounts, void* stream) {
    clear_error();
    Plan* p = (Plan*)plan;
    Cells* a = (Cells*)c1;
    Cells* b = (Cells*)c2;
    if (!p || !a || !d_counts) {
        set_error("count_pairs: null plan, cells or output");
        return FCFC_EINVAL;
    }
    if (a->plan_id != p->id || (b && b->plan_id != p->id)) {
        set_error("count_pairs: cell sets were built on a different plan");
        return FCFC_EGRID;
    }
    fcfc_status s = count_pairs(p, a, b, d_counts, d_wcounts, (hipStream_t)stream);
    if (s == FCFC_OK) {
        p->last_counts = d_counts;
        p->last_counts_n = 0;
    }
    return s;
}

extern "C" fcfc_status fcfc_plan_stats(fcfc_plan_t plan, fcfc_stats* out) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || !out) return FCFC_EINVAL;
    if (!p->have_stats) {
        set_error("plan_stats: no count has run on this plan");
        return FCFC_ESTATE;
    }
    unsigned long long h[8];
    FCFC_HIP(hipMemcpyAsync(h, p->stats_dev, 64, hipMemcpyDeviceToHost, p->last_stream));
    std::vector<int64_t> cnt((size_t)(p->last_counts_n > 0 ? p->last_counts_n : p->nbins));
    if (p->last_counts)
        FCFC_HIP(hipMemcpyAsync(cnt.data(), p->last_counts, cnt.size() * 8, hipMemcpyDeviceToHost, p->last_stream));
    FCFC_HIP(hipStreamSynchronize(p->last_stream));
    float ms = 0;
    if (hipEventElapsedTime(&ms, p->ev0, p->ev1) != hipSuccess) ms = -1;
    p->stats.candidates = (int64_t)h[0];
    p->stats.rechecks = (int64_t)h[1];
    p->stats.flushes = (int64_t)h[6];
    int64_t tot = 0;
    for (int64_t v : cnt) tot += v;
    p->stats.in_range = tot;
    p->stats.kernel_ms = ms;
    if (p->stats.order_used == FCFC_ORDER_LEARNED && h[5] != 0) p->stats.order_used = FCFC_ORDER_HEURISTIC;
    *out = p->stats;
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_weight_scale(double wmin1, double wmax1, double wmin2, double wmax2, int32_t nfactors,
                                         int32_t* S) {
    clear_error();
    if (!S || (nfactors != 2 && nfactors != 3)) {
        set_error("weight_scale: null S or nfactors not 2 or 3");
        return FCFC_EINVAL;
    }
    const double v[4] = {wmin1, wmax1, wmin2, wmax2};
    for (double x : v) {
        if (!(x >= 0.0) || !isfinite(x)) {
            set_error("weight_scale: arguments must be finite and >= 0");
            return FCFC_EINVAL;
        }
    }
    int s = 0;
    FCFC_TRY(weight_scale_rule(wmin1, wmax1, wmin2, wmax2, nfactors, &s));
    *S = s;
    return FCFC_OK;
}

extern "C" void fcfc_cells_free(fcfc_cells_t cells) {
    Cells* c = (Cells*)cells;
    if (!c) return;
    if (c->block) {
        // as hipFree would, wait for all work on the device (counts that read
        // the cell set may still be in flight), then hand the block back to
        // the library's pool; the free completes before this returns, so any
        // stream may reuse the memory
        (void)hipDeviceSynchronize();
        dev_free(c->block, nullptr);
        (void)hipStreamSynchronize(nullptr);
    }
    delete c;
}

extern "C" fcfc_status fcfc_cells_info(fcfc_cells_t cells, int64_t* n_points, int64_t* n_cells) {
    Cells* c = (Cells*)cells;
    if (!c) return FCFC_EINVAL;
    if (n_points) *n_points = c->n;
    if (n_cells) *n_cells = c->tree ? (int64_t)tree_leaves(c) : c->grid.ncell();
    return FCFC_OK;
}
