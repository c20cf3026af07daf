// tune.cpp -- the autotuner: picks the tuning knobs of a count (cells per
// prune radius, histogram copies, tile width, look-up table length,
// workgroup size, work order) by timing
// real builds and counts on a sample catalogue.  The analytic cell size and
// its neighbours are always tried; the learned cost model, when given, adds
// the two cell sizes it predicts fastest; measured GPU time decides.  Knobs never change a count.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

using namespace fcfc;

namespace {

struct Ctx {
    int32_t kind, los, n1, n2;
    const double *e1, *e2;
    double L;
    const fcfc_catalog *c1, *c2;
    bool weighted;
    hipStream_t st;
    int64_t* d_counts = nullptr;
    double* d_w = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    fcfc_model_t model = nullptr;
};

// GPU time (ms) of build + count under tuning t: the best of `reps` runs
// (the model is attached when t asks for the learned order).
// Returns FCFC_ERANGE (and leaves *ms alone) where the tuning is not possible.
fcfc_status time_config(Ctx& c, const fcfc_tuning& t, int reps, double* ms) {
    fcfc_plan_t pl = nullptr;
    FCFC_TRY(fcfc_plan_create(c.kind, c.los, c.e1, c.n1, c.e2, c.n2, c.L, &t, &pl));
    fcfc_status s = FCFC_OK;
    if (t.order == FCFC_ORDER_LEARNED) s = fcfc_plan_set_model(pl, c.model);
    if (s == FCFC_OK && c.L <= 0) {
        fcfc_catalog both[2] = {*c.c1, c.c2 ? *c.c2 : fcfc_catalog{nullptr, nullptr, 0}};
        s = fcfc_plan_fit_bounds(pl, both, c.c2 ? 2 : 1, c.st);
    }
    double best = INFINITY;
    for (int r = 0; s == FCFC_OK && r < reps; r++) {
        fcfc_cells_t a = nullptr, b = nullptr;
        if (hipEventRecord(c.ev0, c.st) != hipSuccess) s = FCFC_EHIP;
        if (s == FCFC_OK) s = fcfc_build_cells(pl, c.c1, c.st, &a);
        if (s == FCFC_OK && c.c2) s = fcfc_build_cells(pl, c.c2, c.st, &b);
        if (s == FCFC_OK) s = fcfc_count_pairs(pl, a, b, c.d_counts, c.weighted ? c.d_w : nullptr, c.st);
        if (s == FCFC_OK && hipEventRecord(c.ev1, c.st) != hipSuccess) s = FCFC_EHIP;
        if (s == FCFC_OK && hipEventSynchronize(c.ev1) != hipSuccess) s = FCFC_EHIP;
        float e = 0;
        if (s == FCFC_OK && hipEventElapsedTime(&e, c.ev0, c.ev1) != hipSuccess) s = FCFC_EHIP;
        if (s == FCFC_OK) best = std::min(best, (double)e);
        fcfc_cells_free(a);
        fcfc_cells_free(b);
    }
    fcfc_plan_free(pl);
    if (s == FCFC_OK) *ms = best;
    return s;
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; i++) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Cache signature: library version, device, bins, box, line of sight,
// weighting, and the catalogue sizes rounded to half-octaves.
std::string signature(const Ctx& c, const fcfc_tuning& base) {
    uint64_t h = fnv1a(c.e1, sizeof(double) * (size_t)(c.n1 + 1));
    if (c.e2 && c.n2 > 0) h = fnv1a(c.e2, sizeof(double) * (size_t)(c.n2 + 1), h);
    h = fnv1a(&base, sizeof(base), h);
    char dev[256] = "unknown";
    int d = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&d) == hipSuccess && hipGetDeviceProperties(&prop, d) == hipSuccess)
        snprintf(dev, sizeof(dev), "%s", prop.gcnArchName);
    for (char* q = dev; *q; q++)
        if (*q == ' ' || *q == '\t') *q = '_';
    auto bucket = [](int64_t n) { return n > 0 ? (int)floor(2.0 * log2((double)n)) : -1; };
    char buf[512];
    snprintf(buf, sizeof(buf), "v%d|%s|k%d|l%d|b%d|L%.17g|w%d|n%d|m%d|e%016llx", fcfc_version(), dev, c.kind, c.los,
             c.n1 * 1000 + c.n2, c.L, (int)c.weighted, bucket(c.c1->n), c.c2 ? bucket(c.c2->n) : -1,
             (unsigned long long)h);
    return buf;
}

bool cache_lookup(const char* path, const std::string& sig, fcfc_tuning* t, double* ms) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool hit = false;
    while (fgets(line, sizeof(line), f)) {
        char s[600];
        int k, tile, seg, cop, lut, ord, gw;
        double m;
        if (sscanf(line, "%599s %d %d %d %d %d %d %d %lf", s, &k, &tile, &seg, &cop, &lut, &ord, &gw, &m) == 9 &&
            sig == s && k >= 1 && k <= 8 && (tile == 64 || tile == 128) && seg >= 0 && seg <= 64 &&
            (cop == 1 || cop == 2 || cop == 4) && lut >= 10 && lut <= 15 && ord >= 0 && ord <= 2 && gw >= 0 &&
            gw <= 16 && isfinite(m)) {
            t->order = ord;
            t->group_waves = gw;
            t->cells_per_rmax = k;
            t->tile_points = tile;
            t->seg_cells = seg;
            t->hist_copies = cop;
            t->lut_log2 = lut;
            *ms = m;
            hit = true;  // the last matching line wins
        }
    }
    fclose(f);
    return hit;
}

void cache_store(const char* path, const std::string& sig, const fcfc_tuning& t, double ms) {
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d %d %d %.6f\n", sig.c_str(), t.cells_per_rmax, t.tile_points, t.seg_cells,
            t.hist_copies, t.lut_log2, t.order, t.group_waves, ms);
    fclose(f);
}

}  // namespace

extern "C" fcfc_status fcfc_autotune(fcfc_model_t model, int32_t kind, int32_t los, const double* edges1, int32_t n1,
                                     const double* edges2, int32_t n2, double box_L, const fcfc_tuning* base,
                                     const fcfc_catalog* c1, const fcfc_catalog* c2, int32_t weighted,
                                     const char* cache_path, void* stream, fcfc_tuning* best, double* best_ms,
                                     double* heuristic_ms, int32_t* trials) {
    clear_error();
    if (!c1 || !best || !edges1 || n1 < 1) {
        set_error("autotune: null catalogue, edges or output");
        return FCFC_EINVAL;
    }
    if (weighted && (!c1->w || (c2 && !c2->w))) {
        set_error("autotune: weighted tuning needs weights in every catalogue");
        return FCFC_EINVAL;
    }
    Ctx c{kind, los, n1, n2, edges1, edges2, box_L, c1, c2, weighted != 0, (hipStream_t)stream};
    c.model = model;
    fcfc_tuning t0{};
    if (base) t0 = *base;
    t0.record_timing = 0;
    if (t0.n_hint <= 0) t0.n_hint = (int32_t)std::min<int64_t>(std::max(c1->n, c2 ? c2->n : 0), 0x7fffffff);
    if (trials) *trials = 0;
    if (heuristic_ms) *heuristic_ms = NAN;
    const std::string sig = signature(c, t0);
    double cached = 0;
    fcfc_tuning tc = t0;
    if (cache_path && cache_lookup(cache_path, sig, &tc, &cached)) {
        *best = tc;
        if (best_ms) *best_ms = cached;
        return FCFC_OK;
    }

    // the analytic (heuristic) tuning: every knob left to the library
    int32_t kh = 0;
    FCFC_TRY(fcfc_choose_cells(nullptr, kind, los, edges1, n1, edges2, n2, box_L, &t0, c1, c2, stream, &kh, nullptr));
    // cell sizes to try: the analytic one, its neighbours, and the model's two
    // best (a proposal adds candidates, never takes the neighbours away)
    std::vector<int> ks{kh};
    if (kh > 1) ks.push_back(kh - 1);
    if (kh < 6) ks.push_back(kh + 1);
    if (model) {
        double pred[6];
        int32_t kl = 0;
        FCFC_TRY(fcfc_choose_cells(model, kind, los, edges1, n1, edges2, n2, box_L, &t0, c1, c2, stream, &kl, pred));
        std::vector<int> order;
        for (int k = 1; k <= 6; k++)
            if (isfinite(pred[k - 1])) order.push_back(k);
        std::sort(order.begin(), order.end(), [&](int a, int b) { return pred[a - 1] < pred[b - 1]; });
        for (size_t i = 0; i < order.size() && i < 2; i++) ks.push_back(order[i]);
    }
    std::sort(ks.begin() + 1, ks.end());
    ks.erase(std::unique(ks.begin() + 1, ks.end()), ks.end());

    const int64_t nb = (int64_t)n1 * (kind == FCFC_BIN_S ? 1 : n2);
    if (hipMalloc((void**)&c.d_counts, (size_t)nb * 8) != hipSuccess ||
        (c.weighted && hipMalloc((void**)&c.d_w, (size_t)nb * 8) != hipSuccess)) {
        if (c.d_counts) (void)hipFree(c.d_counts);
        set_error("autotune: cannot allocate %lld histogram bins", (long long)nb);
        return FCFC_ENOMEM;
    }
    fcfc_status s = FCFC_OK;
    if (hipEventCreate(&c.ev0) != hipSuccess || hipEventCreate(&c.ev1) != hipSuccess) s = FCFC_EHIP;
    int ntried = 0;
    fcfc_tuning bt = t0;
    double bms = INFINITY;
    // time t; keep it as the best when faster; returns its time (infinite
    // when the setting is not possible or an error stopped the search)
    auto consider = [&](const fcfc_tuning& t) -> double {
        if (s != FCFC_OK) return INFINITY;
        double ms = INFINITY;
        fcfc_status r = time_config(c, t, 2, &ms);
        ntried++;
        if (r == FCFC_ERANGE) return INFINITY;  // not possible (grid, LDS): skip
        if (r != FCFC_OK) {
            s = r;
            return INFINITY;
        }
        if (ms < bms) {
            bms = ms;
            bt = t;
        }
        return ms;
    };
    // 1. the analytic tuning, then the other cell sizes; the fastest of the
    // analytic size and its neighbours is also kept (the model-free start)
    fcfc_tuning bt_free = t0;
    double bms_free = INFINITY;
    for (size_t i = 0; i < ks.size(); i++) {
        if (i > 0 && ks[i] == kh) continue;
        fcfc_tuning t = t0;
        t.cells_per_rmax = ks[i];
        const double ms = consider(t);
        if (i == 0 && heuristic_ms) *heuristic_ms = ms;
        if (abs(ks[i] - kh) <= 1 && ms < bms_free) {
            bms_free = ms;
            bt_free = t;
        }
    }
    // 2.-6. coordinate descent from a start: histogram copies, tile width,
    // look-up table length, workgroup size and, with a model, the learned order
    auto descend = [&](const fcfc_tuning& start, double start_ms) {
        bt = start;
        bms = start_ms;
        const int copies[2] = {2, 4};
        for (int cp : copies) {
            fcfc_tuning t = bt;
            if ((bt.hist_copies == 0 ? 1 : bt.hist_copies) == cp) continue;
            t.hist_copies = cp;
            consider(t);
        }
        {
            fcfc_tuning t = bt;
            t.tile_points = (bt.tile_points == 64) ? 128 : 64;
            consider(t);
        }
        const int luts[2] = {12, 14};
        for (int lg : luts) {
            fcfc_tuning t = bt;
            if ((bt.lut_log2 == 0 ? 13 : bt.lut_log2) == lg) continue;
            t.lut_log2 = lg;
            consider(t);
        }
        const int gws[3] = {16, 14, 12};
        {
            const fcfc_tuning t1 = bt;
            for (int gw : gws) {
                if (t1.group_waves == gw) continue;
                fcfc_tuning t = t1;
                t.group_waves = gw;
                consider(t);
            }
        }
        if (model && bt.order != FCFC_ORDER_LEARNED) {
            fcfc_tuning t = bt;
            t.order = FCFC_ORDER_LEARNED;
            consider(t);
        }
    };
    descend(bt, bms);
    // A cell size the model proposed may win the first step by timing noise
    // alone; the other knobs are then searched from the model-free start too,
    // so that a model only ever adds candidates to the model-free search.
    if (model && isfinite(bms_free) && bt_free.cells_per_rmax != bt.cells_per_rmax) {
        const fcfc_tuning best_a = bt;
        const double ms_a = bms;
        descend(bt_free, bms_free);
        if (!(bms < ms_a)) {
            bt = best_a;
            bms = ms_a;
        }
    }
    if (c.ev0) (void)hipEventDestroy(c.ev0);
    if (c.ev1) (void)hipEventDestroy(c.ev1);
    (void)hipFree(c.d_counts);
    if (c.d_w) (void)hipFree(c.d_w);
    if (trials) *trials = ntried;
    FCFC_TRY(s);
    if (!isfinite(bms)) {
        set_error("autotune: no tuning could be run");
        return FCFC_ERANGE;
    }
    // make every knob explicit
    if (bt.hist_copies == 0) bt.hist_copies = 1;
    if (bt.tile_points == 0) bt.tile_points = 128;
    if (bt.lut_log2 == 0) bt.lut_log2 = 13;
    *best = bt;
    if (best_ms) *best_ms = bms;
    if (cache_path) cache_store(cache_path, sig, bt, bms);
    return FCFC_OK;
}
