// plan.cpp -- host-side planning: validation of bins, squared edges, the
// grid, the pruned row stencil, FP32 error bands and the squared-separation
// look-up tables.
#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "internal.h"

namespace fcfc {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

static const double U32 = 5.9604644775390625e-08;  // 2^-24, FP32 unit round-off
// Relative error assumed for the hardware reciprocal and reciprocal square
// root (v_rcp_f32, v_rsq_f32); a GPU test measures the true maximum over the
// inputs the kernels use and checks it stays below this.
static const double TRANS_REL = 4.0 * 1.1920928955078125e-07;
double trans_rel_bound() { return TRANS_REL; }

static std::atomic<uint64_t> g_plan_id{1};

// ---------------------------------------------------------------------------
// stencil of B rows for an A row: (dy, dz) with the smallest distance between
// the two rows below the prune radius, and kx the largest x-index difference
// that can still hold a pair in range (Sect. 2.1: the distance range between
// cells depends only on index differences).
// ---------------------------------------------------------------------------
int stencil_rows(const Plan* p, bool half, std::vector<int4>& rows) {
    rows.clear();
    const Grid& g = p->grid;
    double s = g.side;
    double reff = p->rprune * (1.0 + 1e-7) + 1e-9 * s;
    int K = (int)ceil(reff / s) + 1;
    int Ky = K, Kz = K;
    if (g.L <= 0) {
        Ky = std::min(K, g.ny - 1);
        Kz = std::min(K, g.nz - 1);
    }
    for (int dz = -Kz; dz <= Kz; dz++) {
        for (int dy = -Ky; dy <= Ky; dy++) {
            if (half && (dz < 0 || (dz == 0 && dy < 0))) continue;
            double ty = std::max(abs(dy) - 1, 0) * s;
            double tz = std::max(abs(dz) - 1, 0) * s;
            double t2 = ty * ty + tz * tz;
            if (t2 >= reff * reff) continue;
            const double reach = sqrt(reff * reff - t2) / s;  // largest |dx| of a pair in range, in cells
            const int kx = (int)floor(reach) + 1;
            float rf = (float)reach;
            if ((double)rf < reach) rf = nextafterf(rf, INFINITY);
            int rbits;
            memcpy(&rbits, &rf, 4);
            rows.push_back(make_int4(dy, dz, kx, rbits));
        }
    }
    return (int)rows.size();
}

// Cells per prune radius: the finest grid that still holds about 24 points
// per cell on average (tiles of 64 lanes stay mostly within one or two cells).
int choose_k(const Plan* p, int64_t n_hint) {
    if (p->tune.cells_per_rmax > 0) return std::min(8, p->tune.cells_per_rmax);
    if (n_hint <= 0) return 2;
    double vol;
    if (p->L > 0) {
        vol = p->L * p->L * p->L;
    } else {
        const Grid& g = p->grid;
        vol = std::max(1e-30, (double)g.nx * g.ny * g.nz * g.side * g.side * g.side);
    }
    double rho = (double)n_hint / vol;
    int best = 1;
    for (int k = 1; k <= 6; k++) {
        double side = p->rprune / k;
        if (rho * side * side * side >= 24.0) best = k;
    }
    return best;
}

fcfc_status plan_finalize_grid(Plan* p) {
    Grid& g = p->grid;
    int k = choose_k(p, p->tune.n_hint);
    // cells a hair wider than r/k: with the side exactly r/k, the prune margin
    // would keep one more cell on every side of the stencil (rows whose
    // nearest gap is exactly r could never hold a pair, but cannot be told
    // apart from rows just inside it)
    double target = p->rprune / k * (1.0 + 1e-6);
    const int64_t max_cells = (int64_t)1 << 26;
    if (p->L > 0) {
        int64_t n = (int64_t)floor(p->L / target);
        if (n < 1) n = 1;
        while (n * n * n > max_cells) n--;
        if (n > 1023) n = 1023;
        g.nx = g.ny = g.nz = (int)n;
        g.lo[0] = g.lo[1] = g.lo[2] = 0.0;
        g.side = p->L / (double)n;
        g.L = p->L;
    } else {
        // lo and the extent were stored in lo[] and side (= extent max) by the caller
        double ext[3];
        for (int a = 0; a < 3; a++) ext[a] = p->grid_ext[a];
        double side = target;
        for (;;) {
            int64_t n[3];
            for (int a = 0; a < 3; a++) {
                n[a] = (int64_t)ceil(ext[a] / side);
                if (n[a] < 1) n[a] = 1;
            }
            if (n[0] * n[1] * n[2] <= max_cells && n[0] < 32768 && n[1] < 32768 && n[2] < 32768) {
                g.nx = (int)n[0];
                g.ny = (int)n[1];
                g.nz = (int)n[2];
                break;
            }
            side *= 1.25;
        }
        g.side = side;
        g.L = 0;
    }
    g.k = k;
    return FCFC_OK;
}

// ---------------------------------------------------------------------------
// FP32 error bands.
// Kernel arithmetic for one displacement component (cell-local frame):
//   a' = fl32(x_a - o_A),  b' = fl32(x_b - o_B)         |a'|,|b'| <= side
//   D  = fl32(fl32(dc) * fl32(side)),  dc = unwrapped cell-index difference
//   a'' = fl32(a' - D),  d = fl32(b' - a'')
// For a pair that can matter (|d| <= r, hence |D| <= r + 2 side) each of the
// roundings is bounded by u*|result|, giving
//   |d32 - d| <= u (3 side + 3 (r + 2 side) + r) = u (9 side + 4 r),
// plus FP64 rounding of cell origins (~1e-16 of the coordinates).  The bound
// used is twice that.  The squared quantities built from three (or two)
// components then satisfy |Q32 - Q64| <= 2 sqrt(3) e sqrt(Q) + 3 e^2 + 3.3 u Q.
// ---------------------------------------------------------------------------
static float f32_down(double v) {
    float f = (float)v;
    if ((double)f > v) f = nextafterf(f, -INFINITY);
    return f;
}
static float f32_up(double v) {
    float f = (float)v;
    if ((double)f < v) f = nextafterf(f, INFINITY);
    return f;
}

static fcfc_status build_lut(Lut1D& t, const std::vector<double>& edges, const ErrModel& m,
                             int log2_target) {
    t.n = (int)edges.size() - 1;
    t.E.resize(t.n + 1);
    t.lo.resize(t.n + 1);
    t.hi.resize(t.n + 1);
    double worst = 0;
    for (int k = 0; k <= t.n; k++) {
        double E = edges[k] * edges[k];
        t.E[k] = E;
        if (E == 0.0) {  // no separation is below 0: the edge is never ambiguous
            t.lo[k] = 0.f;
            t.hi[k] = 0.f;
            continue;
        }
        double d0 = m(E);
        double dk = 1.5 * m(E + 2.0 * d0) + 2.0 * E * 1.1920928955078125e-07;
        t.lo[k] = f32_down(E - dk);
        t.hi[k] = f32_up(E + dk);
        if (t.lo[k] < 0.f) t.lo[k] = 0.f;
        worst = std::max(worst, dk / E);
    }
    for (int k = 1; k <= t.n; k++) {
        if (!(t.lo[k] >= t.lo[k - 1]) || !(t.hi[k] >= t.hi[k - 1])) {
            set_error("bin edges too close for FP32 banding near edge %d", k);
            return FCFC_EEDGES;
        }
    }
    t.band_rel = worst;
    t.vmax = t.hi[t.n];
    // scale: a power of two giving at most 2^log2_target entries
    double target = ldexp(1.0, log2_target);
    int e;
    frexp(target / (double)t.vmax, &e);  // target/vmax = f * 2^e, f in [0.5,1)
    double scale = ldexp(1.0, e - 1);     // <= target / vmax
    t.scale = (float)scale;
    int64_t nt = (int64_t)ceil((double)t.vmax * scale) + 1;
    if (nt > 32767) nt = 32767;  // cannot happen with log2_target <= 14
    t.tab.assign((size_t)nt, LUT_NONE);
    for (int64_t j = 0; j < nt; j++) {
        double a = (double)j / scale, b = (double)(j + 1) / scale;  // entry [a, b)
        int klo = -1;
        for (int k = 0; k <= t.n; k++) {
            if (t.hi[k] <= t.lo[k]) continue;  // empty band
            if ((double)t.lo[k] < b && (double)t.hi[k] > a) {
                klo = k;
                break;
            }
        }
        if (klo >= 0) {
            t.tab[j] = lut_hot_code(klo);
        } else {
            int c = 0;
            for (int k = 0; k <= t.n; k++)
                if ((double)t.hi[k] <= a) c = k + 1;
            t.tab[j] = (c >= 1 && c <= t.n) ? (int16_t)(c - 1) : (int16_t)LUT_NONE;
        }
    }
    return FCFC_OK;
}

fcfc_status plan_bin_table(Plan* p, const Lut1D** out) {
    if (p->lutbin.n == 0) {
        // a value rounded to FP32 moves by at most half an ulp; the bands
        // build_lut adds around every edge (2 u of the edge) cover that
        const ErrModel rounding_only;
        const int lg = p->tune.lut_log2 > 0 ? std::min(14, std::max(8, p->tune.lut_log2)) : 14;
        fcfc_status s = build_lut(p->lutbin, p->e1, rounding_only, lg);
        if (s != FCFC_OK) {
            p->lutbin = Lut1D();
            return s;
        }
    }
    *out = &p->lutbin;
    return FCFC_OK;
}

fcfc_status plan_side_table(Plan* p, double e_axis, const Lut1D** out) {
    if (p->luttri.n == 0 || p->luttri_e != e_axis) {
        // |Q32 - Q64| <= 2 sqrt3 e sqrt(Q) + 3 e^2 + 3.3 u Q for a squared
        // length formed by an fma chain from FP32 components each within e of
        // the FP64 ones (the same form as the pair counts' squared separation)
        ErrModel m;
        m.A = 2.0 * sqrt(3.0) * e_axis;
        m.B = 3.0 * e_axis * e_axis;
        m.C = 3.3 * U32 + 1e-15;
        const int lg = p->tune.lut_log2 > 0 ? std::min(14, std::max(8, p->tune.lut_log2)) : 13;
        Lut1D t;
        FCFC_TRY(build_lut(t, p->e1, m, lg));
        p->luttri = t;
        p->luttri_e = e_axis;
    }
    *out = &p->luttri;
    return FCFC_OK;
}

fcfc_status plan_finalize_numerics(Plan* p) {
    const Grid& g = p->grid;
    const double u = U32;
    double r = p->rprune;
    // cell-local coordinates (grid) or leaf-local ones (tree, once a count
    // has met the trees: the largest coordinate relative to a leaf origin)
    double side = ((p->tune.tree_leaf > 0 && p->tree_side > 0) ? p->tree_side : g.side) * (1.0 + 1e-6);
    double coord = std::max(p->coord_max, p->L);
    double e = 2.0 * u * (9.0 * side + 4.0 * r * 1.01) + 8e-16 * (coord + r) * 4.0;
    p->e_axis = e;
    ErrModel d2m;
    d2m.A = 2.0 * sqrt(3.0) * e;
    d2m.B = 3.0 * e * e;
    d2m.C = 3.3 * u + 1e-15;
    int lg = p->tune.lut_log2 > 0 ? std::min(14, std::max(8, p->tune.lut_log2)) : 13;

    // With the default size, larger tables are built too (twice the entries
    // for s and (s, mu); for the (s_perp, pi) pair, whose default tables are
    // half size, four times); a count uses them when they leave as many waves
    // resident.
    const bool big = p->tune.lut_log2 <= 0;
    p->has_big = false;
    p->lut1b = Lut1D();
    p->lut2b = Lut1D();
    if (p->kind == FCFC_BIN_S || p->kind == FCFC_BIN_S_MU) {
        FCFC_TRY(build_lut(p->lut1, p->e1, d2m, lg));
        if (big) FCFC_TRY(build_lut(p->lut1b, p->e1, d2m, lg + 1));
        p->r2prune32 = p->lut1.vmax;
        p->lut2 = Lut1D();
    } else {
        ErrModel m1 = d2m, m2 = d2m;
        if (p->los == FCFC_LOS_MIDPOINT) {
            // Kernel: l = fl(2 fl(x_a) + d) per axis, dot = d.l and ll = |l|^2 by
            // fma chains, pi^2 = fl(fl(dot^2) rcp(ll)).  Per axis l is off by at
            // most el (the rounding of the absolute FP32 coordinate, doubled, the
            // displacement's error e and the rounding of the sum).  With
            // pi = d.l / |l|, d_perp the transverse part of d and |l| >= lmin (twice
            // the distance from the observer to the box), dot32 / |l32| is off by at
            // most
            //   dpi = sqrt3 e + |d_perp| sqrt3 el / (lmin - sqrt3 el) + 3 u r
            // (the displacement error along l; the turn of l, felt only through
            // d_perp; the fma chain).  Squaring, the rounded reciprocal (relative
            // error TRANS_REL), |l32|^2's chain and the product add a relative rel.
            // A pair whose pi decides its bin has s_perp below the top s_perp edge
            // (else the s_perp test drops or rechecks it), and one whose s_perp
            // decides has pi below the top pi edge, so
            //   |pi2_32 - pi^2|     <= (2 dpi pi + dpi^2)(1 + rel) + rel pi^2,
            //   |sp2_32 - s_perp^2| <= the d2 error at d2 <= s_perp^2 + P2, plus the
            //                          pi^2 error at P2, plus the rounding of the
            //                          difference (u s_perp^2).
            // Each of these terms is taken 1.5 times for margin.
            const double M = 1.5;
            const double R = p->coord_max;
            const double el = (2.0 * u * R + e + u * (2.0 * R + r)) * (1.0 + 1e-6);
            const double lmin = 2.0 * p->obs_dist;
            const double lguard = lmin - sqrt(3.0) * el;
            if (!(lguard > 0.5 * lmin)) {
                set_error("mid-point line of sight: the box lies too close to the observer for FP32");
                return FCFC_ERANGE;
            }
            const double sp_max = p->e1.back() * (1.0 + 1e-6);
            const double dpi = (sqrt(3.0) * e + sp_max * sqrt(3.0) * el / lguard + 3.0 * u * r) * (1.0 + 1e-6);
            const double rel = 5.0 * u + TRANS_REL + 1e-12;
            m2.A += M * 2.0 * dpi * (1.0 + rel);
            m2.B += M * dpi * dpi * (1.0 + rel);
            m2.C += M * rel;
            const double P2 = p->e2.back() * p->e2.back() * (1.0 + 1e-3) + 1.0;
            m1.B += M * (d2m.A * sqrt(P2) + d2m.C * P2) +
                    M * ((2.0 * dpi * sqrt(P2) + dpi * dpi) * (1.0 + rel) + rel * P2);
            m1.C += M * u;
        }
        FCFC_TRY(build_lut(p->lut1, p->e1, m1, std::max(8, lg - 1)));
        FCFC_TRY(build_lut(p->lut2, p->e2, m2, std::max(8, lg - 1)));
        if (big) {
            FCFC_TRY(build_lut(p->lut1b, p->e1, m1, std::min(14, lg + 1)));
            FCFC_TRY(build_lut(p->lut2b, p->e2, m2, std::min(14, lg + 1)));
        }
        double S = p->lut1.E[p->n1] + p->lut2.E[p->n2];
        p->r2prune32 = f32_up(S + 1.5 * d2m(S) + 2.0 * S * 1.2e-7);
    }
    // mu band: tol(mu*n) = n (A/s + B/s^2 + C) with 1/s taken from rsq(d2)
    if (p->kind == FCFC_BIN_S_MU) {
        double n = p->n2;
        if (p->los == FCFC_LOS_Z) {
            p->mu_tolA = (float)(2.0 * n * (1.0 + sqrt(3.0)) * e);
            p->mu_tolB = (float)(2.0 * n * 1.5 * e * e);
            p->mu_tolC = (float)(2.0 * n * (TRANS_REL + 4.0 * u));
        } else {
            double R = p->coord_max;
            double el = 2.0 * (2.0 * u * R + e + u * (2.0 * R + r)) * 2.0;
            double lmin = 2.0 * p->obs_dist;
            p->mu_tolA = (float)(2.0 * n * 2.0 * sqrt(3.0) * e);
            p->mu_tolB = (float)(2.0 * n * 1.5 * e * e);
            p->mu_tolC = (float)(2.0 * n * (2.0 * sqrt(3.0) * el / lmin + 2.0 * TRANS_REL + 8.0 * u));
        }
        // below this separation the mu band is wide: always recheck
        p->d2small = (float)std::max(1e-30, (64.0 * e) * (64.0 * e));
        // The kernel evaluates the band as A' rs + C with one fma: for every pair
        // it does not recheck, d2 >= d2small, so B rs^2 <= (B / sqrt(d2small)) rs.
        const double Aeff = ((double)p->mu_tolA + (double)p->mu_tolB / sqrt((double)p->d2small)) * (1.0 + 1e-6);
        p->mu_tolA = f32_up(Aeff);
        p->mu_tolB = 0.f;
    } else {
        p->d2small = 0.f;
    }
    p->has_big = big;
    p->numerics_ready = true;
    p->stats.band_d2_rel = std::max(p->lut1.band_rel, p->lut2.band_rel);
    p->stats.lut_entries = (int32_t)p->lut1.tab.size();
    return FCFC_OK;
}

}  // namespace fcfc

using namespace fcfc;

extern "C" const char* fcfc_last_error(void) { return fcfc::last_error(); }

extern "C" const char* fcfc_status_str(fcfc_status s) {
    switch (s) {
        case FCFC_OK: return "ok";
        case FCFC_EINVAL: return "invalid argument";
        case FCFC_ENOMEM: return "out of memory";
        case FCFC_EBOX: return "point outside the box";
        case FCFC_ENONFINITE: return "non-finite position or weight";
        case FCFC_ERANGE: return "value out of supported range";
        case FCFC_EEDGES: return "invalid bin edges";
        case FCFC_EGRID: return "cell sets built on different plans";
        case FCFC_EHIP: return "HIP runtime error";
        case FCFC_EMODEL: return "scheduler model unusable";
        case FCFC_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

extern "C" int32_t fcfc_version(void) { return 1; }

static bool strictly_increasing(const double* e, int n) {
    for (int k = 0; k <= n; k++) {
        if (!isfinite(e[k]) || e[k] < 0) return false;
        if (k > 0 && !(e[k] > e[k - 1])) return false;
    }
    return true;
}

extern "C" fcfc_status fcfc_plan_create(int32_t kind, int32_t los, const double* edges1, int32_t n1,
                                        const double* edges2, int32_t n2, double box_L,
                                        const fcfc_tuning* tune, fcfc_plan_t* out) {
    clear_error();
    if (!out || !edges1 || n1 < 1 || n1 > 32000) {
        set_error("plan_create: null output, missing edges1 or n1 out of [1,32000]");
        return FCFC_EINVAL;
    }
    if (kind < FCFC_BIN_S || kind > FCFC_BIN_SPERP_PI || los < FCFC_LOS_Z || los > FCFC_LOS_MIDPOINT) {
        set_error("plan_create: unknown kind %d or line of sight %d", kind, los);
        return FCFC_EINVAL;
    }
    if (kind != FCFC_BIN_S && (!edges2 || n2 < 1 || n2 > 32000)) {
        set_error("plan_create: edges2 required with n2 in [1,32000]");
        return FCFC_EINVAL;
    }
    if (!(box_L >= 0) || !isfinite(box_L)) {
        set_error("plan_create: box_L must be finite and >= 0");
        return FCFC_EINVAL;
    }
    if (tune && tune->tree_leaf != 0 && (tune->tree_leaf < 32 || tune->tree_leaf > 128 || box_L > 0)) {
        set_error("plan_create: tree_leaf must be 0 or 32..128, and trees need an open box");
        return FCFC_EINVAL;
    }
    if (kind == FCFC_BIN_S) los = FCFC_LOS_Z;
    if (box_L > 0 && los == FCFC_LOS_MIDPOINT) {
        set_error("plan_create: the mid-point line of sight needs an open box");
        return FCFC_EINVAL;
    }
    if (!strictly_increasing(edges1, n1)) {
        set_error("plan_create: edges1 must be finite, >= 0 and strictly increasing");
        return FCFC_EEDGES;
    }
    if (kind != FCFC_BIN_S && !strictly_increasing(edges2, n2)) {
        set_error("plan_create: edges2 must be finite, >= 0 and strictly increasing");
        return FCFC_EEDGES;
    }
    if (kind == FCFC_BIN_S_MU) {
        for (int j = 0; j <= n2; j++) {
            if (edges2[j] != (double)j / (double)n2) {
                set_error("plan_create: mu edges must be k/n2 (uniform over [0,1]); edge %d is %.17g", j,
                          edges2[j]);
                return FCFC_EEDGES;
            }
        }
    }
    Plan* p = new (std::nothrow) Plan();
    if (!p) return FCFC_ENOMEM;
    p->kind = kind;
    p->los = los;
    p->n1 = n1;
    p->n2 = (kind == FCFC_BIN_S) ? 1 : n2;
    p->nbins = p->n1 * p->n2;
    p->e1.assign(edges1, edges1 + n1 + 1);
    if (kind != FCFC_BIN_S) p->e2.assign(edges2, edges2 + n2 + 1);
    p->L = box_L;
    if (tune) p->tune = *tune;
    // Work items hold at most 128 A points x b_chunk B points, and a wavefront
    // empties the LDS histograms after claiming 2^flush_log2 <= 2^26 pairs, so
    // the up to 16 wavefronts of a workgroup add at most
    // 16 (2^26 + 2^7 2^19) = 2^31 increments to a 32-bit LDS counter between
    // two merges.
    if (p->tune.b_chunk != 0 && (p->tune.b_chunk < 256 || p->tune.b_chunk > (1 << 19))) {
        delete p;
        set_error("plan_create: b_chunk must be 0 or lie in [256, 2^19]");
        return FCFC_EINVAL;
    }
    if (p->tune.flush_log2 < 0 || p->tune.flush_log2 > 26) {
        delete p;
        set_error("plan_create: flush_log2 must lie in [0, 26]");
        return FCFC_EINVAL;
    }
    if (p->tune.shard_count < 0 || (p->tune.shard_count > 1 &&
                                    (p->tune.shard_index < 0 || p->tune.shard_index >= p->tune.shard_count))) {
        delete p;
        set_error("plan_create: shard_index must lie in [0, shard_count)");
        return FCFC_EINVAL;
    }
    if (kind == FCFC_BIN_SPERP_PI)
        p->rprune = sqrt(edges1[n1] * edges1[n1] + edges2[n2] * edges2[n2]) * (1.0 + 1e-12);
    else
        p->rprune = edges1[n1];
    if (!(p->rprune > 0)) {
        delete p;
        set_error("plan_create: largest separation must be > 0");
        return FCFC_EEDGES;
    }
    p->id = g_plan_id.fetch_add(1);
    // histogram in LDS: counts (4 B x copies) + weighted limbs (16 B) must fit
    int64_t lds_hist = (int64_t)p->nbins * 4;
    if (lds_hist > 96 * 1024) {
        delete p;
        set_error("plan_create: %d bins do not fit the LDS histogram (max %d)", p->nbins, 96 * 1024 / 4);
        return FCFC_ERANGE;
    }
    if (box_L > 0) {
        if (p->rprune > 0.5 * box_L) {
            delete p;
            set_error("plan_create: prune radius %.17g exceeds L/2 = %.17g", p->rprune, 0.5 * box_L);
            return FCFC_ERANGE;
        }
        p->coord_max = box_L;
        fcfc_status s = plan_finalize_grid(p);
        if (s == FCFC_OK) s = plan_finalize_numerics(p);
        if (s != FCFC_OK) {
            delete p;
            return s;
        }
        p->grid_set = true;
    }
    *out = (fcfc_plan_t)p;
    return FCFC_OK;
}

fcfc_status fcfc::weight_scale_rule(double wmin1, double wmax1, double wmin2, double wmax2, int nfactors, int* S) {
    *S = 0;
    if (nfactors == 3) {
        wmin2 = wmin1;
        wmax2 = wmax1;
    }
    if (!(wmin1 > 0 && wmin2 > 0)) return FCFC_OK;  // every product is zero
    // products of FP64 weights are rounded, and rounding is monotone, so the
    // smallest and largest non-zero magnitudes are these (pairs: a b;
    // triangles: fl(fl(a b) c))
    const double pmin = nfactors == 3 ? (wmin1 * wmin1) * wmin1 : wmin1 * wmin2;
    const double pmax = nfactors == 3 ? (wmax1 * wmax1) * wmax1 : wmax1 * wmax2;
    if (!(pmax <= DBL_MAX)) {
        set_error("weights: the largest weight product overflows FP64 (max |w| %.3g)", wmax1);
        return FCFC_ERANGE;
    }
    if (!(pmin >= DBL_MIN)) {
        // a zero or subnormal product has lost bits: no common scale makes
        // every product an integer without rounding it
        set_error("weights: the smallest weight product underflows FP64 (min non-zero |w| %.3g and %.3g)", wmin1,
                  wmin2);
        return FCFC_ERANGE;
    }
    // pmin = f 2^e with f in [0.5, 1): every product >= pmin is a multiple of
    // ulp(pmin) = 2^(e - 53), so it becomes an integer once scaled by 2^(53 - e)
    int e = 0;
    frexp(pmin, &e);
    const int s = 53 - e;
    if (s > 1023) {
        set_error("weights: products near %.3g need a scale 2^%d beyond FP64", pmin, s);
        return FCFC_ERANGE;
    }
    if (!(ldexp(pmax, s) < ldexp(1.0, 62))) {
        set_error("weights: dynamic range too wide for exact accumulation (max/min weight product %.3g)",
                  pmax / pmin);
        return FCFC_ERANGE;
    }
    *S = s;
    return FCFC_OK;
}

fcfc_status fcfc::fcfc_set_bounds_internal(Plan* p, const double lo[3], const double hi[3]) {
    for (int a = 0; a < 3; a++) {
        if (!isfinite(lo[a]) || !isfinite(hi[a]) || !(hi[a] >= lo[a])) {
            set_error("bounds must be finite with hi >= lo");
            return FCFC_EINVAL;
        }
    }
    double cmax = 0, d2 = 0;
    for (int a = 0; a < 3; a++) {
        cmax = std::max(cmax, std::max(fabs(lo[a]), fabs(hi[a])));
        double c = 0;
        if (lo[a] > 0) c = lo[a];
        else if (hi[a] < 0) c = -hi[a];
        d2 += c * c;
    }
    p->coord_max = cmax;
    p->obs_dist = sqrt(d2);
    if (p->los == FCFC_LOS_MIDPOINT && p->kind != FCFC_BIN_S && !(p->obs_dist > 1e-3 * (cmax + 1.0))) {
        set_error("mid-point line of sight: the origin (observer) must lie outside the catalogue box");
        return FCFC_ERANGE;
    }
    for (int a = 0; a < 3; a++) {
        p->grid.lo[a] = lo[a];
        p->grid_ext[a] = hi[a] - lo[a];
        p->grid_hi[a] = hi[a];
    }
    fcfc_status s = plan_finalize_grid(p);
    if (s == FCFC_OK) s = plan_finalize_numerics(p);
    if (s != FCFC_OK) return s;
    p->grid_set = true;
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_plan_set_bounds(fcfc_plan_t plan, const double lo[3], const double hi[3]) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || !lo || !hi) return FCFC_EINVAL;
    if (p->L > 0 || p->grid_set) {
        set_error("set_bounds: periodic plan or grid already fixed");
        return FCFC_ESTATE;
    }
    return fcfc_set_bounds_internal(p, lo, hi);
}

extern "C" fcfc_status fcfc_plan_numerics(fcfc_plan_t plan, fcfc_numerics* out) {
    clear_error();
    const Plan* p = (const Plan*)plan;
    if (!p || !out) return FCFC_EINVAL;
    if (!p->numerics_ready) {
        set_error("plan_numerics: the grid is not fixed yet (set or fit the bounds first)");
        return FCFC_ESTATE;
    }
    fcfc_numerics n{};
    n.nx = p->grid.nx;
    n.ny = p->grid.ny;
    n.nz = p->grid.nz;
    n.cells_per_rmax = p->grid.k;
    for (int a = 0; a < 3; a++) n.lo[a] = p->L > 0 ? 0.0 : p->grid.lo[a];
    n.side = p->grid.side;
    n.e_axis = p->e_axis;
    n.side32 = (float)p->grid.side;
    n.r2prune32 = p->r2prune32;
    n.d2small = p->d2small;
    n.mu_tolA = p->mu_tolA;
    n.mu_tolC = p->mu_tolC;
    n.trans_rel = (float)trans_rel_bound();
    n.has_big = p->has_big ? 1 : 0;
    *out = n;
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_plan_table(fcfc_plan_t plan, int32_t which, double* E, float* lo, float* hi,
                                       int16_t* tab, int64_t cap, int64_t* n_entries, float* scale, float* vmax) {
    clear_error();
    const Plan* p = (const Plan*)plan;
    if (!p) return FCFC_EINVAL;
    if (!p->numerics_ready) {
        set_error("plan_table: the grid is not fixed yet (set or fit the bounds first)");
        return FCFC_ESTATE;
    }
    const Lut1D* t = nullptr;
    switch (which) {
        case 0: t = &p->lut1; break;
        case 1: t = &p->lut2; break;
        case 2: t = p->has_big ? &p->lut1b : nullptr; break;
        case 3: t = p->has_big ? &p->lut2b : nullptr; break;
        default: break;
    }
    if (!t || t->n == 0) {
        set_error("plan_table: no table %d in this plan", which);
        return FCFC_EINVAL;
    }
    if (E) memcpy(E, t->E.data(), sizeof(double) * (size_t)(t->n + 1));
    if (lo) memcpy(lo, t->lo.data(), sizeof(float) * (size_t)(t->n + 1));
    if (hi) memcpy(hi, t->hi.data(), sizeof(float) * (size_t)(t->n + 1));
    const int64_t nt = (int64_t)t->tab.size();
    if (tab && cap > 0) memcpy(tab, t->tab.data(), sizeof(int16_t) * (size_t)std::min(cap, nt));
    if (n_entries) *n_entries = nt;
    if (scale) *scale = t->scale;
    if (vmax) *vmax = t->vmax;
    return FCFC_OK;
}

extern "C" void fcfc_plan_free(fcfc_plan_t plan) {
    Plan* p = (Plan*)plan;
    if (!p) return;
    if (p->stats_dev) (void)hipFree(p->stats_dev);
    if (p->timing_dev) (void)hipFree(p->timing_dev);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    delete p;
}
