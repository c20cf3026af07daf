/*
 * fcfc_oracle.c -- CPU reference ("oracle") for exact pair counting.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * definition that the GPU library is checked against.  Nothing in the product
 * path may link, load or call it; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark do.  It shares no code, header or table
 * with the HIP library.
 *
 * What is computed (Zhao, "Fast Correlation Function Calculator", FCFC):
 *   for every pair of points -- each unordered pair once for an auto count
 *   (Sect. 3.1, the de-duplication of node pairs of the same tree), every
 *   ordered pair (i in cat1, j in cat2) for a cross count -- form the
 *   separation quantities of Sect. 2.5:
 *       s = |s2 - s1|,  pi = |s.l| / |l|,  sigma = sqrt(s^2 - pi^2),  mu = pi/s,
 *   with l = s1 + s2 (observational line of sight) or l = e_z (simulation
 *   line of sight), and add the pair to the histogram bin whose half-open
 *   interval contains it.  Bins are compared through squared edges
 *   (Sect. 3.2.1: squared distances against pre-computed squared edges,
 *   zero-based bin indices, s_min^2 <= s^2 < s_max^2 as in the linear and
 *   logarithmic index maps of Sect. 3.2.2).
 *
 * Readings where the paper is silent (the same readings the GPU path follows):
 *   - Every operation is IEEE-754 binary64, round to nearest even, evaluated
 *     exactly in the order written below, with no fused multiply-add (this
 *     file must be compiled with -ffp-contract=off).
 *   - Periodic boxes use the minimum image per axis:
 *       h = L/2; if (d > h) d -= L; else if (d < -h) d += L.
 *     (Sect. 3.1 only states that wrap offsets are applied per node pair.)
 *   - d2 = (dx*dx + dy*dy) + dz*dz.
 *   - s bin k:   E[k] <= d2 < E[k+1], E[k] = e[k]*e[k].
 *   - mu bin:    mu is never formed; with M[j] = m[j]*m[j] and PI2 the squared
 *                line-of-sight separation, the bin is the largest j in [0,n]
 *                with M[j]*d2 <= PI2.  j == n means mu >= m[n]: such a pair
 *                belongs to the last bin when m[n] == 1 (mu = 1 is kept), and
 *                is dropped otherwise.  d2 == 0 gives mu = 0.
 *   - PI2 = dz*dz for the z line of sight;  for the mid-point line of sight
 *                l = s1 + s2,  dot = (dx*lx + dy*ly) + dz*lz,
 *                ll = (lx*lx + ly*ly) + lz*lz,  PI2 = (dot*dot)/ll (0 if ll==0).
 *   - sigma^2:   dx*dx + dy*dy for the z line of sight; d2 - PI2 clamped at 0
 *                for the mid-point line of sight.
 *   - pair weight = w_i * w_j (one FP64 product); a bin's weighted count is the
 *     exact real sum of those products rounded once to FP64.  The sum is kept
 *     exactly in 128-bit fixed point (every product is an integer multiple of
 *     a common power of two) and rounded to nearest-even at the end.
 *
 * Two counters are provided: a brute-force O(N1*N2) double loop, and a plain
 * cell-list version that only skips cells that cannot hold a pair in range and
 * classifies every remaining pair with the very same per-pair function.
 *
 * Parity status: every function here is pinned by tests against hand-computed
 * cases, lattice closed forms, exact counting identities, uniform-box
 * statistics, an independent library neighbour counter and exactly rounded
 * sums (tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KIND_S 0
#define ORC_KIND_S_MU 1
#define ORC_KIND_SPERP_PI 2
#define ORC_LOS_Z 0
#define ORC_LOS_MID 1

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_EOVERFLOW -3

typedef struct {
    int kind, los;
    double L;             /* > 0: periodic cube [0,L)^3;  0: open */
    double *E1;           /* n1+1 squared edges of the first dimension (s or sigma) */
    int n1;
    double *E2;           /* n2+1 squared edges of the second dimension (mu or pi) */
    int n2;
    int mu_top_closed;    /* last mu edge is exactly 1 */
} orc_spec;

/* Bin of a squared quantity v against squared edges E[0..n]:
 * k with E[k] <= v < E[k+1], or -1.  Reverse traversal (Sect. 3.2.1). */
static int orc_bin(const double *E, int n, double v)
{
    if (!(v >= E[0]) || v >= E[n]) return -1;
    for (int k = n - 1; k >= 0; k--)
        if (v >= E[k]) return k;
    return -1;
}

/* mu bin from the squared forms described in the header. */
static int orc_mu_bin(const orc_spec *sp, double d2, double pi2)
{
    const double *M = sp->E2;
    int n = sp->n2;
    if (d2 == 0.0) {
        /* mu = 0 */
        if (M[0] <= 0.0) return 0;
        return -1;
    }
    int j = -1;
    for (int t = n; t >= 0; t--) {
        if (M[t] * d2 <= pi2) { j = t; break; }
    }
    if (j < 0) return -1;
    if (j == n) return sp->mu_top_closed ? n - 1 : -1;
    return j;
}

/* Flat bin index (row-major [n1][n2], or [n1] for s) of the pair (i, j), or -1.
 * (xi,yi,zi) is the point of the first catalogue, (xj,yj,zj) of the second. */
static long orc_classify(const orc_spec *sp, double xi, double yi, double zi,
                         double xj, double yj, double zj)
{
    double dx = xj - xi;
    double dy = yj - yi;
    double dz = zj - zi;
    if (sp->L > 0.0) {
        double L = sp->L;
        double h = L * 0.5;
        if (dx > h) dx -= L; else if (dx < -h) dx += L;
        if (dy > h) dy -= L; else if (dy < -h) dy += L;
        if (dz > h) dz -= L; else if (dz < -h) dz += L;
    }
    double d2 = (dx * dx + dy * dy) + dz * dz;

    double pi2 = 0.0;
    if (sp->kind != ORC_KIND_S) {
        if (sp->los == ORC_LOS_Z) {
            pi2 = dz * dz;
        } else {
            double lx = xi + xj;
            double ly = yi + yj;
            double lz = zi + zj;
            double dot = (dx * lx + dy * ly) + dz * lz;
            double ll = (lx * lx + ly * ly) + lz * lz;
            pi2 = (ll > 0.0) ? (dot * dot) / ll : 0.0;
        }
    }

    if (sp->kind == ORC_KIND_S) {
        return orc_bin(sp->E1, sp->n1, d2);
    }
    if (sp->kind == ORC_KIND_S_MU) {
        int k = orc_bin(sp->E1, sp->n1, d2);
        if (k < 0) return -1;
        int j = orc_mu_bin(sp, d2, pi2);
        if (j < 0) return -1;
        return (long)k * sp->n2 + j;
    }
    /* sigma, pi */
    double sp2;
    if (sp->los == ORC_LOS_Z) {
        sp2 = dx * dx + dy * dy;
    } else {
        sp2 = d2 - pi2;
        if (sp2 < 0.0) sp2 = 0.0;
    }
    int k = orc_bin(sp->E1, sp->n1, sp2);
    if (k < 0) return -1;
    int j = orc_bin(sp->E2, sp->n2, pi2);
    if (j < 0) return -1;
    return (long)k * sp->n2 + j;
}

/* ---------------------------------------------------------------------------
 * Exact weighted sums.  With pmin the smallest non-zero |w_i*w_j| that can
 * occur (the product of the smallest non-zero |weights|, rounded: rounding is
 * monotone), every non-zero product p has ulp(p) >= 2^(e-53) where
 * pmin = f*2^e, f in [0.5,1).  Hence p * 2^S is an integer for S = 53 - e, and
 * an __int128 sum of those integers is exact while it fits.
 * ------------------------------------------------------------------------- */
static double orc_min_abs_nonzero(const double *w, int64_t n)
{
    double m = INFINITY;
    for (int64_t i = 0; i < n; i++) {
        double a = fabs(w[i]);
        if (a > 0.0 && a < m) m = a;
    }
    return m;
}

static double orc_max_abs(const double *w, int64_t n)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double a = fabs(w[i]);
        if (a > m) m = a;
    }
    return m;
}

/* round-to-nearest-even of the exact value q * 2^(-S) */
static double orc_i128_to_double(__int128 q, int S)
{
    if (q == 0) return 0.0;
    int neg = q < 0;
    unsigned __int128 m = neg ? (unsigned __int128)(-(q + 1)) + 1u : (unsigned __int128)q;
    int nbits = 0;
    for (unsigned __int128 t = m; t != 0; t >>= 1) nbits++;
    double r;
    if (nbits <= 53) {
        r = ldexp((double)(uint64_t)m, -S);
    } else {
        int sh = nbits - 53;
        unsigned __int128 top = m >> sh;
        unsigned __int128 rem = m - (top << sh);
        unsigned __int128 half = (unsigned __int128)1 << (sh - 1);
        if (rem > half || (rem == half && (top & 1u))) top += 1u;
        r = ldexp((double)(uint64_t)top, sh - S);
    }
    return neg ? -r : r;
}

typedef struct {
    int weighted;
    int S;              /* fixed-point scale exponent */
    double two_S;       /* 2^S */
} orc_wspec;

static int orc_prepare_weights(orc_wspec *ws, const double *w1, int64_t n1,
                               const double *w2, int64_t n2, double npairs)
{
    ws->weighted = 1;
    double m1 = orc_min_abs_nonzero(w1, n1), m2 = orc_min_abs_nonzero(w2, n2);
    double M1 = orc_max_abs(w1, n1), M2 = orc_max_abs(w2, n2);
    if (!isfinite(M1) || !isfinite(M2)) return ORC_EINVAL;
    if (isinf(m1) || isinf(m2)) { /* all weights zero: every product is 0 */
        ws->S = 0; ws->two_S = 1.0; return ORC_OK;
    }
    double pmin = m1 * m2;
    if (pmin == 0.0) return ORC_EINVAL;   /* products would underflow */
    int e;
    frexp(pmin, &e);
    ws->S = 53 - e;
    ws->two_S = ldexp(1.0, ws->S);
    /* every |p * 2^S| <= M1*M2*2^S; the bin sum must stay below 2^126 */
    double bound = (M1 * M2) * ws->two_S * (npairs + 1.0);
    if (!(bound < ldexp(1.0, 126))) return ORC_EOVERFLOW;
    return ORC_OK;
}

static int orc_spec_init(orc_spec *sp, int kind, int los, double L,
                         const double *e1, int n1, const double *e2, int n2)
{
    memset(sp, 0, sizeof(*sp));
    if (kind < 0 || kind > 2 || los < 0 || los > 1 || n1 < 1) return ORC_EINVAL;
    if (!(L >= 0.0) || !isfinite(L)) return ORC_EINVAL;
    if (kind != ORC_KIND_S && (n2 < 1 || !e2)) return ORC_EINVAL;
    if (L > 0.0 && los == ORC_LOS_MID && kind != ORC_KIND_S) return ORC_EINVAL;
    sp->kind = kind; sp->los = los; sp->L = L; sp->n1 = n1;
    sp->n2 = (kind == ORC_KIND_S) ? 1 : n2;
    sp->E1 = (double *)malloc(sizeof(double) * (size_t)(n1 + 1));
    sp->E2 = (double *)malloc(sizeof(double) * (size_t)(sp->n2 + 1));
    if (!sp->E1 || !sp->E2) return ORC_ENOMEM;
    for (int k = 0; k <= n1; k++) {
        if (!(e1[k] >= 0.0) || !isfinite(e1[k])) return ORC_EINVAL;
        if (k > 0 && !(e1[k] > e1[k - 1])) return ORC_EINVAL;
        sp->E1[k] = e1[k] * e1[k];
    }
    if (kind == ORC_KIND_S) {
        sp->E2[0] = 0.0; sp->E2[1] = 1.0;
    } else {
        for (int k = 0; k <= n2; k++) {
            if (!(e2[k] >= 0.0) || !isfinite(e2[k])) return ORC_EINVAL;
            if (k > 0 && !(e2[k] > e2[k - 1])) return ORC_EINVAL;
            if (kind == ORC_KIND_S_MU && e2[k] > 1.0) return ORC_EINVAL;
            sp->E2[k] = e2[k] * e2[k];
        }
        sp->mu_top_closed = (kind == ORC_KIND_S_MU && e2[n2] == 1.0);
    }
    return ORC_OK;
}

static void orc_spec_free(orc_spec *sp)
{
    free(sp->E1); free(sp->E2);
    sp->E1 = sp->E2 = NULL;
}

/* Per-thread accumulators, summed at the end. */
typedef struct {
    int64_t *cnt;
    __int128 *wsum;
} orc_acc;

static int orc_acc_alloc(orc_acc *a, long nbins, int weighted)
{
    a->cnt = (int64_t *)calloc((size_t)nbins, sizeof(int64_t));
    a->wsum = weighted ? (__int128 *)calloc((size_t)nbins, sizeof(__int128)) : NULL;
    return (a->cnt && (!weighted || a->wsum)) ? ORC_OK : ORC_ENOMEM;
}

static inline void orc_acc_add(orc_acc *a, const orc_wspec *ws, long b,
                               double wi, double wj)
{
    a->cnt[b] += 1;
    if (ws->weighted) {
        double p = wi * wj;
        a->wsum[b] += (__int128)(p * ws->two_S);
    }
}

static int orc_check_points(const double *x, int64_t n, double L)
{
    for (int64_t i = 0; i < 3 * n; i++) {
        if (!isfinite(x[i])) return ORC_EINVAL;
        if (L > 0.0 && !(x[i] >= 0.0 && x[i] < L)) return ORC_EINVAL;
    }
    return ORC_OK;
}

static int orc_finish(orc_acc *acc, int nth, long nbins, const orc_wspec *ws,
                      int64_t *counts, double *wcounts)
{
    for (long b = 0; b < nbins; b++) {
        int64_t c = 0;
        __int128 s = 0;
        for (int t = 0; t < nth; t++) {
            c += acc[t].cnt[b];
            if (ws->weighted) s += acc[t].wsum[b];
        }
        counts[b] = c;
        if (ws->weighted && wcounts) wcounts[b] = orc_i128_to_double(s, ws->S);
    }
    return ORC_OK;
}

static void orc_acc_free(orc_acc *acc, int nth)
{
    for (int t = 0; t < nth; t++) { free(acc[t].cnt); free(acc[t].wsum); }
    free(acc);
}

/* ---------------------------------------------------------------------------
 * Brute force.  is_auto != 0: pairs i < j of catalogue 1 (x2/w2/n2 ignored).
 * Otherwise every (i, j), i in catalogue 1, j in catalogue 2.
 * Weighted iff wcounts != NULL (then w1, and w2 for a cross count, are given).
 * Outputs are overwritten.  Returns 0 or a negative error code.
 * ------------------------------------------------------------------------- */
int oracle_count_brute(const double *x1, const double *w1, int64_t n1,
                       const double *x2, const double *w2, int64_t n2,
                       int is_auto, int kind, int los, double L,
                       const double *e1, int nb1, const double *e2, int nb2,
                       int64_t *counts, double *wcounts, int nthreads)
{
    orc_spec sp;
    int rc = orc_spec_init(&sp, kind, los, L, e1, nb1, e2, nb2);
    if (rc) { orc_spec_free(&sp); return rc; }
    if (is_auto) { x2 = x1; w2 = w1; n2 = n1; }
    if (n1 < 0 || n2 < 0 || (n1 > 0 && !x1) || (n2 > 0 && !x2)) { orc_spec_free(&sp); return ORC_EINVAL; }
    if (orc_check_points(x1, n1, L) || orc_check_points(x2, n2, L)) { orc_spec_free(&sp); return ORC_EINVAL; }
    long nbins = (long)sp.n1 * sp.n2;
    orc_wspec ws = {0, 0, 1.0};
    if (wcounts) {
        if (!w1 || !w2) { orc_spec_free(&sp); return ORC_EINVAL; }
        rc = orc_prepare_weights(&ws, w1, n1, w2, n2, (double)n1 * (double)n2);
        if (rc) { orc_spec_free(&sp); return rc; }
    }
    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    orc_acc *acc = (orc_acc *)calloc((size_t)nth, sizeof(orc_acc));
    if (!acc) { orc_spec_free(&sp); return ORC_ENOMEM; }
    for (int t = 0; t < nth; t++)
        if (orc_acc_alloc(&acc[t], nbins, ws.weighted)) { orc_acc_free(acc, nth); orc_spec_free(&sp); return ORC_ENOMEM; }

#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
    for (int64_t i = 0; i < n1; i++) {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double xi = x1[3 * i], yi = x1[3 * i + 1], zi = x1[3 * i + 2];
        double wi = ws.weighted ? w1[i] : 0.0;
        int64_t j0 = is_auto ? i + 1 : 0;
        for (int64_t j = j0; j < n2; j++) {
            long b = orc_classify(&sp, xi, yi, zi, x2[3 * j], x2[3 * j + 1], x2[3 * j + 2]);
            if (b >= 0) orc_acc_add(&acc[t], &ws, b, wi, ws.weighted ? w2[j] : 0.0);
        }
    }
    orc_finish(acc, nth, nbins, &ws, counts, wcounts);
    orc_acc_free(acc, nth);
    orc_spec_free(&sp);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Plain cell list (Sect. 2.1: axis-aligned cells, points grouped per cell).
 * Cell side >= cell_size; a point's neighbour cells are all cells within
 * ceil(r_prune / side) + 1 cells per axis (wrapped and de-duplicated for a
 * periodic box), where r_prune = s_max, or sqrt(sigma_max^2 + pi_max^2).  This
 * holds every partner in range with a whole cell of margin.  A neighbour cell
 * is skipped when the point's distance to it exceeds r_prune (the pruning of
 * node pairs whose minimum separation is beyond the largest edge, Sect. 3.1):
 * per axis the gap between the point's coordinate and the cell's slab, the
 * smallest over every wrap offset that reaches the cell; the test keeps a
 * relative margin of 1e-9 for the rounding of the slab bounds and of the
 * pair's own separation.  Every remaining candidate is classified by the same
 * per-pair function as the brute force.
 * ------------------------------------------------------------------------- */
typedef struct {
    int n[3];
    double lo[3], side[3];
    int64_t *start;   /* ncell + 1 */
    int64_t *order;   /* point indices grouped by cell, ascending within a cell */
} orc_grid;

static long orc_cell_of(const orc_grid *g, double x, double y, double z)
{
    double v[3] = {x, y, z};
    long c[3];
    for (int a = 0; a < 3; a++) {
        double f = floor((v[a] - g->lo[a]) / g->side[a]);
        long k = (long)f;
        if (f < 0) k = 0;
        if (k > g->n[a] - 1) k = g->n[a] - 1;
        c[a] = k;
    }
    return (c[2] * g->n[1] + c[1]) * g->n[0] + c[0];
}

static int orc_grid_build(orc_grid *g, const double *x, int64_t n)
{
    long ncell = (long)g->n[0] * g->n[1] * g->n[2];
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    long *cell = (long *)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
    if (!g->start || !g->order || !cell) { free(cell); return ORC_ENOMEM; }
    for (int64_t i = 0; i < n; i++) {
        cell[i] = orc_cell_of(g, x[3 * i], x[3 * i + 1], x[3 * i + 2]);
        g->start[cell[i] + 1]++;
    }
    for (long c = 0; c < ncell; c++) g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    if (!fill) { free(cell); return ORC_ENOMEM; }
    for (long c = 0; c < ncell; c++) fill[c] = g->start[c];
    for (int64_t i = 0; i < n; i++) g->order[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
    return ORC_OK;
}

static void orc_grid_free(orc_grid *g)
{
    free(g->start); free(g->order);
    g->start = NULL; g->order = NULL;
}

int oracle_count_grid(const double *x1, const double *w1, int64_t n1,
                      const double *x2, const double *w2, int64_t n2,
                      int is_auto, int kind, int los, double L,
                      const double *e1, int nb1, const double *e2, int nb2,
                      double cell_size,
                      int64_t *counts, double *wcounts, int nthreads)
{
    orc_spec sp;
    int rc = orc_spec_init(&sp, kind, los, L, e1, nb1, e2, nb2);
    if (rc) { orc_spec_free(&sp); return rc; }
    if (is_auto) { x2 = x1; w2 = w1; n2 = n1; }
    if (n1 < 0 || n2 < 0 || (n1 > 0 && !x1) || (n2 > 0 && !x2) || !(cell_size > 0.0)) { orc_spec_free(&sp); return ORC_EINVAL; }
    if (orc_check_points(x1, n1, L) || orc_check_points(x2, n2, L)) { orc_spec_free(&sp); return ORC_EINVAL; }
    long nbins = (long)sp.n1 * sp.n2;
    orc_wspec ws = {0, 0, 1.0};
    if (wcounts) {
        if (!w1 || !w2) { orc_spec_free(&sp); return ORC_EINVAL; }
        rc = orc_prepare_weights(&ws, w1, n1, w2, n2, (double)n1 * (double)n2);
        if (rc) { orc_spec_free(&sp); return rc; }
    }
    double rmax = (kind == ORC_KIND_SPERP_PI) ? sqrt(e1[nb1] * e1[nb1] + e2[nb2] * e2[nb2]) : e1[nb1];

    orc_grid g;
    memset(&g, 0, sizeof(g));
    for (int a = 0; a < 3; a++) {
        if (L > 0.0) {
            long n = (long)floor(L / cell_size);
            if (n < 1) n = 1;
            if (n > 256) n = 256;
            g.n[a] = (int)n;
            g.lo[a] = 0.0;
            g.side[a] = L / (double)n;
        } else {
            double lo = INFINITY, hi = -INFINITY;
            for (int64_t i = 0; i < n1; i++) { if (x1[3 * i + a] < lo) lo = x1[3 * i + a]; if (x1[3 * i + a] > hi) hi = x1[3 * i + a]; }
            for (int64_t i = 0; i < n2; i++) { if (x2[3 * i + a] < lo) lo = x2[3 * i + a]; if (x2[3 * i + a] > hi) hi = x2[3 * i + a]; }
            if (!(hi >= lo)) { lo = 0.0; hi = 0.0; }
            long n = (long)ceil((hi - lo) / cell_size);
            if (n < 1) n = 1;
            if (n > 256) n = 256;
            g.n[a] = (int)n;
            g.lo[a] = lo;
            g.side[a] = (hi - lo) / (double)n;
            if (!(g.side[a] > 0.0)) g.side[a] = 1.0;
        }
    }
    orc_grid g2 = g;
    g2.start = NULL; g2.order = NULL;
    if (orc_grid_build(&g2, x2, n2)) { orc_grid_free(&g2); orc_spec_free(&sp); return ORC_ENOMEM; }
    int reach[3];
    for (int a = 0; a < 3; a++) reach[a] = (int)ceil(rmax / g.side[a]) + 1;
    /* cells farther than this from a point hold no partner in range */
    double cmag = (L > 0.0) ? L : 0.0;
    for (int a = 0; a < 3; a++) {
        double m = fabs(g.lo[a]) + g.side[a] * (double)g.n[a];
        if (m > cmag) cmag = m;
    }
    double lim = rmax * (1.0 + 1e-9) + 1e-9 * cmag;
    double lim2 = lim * lim;

    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    orc_acc *acc = (orc_acc *)calloc((size_t)nth, sizeof(orc_acc));
    if (!acc) { orc_grid_free(&g2); orc_spec_free(&sp); return ORC_ENOMEM; }
    for (int t = 0; t < nth; t++)
        if (orc_acc_alloc(&acc[t], nbins, ws.weighted)) { orc_acc_free(acc, nth); orc_grid_free(&g2); orc_spec_free(&sp); return ORC_ENOMEM; }

#pragma omp parallel num_threads(nth)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        /* per-axis neighbour index lists (wrapped and de-duplicated), with the
         * smallest gap between the point and each listed cell's slab */
        int *lst[3];
        double *gap[3];
        int cnt[3];
        for (int a = 0; a < 3; a++) {
            lst[a] = (int *)malloc(sizeof(int) * (size_t)(2 * reach[a] + 1));
            gap[a] = (double *)malloc(sizeof(double) * (size_t)(2 * reach[a] + 1));
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n1; i++) {
            double xi = x1[3 * i], yi = x1[3 * i + 1], zi = x1[3 * i + 2];
            double wi = ws.weighted ? w1[i] : 0.0;
            long ci = orc_cell_of(&g2, xi, yi, zi);
            long c3[3] = {ci % g.n[0], (ci / g.n[0]) % g.n[1], ci / ((long)g.n[0] * g.n[1])};
            double pv[3] = {xi, yi, zi};
            for (int a = 0; a < 3; a++) {
                cnt[a] = 0;
                for (int d = -reach[a]; d <= reach[a]; d++) {
                    long c = c3[a] + d;
                    /* the slab of this offset, unwrapped */
                    double slo = g.lo[a] + (double)c * g.side[a];
                    double shi = slo + g.side[a];
                    double gp = 0.0;
                    if (pv[a] < slo) gp = slo - pv[a];
                    else if (pv[a] > shi) gp = pv[a] - shi;
                    if (L > 0.0) {
                        c %= g.n[a];
                        if (c < 0) c += g.n[a];
                    } else if (c < 0 || c >= g.n[a]) {
                        continue;
                    }
                    int seen = -1;
                    for (int q = 0; q < cnt[a]; q++) if (lst[a][q] == (int)c) seen = q;
                    if (seen < 0) {
                        lst[a][cnt[a]] = (int)c;
                        gap[a][cnt[a]] = gp;
                        cnt[a]++;
                    } else if (gp < gap[a][seen]) {
                        gap[a][seen] = gp;
                    }
                }
            }
            for (int qz = 0; qz < cnt[2]; qz++)
                for (int qy = 0; qy < cnt[1]; qy++)
                    for (int qx = 0; qx < cnt[0]; qx++) {
                        double gsq = (gap[0][qx] * gap[0][qx] + gap[1][qy] * gap[1][qy]) + gap[2][qz] * gap[2][qz];
                        if (gsq > lim2) continue;
                        long c = ((long)lst[2][qz] * g.n[1] + lst[1][qy]) * g.n[0] + lst[0][qx];
                        for (int64_t p = g2.start[c]; p < g2.start[c + 1]; p++) {
                            int64_t j = g2.order[p];
                            if (is_auto && j <= i) continue;
                            long b = orc_classify(&sp, xi, yi, zi, x2[3 * j], x2[3 * j + 1], x2[3 * j + 2]);
                            if (b >= 0) orc_acc_add(&acc[t], &ws, b, wi, ws.weighted ? w2[j] : 0.0);
                        }
                    }
        }
        for (int a = 0; a < 3; a++) { free(lst[a]); free(gap[a]); }
    }
    orc_finish(acc, nth, nbins, &ws, counts, wcounts);
    orc_acc_free(acc, nth);
    orc_grid_free(&g2);
    orc_spec_free(&sp);
    return ORC_OK;
}

/* Canonical classification of a single pair, exported for tests of individual
 * pairs (returns the flat bin or -1; -2 on a bad specification). */
long oracle_classify_pair(const double *p1, const double *p2, int kind, int los, double L,
                          const double *e1, int nb1, const double *e2, int nb2)
{
    orc_spec sp;
    if (orc_spec_init(&sp, kind, los, L, e1, nb1, e2, nb2)) { orc_spec_free(&sp); return -2; }
    long b = orc_classify(&sp, p1[0], p1[1], p1[2], p2[0], p2[1], p2[2]);
    orc_spec_free(&sp);
    return b;
}

/* The same classification for n pairs (p1[3i..], p2[3i..]) into out[i]; returns
 * ORC_OK, or -2 on a bad specification. */
int oracle_classify_pairs(const double *p1, const double *p2, int64_t n, int kind, int los, double L,
                          const double *e1, int nb1, const double *e2, int nb2, long *out)
{
    orc_spec sp;
    if (orc_spec_init(&sp, kind, los, L, e1, nb1, e2, nb2)) { orc_spec_free(&sp); return -2; }
    for (int64_t i = 0; i < n; i++)
        out[i] = orc_classify(&sp, p1[3 * i], p1[3 * i + 1], p1[3 * i + 2],
                              p2[3 * i], p2[3 * i + 1], p2[3 * i + 2]);
    orc_spec_free(&sp);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Triangle counts (the three-point extension; Sect. 6 lists three-point
 * statistics as future work, so the definition is the plain one built from
 * the separation of Sect. 2.5 and the squared-edge bins of Sect. 3.2):
 *   every set {i, j, k} of three distinct points is counted once when each of
 *   its three sides s = |x_b - x_a| (minimum image in a periodic box) lies in
 *   [e_0, e_n); its bin is (a, b, c), the three side bins sorted so that
 *   a <= b <= c, in the row-major [n][n][n] histogram (entries with a > b or
 *   b > c stay zero).  Each side is classified by orc_classify, the same
 *   per-pair function as the pair counts.
 * Two counters: the plain triple loop over i < j < k, and a neighbour-list
 * version: for each i, the j > i with side ij in range; then every pair of
 * them whose third side is in range.  A triangle with all sides in range is
 * found exactly once, from its lowest index.
 * Weighted (neighbour-list counter, w non-NULL): a triangle's weight is the
 * product of its three point weights taken in ascending order of value,
 * fl(fl(a*b)*c), so that it does not depend on the order of the points; a
 * bin's weighted count is the exact real sum of those products rounded once
 * to FP64, kept exactly in 128-bit fixed point as for pairs (every product
 * is an integer multiple of 2^-S, S from the smallest possible product).
 * ------------------------------------------------------------------------- */
static long orc_tri_index(int n, int b1, int b2, int b3)
{
    int t;
    if (b1 > b2) { t = b1; b1 = b2; b2 = t; }
    if (b2 > b3) { t = b2; b2 = b3; b3 = t; }
    if (b1 > b2) { t = b1; b1 = b2; b2 = t; }
    return ((long)b1 * n + b2) * n + b3;
}

int oracle_triplets_brute(const double *x, int64_t n, double L, const double *e, int nb,
                          int64_t *counts, int nthreads)
{
    orc_spec sp;
    int rc = orc_spec_init(&sp, ORC_KIND_S, ORC_LOS_Z, L, e, nb, NULL, 0);
    if (rc) { orc_spec_free(&sp); return rc; }
    if (n < 0 || (n > 0 && !x) || orc_check_points(x, n, L)) { orc_spec_free(&sp); return ORC_EINVAL; }
    long nbins = (long)nb * nb * nb;
    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    int64_t *acc = (int64_t *)calloc((size_t)nth * (size_t)nbins, sizeof(int64_t));
    if (!acc) { orc_spec_free(&sp); return ORC_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 4) num_threads(nth)
    for (int64_t i = 0; i < n; i++) {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t *h = acc + (size_t)t * (size_t)nbins;
        for (int64_t j = i + 1; j < n; j++) {
            long bij = orc_classify(&sp, x[3 * i], x[3 * i + 1], x[3 * i + 2], x[3 * j], x[3 * j + 1], x[3 * j + 2]);
            if (bij < 0) continue;
            for (int64_t k = j + 1; k < n; k++) {
                long bik = orc_classify(&sp, x[3 * i], x[3 * i + 1], x[3 * i + 2], x[3 * k], x[3 * k + 1], x[3 * k + 2]);
                if (bik < 0) continue;
                long bjk = orc_classify(&sp, x[3 * j], x[3 * j + 1], x[3 * j + 2], x[3 * k], x[3 * k + 1], x[3 * k + 2]);
                if (bjk < 0) continue;
                h[orc_tri_index(nb, (int)bij, (int)bik, (int)bjk)]++;
            }
        }
    }
    for (long b = 0; b < nbins; b++) {
        int64_t v = 0;
        for (int t = 0; t < nth; t++) v += acc[(size_t)t * (size_t)nbins + b];
        counts[b] = v;
    }
    free(acc);
    orc_spec_free(&sp);
    return ORC_OK;
}

static double orc_tri_weight(double a, double b, double c)
{
    double t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    return (a * b) * c;
}

int oracle_triplets_list_w(const double *x, const double *w, int64_t n, double L, const double *e, int nb,
                           int64_t *counts, double *wcounts, int nthreads);

int oracle_triplets_list(const double *x, int64_t n, double L, const double *e, int nb,
                         int64_t *counts, int nthreads)
{
    return oracle_triplets_list_w(x, NULL, n, L, e, nb, counts, NULL, nthreads);
}

int oracle_triplets_list_w(const double *x, const double *w, int64_t n, double L, const double *e, int nb,
                           int64_t *counts, double *wcounts, int nthreads)
{
    orc_spec sp;
    int rc = orc_spec_init(&sp, ORC_KIND_S, ORC_LOS_Z, L, e, nb, NULL, 0);
    if (rc) { orc_spec_free(&sp); return rc; }
    if (n < 0 || (n > 0 && !x) || orc_check_points(x, n, L)) { orc_spec_free(&sp); return ORC_EINVAL; }
    long nbins = (long)nb * nb * nb;
    int weighted = (w != NULL && wcounts != NULL);
    int S = 0;
    if (weighted) {
        double m = orc_min_abs_nonzero(w, n), M = orc_max_abs(w, n);
        if (m < INFINITY) {
            double pmin = (m * m) * m, pmax = (M * M) * M;
            int ex;
            frexp(pmin, &ex);
            S = 53 - ex;
            if (!(ldexp(pmax, S) < ldexp(1.0, 62))) { orc_spec_free(&sp); return ORC_EINVAL; }
        }
    }
    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    int64_t *acc = (int64_t *)calloc((size_t)nth * (size_t)nbins, sizeof(int64_t));
    __int128 *wacc = weighted ? (__int128 *)calloc((size_t)nth * (size_t)nbins, sizeof(__int128)) : NULL;
    if (weighted && !wacc) { free(acc); orc_spec_free(&sp); return ORC_ENOMEM; }
    int64_t *nbr = (int64_t *)malloc((size_t)nth * (size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    long *nbin = (long *)malloc((size_t)nth * (size_t)(n > 0 ? n : 1) * sizeof(long));
    if (!acc || !nbr || !nbin) { free(acc); free(nbr); free(nbin); orc_spec_free(&sp); return ORC_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 4) num_threads(nth)
    for (int64_t i = 0; i < n; i++) {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t *h = acc + (size_t)t * (size_t)nbins;
        __int128 *hw = weighted ? wacc + (size_t)t * (size_t)nbins : NULL;
        int64_t *lj = nbr + (size_t)t * (size_t)n;
        long *lb = nbin + (size_t)t * (size_t)n;
        int64_t m = 0;
        for (int64_t j = i + 1; j < n; j++) {
            long b = orc_classify(&sp, x[3 * i], x[3 * i + 1], x[3 * i + 2], x[3 * j], x[3 * j + 1], x[3 * j + 2]);
            if (b >= 0) { lj[m] = j; lb[m] = b; m++; }
        }
        for (int64_t p = 0; p < m; p++) {
            const double *xp = x + 3 * lj[p];
            for (int64_t q = p + 1; q < m; q++) {
                const double *xq = x + 3 * lj[q];
                long bpq = orc_classify(&sp, xp[0], xp[1], xp[2], xq[0], xq[1], xq[2]);
                if (bpq < 0) continue;
                long slot = orc_tri_index(nb, (int)lb[p], (int)lb[q], (int)bpq);
                h[slot]++;
                if (weighted) {
                    double tw = orc_tri_weight(w[i], w[lj[p]], w[lj[q]]);
                    hw[slot] += (__int128)ldexp(tw, S);
                }
            }
        }
    }
    for (long b = 0; b < nbins; b++) {
        int64_t v = 0;
        __int128 vw = 0;
        for (int t = 0; t < nth; t++) {
            v += acc[(size_t)t * (size_t)nbins + b];
            if (weighted) vw += wacc[(size_t)t * (size_t)nbins + b];
        }
        counts[b] = v;
        if (weighted) wcounts[b] = orc_i128_to_double(vw, S);
    }
    free(acc);
    free(wacc);
    free(nbr);
    free(nbin);
    orc_spec_free(&sp);
    return ORC_OK;
}

int oracle_version(void) { return 1; }
