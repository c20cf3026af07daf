// estimators.hip -- from pair counts to correlation functions, on the GPU:
// linear estimators over normalised pair counts (Landy-Szalay, Peebles-Hauser,
// Szapudi-Szalay and any other linear form), the analytic RR of a periodic
// box, Legendre multipoles of xi(s, mu) and the projected w_p(s_perp)
// (Sect. 1 and App. D).  Everything is FP64.
#include <math.h>

#include "internal.h"

namespace fcfc {

constexpr int XI_MAX_TERMS = 8;

struct XiArgs {
    const double* terms[XI_MAX_TERMS];
    double coef[XI_MAX_TERMS];  // coefficient / normalisation of each term
    int nterms;
    int den;                    // term used as the denominator
    double den_scale;           // 1 / its normalisation
};

// xi = (sum_t coef_t X_t / n_t) / (X_den / n_den); a bin whose denominator is
// zero gets NaN
__global__ void k_xi(XiArgs a, int64_t nbins, double* __restrict__ xi) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    double num = 0.0;
    for (int t = 0; t < a.nterms; t++) num += a.coef[t] * a.terms[t][b];
    const double den = a.terms[a.den][b] * a.den_scale;
    xi[b] = (den != 0.0) ? num / den : NAN;
}

// Analytic pair count of a uniform periodic box: npairs * V_bin / L^3, with
// V_bin the volume of the bin in separation space (pairs at +-pi and at
// mu = |pi| / s are both in one bin).
__global__ void k_analytic_rr(int kind, const double* __restrict__ e1, int n1, const double* __restrict__ e2,
                              int n2, double scale, double* __restrict__ rr) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = (kind == FCFC_BIN_S) ? n1 : n1 * n2;
    if (b >= nb) return;
    const int i = (kind == FCFC_BIN_S) ? b : b / n2;
    const int j = (kind == FCFC_BIN_S) ? 0 : b % n2;
    double v;
    if (kind == FCFC_BIN_S) {
        v = (4.0 * M_PI / 3.0) * (e1[i + 1] * e1[i + 1] * e1[i + 1] - e1[i] * e1[i] * e1[i]);
    } else if (kind == FCFC_BIN_S_MU) {
        // a shell times the fraction dmu of the full sphere (mu = |cos theta|)
        v = (4.0 * M_PI / 3.0) * (e1[i + 1] * e1[i + 1] * e1[i + 1] - e1[i] * e1[i] * e1[i]) * (e2[j + 1] - e2[j]);
    } else {
        // a cylindrical annulus in s_perp, both signs of pi
        v = M_PI * (e1[i + 1] * e1[i + 1] - e1[i] * e1[i]) * 2.0 * (e2[j + 1] - e2[j]);
    }
    rr[b] = scale * v;
}

// integral of the Legendre polynomial P_l over [a, b] (Bonnet recursion for
// P_l; for l >= 1 the antiderivative is (P_{l+1} - P_{l-1}) / (2 l + 1))
__device__ inline void legendre_pair(int l, double x, double& pm1, double& pl, double& pp1) {
    double p0 = 1.0, p1 = x;
    if (l == 0) {
        pm1 = 0.0;
        pl = 1.0;
        pp1 = x;
        return;
    }
    for (int k = 1; k < l; k++) {
        const double p2 = ((2.0 * k + 1.0) * x * p1 - (double)k * p0) / (double)(k + 1);
        p0 = p1;
        p1 = p2;
    }
    pm1 = p0;
    pl = p1;
    pp1 = ((2.0 * l + 1.0) * x * p1 - (double)l * p0) / (double)(l + 1);
}
__device__ inline double legendre_integral(int l, double a, double b) {
    if (l == 0) return b - a;
    double am, al, ap, bm, bl, bp;
    legendre_pair(l, a, am, al, ap);
    legendre_pair(l, b, bm, bl, bp);
    return ((bp - bm) - (ap - am)) / (2.0 * l + 1.0);
}

// xi_l(s_i) = (2 l + 1) sum_j xi(s_i, mu_j) int_{mu_j}^{mu_j+1} P_l(mu) dmu for
// xi constant within each mu bin; out[k * ns + i] for the k-th requested l
__global__ void k_multipoles(const double* __restrict__ xi, int ns, int nmu, const double* __restrict__ mu,
                             const int* __restrict__ ells, int nell, double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns * nell) return;
    const int k = t / ns, i = t % ns;
    const int l = ells[k];
    double acc = 0.0;
    for (int j = 0; j < nmu; j++) acc += xi[(int64_t)i * nmu + j] * legendre_integral(l, mu[j], mu[j + 1]);
    out[t] = (2.0 * l + 1.0) * acc;
}

// w_p(s_perp_i) = 2 sum_j xi(s_perp_i, pi_j) dpi_j over the pi bins up to pi_max
__global__ void k_wp(const double* __restrict__ xi, int nsp, int npi, const double* __restrict__ pi,
                     double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsp) return;
    double acc = 0.0;
    for (int j = 0; j < npi; j++) acc += xi[(int64_t)i * npi + j] * (pi[j + 1] - pi[j]);
    out[i] = 2.0 * acc;
}

static fcfc_status upload_edges(const double* h, int n, double** d, hipStream_t st) {
    if (dev_alloc((void**)d, sizeof(double) * (size_t)(n + 1), st) != FCFC_OK) {
        set_error("estimators: cannot allocate %d edges", n + 1);
        return FCFC_ENOMEM;
    }
    FCFC_HIP(hipMemcpyAsync(*d, h, sizeof(double) * (size_t)(n + 1), hipMemcpyHostToDevice, st));
    return FCFC_OK;
}

}  // namespace fcfc

using namespace fcfc;

extern "C" fcfc_status fcfc_xi(int32_t nterms, const double* const* d_terms, const double* coef, const double* norm,
                               int32_t den, int64_t nbins, double* d_xi, void* stream) {
    clear_error();
    if (nterms < 1 || nterms > XI_MAX_TERMS || !d_terms || !coef || !norm || den < 0 || den >= nterms ||
        nbins < 0 || (nbins > 0 && !d_xi)) {
        set_error("xi: need 1..%d terms, coefficients, normalisations and a denominator term", XI_MAX_TERMS);
        return FCFC_EINVAL;
    }
    XiArgs a{};
    a.nterms = nterms;
    a.den = den;
    for (int t = 0; t < nterms; t++) {
        if (!d_terms[t] || !(norm[t] > 0) || !isfinite(coef[t])) {
            set_error("xi: term %d needs a device array and a positive normalisation", t);
            return FCFC_EINVAL;
        }
        a.terms[t] = d_terms[t];
        a.coef[t] = coef[t] / norm[t];
    }
    a.den_scale = 1.0 / norm[den];
    if (nbins == 0) return FCFC_OK;
    hipLaunchKernelGGL(k_xi, dim3((unsigned)((nbins + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a, nbins, d_xi);
    FCFC_HIP(hipGetLastError());
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_pair_norm(int64_t n1, int64_t n2, double* out) {
    clear_error();
    if (!out || n1 < 0) {
        set_error("pair_norm: null output or negative size");
        return FCFC_EINVAL;
    }
    const __int128 a = n1;
    const __int128 pairs = n2 < 0 ? a * (a - 1) / 2 : a * (__int128)n2;
    *out = (double)pairs;
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_landy_szalay(const double* d_dd, const double* d_dr, const double* d_rr, int64_t n_d,
                                         int64_t n_r, int64_t nbins, double* d_xi, void* stream) {
    clear_error();
    if (!d_dd || !d_dr || !d_rr || n_d < 2 || n_r < 2) {
        set_error("landy_szalay: need DD, DR and RR and at least 2 data and 2 random points");
        return FCFC_EINVAL;
    }
    double norm[3];
    FCFC_TRY(fcfc_pair_norm(n_d, -1, &norm[0]));
    FCFC_TRY(fcfc_pair_norm(n_d, n_r, &norm[1]));
    FCFC_TRY(fcfc_pair_norm(n_r, -1, &norm[2]));
    const double* terms[3] = {d_dd, d_dr, d_rr};
    const double coef[3] = {1.0, -2.0, 1.0};
    return fcfc_xi(3, terms, coef, norm, 2, nbins, d_xi, stream);
}

extern "C" fcfc_status fcfc_analytic_rr(fcfc_plan_t plan, double npairs, double* d_rr, void* stream) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || !d_rr || !(npairs >= 0) || !isfinite(npairs)) return FCFC_EINVAL;
    if (p->L <= 0) {
        set_error("analytic_rr: needs a periodic plan");
        return FCFC_ESTATE;
    }
    if (p->kind == FCFC_BIN_S_MU && p->los != FCFC_LOS_Z) {
        set_error("analytic_rr: (s, mu) needs the line of sight z");
        return FCFC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    double *e1 = nullptr, *e2 = nullptr;
    FCFC_TRY(upload_edges(p->e1.data(), p->n1, &e1, st));
    if (p->kind != FCFC_BIN_S) {
        fcfc_status s = upload_edges(p->e2.data(), p->n2, &e2, st);
        if (s != FCFC_OK) {
            dev_free(e1, st);
            return s;
        }
    }
    const double scale = npairs / (p->L * p->L * p->L);
    hipLaunchKernelGGL(k_analytic_rr, dim3((p->nbins + 255) / 256), dim3(256), 0, st, p->kind, e1, p->n1, e2, p->n2,
                       scale, d_rr);
    fcfc_status s = (hipGetLastError() == hipSuccess) ? FCFC_OK : FCFC_EHIP;
    dev_free(e1, st);
    if (e2) dev_free(e2, st);
    if (s != FCFC_OK) set_error("analytic_rr: launch failed");
    return s;
}

extern "C" fcfc_status fcfc_multipoles(const double* d_xi, int32_t ns, const double* mu_edges, int32_t nmu,
                                       const int32_t* ells, int32_t nell, double* d_out, void* stream) {
    clear_error();
    if (!d_xi || !mu_edges || !ells || !d_out || ns < 1 || nmu < 1 || nell < 1) return FCFC_EINVAL;
    for (int k = 0; k < nell; k++)
        if (ells[k] < 0 || ells[k] > 64) {
            set_error("multipoles: orders must lie in [0, 64]");
            return FCFC_EINVAL;
        }
    hipStream_t st = (hipStream_t)stream;
    double* mu = nullptr;
    FCFC_TRY(upload_edges(mu_edges, nmu, &mu, st));
    int* dl = nullptr;
    if (dev_alloc((void**)&dl, sizeof(int) * (size_t)nell, st) != FCFC_OK) {
        dev_free(mu, st);
        set_error("multipoles: cannot allocate");
        return FCFC_ENOMEM;
    }
    fcfc_status s = FCFC_OK;
    if (hipMemcpyAsync(dl, ells, sizeof(int) * (size_t)nell, hipMemcpyHostToDevice, st) != hipSuccess) s = FCFC_EHIP;
    if (s == FCFC_OK) {
        hipLaunchKernelGGL(k_multipoles, dim3((ns * nell + 255) / 256), dim3(256), 0, st, d_xi, ns, nmu, mu, dl, nell,
                           d_out);
        if (hipGetLastError() != hipSuccess) s = FCFC_EHIP;
    }
    dev_free(mu, st);
    dev_free(dl, st);
    if (s != FCFC_OK) set_error("multipoles: HIP failure");
    return s;
}

extern "C" fcfc_status fcfc_wp(const double* d_xi, int32_t nsp, const double* pi_edges, int32_t npi, double* d_out,
                               void* stream) {
    clear_error();
    if (!d_xi || !pi_edges || !d_out || nsp < 1 || npi < 1) return FCFC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    double* pe = nullptr;
    FCFC_TRY(upload_edges(pi_edges, npi, &pe, st));
    hipLaunchKernelGGL(k_wp, dim3((nsp + 255) / 256), dim3(256), 0, st, d_xi, nsp, npi, pe, d_out);
    fcfc_status s = (hipGetLastError() == hipSuccess) ? FCFC_OK : FCFC_EHIP;
    dev_free(pe, st);
    if (s != FCFC_OK) set_error("wp: launch failed");
    return s;
}
