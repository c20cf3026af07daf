"""CPU oracle of the estimators -- TEST INFRASTRUCTURE ONLY.

Only the test suite may import this module; the library shares no code with it.
Plain float64 definitions, in the paper's terms:

* a correlation-function estimator is a linear form in normalised pair counts
  divided by one of them: Landy-Szalay (DD - 2 DR + RR) / RR (Sect. 1),
  Peebles-Hauser DD / RR - 1 and Szapudi-Szalay for cross correlations
  (App. D); each count X is normalised by its number of pairs n_X;
* the analytic RR of a periodic box (App. D) is the number of pairs times the
  separation-space volume of the bin over the box volume;
* the multipoles xi_l(s) = (2 l + 1) int_0^1 xi(s, mu) P_l(mu) dmu and the
  projected w_p(s_perp) = 2 int_0^pi_max xi(s_perp, pi) dpi (App. D), with xi
  constant within each bin.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def xi_linear(terms, coef, norm, den):
    """(sum_t coef_t X_t / norm_t) / (X_den / norm_den), NaN where the denominator is 0."""
    num = np.zeros_like(np.asarray(terms[0], dtype=np.float64))
    for x, c, n in zip(terms, coef, norm):
        num = num + (c / n) * np.asarray(x, dtype=np.float64)
    d = np.asarray(terms[den], dtype=np.float64) / norm[den]
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(d != 0, num / np.where(d != 0, d, 1.0), np.nan)


def bin_volumes(kind, e1, e2=None):
    """Separation-space volume of each bin: shell (s); shell x dmu ((s, mu), mu = |cos|);
    annulus x 2 dpi ((s_perp, pi), both signs of pi)."""
    e1 = np.asarray(e1, dtype=np.float64)
    shell = 4.0 * np.pi / 3.0 * (e1[1:] ** 3 - e1[:-1] ** 3)
    if kind == "s":
        return shell
    e2 = np.asarray(e2, dtype=np.float64)
    if kind == "smu":
        return np.outer(shell, np.diff(e2))
    annulus = np.pi * (e1[1:] ** 2 - e1[:-1] ** 2)
    return np.outer(annulus, 2.0 * np.diff(e2))


def analytic_rr(kind, e1, e2, L, npairs):
    return npairs * bin_volumes(kind, e1, e2) / float(L) ** 3


def legendre_bin_integrals(ell, edges):
    """int P_ell over each [edges_j, edges_j+1]."""
    anti = npleg.Legendre.basis(ell).integ()
    v = anti(np.asarray(edges, dtype=np.float64))
    return np.diff(v)


def multipoles(xi_smu, mu_edges, ells=(0, 2, 4)):
    x = np.asarray(xi_smu, dtype=np.float64)
    return np.stack([(2 * l + 1) * (x @ legendre_bin_integrals(l, mu_edges)) for l in ells])


def wp(xi_spi, pi_edges):
    return 2.0 * (np.asarray(xi_spi, dtype=np.float64) @ np.diff(np.asarray(pi_edges, dtype=np.float64)))
