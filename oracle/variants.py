"""Other ways to average over the stochastic orbitals in eq:sigma_2.

The paper writes the two RS-SRI vertices of eq:sigma_2 as averages over
independent sets theta and theta'.  The default estimator (selfenergy.py)
pairs vector s of one set with vector s of the other and keeps the
range-separated vertex L/S-resolved.  Two variants:

Control-variate form.  E[R (x) R] = sum_Q K_Q (x) K_Q = v (eq:abgd_l) and
E[R^L (x) R^L] = sum_Q K^L_Q (x) K^L_Q = D, so with D exact

  v ~= D + R (x) R - R^L (x) R^L

is unbiased, and for independent theta, theta' so is

  Sigma ~= Sigma[D, D] + chain(R_xi, R'_eta) - chain(R^L_xi, R'^L_eta),
  chain(a, b) = Sigma[a (x) a, b (x) b]   (eq:sigma, bilinear form),

whose expectation is Sigma[v, v] - Sigma[D, D] + Sigma[D, D].  It needs
four N x N products per chain (a G, (a G) b, M Gbar, T M) -- 8 per pair
instead of the 24 of the L/S-resolved form -- but the cross terms D (x) S
are now sampled rather than exact.

Double sum.  Read literally, <>_theta <>_theta' averages over all N_s^2
combinations of one vector from each set: Sigma_s for every (xi_i, eta_j),
averaged over i and j.  Each term is the pair estimator of selfenergy.py, so
the double average is unbiased; its terms are not independent (they share
vectors), and its standard error is that of a two-sample U-statistic.

Every function cites the passage it follows; nothing here is shared with
the GPU path.
"""
from __future__ import annotations

import numpy as np

from . import selfenergy as se


def chain(a: np.ndarray, b: np.ndarray, g: np.ndarray, gb: np.ndarray) -> np.ndarray:
    """Sigma[a (x) a, b (x) b] of eq:sigma for symmetric a, b."""
    return se.sigma_bilinear(a, a, b, b, g, gb)


def sigma_pair_cv(xt, xl, yt, yl, g, gb) -> np.ndarray:
    """One pair of the control-variate estimator, without Sigma[D, D]:
    chain(R_xi, R_eta) - chain(R^L_xi, R^L_eta)."""
    return chain(xt, yt, g, gb) - chain(xl, yl, g, gb)


def sigma_double(split, xl, xs, yl, ys, g, gb) -> np.ndarray:
    """The double average (1/N_s^2) sum_{i,j} Sigma_ij of the pair estimator
    over every combination of a first-set vector i and a second-set vector j
    (without Sigma[D, D], unsymmetrised).  Returns (mean, per-combination
    list [N_s][N_s] of matrices)."""
    ns = xl.shape[0]
    per = [[se.sigma_pair(split, xl[i], xs[i], yl[j], ys[j], g, gb) for j in range(ns)] for i in range(ns)]
    mean = sum(per[i][j] for i in range(ns) for j in range(ns)) / float(ns * ns)
    return mean, per


def double_mean_stderr(e: np.ndarray):
    """Mean and standard error of the double average of a two-sample
    statistic e[i][j] (i over the first set, j over the second): to first
    order the U-statistic variance is Var_i(mean_j e_ij) / N_s +
    Var_j(mean_i e_ij) / N_s (Hoeffding's decomposition; sample variances
    with ddof = 1)."""
    e = np.asarray(e, dtype=np.float64)
    ni, nj = e.shape
    rows = e.mean(axis=1)
    cols = e.mean(axis=0)
    var = rows.var(ddof=1) / ni + cols.var(ddof=1) / nj
    return float(e.mean()), float(np.sqrt(var))
