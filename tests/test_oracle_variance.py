"""Exact pair-estimator variance (oracle/variance.py) and what it says about
proposals over the auxiliary index.

Pins: the quadratic and quartic forms reproduce selfenergy.sigma_pair's
energy for arbitrary real vectors; the fourth-moment matrices equal
enumeration over each distribution's outcomes; the exact mean and variance
equal enumeration over every pair of +-1 vectors on a small chain.

Then what a proposal over the auxiliary index can gain, exactly, on the
chains the method runs on: k = 1 importance draws (best weights over many
starts) against +-1 vectors, and stratified vectors (classes Q mod K) whose
class make-up decides whether they win or lose."""
import itertools

import numpy as np
import pytest
from scipy.optimize import minimize

import chain_inputs as ci
from oracle import green, integrals, selfenergy as se, split as sp, variance as va


def _chain(nd, eps=1e-2, beta=20.0, ntau=6):
    geo = ci.chain_geometry(nd)
    f = ci.fock_tight_binding(geo.x)
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    e, c = green.orbitals(f)
    tau, w = green.tau_grid(beta, ntau)
    g, gb = green.green_tau(e, c, green.midgap_mu(e, geo.n // 2), beta, tau)
    return b, sp.split_b(b, eps), g, gb, w


def _energy(b, spl, th, thp, g, gb, w):
    _, xl, xs = sp.r_vectors(b, spl, th[None])
    _, yl, ys = sp.r_vectors(b, spl, thp[None])
    return sum(w[t] * np.sum(se.sigma_pair(spl, xl[0], xs[0], yl[0], ys[0], g[t], gb[t]) * gb[t].T)
               for t in range(len(w)))


def _poly(x, y, wm, th, thp):
    q, qp = np.outer(th, th).reshape(-1), np.outer(thp, thp).reshape(-1)
    return x.reshape(-1) @ q + y.reshape(-1) @ qp + q @ wm @ qp


def test_forms_reproduce_the_pair_energy():
    b, spl, g, gb, w = _chain(2, ntau=3)
    x, y, wm = va.pair_forms(b, spl, g, gb, w)
    r = np.random.default_rng(0)
    for _ in range(3):
        th, thp = r.standard_normal(b.shape[0]), r.standard_normal(b.shape[0])
        want = _energy(b, spl, th, thp, g, gb, w)
        assert abs(_poly(x, y, wm, th, thp) - want) < 1e-12 * max(1.0, abs(want))


def _enum_m4(outcomes, probs, na):
    m = np.zeros((na * na, na * na))
    for th, pr in zip(outcomes, probs):
        q = np.outer(th, th).reshape(-1)
        m += pr * np.outer(q, q)
    return m


def test_fourth_moments_by_enumeration():
    na = 5
    signs = np.array(list(itertools.product([1.0, -1.0], repeat=na)))
    assert np.allclose(va.m4_pm1(na), _enum_m4(signs, np.full(len(signs), 1.0 / len(signs)), na), atol=1e-14)
    p = np.array([0.1, 0.3, 0.2, 0.15, 0.25])
    outs = [np.eye(na)[a] / np.sqrt(p[a]) for a in range(na)]
    assert np.allclose(va.m4_importance(p), _enum_m4(outs, p, na), atol=1e-12)
    pi = np.array([0.3, 0.7])
    outs, probs = [], []
    for c in range(2):
        mem = np.arange(c, na, 2)
        for s in itertools.product([1.0, -1.0], repeat=len(mem)):
            th = np.zeros(na)
            th[mem] = np.array(s) / np.sqrt(pi[c])
            outs.append(th)
            probs.append(pi[c] / 2 ** len(mem))
    assert np.allclose(va.m4_stratified(pi, 2, na), _enum_m4(outs, probs, na), atol=1e-12)


def test_exact_variance_by_enumeration_of_pm1_pairs():
    b, spl, g, gb, w = _chain(1, eps=0.1, ntau=3)           # N_aux = 6: 4096 pairs
    x, y, wm = va.pair_forms(b, spl, g, gb, w)
    signs = np.array(list(itertools.product([1.0, -1.0], repeat=b.shape[0])))
    vals = np.array([_poly(x, y, wm, th, thp) for th in signs for thp in signs])
    mean, var = va.mean_var(x, y, wm, va.m4_pm1(b.shape[0]))
    assert abs(mean - vals.mean()) < 1e-12 * abs(vals).max()
    assert abs(var - vals.var()) < 1e-10 * vals.var()
    # and the mixture form agrees with the dense one
    terms = va.mixture_terms(x, y, wm, [va.m4_pm1(6, np.arange(c, 6, 2)) for c in range(2)])
    pi = np.array([0.4, 0.6])
    assert abs(va.mixture_var(terms, pi) - va.mean_var(x, y, wm, va.m4_stratified(pi, 2, 6))[1]) < 1e-10 * var


def _best(terms, n, starts):
    """Smallest variance over the simplex (softmax parameters, several starts)."""
    f = lambda z: va.mixture_var(terms, np.exp(z - z.max()) / np.exp(z - z.max()).sum())
    best = np.inf
    for z0 in starts(n):
        res = minimize(f, z0, method="L-BFGS-B")
        best = min(best, res.fun, f(z0))
    return best


def _starts(n):
    r = np.random.default_rng(7)
    return [np.zeros(n)] + [r.standard_normal(n) for _ in range(4)]


@pytest.mark.parametrize("nd", [3, 5])
def test_exact_variances_rank_the_samplers(nd):
    """Exact per-pair variances on the chain (eps = 1e-2), relative to +-1
    vectors: k = 1 importance draws lose even with the best weights;
    stratified vectors with classes that mix the three kinds of
    auxiliary centre (K = 4) win; classes of one kind (K = 6, a multiple of
    three) lose."""
    b, spl, g, gb, w = _chain(nd)
    na = b.shape[0]
    x, y, wm = va.pair_forms(b, spl, g, gb, w)
    _, v_pm1 = va.mean_var(x, y, wm, va.m4_pm1(na))
    imp = _best(va.importance_terms(x, y, wm), na, _starts) / v_pm1
    strat = {}
    for k in (4, 6):
        terms = va.mixture_terms(x, y, wm, [va.m4_pm1(na, np.arange(c, na, k)) for c in range(k)])
        strat[k] = va.mixture_var(terms, np.full(k, 1.0 / k)) / v_pm1
    print(f"{nd} dimers, variance / +-1: importance (best p) {imp:.2f}, stratified K=4 {strat[4]:.3f}, "
          f"K=6 {strat[6]:.3f}")
    assert imp > 1.0
    assert strat[4] < 0.5
    assert strat[6] > 1.0
