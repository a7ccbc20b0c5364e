"""Pins of the estimator variants of eq:sigma_2 (oracle/variants.py): the
single-vertex chain against the 4-index definition of eq:sigma, the
control-variate and pair estimators against deterministic RI by exact
enumeration of every sign pattern, and the U-statistic standard error on a
case where it is known in closed form."""
import itertools

import numpy as np

import chain_inputs as ci
from oracle import integrals, green, selfenergy as se, split as sp, variants as va


def _tiny(naux=5, n=4, seed=3):
    """A random symmetric factor tensor small enough to enumerate every sign
    vector (2^naux), with a real Green's function."""
    b = ci.random_three_index(naux, n, seed) * 0.3
    f = ci.random_symmetric(n, seed + 1)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, n // 2)
    g, gb = green.green_tau(e, c, mu, 7.0, [1.3])
    spl = sp.split_b(b, 0.35)
    return b, spl, g[0], gb[0]


def test_chain_is_eq_sigma_with_one_bilinear_vertex_each():
    b, spl, g, gb = _tiny()
    a, d = b[0], b[1] + 0.5 * b[2]
    v1 = np.einsum("ij,kl->ijkl", a, a)
    v2 = np.einsum("ij,kl->ijkl", d, d)
    ref = se.sigma_bruteforce(v1, v2, g, gb)
    assert np.allclose(va.chain(a, d, g, gb), ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def _signs(naux):
    return np.array(list(itertools.product([1.0, -1.0], repeat=naux)))


def test_control_variate_estimator_is_unbiased_by_enumeration():
    """Averaged over every pair of sign vectors, chain(R, R') - chain(R^L,
    R'^L) equals Sigma_RI - Sigma[D, D] exactly (E[theta theta^T] = I)."""
    b, spl, g, gb = _tiny()
    th = _signs(b.shape[0])
    rt, rl, _ = sp.r_vectors(b, spl, th)
    acc = np.zeros_like(g)
    for i in range(th.shape[0]):
        for j in range(th.shape[0]):
            acc += va.sigma_pair_cv(rt[i], rl[i], rt[j], rl[j], g, gb)
    acc /= th.shape[0] ** 2
    want = se.sigma_ri(b, g, gb) - se.sigma_dd(spl, g, gb)
    assert np.abs(spl.kl_dense()).max() > 0 and np.abs(b - spl.kl_dense()).max() > 0   # both parts present
    assert np.allclose(acc, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_double_sum_terms_are_the_pair_estimator_and_unbiased():
    """The double average over sets of two vectors each, averaged over every
    choice of the four sign vectors, equals Sigma_RI - Sigma[D, D]; and its
    (i, i) terms are the paired estimator's."""
    b, spl, g, gb = _tiny(naux=4)
    th = _signs(b.shape[0])
    _, xl, xs = sp.r_vectors(b, spl, th)
    m = th.shape[0]
    acc = np.zeros_like(g)
    count = 0
    for i0, i1 in itertools.product(range(m), repeat=2):
        for j0 in range(m):
            j1 = (j0 * 7 + i0 + 3) % m              # a fixed bijection of the last index keeps the sum complete
            mean, per = va.sigma_double(spl, xl[[i0, i1]], xs[[i0, i1]], xl[[j0, j1]], xs[[j0, j1]], g, gb)
            acc += mean
            count += 1
    acc /= count
    want = se.sigma_ri(b, g, gb) - se.sigma_dd(spl, g, gb)
    assert np.allclose(acc, want, rtol=0, atol=1e-12 * np.abs(want).max())
    mean, per = va.sigma_double(spl, xl[[1, 2]], xs[[1, 2]], xl[[3, 5]], xs[[3, 5]], g, gb)
    assert np.array_equal(per[0][0], se.sigma_pair(spl, xl[1], xs[1], xl[3], xs[3], g, gb))


def test_double_stderr_closed_form_for_additive_samples():
    """For e_ij = a_i + b_j the double mean is mean(a) + mean(b) and the
    first-order U-statistic variance is Var(a)/n_i + Var(b)/n_j exactly."""
    r = np.random.default_rng(0)
    a, bb = r.standard_normal(7), 3.0 * r.standard_normal(5)
    e = a[:, None] + bb[None, :]
    m, s = va.double_mean_stderr(e)
    assert abs(m - (a.mean() + bb.mean())) < 1e-14
    assert abs(s - np.sqrt(a.var(ddof=1) / 7 + bb.var(ddof=1) / 5)) < 1e-14


def test_control_variate_variance_exceeds_the_range_separated_one():
    """Exact per-pair variances of the trace Tr(Sigma_s Gbar) by enumeration:
    the control-variate form samples the D (x) S cross terms that the
    L/S-resolved form keeps exact, and pays for it in variance."""
    b, spl, g, gb = _tiny()
    th = _signs(b.shape[0])
    rt, rl, rs = sp.r_vectors(b, spl, th)
    cv, rs_ = [], []
    for i in range(0, th.shape[0], 3):
        for j in range(1, th.shape[0], 5):
            cv.append(np.sum(va.sigma_pair_cv(rt[i], rl[i], rt[j], rl[j], g, gb) * gb.T))
            rs_.append(np.sum(se.sigma_pair(spl, rl[i], rs[i], rl[j], rs[j], g, gb) * gb.T))
    assert np.var(cv) > np.var(rs_)
