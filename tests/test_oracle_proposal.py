"""Pins of the proposal part of the oracle: exact gradients against central
finite differences, a training step that lowers the loss, per-Q tables
against the direct energy of eq:sigma, and the variance gain of importance
sampling (evaluated exactly by enumeration)."""
import numpy as np

import chain_inputs as ci
from oracle import energy, green, integrals, proposal as pr, rng, selfenergy as se, split as sp


def _chains(count=2, seed=0):
    out = []
    for k in range(count):
        r = np.random.default_rng(seed + k)
        naux = 9 + 3 * k
        phi = r.standard_normal((naux, pr.D_IN))
        t = r.random(naux) + 0.1
        out.append((phi, t / t.sum()))
    return out


def test_mlp_gradients_match_central_differences():
    ch = _chains()
    m = pr.init_mlp(3, np.zeros(pr.D_IN), np.ones(pr.D_IN))
    gw1, gb1, gw2 = pr.gradients(m, ch)
    h = 1e-6
    for arr, grad in ((m.w1, gw1), (m.b1, gb1), (m.w2, gw2)):
        flat = arr.reshape(-1)
        gflat = grad.reshape(-1)
        for i in np.random.default_rng(1).choice(flat.shape[0], 12, replace=False):
            old = flat[i]
            flat[i] = old + h
            lp = pr.loss(m, ch)
            flat[i] = old - h
            lm = pr.loss(m, ch)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd))


def test_adam_training_lowers_loss():
    ch = _chains(3, seed=5)
    m = pr.init_mlp(0, np.zeros(pr.D_IN), np.ones(pr.D_IN))
    st = pr.adam_init(m)
    l0 = pr.loss(m, ch)
    for _ in range(200):
        pr.adam_step(m, st, pr.gradients(m, ch), lr=1e-2)
    assert pr.loss(m, ch) < 0.5 * l0


def test_proposal_is_a_distribution_with_floor():
    z = np.random.default_rng(2).standard_normal(50) * 5
    p = pr.proposal(z, 0.1)
    assert abs(p.sum() - 1.0) < 1e-14
    assert p.min() >= 0.1 / 50 - 1e-18


def _tiny_tables():
    geo = ci.chain_geometry(2)
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    f = ci.fock_tight_binding(geo.x)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, geo.n // 2)
    tau, w = green.tau_grid(20.0, 4)
    g, gb = green.green_tau(e, c, mu, 20.0, tau)
    spl = sp.split_b(b, 5e-2)
    bt = pr.truncate(b)
    return b, bt, spl, g, gb, w, pr.pair_tables(bt, spl.kl_dense(), g, gb, w)


def test_pair_table_is_the_energy_of_eq_sigma():
    b, bt, spl, g, gb, w, tab = _tiny_tables()
    kl = spl.kl_dense()
    for q, r in ((0, 1), (3, 5), (7, 2)):
        direct = sum(w[t] * energy.trace_product(se.sigma_bilinear(bt[q], bt[q], kl[r], kl[r], g[t], gb[t]), gb[t])
                     for t in range(len(w)))
        assert abs(tab["BK"][q, r] - direct) < 1e-12 * max(1.0, abs(direct))


def test_importance_variance_gain_by_enumeration():
    """Exact per-pair variance of the k=1 estimator for uniform p and for
    p proportional to the targets: the targeted proposal is not worse."""
    b, bt, spl, g, gb, w, tab = _tiny_tables()
    t = pr.targets_from_tables(tab)
    naux = b.shape[0]
    eye = np.eye(naux)

    def pair_e(q, r, p):
        _, xl, xs = sp.r_vectors(b, spl, eye[q:q + 1] / np.sqrt(p[q]))
        _, yl, ys = sp.r_vectors(b, spl, eye[r:r + 1] / np.sqrt(p[r]))
        return sum(w[k] * energy.trace_product(se.sigma_pair(spl, xl[0], xs[0], yl[0], ys[0], g[k], gb[k]), gb[k])
                   for k in range(len(w)))

    def variance(p):
        vals = np.array([[pair_e(q, r, p) for r in range(naux)] for q in range(naux)])
        wts = p[:, None] * p[None, :]
        mean = np.sum(wts * vals)
        return np.sum(wts * (vals - mean) ** 2), mean

    vu, mu_ = variance(np.full(naux, 1.0 / naux))
    pt = 0.9 * t / t.sum() + 0.1 / naux
    vt, mt = variance(pt)
    assert abs(mu_ - mt) < 1e-10 * abs(mu_)         # both unbiased for the same value
    assert vt < vu


def test_stratified_variance_gain_by_enumeration():
    """Stratified vectors with class weights from the targets (pi_c summed over
    the class members' t_Q) against equal class weights: both unbiased for the
    same value, the targeted ones with lower variance (exact, enumerating
    every class and sign state of both vectors)."""
    import itertools
    b, bt, spl, g, gb, w, tab = _tiny_tables()
    t = pr.targets_from_tables(tab)
    naux, nclass = b.shape[0], 6

    def states(pi):
        th, prob = [], []
        for c in range(nclass):
            mem = np.arange(naux)[np.arange(naux) % nclass == c]
            for sg in itertools.product([1.0, -1.0], repeat=mem.shape[0]):
                v = np.zeros(naux)
                v[mem] = np.array(sg) / np.sqrt(pi[c])
                th.append(v)
                prob.append(pi[c] / 2.0 ** mem.shape[0])
        return np.array(th), np.array(prob)

    def moments(pi):
        th, prob = states(pi)
        _, rl, rs = sp.r_vectors(b, spl, th)
        m1 = m2 = 0.0
        for a in range(th.shape[0]):
            for c in range(th.shape[0]):
                e = sum(w[k] * energy.trace_product(se.sigma_pair(spl, rl[a], rs[a], rl[c], rs[c], g[k], gb[k]), gb[k])
                        for k in range(len(w)))
                m1 += prob[a] * prob[c] * e
                m2 += prob[a] * prob[c] * e * e
        return m1, m2 - m1 * m1

    mu_u, var_u = moments(np.full(nclass, 1.0 / nclass))
    mu_t, var_t = moments(pr.class_probabilities(t / t.sum(), nclass))
    assert abs(mu_u - mu_t) < 1e-10 * abs(mu_u)
    assert var_t < var_u
