"""Pins of the oracle's auxiliary functions: the proposal features, the density
matrix, the per-Q targets, the network initialisation and optimiser, and the
RI factor contraction of eq:K_ijQ.

Each test fixes a value by a route other than the function under test:
designed inputs with hand-known answers, a second formula for the same
quantity (the particle number, the Green's function at the other end of the
interval, the Coulomb/exchange map of eq:sigma), or a closed form of the
algorithm (Adam's first step)."""
import numpy as np

import chain_inputs as ci
from oracle import energy, green, integrals, proposal as pr, rng, selfenergy as se, split as sp


# ---------------------------------------------------------------------------
# raw_features
# ---------------------------------------------------------------------------

def test_features_on_designed_inputs():
    """Hand-evaluated features: atoms at 0, 1, 5 with centres at -1, 0, 2,
    4.5, 5; B_Q = (Q+1) * A with A a fixed non-symmetric 3x3 pattern whose
    Frobenius norm is known; K_Q = B_Q / 4 (so B_Q - K_Q = 3/4 B_Q); P = a
    single off-diagonal element (selects one entry, catching a transpose)."""
    x = np.array([0.0, 1.0, 5.0])
    xq = np.array([-1.0, 0.0, 2.0, 4.5, 5.0])
    a = np.array([[1.0, 2.0, 0.0],
                  [0.0, 0.0, 2.0],
                  [0.0, 4.0, 0.0]])          # ||A||_F = sqrt(1 + 4 + 4 + 16) = 5
    b = np.stack([(q + 1.0) * a for q in range(5)])
    kl = b / 4.0
    p = np.zeros((3, 3))
    p[0, 1] = 0.5                             # picks B_Q[0, 1] = 2 (Q+1); B_Q[1, 0] = 0
    phi = pr.raw_features(x, xq, b, kl, p)
    d_end = np.array([-1.0, 0.0, 2.0, 0.5, 0.0])   # distance to the nearer end
    for q in range(5):
        assert abs(phi[q, 0] - np.tanh(d_end[q] / 4.0)) < 1e-15
        assert abs(phi[q, 1] - np.log(5.0 * (q + 1))) < 1e-13
        assert abs(phi[q, 2] - np.log(0.75 * 5.0 * (q + 1))) < 1e-13
        assert abs(phi[q, 3] - (q + 1.0)) < 1e-14


def test_features_mirror_symmetry_of_the_chain():
    """The synthetic chain is mirror-symmetric (0.74/1.5 spacings with whole
    dimers), and so are its centres and B: every feature of centre Q equals
    that of centre N_aux-1-Q, with the mid-gap density of the mirrored chain."""
    geo = ci.chain_geometry(3)
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    f = ci.fock_tight_binding(geo.x)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, geo.n // 2)
    dens = pr.density_matrix(e, c, mu, 40.0)
    spl = sp.split_b(b, 1e-2)
    phi = pr.raw_features(geo.x, geo.xq, b, spl.kl_dense(), dens)
    assert np.allclose(phi, phi[::-1], rtol=0, atol=1e-12)
    assert phi[1, 0] == 0.0                  # the first atom sits on the chain end


# ---------------------------------------------------------------------------
# density_matrix
# ---------------------------------------------------------------------------

def _tb_orbitals(nd=4):
    geo = ci.chain_geometry(nd)
    f = ci.fock_tight_binding(geo.x)
    e, c = green.orbitals(f)
    return geo, e, c, green.midgap_mu(e, geo.n // 2)


def test_density_is_minus_two_g_at_beta_minus():
    """P = -2 G(beta-): the oracle's G(tau) at tau = beta (the (1-f) e^{-e~ tau}
    branch) and its G(beta - tau) at tau = 0 (the f e^{e~ tau} branch) are two
    routes to G(beta-); P must equal -2 times both."""
    geo, e, c, mu = _tb_orbitals()
    beta = 7.0
    g, gb = green.green_tau(e, c, mu, beta, [beta, 0.0])
    p = pr.density_matrix(e, c, mu, beta)
    assert np.allclose(p, -2.0 * g[0], rtol=0, atol=1e-13)
    assert np.allclose(p, -2.0 * gb[1], rtol=0, atol=1e-13)


def test_density_trace_and_idempotency():
    """Tr P = N_e = 2 sum f (Section III's particle number) and, with the
    mid-gap chemical potential at large beta, P/2 is the projector onto the
    occupied orbitals: (P/2)^2 = P/2 and Tr P = N."""
    geo, e, c, mu = _tb_orbitals()
    p_warm = pr.density_matrix(e, c, mu, 3.0)
    assert abs(np.trace(p_warm) - green.electron_count(e, c, mu, 3.0)) < 1e-12
    p = pr.density_matrix(e, c, mu, 500.0)
    h = 0.5 * p
    assert abs(np.trace(p) - geo.n) < 1e-10
    assert np.abs(h @ h - h).max() < 1e-10


# ---------------------------------------------------------------------------
# targets_from_tables
# ---------------------------------------------------------------------------

def test_targets_equal_the_direct_contributions():
    """t_Q = |cL_Q| + |cR_Q| + sum_Q' |d_QQ'| with, for S_Q = B_Q (x) B_Q -
    K_Q (x) K_Q and the tau-quadrature of Tr(Sigma Gb):
      d_QQ' = int Tr(Sigma[S_Q, S_Q'] Gb)   (the bilinear pieces of eq:sigma),
      cL_Q  = int Tr(Sigma[D, S_Q] Gb)      (Coulomb/exchange map of D),
      cR_Q  = int Tr(Sigma[S_Q, D] Gb).
    G and Gb are random non-symmetric matrices here, so that left and right
    contributions differ and a swapped table axis is caught."""
    geo = ci.chain_geometry(2)
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    spl = sp.split_b(b, 5e-2)
    kl = spl.kl_dense()
    bt = pr.truncate(b)
    n, naux = geo.n, geo.naux
    r = np.random.default_rng(7)
    g = r.standard_normal((2, n, n)) * 0.3
    gb = r.standard_normal((2, n, n)) * 0.3
    w = np.array([0.7, 1.3])
    tab = pr.pair_tables(bt, kl, g, gb, w)
    t = pr.targets_from_tables(tab)

    def integ(sig_of_t):
        return sum(w[k] * energy.trace_product(sig_of_t(k), gb[k]) for k in range(2))

    # the D vertex built from the same blocks as the split
    def s_terms(q):
        return [(bt[q], bt[q], 1.0), (kl[q], kl[q], -1.0)]

    d = np.zeros((naux, naux))
    for q in range(naux):
        for r_ in range(naux):
            d[q, r_] = integ(lambda k: se.sigma_terms(s_terms(q), s_terms(r_), g[k], gb[k]))
    cl = np.zeros(naux)
    cr = np.zeros(naux)
    for q in range(naux):
        cl[q] = integ(lambda k: sum(cf * se.sigma_d_left(spl, a_, b_, g[k], gb[k]) for a_, b_, cf in s_terms(q)))
        cr[q] = integ(lambda k: sum(cf * se.sigma_d_right(spl, a_, b_, g[k], gb[k]) for a_, b_, cf in s_terms(q)))
    assert np.abs(cl - cr).max() > 1e-3 * np.abs(cl).max()      # the test can see an axis swap
    want = np.abs(cl) + np.abs(cr) + np.abs(d).sum(axis=1)
    assert np.allclose(t, want, rtol=1e-11, atol=1e-14 * np.abs(want).max())


# ---------------------------------------------------------------------------
# init_mlp, adam_step
# ---------------------------------------------------------------------------

def test_init_mlp_ranges_and_moments():
    """Weights uniform on (-1/sqrt(fan_in), 1/sqrt(fan_in)) per layer (fan_in =
    D_IN for W1 and b1, HIDDEN for w2): bounds, mean ~ 0, variance
    1/(3 fan_in) within sampling error, reproducible per seed."""
    m = pr.init_mlp(11, np.zeros(pr.D_IN), np.ones(pr.D_IN))
    m2 = pr.init_mlp(11, np.zeros(pr.D_IN), np.ones(pr.D_IN))
    m3 = pr.init_mlp(12, np.zeros(pr.D_IN), np.ones(pr.D_IN))
    assert np.array_equal(m.w1, m2.w1) and not np.array_equal(m.w1, m3.w1)
    for arr, fan in ((m.w1, pr.D_IN), (m.b1, pr.D_IN), (m.w2, pr.HIDDEN)):
        lim = 1.0 / np.sqrt(fan)
        assert np.abs(arr).max() < lim
        var = 1.0 / (3.0 * fan)
        nel = arr.size
        assert abs(arr.mean()) < 4.0 * np.sqrt(var / nel)
        assert abs(arr.var() / var - 1.0) < 4.0 * np.sqrt(0.8 / nel)   # Var(u^2)/E(u^2)^2 = 4/5
    # the layout: W1 takes the first HIDDEN*D_IN words of stream 2, row-major
    u = rng.uniform_from_word(rng.words(11, 2, 0, np.array([0, 1, pr.D_IN])))
    assert m.w1[0, 0] == (2.0 * u[0] - 1.0) / np.sqrt(pr.D_IN)
    assert m.w1[0, 1] == (2.0 * u[1] - 1.0) / np.sqrt(pr.D_IN)
    assert m.w1[1, 0] == (2.0 * u[2] - 1.0) / np.sqrt(pr.D_IN)


def test_adam_first_step_closed_form():
    """With zero moments the bias-corrected first Adam step moves every
    parameter by exactly -lr g / (|g| + eps) (Kingma & Ba 2015, Sec. 2)."""
    m = pr.init_mlp(0, np.zeros(pr.D_IN), np.ones(pr.D_IN))
    st = pr.adam_init(m)
    r = np.random.default_rng(3)
    grads = [r.standard_normal(m.w1.shape), r.standard_normal(m.b1.shape) * 1e-3,
             r.standard_normal(m.w2.shape) * 1e3]
    before = [m.w1.copy(), m.b1.copy(), m.w2.copy()]
    lr, eps = 3e-3, 1e-8
    pr.adam_step(m, st, grads, lr=lr, eps=eps)
    for p0, p1, gr in zip(before, [m.w1, m.b1, m.w2], grads):
        assert np.allclose(p1 - p0, -lr * gr / (np.abs(gr) + eps), rtol=1e-9, atol=1e-18)


def test_adam_constant_gradient_moves_by_lr_every_step():
    """Under a constant gradient the bias corrections make m_hat = g and
    v_hat = g^2 at every step, so each step is -lr g/(|g|+eps); without the
    corrections the second and later steps would differ."""
    m = pr.init_mlp(1, np.zeros(pr.D_IN), np.ones(pr.D_IN))
    st = pr.adam_init(m)
    r = np.random.default_rng(4)
    grads = [r.standard_normal(m.w1.shape), r.standard_normal(m.b1.shape), r.standard_normal(m.w2.shape)]
    lr = 1e-2
    for _ in range(5):
        before = [m.w1.copy(), m.b1.copy(), m.w2.copy()]
        pr.adam_step(m, st, grads, lr=lr)
        for p0, p1, gr in zip(before, [m.w1, m.b1, m.w2], grads):
            assert np.allclose(p1 - p0, -lr * gr / (np.abs(gr) + 1e-8), rtol=1e-9, atol=1e-15)


# ---------------------------------------------------------------------------
# b_from_three_index, inverse_sqrt_spd
# ---------------------------------------------------------------------------

def test_inverse_sqrt_is_an_inverse_square_root():
    v = ci.random_spd(9, 5)
    x = integrals.inverse_sqrt_spd(v)
    assert np.allclose(x, x.T, rtol=0, atol=1e-13)
    assert np.allclose(x @ v @ x, np.eye(9), rtol=0, atol=1e-12)
    assert np.allclose(np.linalg.inv(x @ x), v, rtol=0, atol=1e-11)
    assert np.linalg.eigvalsh(x).min() > 0                      # the positive root


def test_ri_factors_reproduce_the_metric_contraction():
    """eq:vKQKQ with V != I: sum_Q K^Q_ij K^Q_kl = sum_AB (ij|A) (V^-1)_AB (B|kl),
    with V^-1 applied by a linear solve (no square root involved)."""
    n, naux = 4, 11
    ija = ci.random_three_index(naux, n, 21)
    v = ci.random_spd(naux, 22)
    k = integrals.b_from_three_index(ija, v)
    four = integrals.four_index(k)
    flat = ija.reshape(naux, n * n)
    want = (flat.T @ np.linalg.solve(v, flat)).reshape(n, n, n, n)
    assert np.allclose(four, want, rtol=0, atol=1e-12 * np.abs(want).max())
    # V = None is the identity metric
    assert np.array_equal(integrals.b_from_three_index(ija, None), ija)
