"""Pins of the screened front end (oracle/integrals.screen_three_index,
eq:V_ijA, then the second eq:K_ijQ and eq:K_L): a hand-evaluated case, the
limits eps' = 0 (nothing dropped) and eps' large (only the per-j maxima),
the per-j threshold against a loop over elements, and the RS-SRI estimator
built on the screened large part staying unbiased for v = sum_Q K^Q K^Q by
enumeration of every sign vector."""
import itertools

import numpy as np

import chain_inputs as ci
from oracle import green, integrals, selfenergy as se, split as sp


def test_hand_evaluated_case():
    """N = 2, N_aux = 2: column j = 0 holds 4, -1, 0.5, 0.05 ((A, i) =
    (0,0), (0,1), (1,0), (1,1)); its threshold at eps' = 0.1 is 0.1 / 2 * 4 =
    0.2: 0.05 goes.  Column j = 1 holds 2, 0.02, -0.3, 0.19: threshold 0.1;
    0.02 goes, 0.19 stays."""
    ija = np.zeros((2, 2, 2))
    ija[0, 0, 0], ija[0, 1, 0], ija[1, 0, 0], ija[1, 1, 0] = 4.0, -1.0, 0.5, 0.05
    ija[0, 0, 1], ija[0, 1, 1], ija[1, 0, 1], ija[1, 1, 1] = 2.0, 0.02, -0.3, 0.19
    got = integrals.screen_three_index(ija, 0.1)
    want = ija.copy()
    want[1, 1, 0] = 0.0
    want[0, 1, 1] = 0.0
    assert np.array_equal(got, want)


def test_limits():
    ija = ci.random_three_index(7, 6, 3)
    assert np.array_equal(integrals.screen_three_index(ija, 0.0), ija)
    # eps' = N keeps exactly the elements equal in size to their column maximum
    got = integrals.screen_three_index(ija, 6.0)
    m = np.abs(ija).max(axis=(0, 1))
    assert np.array_equal(got != 0, np.abs(ija) == m[None, None, :])


def test_threshold_is_per_j_by_element_loop():
    """The inclusive per-j test of eq:V_ijA checked element by element on a
    chain-shaped tensor (columns far apart have very different maxima)."""
    geo = ci.chain_geometry(4)
    ija = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    ija[:, :, 3] *= 1e-3                      # one weak column: a global threshold would drop it
    eps_p = 0.02
    got = integrals.screen_three_index(ija, eps_p)
    naux, n, _ = ija.shape
    for j in range(n):
        m_j = max(abs(ija[a, i, j]) for a in range(naux) for i in range(n))
        for a in range(naux):
            for i in range(n):
                keep = abs(ija[a, i, j]) >= eps_p / n * m_j
                assert got[a, i, j] == (ija[a, i, j] if keep else 0.0)
    assert np.count_nonzero(got[:, :, 3]) > 0


def _signs(naux):
    return np.array(list(itertools.product([1.0, -1.0], repeat=naux)))


def test_estimator_on_the_screened_large_part_is_unbiased():
    """K from the full (ij|A), K^L from the screened one (then eq:K_L): the
    average over every sign vector of D + R^L R^S + R^S R^L + R^S R^S is
    v = sum_Q K^Q K^Q, and so the pair estimator averages to the
    deterministic RI self-energy."""
    naux, n = 5, 4
    ija = ci.random_three_index(naux, n, 11) * 0.4
    v = ci.random_spd(naux, 12)
    k_full = integrals.b_from_three_index(ija, v)
    k_lpre = integrals.b_from_three_index(integrals.screen_three_index(ija, 1.5), v)
    spl = sp.split_b(k_lpre, 0.2)
    assert np.abs(k_full - spl.kl_dense()).max() > 1e-3          # the large part is not K masked
    th = _signs(naux)
    r, rl, rs = sp.r_vectors(k_full, spl, th)
    assert np.allclose(r, np.einsum("sq,qij->sij", th, k_full))
    f = ci.random_symmetric(n, 13)
    e, c = green.orbitals(f)
    g, gb = green.green_tau(e, c, green.midgap_mu(e, n // 2), 8.0, [1.1])
    acc = np.zeros((n, n))
    m = th.shape[0]
    for i in range(m):
        for j in range(m):
            acc += se.sigma_pair(spl, rl[i], rs[i], rl[j], rs[j], g[0], gb[0])
    acc /= m * m
    want = se.sigma_ri(k_full, g[0], gb[0]) - se.sigma_dd(spl, g[0], gb[0])
    assert np.allclose(acc, want, rtol=0, atol=1e-12 * np.abs(want).max())
