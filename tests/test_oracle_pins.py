"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
literal 4-index sum of eq:sigma, closed forms in the orbital basis, the
textbook MP2 limit, matrix exponentials, exhaustive enumeration of the
stochastic orbitals, exact limits of the range separation, and published
test vectors of the random-number finaliser.
"""
import itertools
import os

import numpy as np
import pytest
import scipy.linalg

import chain_inputs as ci
from oracle import energy, green, integrals, rng, selfenergy as se, split as sp

HERE = os.path.dirname(os.path.abspath(__file__))


def _chain(n_dimer, beta=50.0, ntau=8):
    geo = ci.chain_geometry(n_dimer)
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    f = ci.fock_tight_binding(geo.x)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, geo.n // 2)
    tau, w = green.tau_grid(beta, ntau)
    g, gb = green.green_tau(e, c, mu, beta, tau)
    return dict(geo=geo, b=b, f=f, e=e, c=c, mu=mu, beta=beta, tau=tau, w=w, g=g, gb=gb)


def _random_problem(n, naux, seed):
    b = 0.3 * ci.random_three_index(naux, n, seed)
    f = ci.random_symmetric(n, seed + 1, 0.3)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, n // 2)
    tau, w = green.tau_grid(7.0, 4)
    g, gb = green.green_tau(e, c, mu, 7.0, tau)
    return b, g, gb


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ----------------------------------------------------------------- RNG --------

def test_splitmix_published_vectors():
    """The finaliser reproduces the reference SplitMix64 outputs."""
    gold = []
    with open(os.path.join(HERE, "golden", "splitmix64.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                n, h = line.split()
                gold.append((int(n), int(h, 16)))
    for n, h in gold:
        with np.errstate(over="ignore"):
            z = np.array([np.uint64(n) * rng.GOLDEN], dtype=np.uint64)
        assert int(rng._mix(z)[0]) == h


def test_rademacher_balanced_and_streams_independent():
    t0 = rng.rademacher(0, 0, 256, 600)
    t1 = rng.rademacher(0, 1, 256, 600)
    assert set(np.unique(t0)) == {-1.0, 1.0}
    assert abs(t0.mean()) < 0.01
    # E[theta theta^T] = I within sampling noise (1/sqrt(256) ~ 0.06)
    cov = t0.T @ t0 / 256
    off = cov - np.diag(np.diag(cov))
    assert np.allclose(np.diag(cov), 1.0)
    assert np.abs(off).max() < 0.35
    assert np.mean(t0 == t1) < 0.55
    # counter based: a sub-range equals the slice of a longer draw
    assert np.array_equal(rng.rademacher(0, 0, 8, 600, s0=100), rng.rademacher(0, 0, 256, 600)[100:108])


def test_cdf_sampling_frequencies():
    p = ci.random_weights(12, 3)
    cdf = rng.proposal_cdf(p)
    assert cdf[-1] == 1.0
    q, s = rng.importance_draws(5, 0, 200000, 1, cdf)
    freq = np.bincount(q[:, 0], minlength=12) / 200000
    assert np.abs(freq - p).max() < 4 * np.sqrt(p.max() / 200000) + 1e-3
    assert abs(s.mean()) < 0.01


# ------------------------------------------------------- Green's function -----

def test_green_against_matrix_exponential():
    """G(tau) = -exp(-(F-mu)tau) [1 + exp(-beta(F-mu))]^{-1} for S = I."""
    d = _chain(4, beta=20.0, ntau=5)
    h = d["f"] - d["mu"] * np.eye(d["geo"].n)
    occ = np.linalg.inv(np.eye(d["geo"].n) + scipy.linalg.expm(-d["beta"] * h))
    for t, tv in enumerate(d["tau"]):
        ref = -scipy.linalg.expm(-tv * h) @ occ
        assert _rel(d["g"][t], ref) < 1e-10      # expm itself carries ~1e-12
        refb = -scipy.linalg.expm(-(d["beta"] - tv) * h) @ occ
        assert _rel(d["gb"][t], refb) < 1e-10


def test_green_jump_and_particle_number():
    d = _chain(5, beta=50.0, ntau=4)
    g0, gbeta = green.green_tau(d["e"], d["c"], d["mu"], d["beta"], [1e-14])
    # G(0+) + G(beta-) = -S^{-1} = -I (eq:Smatrix)
    assert np.abs(g0[0] + gbeta[0] + np.eye(d["geo"].n)).max() < 1e-12
    # N_e = -2 Tr G(beta-) S = 2 sum_k f_k, and ~N at half filling up to the
    # thermal tail exp(-beta gap / 2) of each orbital
    ne = green.electron_count(d["e"], d["c"], d["mu"], d["beta"])
    f = green.occupations(d["e"], d["mu"], d["beta"])
    assert abs(ne - 2.0 * f.sum()) < 1e-12
    n = d["geo"].n
    gap = d["e"][n // 2] - d["e"][n // 2 - 1]
    assert abs(ne - n) < 2 * n * np.exp(-0.5 * d["beta"] * gap)


def test_green_nonorthogonal_overlap():
    n = 8
    s = ci.random_overlap(n, 11)
    f = ci.random_symmetric(n, 12, 0.4)
    e, c = green.orbitals(f, s)
    assert np.allclose(c.T @ s @ c, np.eye(n), atol=1e-12)
    assert np.allclose(f @ c, s @ c * e, atol=1e-12)
    mu = green.midgap_mu(e, n // 2)
    g0, gb = green.green_tau(e, c, mu, 30.0, [1e-15])
    assert np.abs(g0[0] + gb[0] + np.linalg.inv(s)).max() < 1e-10


def test_tau_grid_symmetry():
    tau, w = green.tau_grid(50.0, 32)
    assert np.allclose(tau + tau[::-1], 50.0)
    assert abs(w.sum() - 50.0) < 1e-12
    d = _chain(3, beta=50.0, ntau=6)
    # Gb(tau_t) = G(beta - tau_t) = G(tau_{n-1-t}) on the symmetric grid
    assert np.abs(d["gb"] - d["g"][::-1]).max() < 1e-13


# ------------------------------------------------------------ eq:sigma --------

def test_bilinear_form_matches_bruteforce():
    n = 5
    r = [ci.random_symmetric(n, s) for s in range(4)]
    r[1] = np.random.default_rng(9).standard_normal((n, n))   # general, not symmetric
    _, g, gb = _random_problem(n, 3, 20)
    v1 = np.einsum("im,qk->imqk", r[0], r[1])
    v2 = np.einsum("lp,nj->lpnj", r[2], r[3])
    bf = se.sigma_bruteforce(v1, v2, g[1], gb[1])
    assert _rel(se.sigma_bilinear(r[0], r[1], r[2], r[3], g[1], gb[1]), bf) < 1e-13


def test_sigma_ri_matches_bruteforce_random_b():
    b, g, gb = _random_problem(6, 10, 30)
    v = integrals.four_index(b)
    for t in range(2):
        assert _rel(se.sigma_ri(b, g[t], gb[t]), se.sigma_bruteforce(v, v, g[t], gb[t])) < 1e-13


def test_four_index_eightfold_symmetry():
    b = _chain(3)["b"]
    v = integrals.four_index(b)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.abs(v - v.transpose(perm)).max() < 1e-15


def test_sigma_ri_symmetric():
    d = _chain(4)
    s = se.sigma_ri(d["b"], d["g"][2], d["gb"][2])
    assert np.abs(s - s.T).max() < 1e-14 * np.abs(s).max()


def test_sigma_dd_and_cross_terms_match_bruteforce():
    d = _chain(3, ntau=4)
    b = d["b"]
    spl = sp.split_b(b, 1e-2)
    kl = spl.kl_dense()
    dvert = integrals.four_index(kl)
    g, gb = d["g"][1], d["gb"][1]
    assert _rel(se.sigma_dd(spl, g, gb), se.sigma_bruteforce(dvert, dvert, g, gb)) < 1e-13
    th = rng.rademacher(7, 0, 1, b.shape[0])
    thp = rng.rademacher(7, 1, 1, b.shape[0])
    _, xl, xs = sp.r_vectors(b, spl, th)
    _, yl, ys = sp.r_vectors(b, spl, thp)
    sx = (np.einsum("im,qk->imqk", xl[0], xs[0]) + np.einsum("im,qk->imqk", xs[0], xl[0])
          + np.einsum("im,qk->imqk", xs[0], xs[0]))
    sy = (np.einsum("im,qk->imqk", yl[0], ys[0]) + np.einsum("im,qk->imqk", ys[0], yl[0])
          + np.einsum("im,qk->imqk", ys[0], ys[0]))
    # the per-pair estimate of eq:sigma_2 is Sigma[D+S_xi, D+S_eta] - Sigma[D, D]
    full = se.sigma_bruteforce(dvert + sx, dvert + sy, g, gb)
    ref = full - se.sigma_bruteforce(dvert, dvert, g, gb)
    got = se.sigma_pair(spl, xl[0], xs[0], yl[0], ys[0], g, gb)
    assert _rel(got, ref) < 1e-12
    # the JK regrouping equals the per-Q sum of bilinear terms
    per_q = sum(se.sigma_bilinear(kl[q], kl[q], ys[0], yl[0], g, gb) for q in range(kl.shape[0]))
    assert _rel(se.sigma_d_left(spl, ys[0], yl[0], g, gb), per_q) < 1e-13
    per_q = sum(se.sigma_bilinear(xs[0], xl[0], kl[q], kl[q], g, gb) for q in range(kl.shape[0]))
    assert _rel(se.sigma_d_right(spl, xs[0], xl[0], g, gb), per_q) < 1e-13


def test_sigma_matches_orbital_closed_form():
    d = _chain(4, beta=30.0, ntau=3)
    smo = energy.sigma_mo(d["b"], d["e"], d["c"], d["mu"], d["beta"], d["tau"])
    for t in range(3):
        ao = d["c"] @ smo[t] @ d["c"].T
        assert _rel(se.sigma_ri(d["b"], d["g"][t], d["gb"][t]), ao) < 1e-12


# ------------------------------------------------------------ energy ----------

def test_energy_quadrature_converges_to_closed_form():
    d = _chain(3, beta=7.0)
    exact = energy.energy_integral_mo(d["b"], d["e"], d["c"], d["mu"], d["beta"])
    errs = []
    for nt in (4, 8, 16, 32):
        tau, w = green.tau_grid(d["beta"], nt)
        g, gb = green.green_tau(d["e"], d["c"], d["mu"], d["beta"], tau)
        sig = np.array([se.sigma_ri(d["b"], g[t], gb[t]) for t in range(nt)])
        errs.append(abs(np.dot(w, energy.energy_integrand(sig, gb)) - exact) / abs(exact))
    assert errs[-1] < 1e-13
    assert errs[0] > errs[1] > errs[2]


def test_energy_zero_temperature_limit_is_mp2():
    """-GM * int Tr(Sigma Gb) -> textbook closed-shell MP2 as beta -> infinity
    (fixes the sign and factor of eq:corr)."""
    d = _chain(4)
    n_occ = d["geo"].n // 2
    mp2 = energy.mp2_energy(d["b"], d["e"], d["c"], n_occ)
    val = -energy.GM_FACTOR * energy.energy_integral_mo(d["b"], d["e"], d["c"], d["mu"], 2000.0)
    assert mp2 < 0
    assert abs(val - mp2) < 1e-12 * abs(mp2)


def test_energy_quadrature_at_beta50_matches_closed_form():
    d = _chain(5, beta=50.0, ntau=32)
    sig = np.array([se.sigma_ri(d["b"], d["g"][t], d["gb"][t]) for t in range(32)])
    e_quad = energy.energy_total(sig, d["gb"], d["w"])
    e_exact = -energy.GM_FACTOR * energy.energy_integral_mo(d["b"], d["e"], d["c"], d["mu"], 50.0)
    assert abs(e_quad - e_exact) < 1e-6 * abs(e_exact)


# ------------------------------------------------- range separation limits ----

def test_eps_zero_is_deterministic_ri():
    d = _chain(3, ntau=4)
    spl = sp.split_b(d["b"], 0.0)
    th = rng.rademacher(1, 0, 2, d["b"].shape[0])
    r, rl, rs = sp.r_vectors(d["b"], spl, th)
    assert np.abs(rs).max() < 1e-15          # everything is "large"
    g, gb = d["g"][1], d["gb"][1]
    assert np.abs(se.sigma_pair(spl, rl[0], rs[0], rl[1], rs[1], g, gb)).max() < 1e-14
    assert _rel(se.sigma_dd(spl, g, gb), se.sigma_ri(d["b"], g, gb)) < 1e-13


def test_empty_large_part_is_pure_sri():
    """eps > 1 empties K^L, so eq:RS-SRI reduces to the SRI of eq:abgd_l."""
    d = _chain(3, ntau=4)
    spl = sp.split_b(d["b"], 1.5)
    assert spl.nnz == 0
    th = rng.rademacher(2, 0, 1, d["b"].shape[0])
    thp = rng.rademacher(2, 1, 1, d["b"].shape[0])
    r, rl, rs = sp.r_vectors(d["b"], spl, th)
    rp, rlp, rsp = sp.r_vectors(d["b"], spl, thp)
    g, gb = d["g"][2], d["gb"][2]
    ref = se.sigma_bilinear(r[0], r[0], rp[0], rp[0], g, gb)
    assert _rel(se.sigma_pair(spl, rl[0], rs[0], rlp[0], rsp[0], g, gb), ref) < 1e-13


def test_split_threshold_inclusive_and_blocks():
    b = _chain(4)["b"]
    spl = sp.split_b(b, 1e-2)
    kl = spl.kl_dense()
    m = np.abs(b).max()
    keep = np.abs(b) >= 1e-2 * m
    assert np.array_equal(kl != 0, keep)
    # an element exactly at the threshold is kept
    q, i, j = np.unravel_index(np.argmax(np.abs(b)), b.shape)
    b2 = b.copy()
    b2[0, 0, 1] = b2[0, 1, 0] = 1e-2 * m
    spl2 = sp.split_b(b2, 1e-2)
    assert spl2.kl_slice(0)[0, 1] == 1e-2 * m
    assert spl.wmax <= b.shape[1]


# ------------------------------------------------------- enumeration ----------

def _enumerate_setup():
    b = 0.3 * ci.random_three_index(5, 4, 44)
    spl = sp.split_b(b, 0.3)
    assert 0 < spl.nnz < b.size
    f = ci.random_symmetric(4, 45, 0.3)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, 2)
    g, gb = green.green_tau(e, c, mu, 5.0, [1.3])
    return b, spl, g[0], gb[0]


def test_enumeration_of_rademacher_pairs_is_exact():
    """Averaging the pair estimate over all 2^Naux x 2^Naux sign vectors gives
    Sigma_RI - Sigma[D,D] exactly (E[theta theta^T] = I)."""
    b, spl, g, gb = _enumerate_setup()
    naux = b.shape[0]
    signs = np.array(list(itertools.product([1.0, -1.0], repeat=naux)))
    _, rl, rs = sp.r_vectors(b, spl, signs)
    tot = np.zeros((4, 4))
    for a in range(signs.shape[0]):
        for c in range(signs.shape[0]):
            tot += se.sigma_pair(spl, rl[a], rs[a], rl[c], rs[c], g, gb)
    tot /= signs.shape[0] ** 2
    ref = se.sigma_ri(b, g, gb) - se.sigma_dd(spl, g, gb)
    assert _rel(tot, ref) < 1e-12


def test_enumeration_of_importance_draws_is_exact():
    """k = 1 importance vectors: sum_{Q,Q'} p_Q p_Q' (estimate) = Sigma_RI - Sigma_DD."""
    from oracle import proposal
    b, spl, g, gb = _enumerate_setup()
    naux = b.shape[0]
    p = ci.random_weights(naux, 46)
    eye = np.eye(naux)
    tot = np.zeros((4, 4))
    for q in range(naux):
        _, xl, xs = sp.r_vectors(b, spl, eye[q:q + 1] / np.sqrt(p[q]))
        for r in range(naux):
            _, yl, ys = sp.r_vectors(b, spl, -eye[r:r + 1] / np.sqrt(p[r]))
            tot += p[q] * p[r] * se.sigma_pair(spl, xl[0], xs[0], yl[0], ys[0], g, gb)
    ref = se.sigma_ri(b, g, gb) - se.sigma_dd(spl, g, gb)
    assert _rel(tot, ref) < 1e-12
    # the generator builds the same vectors the enumeration uses
    th = proposal.importance_theta(p, 3, 0, 50, 1)
    nzc = np.count_nonzero(th, axis=1)
    assert np.all(nzc == 1)
    qs = np.argmax(np.abs(th), axis=1)
    assert np.allclose(np.abs(th[np.arange(50), qs]), 1.0 / np.sqrt(p[qs]))


def _stratified_states(naux, nclass, pi):
    """Every (class, sign pattern) state of one stratified vector and its
    probability: class c with pi_c, signs of the class members uniform."""
    states, probs = [], []
    for c in range(nclass):
        members = np.arange(naux)[np.arange(naux) % nclass == c]
        for sg in itertools.product([1.0, -1.0], repeat=members.shape[0]):
            th = np.zeros(naux)
            th[members] = np.array(sg) / np.sqrt(pi[c])
            states.append(th)
            probs.append(pi[c] / 2.0 ** members.shape[0])
    return np.array(states), np.array(probs)


def test_enumeration_of_stratified_vectors_is_exact():
    """Stratified vectors (one class drawn per vector, +-1 on its members,
    scaled by 1/sqrt(pi_c)): E[theta theta^T] = I, and the pair estimate
    averaged over all states of both vectors is Sigma_RI - Sigma[D,D]."""
    from oracle import proposal
    b, spl, g, gb = _enumerate_setup()
    naux = b.shape[0]
    p = ci.random_weights(naux, 47)
    nclass = 3
    pi = proposal.class_probabilities(p, nclass)
    th, pr_ = _stratified_states(naux, nclass, pi)
    assert abs(pr_.sum() - 1.0) < 1e-14
    assert _rel(np.einsum("s,si,sj->ij", pr_, th, th), np.eye(naux)) < 1e-14
    _, rl, rs = sp.r_vectors(b, spl, th)
    tot = np.zeros((4, 4))
    for a in range(th.shape[0]):
        for c in range(th.shape[0]):
            tot += pr_[a] * pr_[c] * se.sigma_pair(spl, rl[a], rs[a], rl[c], rs[c], g, gb)
    ref = se.sigma_ri(b, g, gb) - se.sigma_dd(spl, g, gb)
    assert _rel(tot, ref) < 1e-12
    # the generator draws only such states: one class, +-1/sqrt(pi_c) on it
    thg = proposal.stratified_theta(p, nclass, 5, 1, 40)
    for v in thg:
        nz = np.nonzero(v)[0]
        assert np.all(nz % nclass == nz[0] % nclass)
        assert np.allclose(np.abs(v[nz]), 1.0 / np.sqrt(pi[nz[0] % nclass]))
        assert nz.shape[0] == np.count_nonzero(np.arange(naux) % nclass == nz[0] % nclass)
