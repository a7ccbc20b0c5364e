"""Pins of the self-consistent GF2 steps (oracle/scf.py): the Matsubara
transform against the closed-form non-interacting G0(i w), a static
self-energy against the G0 of the shifted Fock matrix (with the 1/n_w
convergence of the tail treatment), the anticommutator jump of the
interacting G, particle-number tuning, the RI Fock build against the 4-index
definition of eq:F, and a fixed point of the whole loop on a tiny chain."""
import numpy as np

import chain_inputs as ci
from oracle import green, integrals, scf, selfenergy as se


def _chain(nd=3, beta=10.0):
    geo = ci.chain_geometry(nd)
    f = ci.fock_tight_binding(geo.x)
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    s = np.eye(geo.n)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, geo.n // 2)
    return geo, f, b, s, e, c, mu, beta


def test_matsubara_transform_of_g0_is_the_closed_form():
    geo, f, b, s, e, c, mu, beta = _chain()
    tau, w = green.tau_grid(beta, 96)
    g, _ = green.green_tau(e, c, mu, beta, tau)
    om = scf.matsubara(beta, 8)
    got = scf.tau_to_iw(g, tau, w, om)
    want = scf.g0_iw(f, s, mu, om)
    assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()


def test_static_self_energy_gives_the_shifted_g0_with_a_one_over_nw_tail():
    """Sigma(i w) = Sigma0 (frequency independent) is a change of F: the Dyson
    G must be G0 of F + Sigma0.  The back-transform subtracts G0 of F, so the
    remainder decays as 1/w^2: its truncated Matsubara sum converges as 1/n_w
    at the ends of [0, beta] (doubling n_w halves the error) and as 1/n_w^3
    inside (the oscillating tail sums away)."""
    geo, f, b, s, e, c, mu, beta = _chain()
    r = np.random.default_rng(1)
    s0 = r.standard_normal((geo.n, geo.n)) * 0.02
    s0 = 0.5 * (s0 + s0.T)
    e2, c2 = green.orbitals(f + s0)
    for tau, rate in (([0.0], 2.0), ([0.7, 3.1, 8.9], 8.0)):
        want, _ = green.green_tau(e2, c2, mu, beta, tau)
        errs = []
        for nw in (400, 800, 1600):
            om = scf.matsubara(beta, nw)
            g, _, _ = scf.green_tau_dyson(f, s, mu, beta, np.broadcast_to(s0, (nw, geo.n, geo.n)), om, tau)
            errs.append(np.abs(g - want).max())
        assert abs(errs[0] / errs[1] - rate) < 0.05 * rate and abs(errs[1] / errs[2] - rate) < 0.05 * rate
        assert errs[2] < (2e-4 if rate == 2.0 else 1e-10) * np.abs(want).max()


def test_interacting_g_keeps_the_anticommutator_jump():
    """G(0+) + G(beta-) = -S^{-1} for any self-energy that decays at high
    frequency (here a one-pole Sigma(i w) = A / (i w - a))."""
    geo, f, b, s, e, c, mu, beta = _chain()
    r = np.random.default_rng(2)
    a_ = r.standard_normal((geo.n, geo.n)) * 0.05
    a_ = a_ @ a_.T
    om = scf.matsubara(beta, 3000)
    sig = np.array([a_ / (1j * wn - 0.3) for wn in om])
    g, _, gbeta = scf.green_tau_dyson(f, s, mu, beta, sig, om, [0.0])
    assert np.abs(g[0] + gbeta + np.eye(geo.n)).max() < 2e-4


def test_mu_tuning_conserves_the_particle_number():
    geo, f, b, s, e, c, mu, beta = _chain()
    om = scf.matsubara(beta, 200)
    r = np.random.default_rng(3)
    a_ = r.standard_normal((geo.n, geo.n)) * 0.05
    sig = np.array([(a_ + a_.T) / (1j * wn + 0.4) for wn in om])
    mu2 = scf.tune_mu(f, s, beta, sig, om, float(geo.n) - 0.3, mu - 1.0, mu + 1.0)
    ne = scf.electron_count(scf.g_beta_minus(f, s, mu2, beta, sig, om), s)
    assert abs(ne - (geo.n - 0.3)) < 1e-9
    # N_e grows with mu
    n_lo = scf.electron_count(scf.g_beta_minus(f, s, mu2 - 0.05, beta, sig, om), s)
    assert n_lo < ne


def test_ri_fock_build_is_eq_F():
    geo, f, b, s, e, c, mu, beta = _chain(2)
    p = 2.0 * (c[:, : geo.n // 2] @ c[:, : geo.n // 2].T)
    v = integrals.four_index(b)
    h = ci.random_symmetric(geo.n, 4, 0.1)
    want = h + np.einsum("kl,ijkl->ij", p, v) - 0.5 * np.einsum("kl,ilkj->ij", p, v)
    assert np.allclose(scf.fock(h, b, p), want, rtol=0, atol=1e-14)
    assert np.allclose(scf.fock(scf.core_hamiltonian(f, b, p), b, p), f, rtol=0, atol=1e-14)


def test_scf_loop_reaches_a_fixed_point():
    """Deterministic RI-GF2 on a 2-dimer chain: Sigma(tau) from G, Dyson with
    mu tuned to N_e = N, Fock update; the density stops changing and N_e is
    conserved throughout."""
    geo, f, b, s, e, c, mu, beta = _chain(2, beta=10.0)
    tau, w = green.tau_grid(beta, 48)
    om = scf.matsubara(beta, 600)
    g, gb = green.green_tau(e, c, mu, beta, tau)
    p0 = -2.0 * green.green_tau(e, c, mu, beta, [0.0])[1][0]
    h = scf.core_hamiltonian(f, b, p0)
    fk, p_prev, dps = f.copy(), p0, []
    for it in range(18):
        sig_tau = np.array([se.sigma_ri(b, g[t], gb[t]) for t in range(len(tau))])
        sig_iw = scf.tau_to_iw(sig_tau, tau, w, om)
        mu = scf.tune_mu(fk, s, beta, sig_iw, om, float(geo.n), mu - 0.5, mu + 0.5)
        g, gb, gbeta = scf.green_tau_dyson(fk, s, mu, beta, sig_iw, om, tau)
        p = -2.0 * gbeta
        assert abs(np.trace(p) - geo.n) < 1e-8
        dps.append(np.abs(p - p_prev).max())
        p_prev = p
        fk = scf.fock(h, b, p)
    # linear convergence, about a decade every two iterations on this chain
    assert dps[-1] < 1e-8 and dps[-1] < 1e-7 * dps[0]
