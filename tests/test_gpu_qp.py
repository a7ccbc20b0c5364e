"""Parity of the quasiparticle energies (gf2_qp_energies) with the oracle
(oracle/qp.py): the one-pole closed form, and the deterministic RI
self-energy of the 10-dimer chain computed on each side independently.

Bar: 1e-9 in E (Eh), or ten times the oracle's own spread under a 1e-14
relative perturbation of its self-energy, whichever is larger: Thiele's
continued fraction amplifies input rounding by its conditioning, which grows
quickly with the number of points for a self-energy with many poles (the
two sides' self-energies differ by about 1e-15)."""
import numpy as np
import pytest

import chain_inputs as ci
from oracle import green, integrals, qp, selfenergy as se

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2005_12338_amd import gf2
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gf2.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("use_s", [False, True])
def test_one_pole_closed_form(ctx, use_s):
    nd, beta, ntau = 5, 20.0, 96
    geo = ci.chain_geometry(nd)
    f = ci.fock_tight_binding(geo.x)
    s = ci.random_overlap(geo.n, 3) if use_s else None
    e, c = green.orbitals(f, s)
    mu = green.midgap_mu(e, geo.n // 2)
    tau, w = green.tau_grid(beta, ntau)
    amp = 0.01 + 0.002 * np.arange(geo.n)
    pole = np.where(e > mu, 1.0, -1.0) * (0.8 + 0.05 * np.arange(geo.n))
    st = -amp[None, :] * np.exp(-np.outer(tau, pole)) / (1.0 + np.exp(-beta * pole))[None, :]
    sc = c if s is None else s @ c
    sig = np.einsum("ik,tk,jk->tij", sc, st, sc)
    E, ok = ctx.qp_energies(f, s, mu, beta, tau, w, torch.tensor(sig, device="cuda"), 16)
    d = e - mu - pole
    want = 0.5 * (e + mu + pole) + np.sign(d) * np.sqrt(0.25 * d * d + amp)
    ref, ok_r = qp.qp_energies(sig, f, s if s is not None else np.eye(geo.n), mu, beta, tau, w, 16, 1e-9)
    assert ok.all() and ok_r.all()
    assert np.abs(E - want).max() < 1e-9
    assert np.abs(E - ref).max() < 1e-10


@pytest.mark.parametrize("n_pade", [1, 8, 32])
def test_ri_self_energy_matches_oracle(ctx, n_pade):
    nd, beta, ntau = 10, 30.0, 48
    geo = ci.chain_geometry(nd)
    f = ci.fock_tight_binding(geo.x)
    tau, w = green.tau_grid(beta, ntau)
    # GPU: deterministic RI self-energy (eps = 0 keeps all of B exactly)
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float64)
    spl = ctx.split(B, 0.0)
    G, Gb, mu = ctx.green_tau(f, tau, beta, n_occ=geo.n // 2)
    det = ctx.sigma_det(spl, G, Gb)
    Sig = ctx.sigma_finalize(det, torch.zeros_like(det), 1)
    E, ok = ctx.qp_energies(f, None, mu, beta, tau, w, Sig, n_pade)
    # oracle: its own RI self-energy
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    e, c = green.orbitals(f)
    mu_o = green.midgap_mu(e, geo.n // 2)
    g, gb = green.green_tau(e, c, mu_o, beta, tau)
    sig_o = np.array([se.sigma_ri(b, g[t], gb[t]) for t in range(ntau)])
    ref, ok_r = qp.qp_energies(sig_o, f, np.eye(geo.n), mu_o, beta, tau, w, n_pade, 1e-9)
    r = np.random.default_rng(1)
    ref2, _ = qp.qp_energies(sig_o * (1.0 + 1e-14 * r.standard_normal(sig_o.shape)), f, np.eye(geo.n), mu_o,
                             beta, tau, w, n_pade, 1e-9)
    spread = np.abs(ref2 - ref).max()
    print(f"n_pade {n_pade}: max |E - E_oracle| {np.abs(E - ref).max():.2e}, oracle spread {spread:.2e}, "
          f"shift from eps {np.abs(E - e).max():.3e}, converged {ok.sum()}/{geo.n}")
    assert np.array_equal(ok, ok_r)
    assert np.abs(E - ref).max() < max(1e-9, 10.0 * spread)
    spl.free()
