"""Pins of the quasiparticle step (oracle/qp.py): the Pade approximant
interpolates its points and reproduces a rational function (a few poles)
off the imaginary axis; the quasiparticle equation against its closed form
for a one-pole self-energy per orbital (a quadratic), through the whole
chain Sigma(tau) -> s_k(i w) -> Pade -> fixed point; Sigma = 0 gives the
orbital energies."""
import numpy as np

import chain_inputs as ci
from oracle import green, qp


def _rational(z):
    a = np.array([0.02, 0.05, 0.01])
    b = np.array([-0.7, 0.4, 1.3])
    return np.sum(a / (z - b))


def test_pade_interpolates_and_continues_a_rational_function():
    beta = 20.0
    for m in (7, 16, 48):
        z = 1j * (2.0 * np.arange(m) + 1.0) * np.pi / beta
        u = np.array([_rational(x) for x in z])
        a = qp.pade_coefficients(z, u)
        assert max(abs(qp.pade_eval(z, a, zi) - ui) for zi, ui in zip(z, u)) < 1e-13
        for x in np.linspace(-2.0, 2.0, 11):
            zz = complex(x, 1e-3)
            assert abs(qp.pade_eval(z, a, zz) - _rational(zz)) < 1e-10 * abs(_rational(zz))


def _one_pole_chain(nd=5, beta=20.0, ntau=96, s=None):
    geo = ci.chain_geometry(nd)
    f = ci.fock_tight_binding(geo.x)
    e, c = green.orbitals(f, s)
    mu = green.midgap_mu(e, geo.n // 2)
    tau, w = green.tau_grid(beta, ntau)
    amp = 0.01 + 0.002 * np.arange(geo.n)                       # weight of orbital k's pole
    pole = np.where(e > mu, 1.0, -1.0) * (0.8 + 0.05 * np.arange(geo.n))   # pole (from mu) beyond its orbital
    # s_k(tau) = -A e^{-b tau} / (1 + e^{-beta b})  <->  s_k(i w) = A / (i w - b)
    st = -amp[None, :] * np.exp(-np.outer(tau, pole)) / (1.0 + np.exp(-beta * pole))[None, :]
    # Sigma(tau) in the basis: S c diag(s_k) c^T S (so that c^T Sigma c = diag(s_k))
    sc = c if s is None else s @ c
    sig = np.einsum("ik,tk,jk->tij", sc, st, sc)
    return f, e, mu, tau, w, amp, pole, sig


def test_quasiparticle_equation_closed_form_for_one_pole():
    """E = eps + A / (E - mu - b): E = (eps + mu + b)/2 + sign(eps - mu - b)
    sqrt((eps - mu - b)^2 / 4 + A)."""
    beta = 20.0
    for s in (None, ci.random_overlap(10, 3)):
        f, e, mu, tau, w, amp, pole, sig = _one_pole_chain(s=s, beta=beta)
        got, ok = qp.qp_energies(sig, f, s if s is not None else np.eye(f.shape[0]), mu, beta, tau, w, 16, 1e-9)
        d = e - mu - pole
        want = 0.5 * (e + mu + pole) + np.sign(d) * np.sqrt(0.25 * d * d + amp)
        assert ok.all()
        assert np.abs(got - want).max() < 1e-9


def test_zero_self_energy_gives_the_orbital_energies():
    geo = ci.chain_geometry(4)
    f = ci.fock_tight_binding(geo.x)
    tau, w = green.tau_grid(20.0, 16)
    e, c = green.orbitals(f)
    got, ok = qp.qp_energies(np.zeros((16, geo.n, geo.n)), f, None, 0.0, 20.0, tau, w, 8, 1e-9)
    assert ok.all() and np.array_equal(got, e)
