"""Parity of the learned-proposal kernels with the oracle (oracle/proposal.py).

Features, tables and targets run in FP64 on the device: 1e-10 relative.
The network runs in FP32 on the device against the FP64 oracle evaluated
with the same (FP32-representable) weights: 1e-5 relative on losses and
logits, 1e-4 of the largest component on gradients.  Initial weights are
bit-exact (same counter words, same FP64 arithmetic, one rounding to FP32).
"""
import numpy as np
import pytest

import chain_inputs as ci
from oracle import green, integrals, proposal as pr, split as sp

from _problems import chain, rel

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


def _oracle_mlp(m):
    return pr.Mlp(m.w1.double().cpu().numpy(), m.b1.double().cpu().numpy(), m.w2.double().cpu().numpy(),
                  m.mean.double().cpu().numpy(), m.std.double().cpu().numpy())


def _chains(seed=0, sizes=(9, 30, 257)):
    """Training chains of ragged lengths: phi ~ N(0, 1) scaled per column,
    t_hat a normalised positive vector."""
    r = np.random.default_rng(seed)
    phis, ts = [], []
    for n in sizes:
        phi = r.standard_normal((n, pr.D_IN)) * np.array([0.5, 2.0, 3.0, 0.1]) + np.array([0.3, -4.0, -9.0, 0.02])
        t = r.random(n) ** 4 + 1e-3
        phis.append(phi)
        ts.append(t / t.sum())
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return phis, ts, off


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_features_match_oracle(ctx):
    pb = chain(9, 50.0, 4, 1e-2)
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float64)
    spl = ctx.split(B, pb["eps"])
    _, Gb0, mu = ctx.green_tau(pb["f"], np.array([0.0]), pb["beta"], n_occ=geo.n // 2)
    phi = torch.empty((geo.naux, 4), dtype=torch.float64, device="cuda")
    ctx.proposal_features(spl, B, geo.x, geo.xq, Gb0[0].contiguous(), phi)
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    e, c = green.orbitals(pb["f"])
    mu_o = green.midgap_mu(e, geo.n // 2)
    ref = pr.raw_features(geo.x, geo.xq, b, sp.split_b(b, pb["eps"]).kl_dense(),
                          pr.density_matrix(e, c, mu_o, pb["beta"]))
    got = phi.cpu().numpy()
    assert np.max(np.abs(got[:, 0] - ref[:, 0])) < 1e-14
    assert np.max(np.abs(got[:, 1] - ref[:, 1])) < 1e-11
    assert np.max(np.abs(got[:, 2] - ref[:, 2])) < 1e-9
    assert rel(got[:, 3], ref[:, 3]) < 1e-10


@pytest.mark.parametrize("n_dimer,eps,rel_cut", [(3, 5e-2, 1e-10), (4, 1e-2, 1e-3)])
def test_pair_tables_and_targets_match_oracle(ctx, n_dimer, eps, rel_cut):
    pb = chain(n_dimer, 20.0, 4, eps)
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float64)
    spl = ctx.split(B, eps)
    tau, w = green.tau_grid(pb["beta"], pb["ntau"])
    G, Gb, _ = ctx.green_tau(pb["f"], tau, pb["beta"], n_occ=geo.n // 2)
    tab = torch.empty((4, geo.naux, geo.naux), dtype=torch.float64, device="cuda")
    t = torch.empty(geo.naux, dtype=torch.float64, device="cuda")
    ctx.proposal_targets(spl, B, G, Gb, w, rel_cut, t, tab)

    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    e, c = green.orbitals(pb["f"])
    mu = green.midgap_mu(e, geo.n // 2)
    g, gb = green.green_tau(e, c, mu, pb["beta"], tau)
    ref = pr.pair_tables(pr.truncate(b, rel_cut), sp.split_b(b, eps).kl_dense(), g, gb, w)
    got = tab.cpu().numpy()
    for k, key in enumerate(("BB", "BK", "KB", "KK")):
        assert rel(got[k], ref[key]) < 1e-10, key
    assert rel(t.cpu().numpy(), pr.targets_from_tables(ref)) < 1e-10


def test_init_matches_oracle(ctx):
    phis, _, _ = _chains()
    phi = np.concatenate(phis)
    m = ctx.mlp()
    ctx.proposal_init(m, _dev(phi), seed=77)
    mean, std = phi.mean(axis=0), phi.std(axis=0)
    ref = pr.init_mlp(77, mean, std)
    assert np.array_equal(m.w1.cpu().numpy(), ref.w1.astype(np.float32))
    assert np.array_equal(m.b1.cpu().numpy(), ref.b1.astype(np.float32))
    assert np.array_equal(m.w2.cpu().numpy(), ref.w2.astype(np.float32))
    assert rel(m.mean.cpu().numpy(), mean) < 1e-6
    assert rel(m.std.cpu().numpy(), std) < 1e-6
    assert float(m.adam_m.abs().max()) == 0.0 and float(m.adam_v.abs().max()) == 0.0


def test_loss_and_gradients_match_oracle(ctx):
    phis, ts, off = _chains(1)
    m = ctx.mlp()
    ctx.proposal_init(m, _dev(np.concatenate(phis)), seed=3)
    loss, grad = ctx.proposal_grad(m, off, _dev(np.concatenate(phis)), _dev(np.concatenate(ts)))
    om = _oracle_mlp(m)
    ch = list(zip(phis, ts))
    lref = pr.loss(om, ch)
    gw1, gb1, gw2 = pr.gradients(om, ch)
    gref = np.concatenate([gw1.reshape(-1), gb1, gw2])
    assert abs(loss - lref) < 1e-5 * abs(lref)
    assert np.max(np.abs(grad - gref)) < 1e-4 * np.max(np.abs(gref))


def test_adam_step_matches_oracle_and_training_lowers_loss(ctx):
    phis, ts, off = _chains(2)
    dphi, dt = _dev(np.concatenate(phis)), _dev(np.concatenate(ts))
    m = ctx.mlp()
    ctx.proposal_init(m, dphi, seed=11)
    om = _oracle_mlp(m)
    ch = list(zip(phis, ts))
    g = pr.gradients(om, ch)
    l0 = pr.loss(om, ch)
    st = pr.adam_init(om)
    pr.adam_step(om, st, g, lr=1e-2)
    hist = ctx.proposal_train(m, off, dphi, dt, steps=1, lr=1e-2)
    assert m.step == 1
    assert abs(hist[0] - l0) < 1e-5 * l0
    # first Adam step moves each weight by lr * g / (|g| + eps): compare where
    # the gradient is clearly non-zero (elsewhere the sign is a rounding call)
    gref = np.concatenate([x.reshape(-1) for x in g])
    new = np.concatenate([m.w1.double().cpu().numpy().reshape(-1), m.b1.double().cpu().numpy(),
                          m.w2.double().cpu().numpy()])
    ref = np.concatenate([om.w1.reshape(-1), om.b1, om.w2])
    big = np.abs(gref) > 1e-3 * np.max(np.abs(gref))
    assert big.sum() > 0.5 * big.size
    assert np.max(np.abs(new[big] - ref[big])) < 1e-5
    hist = ctx.proposal_train(m, off, dphi, dt, steps=300, lr=1e-2)
    assert m.step == 301
    assert hist[-1] < 0.5 * hist[0]
    assert np.all(np.isfinite(hist))


def test_inference_matches_oracle(ctx):
    phis, ts, off = _chains(4)
    m = ctx.mlp()
    dphi = _dev(np.concatenate(phis))
    ctx.proposal_init(m, dphi, seed=5)
    ctx.proposal_train(m, off, dphi, _dev(np.concatenate(ts)), steps=50, lr=1e-2)
    om = _oracle_mlp(m)
    phi = phis[2]
    alpha = 0.2
    p = torch.empty(phi.shape[0], dtype=torch.float64, device="cuda")
    ctx.proposal_infer(m, _dev(phi), alpha, p)
    z, _ = pr.forward(om, phi)
    ref = pr.proposal(z, alpha)
    got = p.cpu().numpy()
    assert rel(got, ref) < 1e-5
    assert abs(got.sum() - 1.0) < 1e-12
    assert got.min() >= alpha / phi.shape[0] * (1 - 1e-12)
    pb = torch.empty_like(p)
    ctx.proposal_infer(m, _dev(phi), alpha, pb, bf16=True)
    gb = pb.cpu().numpy()
    assert abs(gb.sum() - 1.0) < 1e-12
    assert np.max(np.abs(gb - ref) / ref) < 0.1


def test_proposal_rejects_bad_arguments(ctx):
    from paper_2005_12338_amd import gf2
    m = ctx.mlp()
    phi = _dev(np.zeros((5, 4)))
    p = torch.empty(5, dtype=torch.float64, device="cuda")
    with pytest.raises(gf2.Gf2Error):
        ctx.proposal_infer(m, phi, 0.0, p)
    with pytest.raises(gf2.Gf2Error):
        ctx.proposal_train(m, np.array([0, 3, 2]), phi, p, steps=1, lr=1e-2)


def _chain_data(ctx, gf2, nd, eps, ntau, beta=100.0):
    geo = ci.chain_geometry(nd)
    f = ci.fock_tight_binding(geo.x)
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float32)
    spl = ctx.split(B, eps)
    tau, w = gf2.gf2_tau_grid(beta, ntau)
    G, Gb, _ = ctx.green_tau(f, tau, beta, n_occ=geo.n // 2)
    _, Gb0, _ = ctx.green_tau(f, np.array([0.0]), beta, n_occ=geo.n // 2)
    phi = torch.empty((geo.naux, pr.D_IN), dtype=torch.float64, device="cuda")
    ctx.proposal_features(spl, B, geo.x, geo.xq, Gb0[0].contiguous(), phi)
    return geo, B, spl, w, G, Gb, phi


def test_learned_proposal_gains_over_pm1(ctx):
    """What the trained proposal gains over the method without it: the
    network (trained on the per-Q targets of the 20 small training chains)
    and the class count of its stratified vectors (chosen on the same
    chains from the measured per-pair spread) against plain +-1 vectors, on
    the held-out 400-dimer chain (N=800, N_aux=2400, threshold 1e-4).  The
    per-pair variance of E_corr falls far below that of +-1 vectors (the
    bar: at least 20% lower); the means of the learned, the uniform-weight
    and the +-1 estimates agree within four combined standard errors."""
    from paper_2005_12338_amd import training
    eps, ntau, ns = 1e-4, 16, 192
    chains = [training.training_chain(ctx, nd, eps, 100.0, ntau) for nd in ci.training_dimer_counts()]
    m, hist = training.train_network(ctx, chains)
    assert hist[-1] < 0.05 * hist[0]
    k, ratio = training.select_classes(ctx, chains, m)
    for c in chains:
        c["spl"].free()
    held = training.training_chain(ctx, 400, eps, 100.0, ntau)
    pl = training.infer_weights(ctx, m, held)
    pu = np.full(held["geo"].naux, 1.0 / held["geo"].naux)

    def per_pair(**kw):
        _, es = ctx.sigma_tau(held["spl"], held["B"], held["G"], held["Gb"], ns, seed=3, prec="fp32", **kw)
        e = -0.5 * (es.cpu().numpy() @ held["w"])
        return e.mean(), e.std(ddof=1)

    m_rad, s_rad = per_pair()
    m_uni, s_uni = per_pair(p=pu, classes=k)
    m_lrn, s_lrn = per_pair(p=pl, classes=k)
    print(f"class count {k} (training-chain variance ratio {ratio[k]:.3f}); per-pair sigma on N=800: "
          f"+-1 {s_rad:.3e}, learned {s_lrn:.3e} (variance ratio {(s_lrn / s_rad) ** 2:.4f}), "
          f"uniform weights {s_uni:.3e}")
    assert k % 3 != 0
    assert (s_lrn / s_rad) ** 2 < 0.8
    for mm, ss in ((m_uni, s_uni), (m_lrn, s_lrn)):
        assert abs(mm - m_rad) < 4.0 * np.hypot(ss, s_rad) / np.sqrt(ns)
    _auto_early_decision(ctx, held, pl, k)
    held["spl"].free()


def _auto_early_decision(ctx, held, p, k, seed=5):
    """AUTO's decision on its first probe (2 pairs), recomputed here from
    the two pairs in BF16 and BF16X3: with r = 2 std(dE) / (0.1 std(E)), r
    above 3 must send the whole run to BF16X3 at once, with the results of a
    plain BF16X3 run of the same pairs.  The learned vectors' spread is so
    small that r is well above 3 on this chain."""
    e = {}
    for prec in ("bf16", "bf16x3"):
        _, es = ctx.sigma_tau(held["spl"], held["B"], held["G"], held["Gb"], 2, seed=seed, prec=prec, p=p, classes=k)
        e[prec] = -0.5 * (es.cpu().numpy() @ held["w"])
    r = 2.0 * np.std(e["bf16x3"] - e["bf16"], ddof=1) / (0.1 * np.std(e["bf16x3"], ddof=1))
    kw = dict(batch=8, max_pairs=8, seed=seed, p=p, classes=k)
    n_e = float(held["geo"].n)
    _, _, es_a, info = ctx.energy_adaptive_det(held["spl"], held["B"], held["G"], held["Gb"], held["w"], n_e, 1e-3,
                                               prec="auto", **kw)
    _, _, es_x, ref = ctx.energy_adaptive_det(held["spl"], held["B"], held["G"], held["Gb"], held["w"], n_e, 1e-3,
                                              prec="bf16x3", **kw)
    print(f"AUTO first-probe ratio r = {r:.2f}: {info['precision']}, E {info['E']:.12f} "
          f"(BF16X3 run {ref['E']:.12f})")
    assert r > 3.0
    assert info["precision"] == "bf16x3" and info["pairs"] == ref["pairs"] == 8
    assert abs(info["E"] - ref["E"]) < 1e-12 * abs(ref["E"])
    assert abs(info["stderr"] - ref["stderr"]) < 1e-9 * ref["stderr"]
    assert np.allclose(es_a.cpu().numpy(), es_x.cpu().numpy(), rtol=1e-12, atol=0.0)
