"""Parity of the HIP path with the CPU oracle on the same seeded inputs.

Tolerances: FP64 path 1e-10 relative, FP32 path 1e-5 relative (Sigma as
max_t ||dSigma(tau_t)|| / max_t ||Sigma(tau_t)||, energies |dE|/|E|);
integer work (random words, supports, draws) bit-exact.
"""
import numpy as np
import pytest

import chain_inputs as ci
from oracle import energy, green, integrals, proposal as pr, rng, selfenergy as se, split as sp

from _problems import chain, oracle_pairs, oracle_setup, rel

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


def _gpu_inputs(ctx, pb, dtype):
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=dtype)
    tau, w = green.tau_grid(pb["beta"], pb["ntau"])
    G, Gb, mu = ctx.green_tau(pb["f"], tau, pb["beta"], n_occ=geo.n // 2)
    return B, G, Gb, mu, tau, w


def test_rng_words_bit_exact(ctx):
    for seed, stream, s in ((0, 0, 0), (12345, 1, 77), (2 ** 63 + 5, 2, 1 << 29)):
        got = ctx.rng_words(seed, stream, s, 3, 500)
        ref = rng.words(seed, stream, s, np.arange(3, 503, dtype=np.uint64))
        assert np.array_equal(got, ref)


def test_synthetic_b_matches_oracle(ctx):
    pb = chain(7, 50.0, 4, 1e-2)
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float64).cpu().numpy()
    ref = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    assert rel(B, ref) < 1e-14
    B32 = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float32).cpu().numpy()
    assert rel(B32, ref) < 1e-6


def test_general_b_contraction_matches_oracle(ctx):
    n, naux = 6, 20
    ija = ci.random_three_index(naux, n, 5)
    v = ci.random_spd(naux, 6)
    t = torch.tensor(ija, device="cuda")
    B = ctx.build_B(n, naux, ijA=t, V=v, dtype=torch.float64).cpu().numpy()
    ref = integrals.b_from_three_index(ija, v)
    assert rel(B, ref) < 1e-11
    B2 = ctx.build_B(n, naux, ijA=t, V=None, dtype=torch.float64).cpu().numpy()
    assert np.array_equal(B2, ija)


@pytest.mark.parametrize("eps", [0.0, 1e-3, 1e-2, 0.3])
def test_split_supports_and_blocks_exact(ctx, eps):
    pb = chain(6, 50.0, 4, eps)
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float64)
    spl = ctx.split(B, eps)
    ref = sp.split_b(B.cpu().numpy(), eps)
    w, idx, blk, kmax = spl.export()
    assert kmax == ref.kmax
    assert spl.nnz == ref.nnz
    assert spl.wmax == ref.wmax
    for q in range(geo.naux):
        assert w[q] == ref.support[q].shape[0]
        assert np.array_equal(idx[q, :w[q]], ref.support[q])
        assert np.array_equal(blk[q, :w[q], :w[q]], ref.blocks[q])
    spl.free()


def test_split_rejects_wide_support(ctx):
    from paper_2005_12338_amd import gf2
    pb = chain(20, 50.0, 4, 0.0)
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float64)
    with pytest.raises(gf2.Gf2Error) as ei:
        ctx.split(B, 0.0)        # every element kept: supports span all 40 orbitals
    assert ei.value.code == gf2.GF2_E_ARG


def test_green_matches_oracle(ctx):
    pb = chain(10, 50.0, 16, 1e-2)
    o = oracle_setup(pb)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, torch.float64)
    assert abs(mu - o["mu"]) < 1e-13
    assert rel(G.cpu().numpy(), o["g"]) < 1e-11
    assert rel(Gb.cpu().numpy(), o["gb"]) < 1e-11


def test_green_nonorthogonal_overlap(ctx):
    n = 12
    s = ci.random_overlap(n, 3)
    f = ci.random_symmetric(n, 4, 0.4)
    e, c = green.orbitals(f, s)
    mu = green.midgap_mu(e, n // 2)
    tau, w = green.tau_grid(20.0, 3)
    g, gb = green.green_tau(e, c, mu, 20.0, tau)
    G, Gb, mu_g = ctx.green_tau(f, tau, 20.0, n_occ=n // 2, S=s)
    assert abs(mu_g - mu) < 1e-12
    assert rel(G.cpu().numpy(), g) < 1e-10
    assert rel(Gb.cpu().numpy(), gb) < 1e-10


def test_green_rejects_bad_tau(ctx):
    from paper_2005_12338_amd import gf2
    f = ci.fock_tight_binding(ci.atom_positions(3))
    with pytest.raises(gf2.Gf2Error):
        ctx.green_tau(f, np.array([0.5, 60.0]), 50.0, n_occ=3)


@pytest.mark.parametrize("n_dimer,eps", [(10, 1e-2), (12, 1e-3), (12, 1e-4), (9, 1e-6), (6, 0.0)])
def test_sigma_det_matches_oracle(ctx, n_dimer, eps):
    """Register strip form (supports <= 4, 6, 8) and the LDS tile form (wider)."""
    pb = chain(n_dimer, 50.0, 4, eps)
    o = oracle_setup(pb)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, torch.float64)
    spl = ctx.split(B, pb["eps"])
    got = ctx.sigma_det(spl, G, Gb).cpu().numpy()
    for t in range(pb["ntau"]):
        ref = se.sigma_dd(o["split"], o["g"][t], o["gb"][t])
        assert rel(got[t], ref) < 1e-11


def _check_sigma(ctx, pb, prec, dtype, ns, seed, tol, taus=None, pairs=None):
    o = oracle_setup(pb)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, dtype)
    spl = ctx.split(B, pb["eps"])
    Sigma, es = ctx.sigma_tau(spl, B, G, Gb, ns=ns, seed=seed, prec=prec)
    Sigma = Sigma.cpu().numpy()
    es = es.cpu().numpy()
    taus = list(range(pb["ntau"])) if taus is None else taus
    pairs = list(range(ns)) if pairs is None else pairs
    per = oracle_pairs(o, seed, ns, taus, pairs)
    # per-pair energies e_s(tau) = Tr(Sigma_s Gb)
    e_ref = np.array([[energy.trace_product(per[(t, s)], o["gb"][t]) for t in taus] for s in pairs])
    e_got = es[np.ix_(pairs, taus)]
    assert rel(e_got, e_ref) < tol, rel(e_got, e_ref)
    if len(pairs) == ns:
        for t in taus:
            ref = se.sigma_dd(o["split"], o["g"][t], o["gb"][t])
            acc = sum(per[(t, s)] for s in pairs)
            ref = ref + (acc + acc.T) / (2.0 * ns)
            assert rel(Sigma[t], ref) < tol, (t, rel(Sigma[t], ref))
    return Sigma, es, o, (B, G, Gb, w, spl)


def test_sigma_tau_fp64_tiny_matches_oracle(ctx):
    """Tiny chain: N=20, N_aux=60, beta=50, 32 tau, 64 pairs, eps=1e-2."""
    pb = chain(10, 50.0, 32, 1e-2)
    Sigma, es, o, (B, G, Gb, w, spl) = _check_sigma(ctx, pb, "fp64", torch.float64, 64, 0, 1e-10)
    # energy and its standard error through the C ABI
    e_tot, e_pe, se_ = ctx.energy(torch.tensor(Sigma, device="cuda"), Gb, w, pb["n"],
                                  torch.tensor(es, device="cuda"))
    ref_e = energy.energy_total(Sigma, o["gb"], w)
    assert abs(e_tot - ref_e) < 1e-10 * abs(ref_e)
    e_det = np.array([energy.trace_product(se.sigma_dd(o["split"], o["g"][t], o["gb"][t]), o["gb"][t])
                      for t in range(pb["ntau"])])
    es_tot = energy.sample_energies(e_det, es, w)
    m, s = energy.mean_stderr(es_tot)
    assert abs(m - e_tot) < 1e-12 * abs(e_tot)
    assert abs(s - se_) < 1e-8 * s


def test_sigma_tau_fp64_ragged_tiles(ctx):
    """N=70 spans two 64-wide tiles with a ragged tail."""
    pb = chain(35, 50.0, 3, 1e-2)
    _check_sigma(ctx, pb, "fp64", torch.float64, 5, 3, 1e-10)


def test_sigma_tau_fp32_several_tiles(ctx):
    """N=150 (two 128-wide tiles, ragged), FP32 path, 1e-5."""
    pb = chain(75, 100.0, 3, 1e-3)
    _check_sigma(ctx, pb, "fp32", torch.float32, 4, 1, 1e-5)


def test_sigma_eps_zero_has_no_stochastic_part(ctx):
    pb = chain(5, 20.0, 3, 0.0)
    o = oracle_setup(pb)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, torch.float64)
    spl = ctx.split(B, 0.0)
    Sigma, es = ctx.sigma_tau(spl, B, G, Gb, ns=3, seed=0, prec="fp64")
    assert np.abs(es.cpu().numpy()).max() < 1e-14
    for t in range(3):
        assert rel(Sigma[t].cpu().numpy(), se.sigma_ri(o["b"], o["g"][t], o["gb"][t])) < 1e-11


def test_sigma_pure_sri_matches_oracle(ctx):
    """Threshold above the maximum: B^L = 0, D = 0, and the estimator is the
    plain stochastic RI of Section II (every element stochastic)."""
    pb = chain(10, 50.0, 4, 2.0)
    Sigma, es, o, (B, G, Gb, w, spl) = _check_sigma(ctx, pb, "fp64", torch.float64, 6, 5, 1e-10)
    assert spl.wmax == 0 and spl.nnz == 0
    for t in range(pb["ntau"]):
        assert np.abs(se.sigma_dd(o["split"], o["g"][t], o["gb"][t])).max() == 0.0
    _check_sigma(ctx, chain(40, 100.0, 2, 2.0), "fp32", torch.float32, 3, 1, 1e-5)


def test_sigma_importance_mode_matches_oracle(ctx):
    pb = chain(8, 50.0, 3, 1e-2)
    o = oracle_setup(pb)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, torch.float64)
    spl = ctx.split(B, pb["eps"])
    p = ci.random_weights(pb["naux"], 9)
    ns, k = 6, 2
    Sigma, es = ctx.sigma_tau(spl, B, G, Gb, ns=ns, seed=4, prec="fp64", p=p, k=k)
    th = pr.importance_theta(p, 4, 0, ns, k)
    thp = pr.importance_theta(p, 4, 1, ns, k)
    per = oracle_pairs(o, 4, ns, range(3), range(ns), th, thp)
    e_ref = np.array([[energy.trace_product(per[(t, s)], o["gb"][t]) for t in range(3)] for s in range(ns)])
    assert rel(es.cpu().numpy(), e_ref) < 1e-10


@pytest.mark.parametrize("nclass", [3, 7])
def test_sigma_stratified_mode_matches_oracle(ctx, nclass):
    """Stratified vectors (one class per vector, +-1/sqrt(pi_c) on its
    members), class weights from a random p, pair by pair."""
    pb = chain(8, 50.0, 3, 1e-2)
    o = oracle_setup(pb)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, torch.float64)
    spl = ctx.split(B, pb["eps"])
    p = ci.random_weights(pb["naux"], 19)
    ns = 6
    Sigma, es = ctx.sigma_tau(spl, B, G, Gb, ns=ns, seed=8, prec="fp64", p=p, classes=nclass)
    th = pr.stratified_theta(p, nclass, 8, 0, ns)
    thp = pr.stratified_theta(p, nclass, 8, 1, ns)
    per = oracle_pairs(o, 8, ns, range(3), range(ns), th, thp)
    e_ref = np.array([[energy.trace_product(per[(t, s)], o["gb"][t]) for t in range(3)] for s in range(ns)])
    assert rel(es.cpu().numpy(), e_ref) < 1e-10


def test_sigma_stoch_batches_equal_one_call(ctx):
    """Adaptive sampling in batches (s0 offsets) reproduces one call bitwise."""
    pb = chain(8, 50.0, 3, 1e-2)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, torch.float64)
    spl = ctx.split(B, pb["eps"])
    n = pb["n"]
    s_all = torch.zeros((3, n, n), dtype=torch.float64, device="cuda")
    e_all = torch.zeros((6, 3), dtype=torch.float64, device="cuda")
    ctx.sigma_stoch(spl, B, G, Gb, s_all, ns=6, seed=2, prec="fp64", e_samples=e_all)
    s_b = torch.zeros_like(s_all)
    e_b = torch.zeros_like(e_all)
    ctx.sigma_stoch(spl, B, G, Gb, s_b, ns=4, seed=2, prec="fp64", s0=0, e_samples=e_b[:4])
    ctx.sigma_stoch(spl, B, G, Gb, s_b, ns=2, seed=2, prec="fp64", s0=4, e_samples=e_b[4:])
    assert torch.equal(e_all, e_b)
    assert torch.equal(s_all, s_b)


@pytest.mark.parametrize("prec,n,batch", [("fp64", 70, 3), ("fp32", 150, 2), ("bf16", 200, 2), ("bf16x3", 130, 2),
                                          ("bf16", 150, 3), ("bf16", 300, 2)])
def test_gemm_kernel_matches_torch_reference(ctx, prec, n, batch):
    """The chain's GEMM kernel alone, against a plain PyTorch reference of the
    same product (FP64 / FP32 on the CPU)."""
    ld = (n + 31) // 32 * 32
    g = torch.Generator().manual_seed(7)
    a = torch.randn(batch, n, n, generator=g, dtype=torch.float64)
    b = torch.randn(batch, n, n, generator=g, dtype=torch.float64)

    def pad(x, dt):
        out = torch.zeros(batch, ld, ld, dtype=dt)
        out[:, :n, :n] = x.to(dt)
        return out

    if prec == "fp64":
        A, Bt, ref = pad(a, torch.float64), pad(b, torch.float64), a @ b.transpose(1, 2)
        cdt, tol = torch.float64, 1e-12
    elif prec == "fp32":
        A, Bt = pad(a, torch.float32), pad(b, torch.float32)
        ref = A.double() @ Bt.double().transpose(1, 2)
        ref = ref[:, :n, :n]
        cdt, tol = torch.float32, 1e-5
    elif prec == "bf16":
        A, Bt = pad(a, torch.bfloat16), pad(b, torch.bfloat16)
        ref = (A.float() @ Bt.float().transpose(1, 2))[:, :n, :n].double()
        cdt, tol = torch.float32, 1e-5
    else:
        ah = a.to(torch.bfloat16)
        al = (a - ah.double()).to(torch.bfloat16)
        bh = b.to(torch.bfloat16)
        bl = (b - bh.double()).to(torch.bfloat16)
        A = torch.cat([pad(ah.double(), torch.bfloat16), pad(al.double(), torch.bfloat16)], dim=1)
        Bt = torch.cat([pad(bh.double(), torch.bfloat16), pad(bl.double(), torch.bfloat16)], dim=1)
        ref = a @ b.transpose(1, 2)
        cdt, tol = torch.float32, 3e-5          # x3 products keep ~16 mantissa bits
    C = torch.zeros(batch, ld, ld, dtype=cdt, device="cuda")
    ctx.debug_gemm(prec, n, A.contiguous().cuda(), Bt.contiguous().cuda(), C, batch=batch)
    got = C.cpu().double()[:, :n, :n]
    err = (got - ref).abs().max().item() / ref.abs().max().item()
    assert err < tol, err
    assert torch.count_nonzero(C.cpu()[:, n:, :]) == 0 and torch.count_nonzero(C.cpu()[:, :, n:]) == 0


@pytest.mark.parametrize("n_dimer", [75, 200])
def test_wide_tile_chain_matches_standard_tiles(ctx, n_dimer):
    """N = 150 and 400, where the 160-wide BF16 tiles pad less than 128.
    Mode 1 (deep-K stage only on the wide tile) against mode 0 (128 tiles
    only): the deep-K stage writes FP32, so the two differ by its FP32
    accumulation order alone.  Mode 2 (every launch on the wide tiles) also
    reorders products whose outputs are stored in BF16, so single roundings
    can flip: against the FP32 path it stays at the BF16 level, as mode 0
    does."""
    pb = chain(n_dimer, 100.0, 3, 1e-3)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, torch.float32)
    spl = ctx.split(B, pb["eps"])
    out, ran = {}, {}
    try:
        for mode in (0, 1, 2):
            ctx.set_gemm_tiles(mode)
            ctx.set_profiling(True)
            ctx.profile_read()
            out[mode] = ctx.sigma_tau(spl, B, G, Gb, ns=3, seed=4, prec="bf16")
            ran[mode] = sorted(k for k in ctx.profile_read() if k.endswith("@160"))
    finally:
        ctx.set_profiling(False)
        ctx.set_gemm_tiles(2)
    assert ran[0] == [] and ran[1] == ["gemm_bf16.s4@160"]
    assert ran[2] == ["gemm_bf16.s1@160", "gemm_bf16.s2@160", "gemm_bf16.s3@160", "gemm_bf16.s4@160"]
    S32, e32 = ctx.sigma_tau(spl, B, G, Gb, ns=3, seed=4, prec="fp32")
    (S0, e0), (S1, e1), (S2, e2) = out[0], out[1], out[2]
    assert not torch.equal(e0, e1)
    assert rel(S1.cpu().numpy(), S0.cpu().numpy()) < 1e-6
    assert rel(e1.cpu().numpy(), e0.cpu().numpy()) < 1e-5
    err0 = rel(S0.cpu().numpy(), S32.cpu().numpy())
    err2 = rel(S2.cpu().numpy(), S32.cpu().numpy())
    ee0 = rel(e0.cpu().numpy(), e32.cpu().numpy())
    ee2 = rel(e2.cpu().numpy(), e32.cpu().numpy())
    print(f"n_dimer {n_dimer}: BF16 vs FP32: Sigma rel {err0:.2e} (128 tiles) {err2:.2e} (wide); "
          f"e_s rel {ee0:.2e} {ee2:.2e}")
    assert err2 < 2.0 * err0 + 1e-7 and ee2 < 2.0 * ee0 + 1e-6


@pytest.mark.parametrize("n_dimer", [75, 400])
def test_split_bf16x3_stages_match_the_bf16x3_tile(ctx, n_dimer):
    """Where the 160-wide tile pads less (N = 150, 800), a BF16X3 chain runs
    its launch groups as BF16 products on the 160-wide tiles, each K segment
    A B^T as A_hi B_hi + A_hi B_lo + A_lo B_hi: mode 1 the deep-K stage, mode
    2 (default) also the dual-A stages, whose storage outputs are written as
    hi and lo planes; mode 0 keeps the BF16X3 tile.  The deep-K stage writes
    FP32, so mode 1 differs from mode 0 by the order of the FP32 accumulation
    alone; in mode 2 the hi/lo split of the stored intermediates can round
    differently, at the BF16X3 level.  All stay at that level against FP32."""
    pb = chain(n_dimer, 100.0, 2, 1e-3)
    B, G, Gb, mu, tau, w = _gpu_inputs(ctx, pb, torch.float32)
    spl = ctx.split(B, pb["eps"])
    out, ran = {}, {}
    try:
        for mode in (0, 1, 2):
            ctx.set_gemm_tiles(mode)
            ctx.set_profiling(True)
            ctx.profile_read()
            out[mode] = ctx.sigma_tau(spl, B, G, Gb, ns=2, seed=6, prec="bf16x3")
            ran[mode] = sorted(k for k in ctx.profile_read() if k.startswith("gemm"))
    finally:
        ctx.set_profiling(False)
        ctx.set_gemm_tiles(2)
    assert not any(k.endswith("@160") for k in ran[0])
    assert [k for k in ran[1] if k.endswith("@160")] == ["gemm_bf16x3.s4@160"]
    assert [k for k in ran[2] if k.endswith("@160")] == ["gemm_bf16x3.s1@160", "gemm_bf16x3.s2@160",
                                                          "gemm_bf16x3.s3@160", "gemm_bf16x3.s4@160"]
    S32, e32 = ctx.sigma_tau(spl, B, G, Gb, ns=2, seed=6, prec="fp32")
    S = {m: out[m][0].cpu().numpy() for m in out}
    e = {m: out[m][1].cpu().numpy() for m in out}
    assert rel(S[1], S[0]) < 1e-6
    assert rel(e[1], e[0]) < 1e-5
    assert rel(S[2], S[0]) < 3e-5
    print(f"n_dimer {n_dimer}: BF16X3 vs FP32 Sigma rel {rel(S[0], S32.cpu().numpy()):.2e} (tile), "
          f"{rel(S[1], S32.cpu().numpy()):.2e} (deep-K split), {rel(S[2], S32.cpu().numpy()):.2e} (all split); "
          f"mode 2 vs 0 {rel(S[2], S[0]):.2e}")
    for m in (0, 1, 2):
        assert rel(S[m], S32.cpu().numpy()) < 3e-5
