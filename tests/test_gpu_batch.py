"""Batched chains of uneven size (gf2_sigma_batch) against one call per
instance and against the oracle.

With the same chunk shape the batch runs the same per-unit arithmetic in the
same order as single-instance calls, so results agree bitwise; a tuned shape
regroups the accumulation of pairs (1e-12 relative), and a tuned tile mode
applies to single calls of that size too.
"""
import numpy as np
import pytest

from oracle import energy, green

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


def _instances(ctx, dimers, ntau, eps, dtype, ns):
    out = []
    for i, nd in enumerate(dimers):
        pb = chain(nd, 50.0, ntau, eps)
        geo = pb["geo"]
        B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=dtype)
        tau, w = green.tau_grid(pb["beta"], ntau)
        G, Gb, _ = ctx.green_tau(pb["f"], tau, pb["beta"], n_occ=geo.n // 2)
        out.append(dict(pb=pb, split=ctx.split(B, eps), B=B, G=G, Gb=Gb, ns=ns, seed=i, w=w))
    return out


def _singles(ctx, inst, prec):
    return [ctx.sigma_tau(it["split"], it["B"], it["G"], it["Gb"], ns=it["ns"], seed=it["seed"], prec=prec)
            for it in inst]


def test_batch_fp64_uneven_equals_single_calls_and_oracle(ctx):
    inst = _instances(ctx, [7, 12, 20, 35], 3, 1e-2, torch.float64, 5)
    got = ctx.sigma_batch(inst, prec="fp64")
    ref = _singles(ctx, inst, "fp64")
    for (S, es), (Sr, esr) in zip(got, ref):
        assert torch.equal(S, Sr)
        assert torch.equal(es, esr)
    # the smallest instance against the oracle, pair by pair
    pb = inst[0]["pb"]
    o = oracle_setup(pb)
    per = oracle_pairs(o, 0, 5, range(3), range(5))
    e_ref = np.array([[energy.trace_product(per[(t, s)], o["gb"][t]) for t in range(3)] for s in range(5)])
    assert rel(got[0][1].cpu().numpy(), e_ref) < 1e-10


def test_batch_graph_equals_plain_launches(ctx):
    inst = _instances(ctx, [9, 16, 30], 4, 1e-2, torch.float64, 6)
    a = ctx.sigma_batch(inst, prec="fp64")
    b = ctx.sigma_batch(inst, prec="fp64", graph=True)
    b2 = ctx.sigma_batch(inst, prec="fp64", graph=True)          # a second recording of the same batch
    for (S, es), (Sb, esb), (Sb2, esb2) in zip(a, b, b2):
        assert torch.equal(S, Sb) and torch.equal(S, Sb2)
        assert torch.equal(es, esb) and torch.equal(es, esb2)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_ragged_tiles_autotuned(ctx, prec):
    """Instances spanning one to several 128-wide tiles with ragged tails,
    with the launch shape chosen by the autotuner (persistent or not)."""
    inst = _instances(ctx, [20, 33, 64, 70, 100, 41], 5, 1e-3, torch.float32, 4)
    got = ctx.sigma_batch(inst, prec=prec, autotune=True, graph=True)
    # after the call: in BF16 the tuner may have changed the tile of N = 140,
    # and single calls use its choice too
    ref = _singles(ctx, inst, prec)
    for (S, es), (Sr, esr) in zip(got, ref):
        assert rel(S.cpu().numpy(), Sr.cpu().numpy()) < 1e-12
        assert rel(es.cpu().numpy(), esr.cpu().numpy()) < 1e-12
    # the cached shape is reused on the next call: identical results
    again = ctx.sigma_batch(inst, prec=prec, autotune=True)
    for (S, es), (S2, es2) in zip(got, again):
        assert torch.equal(S, S2) and torch.equal(es, es2)


def test_tile_autotuner_picks_a_mode_per_size():
    """GF2_BATCH_AUTOTUNE times the tile modes on one chain of each BF16 size
    where the 160-wide tile pads less than 128 (N = 150, 160; not N = 80) and
    keeps the fastest per size.  Single calls afterwards use the same tiles
    (the batch equals them up to the regrouping of pairs); each tuned result
    stays at the BF16 level against FP32, as the default tiles do; an
    explicit gf2_set_gemm_tiles discards the choices."""
    from paper_2005_12338_amd import gf2
    c = gf2.Context(0)
    try:
        inst = _instances(c, [75, 40, 80], 3, 1e-3, torch.float32, 3)
        base = c.sigma_batch(inst, prec="bf16")
        s32 = _singles(c, inst, "fp32")
        got = c.sigma_batch(inst, prec="bf16", autotune=True)
        modes = {n: c.tuned_tiles("bf16", n) for n in (150, 80, 160)}
        print("tuned tile modes:", modes)
        assert modes[80] == -1 and modes[150] in (0, 1, 2) and modes[160] in (0, 1, 2)
        assert c.tuned_tiles("fp32", 150) == -1
        ref = _singles(c, inst, "bf16")
        for (S, es), (Sr, esr) in zip(got, ref):
            assert rel(S.cpu().numpy(), Sr.cpu().numpy()) < 1e-12
            assert rel(es.cpu().numpy(), esr.cpu().numpy()) < 1e-12
        for (S, _), (Sb, _), (S3, _) in zip(got, base, s32):
            e_t, e_b = rel(S.cpu().numpy(), S3.cpu().numpy()), rel(Sb.cpu().numpy(), S3.cpu().numpy())
            assert e_t < 2.0 * e_b + 1e-7, (e_t, e_b)
        c.set_gemm_tiles(2)
        assert c.tuned_tiles("bf16", 150) == -1
    finally:
        c.close()


def test_batch_rejects_foreign_split(ctx):
    from paper_2005_12338_amd import gf2
    inst = _instances(ctx, [6, 8], 2, 1e-2, torch.float64, 2)
    inst[1] = dict(inst[1], B=inst[0]["B"])
    with pytest.raises(gf2.Gf2Error):
        ctx.sigma_batch(inst, prec="fp64")


def test_batch_with_importance_and_stratified_items_equals_single_calls(ctx):
    """Items with their own sampling modes (plain, k=2 importance draws,
    stratified with 5 classes) in one FP64 batch: each equals its single
    call bit for bit."""
    import chain_inputs as ci
    inst = _instances(ctx, [8, 14, 21], 3, 1e-2, torch.float64, 4)
    naux = [it["pb"]["geo"].naux for it in inst]
    inst[1] = dict(inst[1], p=ci.random_weights(naux[1], 3), k=2)
    inst[2] = dict(inst[2], p=ci.random_weights(naux[2], 4), classes=5)
    got = ctx.sigma_batch(inst, prec="fp64")
    ref = [ctx.sigma_tau(it["split"], it["B"], it["G"], it["Gb"], ns=it["ns"], seed=it["seed"], prec="fp64",
                         p=it.get("p"), k=it.get("k", 1), classes=it.get("classes", 0)) for it in inst]
    for (S, es), (Sr, esr) in zip(got, ref):
        assert torch.equal(S, Sr)
        assert torch.equal(es, esr)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp64", 1e-10)])
def test_batch_largest_instance_matches_oracle_pair_by_pair(ctx, prec, tol):
    """The largest instance of an uneven multi-instance batch (FP32 and FP64
    launches) against the oracle, every (tau, pair) trace and Sigma."""
    dims, ntau, ns = [9, 31, 16, 48], 3, 4
    inst = _instances(ctx, dims, ntau, 1e-2, torch.float64 if prec == "fp64" else torch.float32, ns)
    got = ctx.sigma_batch(inst, prec=prec)
    k = int(np.argmax(dims))
    pb = inst[k]["pb"]
    o = oracle_setup(pb)
    per = oracle_pairs(o, k, ns, range(ntau), range(ns))
    e_ref = np.array([[energy.trace_product(per[(t, s)], o["gb"][t]) for t in range(ntau)] for s in range(ns)])
    es = got[k][1].cpu().numpy()
    # traces: the bar is relative to the largest per-pair trace (the traces
    # of single pairs scatter around zero)
    assert np.abs(es - e_ref).max() < tol * np.abs(e_ref).max()
    from oracle import selfenergy as se
    acc = np.zeros((ntau, pb["n"], pb["n"]))
    for t in range(ntau):
        acc[t] = sum(per[(t, s)] for s in range(ns))
    sig_ref = np.array([se.sigma_dd(o["split"], o["g"][t], o["gb"][t]) + (acc[t] + acc[t].T) / (2.0 * ns)
                        for t in range(ntau)])
    assert rel(got[k][0].cpu().numpy(), sig_ref) < tol
