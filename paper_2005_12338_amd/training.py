"""Training of the learned proposal on the small training chains, with the
library's own kernels: the network (per-Q features -> weights over the
auxiliary index, gf2_proposal_*) and the class count K of the stratified
vectors that carry its weights.

K is a model choice fitted on the same chains as the network: for every
candidate K the per-pair spread of the energy estimate is measured with
stratified vectors (classes Q mod K, class weights from the network) and
with +-1 vectors, and the K with the smallest mean log variance ratio wins.
The spread depends strongly on K.  A stratified vector estimates the sum
over Q from one class, scaled by 1/pi_c: its variance is that of the class
sums (plus the sign noise of pairs inside a class).  When K is a multiple
of the three auxiliary centres per atom, each class holds one kind of centre
and the class sums differ widely; when the classes mix the kinds evenly and
their members are far apart along the chain, the class sums are nearly
equal and the sign noise nearly vanishes, and the variance falls by orders
of magnitude below that of +-1 vectors.
"""
from __future__ import annotations

import numpy as np

CLASS_CANDIDATES = (8, 10, 14, 16, 20, 22, 25, 26, 28, 32, 34, 38, 40, 44, 50)


def training_chain(ctx, nd: int, eps: float, beta: float, ntau: int):
    """B, split, G, Gbar, tau weights and per-Q features of one chain."""
    import torch
    import chain_inputs as ci
    from . import gf2
    geo = ci.chain_geometry(nd)
    f = ci.fock_tight_binding(geo.x)
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float32)
    spl = ctx.split(B, eps)
    tau, w = gf2.gf2_tau_grid(beta, ntau)
    G, Gb, _ = ctx.green_tau(f, tau, beta, n_occ=geo.n // 2)
    _, gb0, _ = ctx.green_tau(f, np.array([0.0]), beta, n_occ=geo.n // 2)
    phi = torch.empty((geo.naux, 4), dtype=torch.float64, device="cuda")
    ctx.proposal_features(spl, B, geo.x, geo.xq, gb0[0].contiguous(), phi)
    return dict(geo=geo, B=B, spl=spl, G=G, Gb=Gb, w=w, phi=phi)


def train_network(ctx, chains, steps: int = 2000, lr: float = 1e-2, seed: int = 0):
    """Fit the network to the per-Q targets of the chains (full-batch Adam on
    the device).  Returns (mlp, loss history)."""
    import torch
    phis, ts, off = [], [], [0]
    for c in chains:
        t = torch.empty(c["geo"].naux, dtype=torch.float64, device="cuda")
        ctx.proposal_targets(c["spl"], c["B"], c["G"], c["Gb"], c["w"], 1e-10, t)
        phis.append(c["phi"])
        ts.append(t / t.sum())
        off.append(off[-1] + c["geo"].naux)
    m = ctx.mlp()
    phi_all, t_all = torch.cat(phis).contiguous(), torch.cat(ts).contiguous()
    ctx.proposal_init(m, phi_all, seed=seed)
    hist = ctx.proposal_train(m, np.array(off), phi_all, t_all, steps=steps, lr=lr)
    return m, hist


def infer_weights(ctx, mlp, chain, alpha: float = 0.05):
    """The network's weights over the chain's auxiliary index (BF16 inference)."""
    import torch
    p = torch.empty(chain["geo"].naux, dtype=torch.float64, device="cuda")
    ctx.proposal_infer(mlp, chain["phi"], alpha, p, bf16=True)
    return p.cpu().numpy()


def pair_spread(ctx, chain, ns: int, seed: int, prec: str = "fp32", **kw) -> float:
    """Sample standard deviation of the per-pair energy sum_t w_t e_s(tau_t)."""
    _, es = ctx.sigma_tau(chain["spl"], chain["B"], chain["G"], chain["Gb"], ns, seed=seed, prec=prec, **kw)
    e = -0.5 * (es.cpu().numpy() @ chain["w"])
    return float(e.std(ddof=1))


def select_classes(ctx, chains, mlp, candidates=CLASS_CANDIDATES, ns: int = 64, seed: int = 9):
    """The class count with the smallest mean log variance ratio against +-1
    vectors over the chains.  Returns (K, {K: geometric-mean variance ratio})."""
    logs = {k: [] for k in candidates}
    for c in chains:
        s0 = pair_spread(ctx, c, ns, seed)
        p = infer_weights(ctx, mlp, c)
        for k in candidates:
            logs[k].append(2.0 * np.log(pair_spread(ctx, c, ns, seed, p=p, classes=k) / s0))
    ratio = {k: float(np.exp(np.mean(v))) for k, v in logs.items()}
    return min(ratio, key=ratio.get), ratio
