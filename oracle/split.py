"""Range separation of the RI factors (Section II, eq:K_L and what follows).

eq:K_L keeps an element of K^L when |K| >= eps * max|K| (the maximum over
all Q, i, j) and zeroes it otherwise.  With a synthetic K there is no
separate (ij|A), so the earlier per-j threshold eq:V_ijA is not applied and
eq:K_L acts on K directly.  The stochastic vectors then split as
[R^xi]^L = sum_Q K^{L,Q} theta^xi_Q and [R^xi]^S = R^xi - [R^xi]^L.

The large part of each Q is stored as a dense block on its support
S_Q = {i : K^{L,Q}_ij != 0 for some j} (K^Q is symmetric, so rows and
columns share the support).  Functions accept either the full tensor
[N_aux][N][N] or a callable returning one Q slice, so that large chains can
be streamed.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Union

import numpy as np

SliceSource = Union[np.ndarray, Callable[[int], np.ndarray]]


def _slice(b: SliceSource, q: int) -> np.ndarray:
    return np.asarray(b[q] if isinstance(b, np.ndarray) else b(q), dtype=np.float64)


@dataclasses.dataclass
class Split:
    eps: float
    kmax: float
    thresh: float
    n: int
    support: List[np.ndarray]    # S_Q, ascending orbital indices
    blocks: List[np.ndarray]     # K^L[Q][S_Q][:, S_Q] (zeros where below)
    nnz: int                     # number of kept elements of K^L

    @property
    def naux(self) -> int:
        return len(self.support)

    @property
    def wmax(self) -> int:
        return max((s.shape[0] for s in self.support), default=0)

    def kl_slice(self, q: int) -> np.ndarray:
        out = np.zeros((self.n, self.n))
        s = self.support[q]
        out[np.ix_(s, s)] = self.blocks[q]
        return out

    def kl_dense(self) -> np.ndarray:
        return np.stack([self.kl_slice(q) for q in range(self.naux)])


def split_b(b: SliceSource, eps: float, naux: int | None = None) -> Split:
    """eq:K_L applied to K = b: keep |K| >= eps * max|K| (inclusive)."""
    if naux is None:
        naux = b.shape[0]
    kmax = 0.0
    for q in range(naux):
        kmax = max(kmax, float(np.max(np.abs(_slice(b, q)))))
    thresh = eps * kmax
    support, blocks, nnz, n = [], [], 0, 0
    for q in range(naux):
        bq = _slice(b, q)
        n = bq.shape[0]
        keep = np.abs(bq) >= thresh
        nnz += int(np.count_nonzero(keep))
        rows = np.nonzero(np.any(keep, axis=1))[0]
        support.append(rows)
        blk = np.where(keep, bq, 0.0)[np.ix_(rows, rows)]
        blocks.append(np.ascontiguousarray(blk))
    return Split(eps=float(eps), kmax=kmax, thresh=thresh, n=n,
                 support=support, blocks=blocks, nnz=nnz)


def r_vectors(b: SliceSource, split: Split, theta: np.ndarray):
    """R = sum_Q theta_Q K^Q (eq:4 with V = I), [R]^L = sum_Q theta_Q K^{L,Q}
    and [R]^S = R - [R]^L for each row of theta [n_vec][N_aux].  Returns three
    arrays [n_vec][N][N]."""
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    nv, n = theta.shape[0], split.n
    r = np.zeros((nv, n, n))
    rl = np.zeros((nv, n, n))
    for q in range(split.naux):
        bq = _slice(b, q)
        r += theta[:, q, None, None] * bq[None]
        s = split.support[q]
        if s.shape[0]:
            rl[:, s[:, None], s[None, :]] += theta[:, q, None, None] * split.blocks[q][None]
    return r, rl, r - rl
