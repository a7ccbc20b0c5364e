"""Seeded synthetic inputs shaped like the paper's hydrogen dimer chains.

This module is shared by the CPU oracle and the GPU path.  It holds input
generation only -- geometry, the tight-binding Fock matrix, the parameters
of the Gaussian stand-in for the RI factor tensor, the workload table and
seeded random operands for tests.  None of the method's arithmetic (RI
factors, splitting, Green's functions, self-energy, energy) lives here.

The paper's chains (Results section) are STO-3G hydrogen dimer chains with
a cc-pVDZ-RI fitting basis.  No basis-set data or integral engine is
available, so the stand-in is a 1D chain with one s-like function per atom:

* atoms on a line, x_0 = 0, spacings alternating 0.74 (intra-dimer) and
  1.5 bohr (inter-dimer);
* three auxiliary centres per atom: the left bond midpoint, the atom and
  the right bond midpoint, ordered so that x_Q is non-decreasing in Q; the
  chain ends use a mirrored 1.5 bohr bond (so N_aux = 3N);
* the factor tensor B^Q_ij = amp * exp(-a (x_i-x_j)^2)
  * exp(-c (x_Q - (x_i+x_j)/2)^2) with (amp, a, c) = (0.3, 0.8, 1.2),
  evaluated by each side from the geometry and these parameters;
* Fock matrix F_ij = -0.5 exp(-|x_i - x_j|) (tight binding, half filled),
  overlap S = I.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

INTRA_BOND = 0.74   # bohr, strongly bonded pair
INTER_BOND = 1.5    # bohr, weakly bonded pair
B_AMP = 0.3
B_EXP_BOND = 0.8    # exponent on (x_i - x_j)^2
B_EXP_AUX = 1.2     # exponent on (x_Q - (x_i + x_j)/2)^2


def atom_positions(n_dimer: int) -> np.ndarray:
    """Atom coordinates (bohr) of a chain of ``n_dimer`` H2 dimers."""
    n = 2 * int(n_dimer)
    x = np.zeros(n, dtype=np.float64)
    for i in range(1, n):
        x[i] = x[i - 1] + (INTRA_BOND if (i % 2 == 1) else INTER_BOND)
    return x


def aux_centres(x: np.ndarray) -> np.ndarray:
    """Three auxiliary centres per atom: left midpoint, atom, right midpoint."""
    n = x.shape[0]
    left = np.empty(n)
    right = np.empty(n)
    left[0] = x[0] - 0.5 * INTER_BOND
    left[1:] = 0.5 * (x[1:] + x[:-1])
    right[-1] = x[-1] + 0.5 * INTER_BOND
    right[:-1] = 0.5 * (x[1:] + x[:-1])
    xq = np.stack([left, x, right], axis=1).reshape(-1)
    return np.ascontiguousarray(xq)


def fock_tight_binding(x: np.ndarray) -> np.ndarray:
    """Dense tight-binding Fock matrix F_ij = -0.5 exp(-|x_i - x_j|)."""
    d = np.abs(x[:, None] - x[None, :])
    return -0.5 * np.exp(-d)


@dataclasses.dataclass(frozen=True)
class ChainGeometry:
    """Everything a B-factor generator needs, as plain data."""
    x: np.ndarray          # [N] atom positions
    xq: np.ndarray         # [N_aux] auxiliary centres
    amp: float = B_AMP
    a: float = B_EXP_BOND
    c: float = B_EXP_AUX

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def naux(self) -> int:
        return int(self.xq.shape[0])


def chain_geometry(n_dimer: int) -> ChainGeometry:
    x = atom_positions(n_dimer)
    return ChainGeometry(x=x, xq=aux_centres(x))


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_dimer: int
    beta: float
    ntau: int
    ns: int
    eps: float
    precision: str
    seed: int = 0

    @property
    def n(self) -> int:
        return 2 * self.n_dimer

    @property
    def naux(self) -> int:
        return 6 * self.n_dimer

    @property
    def n_elec(self) -> int:
        return self.n           # one electron per hydrogen atom

    @property
    def n_occ(self) -> int:
        return self.n // 2      # closed shell


# The five workloads the method is measured on.  beta / eps / ntau that the
# workload description leaves open are fixed here (beta = 100 for the larger
# chains, eps = 1e-3 for the batch, eps = 1e-4 and 128 tau points for the
# learned-proposal chain).
TINY = Workload("tiny_n20", 10, 50.0, 32, 64, 1e-2, "fp64", 0)
N200 = Workload("chain_n200", 100, 100.0, 64, 256, 1e-3, "fp32", 0)
N800 = Workload("chain_n800", 400, 100.0, 128, 512, 1e-4, "bf16", 0)
N1600 = Workload("chain_n1600_learned", 800, 100.0, 128, 0, 1e-4, "bf16", 0)
BATCH_BETA, BATCH_NTAU, BATCH_NS, BATCH_EPS = 100.0, 64, 128, 1e-3


def batch_dimer_counts(count: int = 96, lo: int = 20, hi: int = 200) -> np.ndarray:
    """Dimer counts of the uneven-size batch (uniform in lo..hi, 20..200 by
    default)."""
    return np.random.default_rng(12345).integers(lo, hi + 1, count)


def batch_workloads(count: int = 96, lo: int = 20, hi: int = 200) -> List[Workload]:
    return [Workload(f"batch_{k}", int(nd), BATCH_BETA, BATCH_NTAU, BATCH_NS,
                     BATCH_EPS, "fp32", seed=k)
            for k, nd in enumerate(batch_dimer_counts(count, lo, hi))]


def training_dimer_counts() -> List[int]:
    """Chains the learned proposal is trained on: 10, 12, ..., 48 dimers."""
    return list(range(10, 50, 2))


# ---------------------------------------------------------------------------
# Seeded random operands for tests of the general (non-synthetic) paths.
# ---------------------------------------------------------------------------

def gaussian_three_index(geo: "ChainGeometry") -> np.ndarray:
    """Raw three-index integrals (ij|A) [N_aux][N][N] of the chain: the same
    Gaussian model as the synthetic factors, amp exp(-a (x_i - x_j)^2)
    exp(-c (x_A - (x_i + x_j)/2)^2), as a host array for both sides."""
    x, xq = geo.x, geo.xq
    d = x[:, None] - x[None, :]
    m = 0.5 * (x[:, None] + x[None, :])
    bond = geo.amp * np.exp(-geo.a * d * d)
    return np.stack([bond * np.exp(-geo.c * (xq[q] - m) ** 2) for q in range(xq.shape[0])])


def aux_metric(xq: np.ndarray, alpha: float = 0.5, shift: float = 0.5) -> np.ndarray:
    """A synthetic Coulomb metric of the auxiliary centres: V_AB =
    exp(-alpha (x_A - x_B)^2) + shift delta_AB (symmetric positive definite:
    a Gaussian kernel matrix plus a positive diagonal)."""
    xq = np.asarray(xq, dtype=np.float64)
    d = xq[:, None] - xq[None, :]
    return np.exp(-alpha * d * d) + shift * np.eye(xq.shape[0])


def random_symmetric(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    r = np.random.default_rng(seed).standard_normal((n, n))
    return scale * 0.5 * (r + r.T)


def random_spd(n: int, seed: int, shift: float = 0.5) -> np.ndarray:
    """A well-conditioned symmetric positive definite matrix."""
    r = np.random.default_rng(seed).standard_normal((n, n)) / np.sqrt(n)
    return r @ r.T + shift * np.eye(n)


def random_three_index(naux: int, n: int, seed: int) -> np.ndarray:
    """A [N_aux][N][N] tensor symmetric in its last two indices."""
    r = np.random.default_rng(seed).standard_normal((naux, n, n))
    return 0.5 * (r + r.transpose(0, 2, 1))


def random_weights(naux: int, seed: int) -> np.ndarray:
    """A strictly positive probability vector over the auxiliary index."""
    w = np.random.default_rng(seed).random(naux) + 0.05
    return w / w.sum()


def random_overlap(n: int, seed: int, off: float = 0.15) -> np.ndarray:
    """A symmetric positive definite matrix with unit diagonal (overlap-like)."""
    r = np.random.default_rng(seed).standard_normal((n, n)) * off / np.sqrt(n)
    s = np.eye(n) + 0.5 * (r + r.T)
    w, v = np.linalg.eigh(s)
    if w.min() < 0.2:
        s = s + (0.2 - w.min()) * np.eye(n)
        d = np.sqrt(np.diag(s))
        s = s / d[:, None] / d[None, :]
    return s
