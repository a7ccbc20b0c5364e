"""Counter-based random numbers for the stochastic orbitals.

The paper draws stochastic orbitals theta^xi_A = +-1 (Section II, the
definition preceding eq:4).  To let two independent implementations draw
the same vectors, every number is a pure function of (seed, stream, sample,
index), built on the SplitMix64 output finaliser of Steele, Lea and Flood
("Fast splittable pseudorandom number generators", OOPSLA 2014):

  mix(z):  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
           z ^= z >> 27; z *= 0x94D049BB133111EB
           z ^= z >> 31
  word(seed, stream, s, q) = mix(seed * 0x9E3779B97F4A7C15
                                 + ((stream << 62) | (s << 32) | q) + 1)

all modulo 2^64.  stream 0 draws the first vertex's orbitals (theta), stream
1 the second vertex's (theta', an independent set, eq:sigma_2).

  sign  = +1 if the top bit of the word is 0 else -1
  u     = (word >> 11) * 2^-53  in [0, 1)

Importance draw j of vector (stream, s) uses q = 2j for its uniform and
q = 2j + 1 for its sign.  A stratified vector (stream, s) draws its class
from the uniform of q = CLASS_Q and takes the signs of its members from
the same words as the +-1 orbitals (q = Q).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= M1
        z ^= z >> np.uint64(27)
        z *= M2
        z ^= z >> np.uint64(31)
    return z


def words(seed: int, stream: int, s, q) -> np.ndarray:
    """64-bit words for every broadcast combination of sample s and index q."""
    s = np.asarray(s, dtype=np.uint64)
    q = np.asarray(q, dtype=np.uint64)
    if np.any(s >= np.uint64(1 << 30)):
        raise ValueError("sample index must be < 2^30")
    ctr = (np.uint64(stream) << np.uint64(62)) | (s << np.uint64(32)) | q
    with np.errstate(over="ignore"):
        base = np.uint64(seed) * GOLDEN
        z = base + ctr + np.uint64(1)
    return _mix(z)


def rademacher(seed: int, stream: int, ns: int, naux: int, s0: int = 0) -> np.ndarray:
    """theta[s][Q] in {+1, -1} (float64) for samples s0 .. s0+ns-1."""
    s = np.arange(s0, s0 + ns, dtype=np.uint64)[:, None]
    q = np.arange(naux, dtype=np.uint64)[None, :]
    w = words(seed, stream, s, q)
    top = (w >> np.uint64(63)).astype(np.int64)
    return np.where(top == 0, 1.0, -1.0)


def uniform_from_word(w: np.ndarray) -> np.ndarray:
    return (np.asarray(w, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def importance_draws(seed: int, stream: int, ns: int, k: int, cdf: np.ndarray,
                     s0: int = 0):
    """k draws per vector: index Q (smallest with u < cdf[Q]) and sign.

    Returns (Q[ns][k] int64, sign[ns][k] float64).
    """
    s = np.arange(s0, s0 + ns, dtype=np.uint64)[:, None]
    j = np.arange(k, dtype=np.uint64)[None, :]
    u = uniform_from_word(words(seed, stream, s, 2 * j))
    sw = words(seed, stream, s, 2 * j + np.uint64(1))
    sign = np.where((sw >> np.uint64(63)) == 0, 1.0, -1.0)
    q = np.searchsorted(cdf, u, side="right")
    q = np.minimum(q, cdf.shape[0] - 1)
    return q.astype(np.int64), sign


CLASS_Q = 0xFFFFFFFF


def class_draws(seed: int, stream: int, ns: int, cdf: np.ndarray, s0: int = 0) -> np.ndarray:
    """One class per vector: the smallest c with u < cdf[c], u from q = CLASS_Q."""
    s = np.arange(s0, s0 + ns, dtype=np.uint64)
    u = uniform_from_word(words(seed, stream, s, np.uint64(CLASS_Q)))
    c = np.searchsorted(cdf, u, side="right")
    return np.minimum(c, cdf.shape[0] - 1).astype(np.int64)


def proposal_cdf(p: np.ndarray) -> np.ndarray:
    """Sequential FP64 prefix sum of p with the last entry forced to 1."""
    p = np.asarray(p, dtype=np.float64)
    cdf = np.empty_like(p)
    acc = 0.0
    for i in range(p.shape[0]):
        acc += float(p[i])
        cdf[i] = acc
    cdf[-1] = 1.0
    return cdf
