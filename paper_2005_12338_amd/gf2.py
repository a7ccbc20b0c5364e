"""ctypes binding of libgf2 (include/gf2.h).

Argument marshalling only: every step of the hot path runs in the
library's HIP kernels.  PyTorch provides device memory and the stream.
The functions keep the C names; ``Context`` wraps them for convenience.
Loading fails loudly if the built library is missing -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgf2.so")

GF2_OK, GF2_E_ARG, GF2_E_DEVICE, GF2_E_NOMEM, GF2_E_NUMERIC, GF2_E_STATE = 0, -1, -2, -3, -4, -5
GF2_F64, GF2_F32 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "auto": 4, "bf16c": 5}
PREC_NAME = {v: k for k, v in PREC.items()}
SAMPLE_RADEMACHER, SAMPLE_IMPORTANCE, SAMPLE_STRATIFIED = 0, 1, 2

_STATUS = {GF2_E_ARG: "GF2_E_ARG", GF2_E_DEVICE: "GF2_E_DEVICE", GF2_E_NOMEM: "GF2_E_NOMEM",
           GF2_E_NUMERIC: "GF2_E_NUMERIC", GF2_E_STATE: "GF2_E_STATE"}


class Gf2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class ChainGeom(C.Structure):
    _fields_ = [("n", C.c_int64), ("naux", C.c_int64), ("x", C.POINTER(C.c_double)),
                ("xq", C.POINTER(C.c_double)), ("amp", C.c_double), ("a", C.c_double),
                ("c", C.c_double)]


class Sampling(C.Structure):
    _fields_ = [("ns", C.c_int64), ("s0", C.c_int64), ("seed", C.c_uint64), ("mode", C.c_int32),
                ("k", C.c_int32), ("p", C.POINTER(C.c_double))]


class BatchItem(C.Structure):
    _fields_ = [("split", C.c_void_p), ("B", C.c_void_p), ("G", C.c_void_p), ("Gbar", C.c_void_p),
                ("ntau", C.c_int64), ("sampling", Sampling), ("Sigma", C.c_void_p), ("e_samples", C.c_void_p)]


BATCH_GRAPH, BATCH_AUTOTUNE = 1, 2


class AdaptiveResult(C.Structure):
    _fields_ = [("e_corr", C.c_double), ("e_corr_per_e", C.c_double), ("stderr_tot", C.c_double),
                ("pairs", C.c_int64), ("precision", C.c_int32), ("bias_probe", C.c_double)]


class MlpC(C.Structure):
    _fields_ = [("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p), ("mean", C.c_void_p),
                ("std", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p), ("step", C.c_int64)]


MLP_IN, MLP_HIDDEN = 4, 128
MLP_NPARAM = MLP_HIDDEN * MLP_IN + 2 * MLP_HIDDEN

_lib: Optional[C.CDLL] = None

_SIGS = {
    "gf2_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "gf2_destroy": (None, [C.c_void_p]),
    "gf2_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gf2_last_error": (C.c_char_p, [C.c_void_p]),
    "gf2_version": (C.c_char_p, []),
    "gf2_build_B": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.POINTER(C.c_double),
                              C.POINTER(ChainGeom), C.c_int, C.c_void_p]),
    "gf2_split": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_double,
                            C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "gf2_split_free": (None, [C.c_void_p]),
    "gf2_split_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_double)]),
    "gf2_tau_grid": (C.c_int, [C.c_double, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gf2_green_tau": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.c_double, C.c_int64, C.c_double, C.c_int64, C.POINTER(C.c_double),
                                C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "gf2_sigma_tau": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                C.POINTER(Sampling), C.c_int, C.c_void_p, C.c_void_p]),
    "gf2_sigma_det": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "gf2_sigma_stoch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                  C.POINTER(Sampling), C.c_int, C.c_void_p, C.c_void_p]),
    "gf2_sigma_stoch_cv": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.POINTER(Sampling), C.c_int, C.c_void_p, C.c_void_p]),
    "gf2_sigma_stoch_double": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.POINTER(Sampling), C.c_int, C.c_void_p, C.c_void_p]),
    "gf2_energy_double": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_double), C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gf2_sigma_finalize": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.c_void_p]),
    "gf2_energy": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_double), C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.POINTER(C.c_double),
                             C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gf2_energy_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int64, C.c_double, C.c_void_p]),
    "gf2_rng_words": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64,
                                C.POINTER(C.c_uint64)]),
    "gf2_set_profiling": (C.c_int, [C.c_void_p, C.c_int]),
    "gf2_set_gemm_tiles": (C.c_int, [C.c_void_p, C.c_int32]),
    "gf2_tuned_tiles": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.POINTER(C.c_int32)]),
    "gf2_debug_gemm": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "gf2_profile_read": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.POINTER(C.c_int32)]),
    "gf2_sigma_batch": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int, C.c_int32]),
    "gf2_energy_adaptive": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.POINTER(C.c_double), C.c_void_p, C.c_double, C.POINTER(Sampling),
                                      C.c_int, C.c_double, C.c_int64, C.c_void_p, C.c_void_p,
                                      C.POINTER(AdaptiveResult)]),
    "gf2_energy_adaptive_det": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                          C.POINTER(C.c_double), C.c_double, C.POINTER(Sampling), C.c_int,
                                          C.c_double, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.POINTER(AdaptiveResult)]),
    "gf2_screen_ijA": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int, C.c_double, C.c_void_p,
                                 C.POINTER(C.c_int64)]),
    "gf2_split_large": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_double,
                                  C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "gf2_qp_energies": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_double, C.c_int64, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_double),
                                  C.POINTER(C.c_int32)]),
    "gf2_dyson": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_double, C.c_int64, C.POINTER(C.c_double),
                            C.POINTER(C.c_double), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gf2_electron_count": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_double, C.c_int64,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p, C.c_int64, C.POINTER(C.c_double)]),
    "gf2_tune_mu": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gf2_fock": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_void_p, C.POINTER(C.c_double)]),
    "gf2_scf_step": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.c_double, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p, C.c_int64, C.c_double, C.c_double,
                               C.c_double, C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "gf2_proposal_features": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
    "gf2_proposal_targets": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                       C.POINTER(C.c_double), C.c_double, C.c_void_p, C.c_void_p]),
    "gf2_proposal_init": (C.c_int, [C.c_void_p, C.POINTER(MlpC), C.c_void_p, C.c_int64, C.c_uint64]),
    "gf2_proposal_grad": (C.c_int, [C.c_void_p, C.POINTER(MlpC), C.c_int32, C.POINTER(C.c_int64), C.c_void_p,
                                    C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gf2_proposal_train": (C.c_int, [C.c_void_p, C.POINTER(MlpC), C.c_int32, C.POINTER(C.c_int64), C.c_void_p,
                                     C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "gf2_proposal_infer": (C.c_int, [C.c_void_p, C.POINTER(MlpC), C.c_void_p, C.c_int64, C.c_double, C.c_int32,
                                     C.c_void_p]),
}


def declared_symbols(header: Optional[str] = None):
    """Names of the functions declared in include/gf2*.h."""
    import re
    inc = os.path.join(os.path.dirname(_PKG), "include")
    names = []
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            names += re.findall(r"^\s*(?:gf2_status|void|const char\*|gf2_\w+\*?)\s+(gf2_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def load() -> C.CDLL:
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2005_12338_amd.build")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dtype(t) -> int:
    """GF2_F64 / GF2_F32 of a torch tensor (raises for anything else)."""
    import torch
    if t.dtype == torch.float64:
        return GF2_F64
    if t.dtype == torch.float32:
        return GF2_F32
    raise TypeError(f"B must be float64 or float32, not {t.dtype}")


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def gf2_tau_grid(beta: float, ntau: int):
    lib = load()
    tau = np.zeros(ntau)
    w = np.zeros(ntau)
    st = lib.gf2_tau_grid(float(beta), int(ntau), _dp(tau), _dp(w))
    if st != GF2_OK:
        raise Gf2Error(st, "gf2_tau_grid")
    return tau, w


@dataclass
class Split:
    handle: C.c_void_p
    n: int
    naux: int
    nnz: int
    wmax: int
    b_ptr: int
    dtype: int
    ctx: "Context"
    large: object = None      # the tensor the large part is read from (kept alive with the handle)

    def free(self):
        if self.handle:
            load().gf2_split_free(self.handle)
            self.handle = None

    def export(self):
        """(w[naux], idx[naux][32], blocks[naux][32][32], kmax) on the host."""
        w = np.zeros(self.naux, dtype=np.int32)
        idx = np.zeros((self.naux, 32), dtype=np.int32)
        blk = np.zeros((self.naux, 32, 32))
        kmax = C.c_double(0)
        self.ctx._check(load().gf2_split_export(self.ctx.h, self.handle, w.ctypes.data, idx.ctypes.data,
                                                blk.ctypes.data, C.byref(kmax)))
        return w, idx, blk, kmax.value

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """A gf2 context bound to a device and torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.gf2_create(C.byref(h), int(device), C.c_void_p(stream.cuda_stream))
        if st != GF2_OK:
            raise Gf2Error(st, "gf2_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.gf2_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != GF2_OK:
            raise Gf2Error(st, self.lib.gf2_last_error(self.h).decode())

    # ---------------------------------------------------------------- B
    def build_B(self, n: int, naux: int, geom=None, ijA=None, V: Optional[np.ndarray] = None,
                dtype=None):
        torch = self.torch
        dtype = dtype or torch.float32
        dt = GF2_F64 if dtype == torch.float64 else GF2_F32
        B = torch.empty((naux, n, n), dtype=dtype, device=self.device)
        g = None
        keep = []
        if ijA is None:
            x = np.ascontiguousarray(geom.x, dtype=np.float64)
            xq = np.ascontiguousarray(geom.xq, dtype=np.float64)
            keep += [x, xq]
            g = ChainGeom(n, naux, _dp(x), _dp(xq), geom.amp, geom.a, geom.c)
        vp = None
        if V is not None:
            V = np.ascontiguousarray(V, dtype=np.float64)
            keep.append(V)
            vp = _dp(V)
        self._check(self.lib.gf2_build_B(self.h, n, naux, _ptr(ijA), vp, C.byref(g) if g else None, dt,
                                         B.data_ptr()))
        return B

    def split(self, B, eps: float) -> Split:
        torch = self.torch
        dt = GF2_F64 if B.dtype == torch.float64 else GF2_F32
        naux, n, _ = B.shape
        h = C.c_void_p()
        nnz = C.c_int64()
        wmax = C.c_int64()
        self._check(self.lib.gf2_split(self.h, B.data_ptr(), dt, n, naux, float(eps), C.byref(h),
                                       C.byref(nnz), C.byref(wmax)))
        return Split(h, n, naux, nnz.value, wmax.value, B.data_ptr(), dt, self)

    def screen_ijA(self, ijA, eps_prime: float):
        """eq:V_ijA on device (ij|A) [naux][n][n]: (screened copy, kept count)."""
        naux, n, _ = ijA.shape
        out = self.torch.empty_like(ijA)
        nnz = C.c_int64()
        self._check(self.lib.gf2_screen_ijA(self.h, n, naux, ijA.data_ptr(), _dtype(ijA), float(eps_prime),
                                            out.data_ptr(), C.byref(nnz)))
        return out, nnz.value

    def split_large(self, B, KL, eps: float) -> Split:
        """The split whose large part comes from KL (screened front end)."""
        naux, n, _ = B.shape
        if KL.shape != B.shape or KL.dtype != B.dtype:
            raise ValueError("KL must match B in shape and dtype")
        h = C.c_void_p()
        nnz = C.c_int64()
        wmax = C.c_int64()
        self._check(self.lib.gf2_split_large(self.h, B.data_ptr(), KL.data_ptr(), _dtype(B), n, naux, float(eps),
                                             C.byref(h), C.byref(nnz), C.byref(wmax)))
        return Split(h, n, naux, nnz.value, wmax.value, B.data_ptr(), _dtype(B), self, KL)

    # ---------------------------------------------------------------- G
    def green_tau(self, F: np.ndarray, tau: np.ndarray, beta: float, mu: float = 0.0, n_occ: int = 0,
                  S: Optional[np.ndarray] = None):
        torch = self.torch
        F = np.ascontiguousarray(F, dtype=np.float64)
        tau = np.ascontiguousarray(tau, dtype=np.float64)
        n = F.shape[0]
        G = torch.empty((tau.shape[0], n, n), dtype=torch.float64, device=self.device)
        Gb = torch.empty_like(G)
        mu_out = C.c_double(0)
        sp = None
        if S is not None:
            S = np.ascontiguousarray(S, dtype=np.float64)
            sp = _dp(S)
        self._check(self.lib.gf2_green_tau(self.h, n, _dp(F), sp, float(mu), int(n_occ), float(beta),
                                           tau.shape[0], _dp(tau), G.data_ptr(), Gb.data_ptr(),
                                           C.byref(mu_out)))
        return G, Gb, mu_out.value

    # ---------------------------------------------------------------- SCF
    @staticmethod
    def _f64(a):
        return None if a is None else np.ascontiguousarray(a, dtype=np.float64)

    def dyson(self, F, S, mu, beta, tau, w, Sigma, nw):
        """G(tau), G(beta - tau) [ntau][n][n] and G(beta-) [n][n] of the Dyson G
        at mu (gf2_dyson)."""
        torch = self.torch
        F, S, tau, w = self._f64(F), self._f64(S), self._f64(tau), self._f64(w)
        n, ntau = F.shape[0], tau.shape[0]
        G = torch.empty((ntau, n, n), dtype=torch.float64, device=self.device)
        Gb = torch.empty_like(G)
        Gbeta = torch.empty((n, n), dtype=torch.float64, device=self.device)
        self._check(self.lib.gf2_dyson(self.h, n, _dp(F), None if S is None else _dp(S), float(mu), float(beta),
                                       ntau, _dp(tau), _dp(w), Sigma.data_ptr(), int(nw), G.data_ptr(),
                                       Gb.data_ptr(), Gbeta.data_ptr()))
        return G, Gb, Gbeta

    def electron_count(self, F, S, mu, beta, tau, w, Sigma, nw) -> float:
        F, S, tau, w = self._f64(F), self._f64(S), self._f64(tau), self._f64(w)
        out = C.c_double(0)
        self._check(self.lib.gf2_electron_count(self.h, F.shape[0], _dp(F), None if S is None else _dp(S),
                                                float(mu), float(beta), tau.shape[0], _dp(tau), _dp(w),
                                                Sigma.data_ptr(), int(nw), C.byref(out)))
        return out.value

    def tune_mu(self, F, S, beta, tau, w, Sigma, nw, n_elec, lo, hi):
        """(mu, N_e reached) with N_e(mu) = n_elec in [lo, hi] (gf2_tune_mu)."""
        F, S, tau, w = self._f64(F), self._f64(S), self._f64(tau), self._f64(w)
        mu, ne = C.c_double(0), C.c_double(0)
        self._check(self.lib.gf2_tune_mu(self.h, F.shape[0], _dp(F), None if S is None else _dp(S), float(beta),
                                         tau.shape[0], _dp(tau), _dp(w), Sigma.data_ptr(), int(nw),
                                         float(n_elec), float(lo), float(hi), C.byref(mu), C.byref(ne)))
        return mu.value, ne.value

    def qp_energies(self, F, S, mu, beta, tau, w, Sigma, n_pade, eta=1e-9, max_iter=200):
        """Quasiparticle energies (gf2_qp_energies): (E [n], converged [n])."""
        F, S, tau, w = self._f64(F), self._f64(S), self._f64(tau), self._f64(w)
        n = F.shape[0]
        e = np.empty(n)
        ok = np.zeros(n, dtype=np.int32)
        self._check(self.lib.gf2_qp_energies(self.h, n, _dp(F), None if S is None else _dp(S), float(mu),
                                             float(beta), tau.shape[0], _dp(tau), _dp(w), Sigma.data_ptr(),
                                             int(n_pade), float(eta), int(max_iter), _dp(e),
                                             ok.ctypes.data_as(C.POINTER(C.c_int32))))
        return e, ok.astype(bool)

    def fock(self, B, h, Gbeta):
        """eq:F on the RI factors, P = -2 G(beta-) (gf2_fock); host [n][n]."""
        h = self._f64(h)
        n, naux = h.shape[0], B.shape[0]
        out = np.empty((n, n))
        self._check(self.lib.gf2_fock(self.h, n, naux, B.data_ptr(), _dtype(B), _dp(h), Gbeta.data_ptr(),
                                      _dp(out)))
        return out

    def scf_step(self, B, h, F, S, beta, tau, w, Sigma, nw, n_elec, lo, hi):
        """One update around the self-energy (gf2_scf_step): returns
        (mu, G, Gbar, G(beta-), new F)."""
        torch = self.torch
        h, F, S, tau, w = self._f64(h), self._f64(F), self._f64(S), self._f64(tau), self._f64(w)
        n, ntau = F.shape[0], tau.shape[0]
        G = torch.empty((ntau, n, n), dtype=torch.float64, device=self.device)
        Gb = torch.empty_like(G)
        Gbeta = torch.empty((n, n), dtype=torch.float64, device=self.device)
        Fo = np.empty((n, n))
        mu = C.c_double(0)
        self._check(self.lib.gf2_scf_step(self.h, n, B.shape[0], B.data_ptr(), _dtype(B), _dp(h), _dp(F),
                                          None if S is None else _dp(S), float(beta), ntau, _dp(tau), _dp(w),
                                          Sigma.data_ptr(), int(nw), float(n_elec), float(lo), float(hi),
                                          C.byref(mu), G.data_ptr(), Gb.data_ptr(), Gbeta.data_ptr(), _dp(Fo)))
        return mu.value, G, Gb, Gbeta, Fo

    # ---------------------------------------------------------------- Sigma
    @staticmethod
    def _sampling(ns, seed, s0=0, p=None, k=1, classes=0):
        """classes > 0: stratified vectors over that many classes, with class
        weights from p (uniform if p is None); else importance draws if p is
        given, else +-1 orbitals."""
        keep = None
        if classes:
            if p is None:
                raise ValueError("stratified sampling needs the per-Q weights p")
            keep = np.ascontiguousarray(p, dtype=np.float64)
            s = Sampling(ns, s0, seed, SAMPLE_STRATIFIED, int(classes), _dp(keep))
        elif p is not None:
            keep = np.ascontiguousarray(p, dtype=np.float64)
            s = Sampling(ns, s0, seed, SAMPLE_IMPORTANCE, k, _dp(keep))
        else:
            s = Sampling(ns, s0, seed, SAMPLE_RADEMACHER, 1, None)
        return s, keep

    def sigma_tau(self, split: Split, B, G, Gb, ns: int, seed: int = 0, prec: str = "fp32", p=None, k=1,
                  s0: int = 0, want_samples: bool = True, classes: int = 0):
        torch = self.torch
        ntau, n, _ = G.shape
        Sigma = torch.empty((ntau, n, n), dtype=torch.float64, device=self.device)
        es = torch.empty((ns, ntau), dtype=torch.float64, device=self.device) if want_samples else None
        smp, keep = self._sampling(ns, seed, s0, p, k, classes)
        self._check(self.lib.gf2_sigma_tau(self.h, split.handle, B.data_ptr(), G.data_ptr(), Gb.data_ptr(),
                                           ntau, C.byref(smp), PREC[prec], Sigma.data_ptr(), _ptr(es)))
        return Sigma, es

    def sigma_det(self, split: Split, G, Gb):
        torch = self.torch
        ntau, n, _ = G.shape
        out = torch.empty((ntau, n, n), dtype=torch.float64, device=self.device)
        self._check(self.lib.gf2_sigma_det(self.h, split.handle, G.data_ptr(), Gb.data_ptr(), ntau,
                                           out.data_ptr()))
        return out

    def sigma_stoch(self, split: Split, B, G, Gb, Sigma_sum, ns: int, seed: int = 0, prec: str = "fp32",
                    p=None, k=1, s0: int = 0, e_samples=None, classes: int = 0):
        ntau = G.shape[0]
        smp, keep = self._sampling(ns, seed, s0, p, k, classes)
        self._check(self.lib.gf2_sigma_stoch(self.h, split.handle, B.data_ptr(), G.data_ptr(),
                                             Gb.data_ptr(), ntau, C.byref(smp), PREC[prec],
                                             Sigma_sum.data_ptr(), _ptr(e_samples)))

    def sigma_stoch_cv(self, split: Split, B, G, Gb, Sigma_sum, ns: int, seed: int = 0, prec: str = "fp32",
                       s0: int = 0, e_samples=None):
        """Control-variate form: adds sum_s [chain(R, R') - chain(R^L, R'^L)]."""
        ntau = G.shape[0]
        smp, keep = self._sampling(ns, seed, s0)
        self._check(self.lib.gf2_sigma_stoch_cv(self.h, split.handle, B.data_ptr(), G.data_ptr(), Gb.data_ptr(),
                                                ntau, C.byref(smp), PREC[prec], Sigma_sum.data_ptr(),
                                                _ptr(e_samples)))

    def sigma_stoch_double(self, split: Split, B, G, Gb, Sigma_sum, ns: int, seed: int = 0, prec: str = "fp32",
                           s0: int = 0, e_samples=None):
        """Double average: adds the pair estimate of every (i, j) < ns combination;
        e_samples [ns*ns][ntau], row i*ns + j."""
        ntau = G.shape[0]
        smp, keep = self._sampling(ns, seed, s0)
        self._check(self.lib.gf2_sigma_stoch_double(self.h, split.handle, B.data_ptr(), G.data_ptr(),
                                                    Gb.data_ptr(), ntau, C.byref(smp), PREC[prec],
                                                    Sigma_sum.data_ptr(), _ptr(e_samples)))

    def energy_double(self, Sigma, Gb, w: np.ndarray, n_elec: float, e_samples, ns: int):
        ntau, n, _ = Sigma.shape
        w = np.ascontiguousarray(w, dtype=np.float64)
        e, epe, se = C.c_double(), C.c_double(), C.c_double()
        self._check(self.lib.gf2_energy_double(self.h, n, ntau, _dp(w), Sigma.data_ptr(), Gb.data_ptr(),
                                               e_samples.data_ptr(), int(ns), float(n_elec), C.byref(e),
                                               C.byref(epe), C.byref(se)))
        return e.value, epe.value, se.value

    def sigma_finalize(self, Sigma_det, Sigma_sum, ns_total: int):
        out = self.torch.empty_like(Sigma_det)
        ntau, n, _ = Sigma_det.shape
        self._check(self.lib.gf2_sigma_finalize(self.h, n, ntau, Sigma_det.data_ptr(), Sigma_sum.data_ptr(),
                                                int(ns_total), out.data_ptr()))
        return out

    def sigma_batch(self, items, prec: str = "fp32", graph: bool = False, autotune: bool = False):
        """items: list of dict(split, B, G, Gb, ns, seed[, s0, p, k]).  Returns
        [(Sigma, e_samples)] in item order."""
        torch = self.torch
        arr = (BatchItem * len(items))()
        outs, keep = [], []
        for i, it in enumerate(items):
            ntau, n, _ = it["G"].shape
            Sigma = torch.empty((ntau, n, n), dtype=torch.float64, device=self.device)
            es = torch.empty((it["ns"], ntau), dtype=torch.float64, device=self.device)
            smp, kp = self._sampling(it["ns"], it.get("seed", 0), it.get("s0", 0), it.get("p"), it.get("k", 1),
                                     it.get("classes", 0))
            keep.append(kp)
            arr[i] = BatchItem(it["split"].handle, it["B"].data_ptr(), it["G"].data_ptr(), it["Gb"].data_ptr(),
                               ntau, smp, Sigma.data_ptr(), es.data_ptr())
            outs.append((Sigma, es))
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_AUTOTUNE if autotune else 0)
        self._check(self.lib.gf2_sigma_batch(self.h, len(items), C.addressof(arr), PREC[prec], flags))
        return outs

    def energy_adaptive(self, split: Split, B, G, Gb, w: np.ndarray, Sigma_det, n_elec: float, target: float,
                        batch: int = 16, max_pairs: int = 4096, seed: int = 0, prec: str = "auto", p=None,
                        k: int = 1, classes: int = 0):
        """Sample pairs in batches until the standard error of the total
        E_corr is below target.  Returns (Sigma, e_samples[:pairs], dict)."""
        torch = self.torch
        ntau, n, _ = G.shape
        w = np.ascontiguousarray(w, dtype=np.float64)
        Sigma = torch.empty((ntau, n, n), dtype=torch.float64, device=self.device)
        es = torch.empty((max_pairs, ntau), dtype=torch.float64, device=self.device)
        smp, keep = self._sampling(batch, seed, 0, p, k, classes)
        r = AdaptiveResult()
        self._check(self.lib.gf2_energy_adaptive(self.h, split.handle, B.data_ptr(), G.data_ptr(), Gb.data_ptr(),
                                                 ntau, _dp(w), Sigma_det.data_ptr(), float(n_elec), C.byref(smp),
                                                 PREC[prec], float(target), int(max_pairs), Sigma.data_ptr(),
                                                 es.data_ptr(), C.byref(r)))
        info = dict(E=r.e_corr, E_per_e=r.e_corr_per_e, stderr=r.stderr_tot, pairs=int(r.pairs),
                    precision=PREC_NAME[int(r.precision)], bias_probe=r.bias_probe)
        return Sigma, es[:r.pairs], info

    def energy_adaptive_det(self, split: Split, B, G, Gb, w: np.ndarray, n_elec: float, target: float,
                            batch: int = 16, max_pairs: int = 4096, seed: int = 0, prec: str = "auto", p=None,
                            k: int = 1, classes: int = 0):
        """energy_adaptive with Sigma[D,D] computed inside, overlapped with the
        first batch of pairs.  Returns (Sigma, Sigma_det, e_samples[:pairs], dict)."""
        torch = self.torch
        ntau, n, _ = G.shape
        w = np.ascontiguousarray(w, dtype=np.float64)
        det = torch.empty((ntau, n, n), dtype=torch.float64, device=self.device)
        Sigma = torch.empty((ntau, n, n), dtype=torch.float64, device=self.device)
        es = torch.empty((max_pairs, ntau), dtype=torch.float64, device=self.device)
        smp, keep = self._sampling(batch, seed, 0, p, k, classes)
        r = AdaptiveResult()
        self._check(self.lib.gf2_energy_adaptive_det(self.h, split.handle, B.data_ptr(), G.data_ptr(),
                                                     Gb.data_ptr(), ntau, _dp(w), float(n_elec), C.byref(smp),
                                                     PREC[prec], float(target), int(max_pairs), det.data_ptr(),
                                                     Sigma.data_ptr(), es.data_ptr(), C.byref(r)))
        info = dict(E=r.e_corr, E_per_e=r.e_corr_per_e, stderr=r.stderr_tot, pairs=int(r.pairs),
                    precision=PREC_NAME[int(r.precision)], bias_probe=r.bias_probe)
        return Sigma, det, es[:r.pairs], info

    # ---------------------------------------------------------------- energy
    def energy(self, Sigma, Gb, w: np.ndarray, n_elec: float, e_samples=None):
        ntau, n, _ = Sigma.shape
        w = np.ascontiguousarray(w, dtype=np.float64)
        e = C.c_double()
        epe = C.c_double()
        se = C.c_double()
        ns = 0 if e_samples is None else e_samples.shape[0]
        self._check(self.lib.gf2_energy(self.h, n, ntau, _dp(w), Sigma.data_ptr(), Gb.data_ptr(),
                                        _ptr(e_samples), ns, float(n_elec), C.byref(e), C.byref(epe),
                                        C.byref(se)))
        return e.value, epe.value, se.value

    def energy_noalloc(self, Sigma, Gb, w_dev, n_elec: float, out, e_samples=None):
        """gf2_energy_noalloc: every argument on the device; out[3] receives
        (E_tot, E_per_e, stderr).  Enqueues kernels only (no allocation, no
        synchronisation)."""
        ntau, n, _ = Sigma.shape
        ns = 0 if e_samples is None else e_samples.shape[0]
        self._check(self.lib.gf2_energy_noalloc(self.h, n, ntau, w_dev.data_ptr(), Sigma.data_ptr(), Gb.data_ptr(),
                                                _ptr(e_samples), ns, float(n_elec), out.data_ptr()))

    def debug_gemm(self, prec: str, n: int, A, Bt, Cout, batch: int = 1):
        """C[b] = A[b] Bt[b]^T with the chain's GEMM kernel (padded square operands)."""
        self._check(self.lib.gf2_debug_gemm(self.h, PREC[prec], n, batch, A.data_ptr(), Bt.data_ptr(),
                                            Cout.data_ptr()))

    def set_gemm_tiles(self, mode):
        """BF16 tile choice where 160 pads less than 128: 2 (default, or True)
        the 160-wide tiles on every product launch, 1 on the deep-K stage only,
        0 (or False) the 128-wide tile everywhere."""
        m = (2 if mode else 0) if isinstance(mode, bool) else int(mode)
        self._check(self.lib.gf2_set_gemm_tiles(self.h, m))

    def tuned_tiles(self, prec: str, n: int) -> int:
        """Tile mode the batch autotuner chose for chains of size n (-1: none)."""
        m = C.c_int32(0)
        self._check(self.lib.gf2_tuned_tiles(self.h, PREC[prec], int(n), C.byref(m)))
        return m.value

    def set_profiling(self, on: bool):
        self._check(self.lib.gf2_set_profiling(self.h, 1 if on else 0))

    def profile_read(self):
        """{kernel class: dict(launches, ms, flops, bytes)} since the last read."""
        cap = 64
        names = C.create_string_buffer(32 * cap)
        la = np.zeros(cap, dtype=np.int64)
        ms = np.zeros(cap)
        fl = np.zeros(cap)
        by = np.zeros(cap)
        cnt = C.c_int32()
        self._check(self.lib.gf2_profile_read(self.h, cap, names, la.ctypes.data, ms.ctypes.data,
                                              fl.ctypes.data, by.ctypes.data, C.byref(cnt)))
        out = {}
        raw = names.raw
        for i in range(cnt.value):
            nm = raw[32 * i:32 * (i + 1)].split(b"\0")[0].decode()
            out[nm] = dict(launches=int(la[i]), ms=float(ms[i]), flops=float(fl[i]), bytes=float(by[i]))
        return out

    # ------------------------------------------------------------ proposal
    def proposal_features(self, split: Split, B, x: np.ndarray, xq: np.ndarray, Gbeta, phi):
        x = np.ascontiguousarray(x, dtype=np.float64)
        xq = np.ascontiguousarray(xq, dtype=np.float64)
        self._check(self.lib.gf2_proposal_features(self.h, split.handle, B.data_ptr(), _dp(x), _dp(xq),
                                                   Gbeta.data_ptr(), phi.data_ptr()))

    def proposal_targets(self, split: Split, B, G, Gb, w: np.ndarray, rel: float, t, tables=None):
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._check(self.lib.gf2_proposal_targets(self.h, split.handle, B.data_ptr(), G.data_ptr(), Gb.data_ptr(),
                                                  w.shape[0], _dp(w), float(rel), t.data_ptr(), _ptr(tables)))

    def mlp(self):
        """A network with device buffers (FP32) owned by the returned object."""
        return Mlp(self.device)

    def proposal_init(self, m: "Mlp", phi, seed: int):
        self._check(self.lib.gf2_proposal_init(self.h, C.byref(m.c), phi.data_ptr(), phi.shape[0], seed))

    def proposal_grad(self, m: "Mlp", chain_off: np.ndarray, phi, t_hat):
        off = np.ascontiguousarray(chain_off, dtype=np.int64)
        loss = C.c_double()
        grad = np.zeros(MLP_NPARAM)
        self._check(self.lib.gf2_proposal_grad(self.h, C.byref(m.c), off.shape[0] - 1,
                                               off.ctypes.data_as(C.POINTER(C.c_int64)), phi.data_ptr(),
                                               t_hat.data_ptr(), C.byref(loss), _dp(grad)))
        return loss.value, grad

    def proposal_train(self, m: "Mlp", chain_off: np.ndarray, phi, t_hat, steps: int, lr: float):
        off = np.ascontiguousarray(chain_off, dtype=np.int64)
        hist = np.zeros(steps)
        self._check(self.lib.gf2_proposal_train(self.h, C.byref(m.c), off.shape[0] - 1,
                                                off.ctypes.data_as(C.POINTER(C.c_int64)), phi.data_ptr(),
                                                t_hat.data_ptr(), steps, float(lr), _dp(hist)))
        return hist

    def proposal_infer(self, m: "Mlp", phi, alpha: float, p, bf16: bool = False):
        self._check(self.lib.gf2_proposal_infer(self.h, C.byref(m.c), phi.data_ptr(), phi.shape[0],
                                                float(alpha), 1 if bf16 else 0, p.data_ptr()))

    def rng_words(self, seed: int, stream: int, s: int, q0: int, count: int) -> np.ndarray:
        out = np.zeros(count, dtype=np.uint64)
        self._check(self.lib.gf2_rng_words(self.h, seed, stream, s, q0, count,
                                            out.ctypes.data_as(C.POINTER(C.c_uint64))))
        return out


class Mlp:
    """Device buffers of one proposal network (gf2_mlp), FP32."""

    def __init__(self, device):
        import torch
        kw = dict(dtype=torch.float32, device=device)
        self.w1 = torch.zeros(MLP_HIDDEN, MLP_IN, **kw)
        self.b1 = torch.zeros(MLP_HIDDEN, **kw)
        self.w2 = torch.zeros(MLP_HIDDEN, **kw)
        self.mean = torch.zeros(MLP_IN, **kw)
        self.std = torch.ones(MLP_IN, **kw)
        self.adam_m = torch.zeros(MLP_NPARAM, **kw)
        self.adam_v = torch.zeros(MLP_NPARAM, **kw)
        self.c = MlpC(self.w1.data_ptr(), self.b1.data_ptr(), self.w2.data_ptr(), self.mean.data_ptr(),
                      self.std.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr(), 0)

    @property
    def step(self) -> int:
        return int(self.c.step)
