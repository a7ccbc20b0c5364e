/*
 * gf2.h -- C ABI of the MI355X (gfx950) RS-SRI-GF2 hot path.
 *
 * The library assembles the imaginary-time second-order self-energy
 * Sigma(tau) and the Galitskii-Migdal correlation energy with the
 * range-separated stochastic resolution of identity of Dou, Chen,
 * Takeshita, Baer, Neuhauser and Rabani (arXiv 2005.12338):
 *
 *   RI factors        K^Q_ij = sum_A (ij|A) V^{-1/2}_AQ          eq:K_ijQ
 *   range separation  [K^Q]^L = K^Q where |K| >= eps max|K|    eq:K_L
 *   stochastic split  R^xi = sum_Q theta_Q K^Q, R^L, R^S = R - R^L (Sec. II)
 *   self-energy       eq:sigma with v from eq:RS-SRI, as in eq:sigma_2
 *   energy            eq:corr, with the sign and factor fixed by the MP2 limit
 *
 * Conventions
 *   - Matrices are row-major; dimensions are int64_t.
 *   - The caller owns every buffer.  Arguments documented as "device" are
 *     device pointers on the context's device (e.g. from torch); "host"
 *     arguments are ordinary host memory.  The library owns only the opaque
 *     context (scratch workspace, tuning table) and split handles.
 *   - Device work is stream-ordered on the context's stream (gf2_create /
 *     gf2_set_stream).  Calls that return host values synchronise that
 *     stream before returning; the others are asynchronous.
 *   - Every call returns a gf2_status.  On failure gf2_last_error(ctx)
 *     describes the cause.  No C++ exception crosses this boundary.  A
 *     context may be used by one host thread at a time.
 *   - Everything runs in this library's HIP kernels (gfx950); there is no CPU
 *     fallback for the device work.
 */
#ifndef GF2_H
#define GF2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GF2_OK = 0,
  GF2_E_ARG = -1,      /* an argument is out of range or inconsistent        */
  GF2_E_DEVICE = -2,   /* a HIP runtime call failed                          */
  GF2_E_NOMEM = -3,    /* device or host allocation failed                   */
  GF2_E_NUMERIC = -4,  /* a non-finite value reached an output               */
  GF2_E_STATE = -5     /* a handle does not belong to the given data / ctx   */
} gf2_status;

typedef enum { GF2_F64 = 0, GF2_F32 = 1 } gf2_dtype;

/* Arithmetic of the stochastic-block products (the 24 dense N x N GEMMs per
 * (tau, pair)).  The deterministic block, traces, accumulation of Sigma and
 * the energy are always FP64.
 *   FP64   : FP64 operands, FP64 MFMA.
 *   FP32   : FP32 operands, FP32 MFMA.
 *   BF16   : BF16 operands, FP32 accumulation (BF16 MFMA).
 *   BF16X3 : each operand split hi = bf16(x), lo = bf16(x - hi); products
 *            hi*hi + hi*lo + lo*hi accumulated in FP32.                     */
typedef enum {
  GF2_PREC_FP64 = 0,
  GF2_PREC_FP32 = 1,
  GF2_PREC_BF16 = 2,
  GF2_PREC_BF16X3 = 3,
  GF2_PREC_AUTO = 4,   /* gf2_energy_adaptive only: BF16 with the
                          two-level correction below, switching to BF16X3
                          when the correction is not precise enough        */
  GF2_PREC_BF16C = 5   /* gf2_sigma_tau / gf2_sigma_stoch only: two-level
                          estimator.  Every pair runs in BF16; the first
                          k = min(ns, 8) pairs also run in BF16X3, and
                          Sigma_sum and the per-pair traces are moved by
                          the mean BF16X3 - BF16 difference of those pairs
                          (ns/k times their summed difference).  BF16
                          rounding biases every pair alike (its second-order
                          terms do not average out over pairs); the
                          correction removes that bias in expectation and
                          leaves std(difference)/sqrt(k) of it            */
} gf2_precision;

/* How the stochastic orbitals are drawn (counter-based SplitMix64, see
 * gf2_rng_word):
 *   RADEMACHER : theta_Q = +-1 for every Q (the paper's orbitals, Sec. II).
 *   IMPORTANCE : theta = (1/sqrt k) sum_j e_j u_{Q_j} / sqrt(p_{Q_j}) with
 *                Q_j drawn from the proposal p and e_j = +-1 (unbiased for
 *                any p > 0 since E[theta theta^T] = I).
 *   STRATIFIED : the auxiliary index is split into k classes Q = c (mod k);
 *                each vector draws one class with probability
 *                pi_c = sum_{Q = c mod k} p_Q (sequential sums, then divided
 *                by their sequential total) from the uniform of word(seed,
 *                stream, s, 0xFFFFFFFF), and theta_Q = e_Q / sqrt(pi_c) on
 *                the class members (e_Q the RADEMACHER sign of the same
 *                (stream, s, Q)), 0 elsewhere.  Members of one class are k
 *                auxiliary functions apart, so the +-1 cross terms between
 *                neighbouring Q vanish; E[theta theta^T] = I for any pi > 0. */
typedef enum {
  GF2_SAMPLE_RADEMACHER = 0,
  GF2_SAMPLE_IMPORTANCE = 1,
  GF2_SAMPLE_STRATIFIED = 2
} gf2_sample_mode;

typedef struct gf2_ctx gf2_ctx;
typedef struct gf2_split_h gf2_split_h;

/* Synthetic chain: B^Q_ij = amp exp(-a (x_i-x_j)^2) exp(-c (x_Q-(x_i+x_j)/2)^2). */
typedef struct {
  int64_t n;          /* number of orbitals N                                */
  int64_t naux;       /* number of auxiliary functions N_aux                 */
  const double* x;    /* host [n] orbital centres                           */
  const double* xq;   /* host [naux] auxiliary centres                      */
  double amp, a, c;
} gf2_chain_geom;

typedef struct {
  int64_t ns;          /* number of stochastic pairs (xi_s, eta_s)          */
  int64_t s0;          /* index of the first pair (counter offset)          */
  uint64_t seed;
  int32_t mode;        /* gf2_sample_mode                                   */
  int32_t k;           /* draws per vector (IMPORTANCE, >= 1) or classes
                          (STRATIFIED, 2 .. naux)                           */
  const double* p;     /* host [naux] proposal (IMPORTANCE, STRATIFIED),
                          positive, sums to 1                               */
} gf2_sampling;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the null stream).  *ctx receives the handle. */
gf2_status gf2_create(gf2_ctx** ctx, int device, void* hip_stream);
void gf2_destroy(gf2_ctx* ctx);
gf2_status gf2_set_stream(gf2_ctx* ctx, void* hip_stream);
/* Message of the last failure on this context ("" if none); owned by ctx. */
const char* gf2_last_error(const gf2_ctx* ctx);
/* Library version string (static storage). */
const char* gf2_version(void);

/* ------------------------------------------------------------ B (a1) ----
 * eq:K_ijQ.  Writes B[naux][n][n] (row-major, device, dtype out_dtype).
 *   ijA == NULL : synthetic chain from *geom (geom->n, geom->naux must equal
 *                 n, naux); V is ignored (V = I).
 *   ijA != NULL : device [naux][n][n] three-index integrals (ij|A) in
 *                 out_dtype; V is host [naux][naux] symmetric positive
 *                 definite (NULL means V = I, i.e. B = ijA).  V^{-1/2} is
 *                 formed from V's eigendecomposition in FP64.
 * Errors: GF2_E_ARG for n, naux <= 0, missing geom in synthetic mode, or a
 * V that is not positive definite. */
gf2_status gf2_build_B(gf2_ctx* ctx, int64_t n, int64_t naux, const void* ijA,
                       const double* V, const gf2_chain_geom* geom,
                       gf2_dtype out_dtype, void* B);

/* ------------------------------------------------------------ split (a2) --
 * eq:K_L on K = B: m = max |B| over all elements; K^L keeps elements with
 * |B| >= eps * m (inclusive) and zeroes the rest.  The handle stores, per Q,
 * the support S_Q (orbitals with a kept element in their row) and the dense
 * block K^L[Q][S_Q][S_Q], plus the gather/scatter maps of the union pattern.
 * B is device [naux][n][n] of dtype `dtype`; it must stay unchanged while the
 * handle is used (the handle records B's address and checks it).
 * Outputs (host): *nnzL kept elements, *wmax = max_Q |S_Q|.
 * Errors: GF2_E_ARG for eps < 0, n or naux <= 0, or a support wider than 32
 * orbitals (the block kernels' limit). */
gf2_status gf2_split(gf2_ctx* ctx, const void* B, gf2_dtype dtype, int64_t n,
                     int64_t naux, double eps, gf2_split_h** out,
                     int64_t* nnzL, int64_t* wmax);

/* gf2_screen_ijA: eq:V_ijA.  (ij|A)^L = (ij|A) where |(ij|A)| >= (eps' / n)
 *   M_j, M_j = max over i and A of |(ij|A)| for orbital j (inclusive), and 0
 *   elsewhere.  ijA and out device [naux][n][n] (A, i, j) of dtype `dtype`
 *   (may alias: the screen is elementwise after the column maxima); the
 *   comparison is made in FP64.  *nnz (host, may be NULL) = kept elements.
 *   Errors: GF2_E_ARG (eps' < 0, sizes, dtype).
 * gf2_split_large: the split of the screened front end.  The large part is
 *   taken from KL, the factors of the screened integrals (gf2_build_B of
 *   gf2_screen_ijA's output: the second eq:K_ijQ), through eq:K_L on KL
 *   itself (|KL| >= eps max|KL|); R = sum_Q theta_Q B^Q still uses the full
 *   B, and R^S = R - R^L.  KL device, same shape and dtype as B, unchanged
 *   while the handle is used.  gf2_split is the case KL = B.  Sampling with
 *   such a split supports +-1, stratified and importance vectors; the
 *   proposal features (gf2_proposal_features) need a split of B itself. */
gf2_status gf2_screen_ijA(gf2_ctx* ctx, int64_t n, int64_t naux, const void* ijA,
                          gf2_dtype dtype, double eps_prime, void* out, int64_t* nnz);
gf2_status gf2_split_large(gf2_ctx* ctx, const void* B, const void* KL, gf2_dtype dtype,
                           int64_t n, int64_t naux, double eps, gf2_split_h** out,
                           int64_t* nnzL, int64_t* wmax);
void gf2_split_free(gf2_split_h* h);
/* Copy the split description to host arrays: support widths w[naux],
 * supports idx[naux][32] (unused slots -1) and blocks blk[naux][32][32]
 * (FP64, zero padded).  Any pointer may be NULL. */
gf2_status gf2_split_export(gf2_ctx* ctx, const gf2_split_h* h, int32_t* w,
                            int32_t* idx, double* blk, double* kmax);

/* ------------------------------------------------------------ tau grid ----
 * Gauss-Legendre nodes and weights mapped to [0, beta] (host arrays [ntau],
 * ascending).  The paper leaves the tau grid open; this is the project's. */
gf2_status gf2_tau_grid(double beta, int64_t ntau, double* tau, double* w);

/* ------------------------------------------------------------ G(tau) (a5) -
 * Non-interacting finite-temperature Green's function (eq:Gij, eq:G0):
 * F C = S C eps (C^T S C = I), e~ = eps - mu, f = 1/(1+exp(beta e~)),
 *   G[t]    = G(tau_t)        = -C diag((1-f) exp(-e~ tau_t)) C^T
 *   Gbar[t] = G(beta - tau_t) = -C diag(f exp(e~ tau_t)) C^T
 * F, S host [n][n] (S NULL = identity); tau host [ntau] in [0, beta], with the
 * end points read as one-sided limits (G(0+), G(beta-)): Gbar at tau = 0 is
 * -C diag(f) C^T = -P/2 for the density matrix P.
 * If n_occ > 0, mu is replaced by the mid-gap value (eps[n_occ-1] +
 * eps[n_occ]) / 2; the value used is returned in *mu_out (host, may be
 * NULL).  G, Gbar: device [ntau][n][n] FP64.
 * Errors: GF2_E_ARG for beta <= 0, tau outside [0, beta], n_occ >= n, or an
 * S that is not positive definite. */
gf2_status gf2_green_tau(gf2_ctx* ctx, int64_t n, const double* F, const double* S,
                         double mu, int64_t n_occ, double beta, int64_t ntau,
                         const double* tau, double* G, double* Gbar, double* mu_out);

/* ------------------------------------------------------------ Sigma (a3-a9)
 * eq:sigma_2 with N_s independent pairs (theta from stream 0, theta' from
 * stream 1):
 *   Sigma(tau) = Sigma[D,D] + (1/N_s) sum_s (Sigma_s + Sigma_s^T)/2,
 *   Sigma_s    = Sigma[D,S_eta_s] + Sigma[S_xi_s,D] + Sigma[S_xi_s,S_eta_s],
 * D = sum_Q K^L_Q (x) K^L_Q and S_xi = R^L(x)R^S + R^S(x)R^L + R^S(x)R^S.
 * Inputs: split handle of B; B device [naux][n][n] (dtype as given to
 * gf2_split); G, Gbar device [ntau][n][n] FP64 (from gf2_green_tau).
 * Outputs (device, FP64): Sigma [ntau][n][n]; e_samples [ns][ntau] with
 * e_s(tau) = Tr(Sigma_s(tau) Gbar(tau)) (the per-pair energy integrand);
 * e_samples may be NULL.
 * Errors: GF2_E_ARG (ns < 1, bad mode, k < 1, proposal not positive),
 * GF2_E_STATE (split handle of another B or context), GF2_E_NUMERIC. */
gf2_status gf2_sigma_tau(gf2_ctx* ctx, const gf2_split_h* split, const void* B,
                         const double* G, const double* Gbar, int64_t ntau,
                         const gf2_sampling* sampling, gf2_precision prec,
                         double* Sigma, double* e_samples);

/* The two halves of gf2_sigma_tau, for adaptive or batched sampling:
 * gf2_sigma_det writes Sigma[D,D] (device [ntau][n][n] FP64); G and Gbar
 * must be symmetric (as gf2_green_tau returns them for a real symmetric
 * Fock matrix): Sigma[D,D] is then symmetric, and supports of at most 8
 * orbitals form its upper triangle and mirror it;
 * gf2_sigma_stoch ADDS sum_s Sigma_s (unsymmetrised, FP64) into Sigma_sum
 * (device [ntau][n][n]; zero it before the first batch) and writes
 * e_samples [ns][ntau] for pairs s0 .. s0+ns-1; gf2_sigma_finalize writes
 * Sigma = Sigma_det + (Sigma_sum + Sigma_sum^T) / (2 ns_total). */
gf2_status gf2_sigma_det(gf2_ctx* ctx, const gf2_split_h* split, const double* G,
                         const double* Gbar, int64_t ntau, double* Sigma_det);
gf2_status gf2_sigma_stoch(gf2_ctx* ctx, const gf2_split_h* split, const void* B,
                           const double* G, const double* Gbar, int64_t ntau,
                           const gf2_sampling* sampling, gf2_precision prec,
                           double* Sigma_sum, double* e_samples);
gf2_status gf2_sigma_finalize(gf2_ctx* ctx, int64_t n, int64_t ntau,
                              const double* Sigma_det, const double* Sigma_sum,
                              int64_t ns_total, double* Sigma);

/* ------------------------------------------------------------ estimator variants
 * Two other readings of the averages <>_theta <>_theta' of eq:sigma_2, with
 * the inputs, outputs and errors of gf2_sigma_stoch (Sigma_sum is ADDED to,
 * unsymmetrised; finish with gf2_sigma_finalize and gf2_sigma_det):
 *
 * gf2_sigma_stoch_cv: the control-variate form.  E[R (x) R] = v and
 *   E[R^L (x) R^L] = D give, per pair, Sigma_s = chain(R_xi, R_eta) -
 *   chain(R^L_xi, R^L_eta) with chain(a, b) = 2 Tr(T) M - T M, M = a G b,
 *   T = M Gbar (eq:sigma with one bilinear vertex each): 8 N x N products
 *   per (tau, pair) instead of 24; unbiased, but the D (x) S cross terms are
 *   sampled.  The difference cancels: use FP32 or FP64 (BF16 rounding of the
 *   two chains is not small next to their difference).  e_samples
 *   [ns][ntau].
 *
 * gf2_sigma_stoch_double: the double average over every combination of a
 *   first-set vector i and a second-set vector j (i, j < ns <= 256): ns^2
 *   pair estimates from 2 ns vectors, each as in gf2_sigma_stoch, added into
 *   Sigma_sum; e_samples [ns * ns][ntau], row i ns + j.  Finish with
 *   gf2_sigma_finalize(..., ns_total = ns * ns, ...) and gf2_energy_double.
 *
 * gf2_energy_double: E_tot as gf2_energy (w host [ntau]; Sigma, Gbar,
 *   e_samples device), and the standard error of the double average to
 *   first order (Hoeffding): sqrt(Var_i(r_i)/ns + Var_j(c_j)/ns), r_i and
 *   c_j the row and column means of the per-combination energies.
 *   GF2_E_ARG unless 2 <= ns <= 256 and ntau <= 512; GF2_E_NUMERIC. */
gf2_status gf2_sigma_stoch_cv(gf2_ctx* ctx, const gf2_split_h* split, const void* B,
                              const double* G, const double* Gbar, int64_t ntau,
                              const gf2_sampling* sampling, gf2_precision prec,
                              double* Sigma_sum, double* e_samples);
gf2_status gf2_sigma_stoch_double(gf2_ctx* ctx, const gf2_split_h* split, const void* B,
                                  const double* G, const double* Gbar, int64_t ntau,
                                  const gf2_sampling* sampling, gf2_precision prec,
                                  double* Sigma_sum, double* e_samples);
gf2_status gf2_energy_double(gf2_ctx* ctx, int64_t n, int64_t ntau, const double* w,
                             const double* Sigma, const double* Gbar,
                             const double* e_samples, int64_t ns, double n_elec,
                             double* E_tot, double* E_per_e, double* stderr_tot);

/* ------------------------------------------------------------ energy (a10)
 * E_tot = -(1/2) sum_t w_t Tr(Sigma(tau_t) Gbar(tau_t)) in FP64 (eq:corr;
 * the -1/2 makes the beta -> infinity limit the closed-shell MP2 energy).
 * Per-pair energies E_s = E_tot - (1/2) sum_t w_t (e_s(tau_t) - mean_s e);
 * stderr = std(E_s, ddof=1)/sqrt(ns).  w host [ntau]; Sigma, Gbar device
 * [ntau][n][n]; e_samples device [ns][ntau] or NULL (then *stderr_tot = 0).
 * Outputs (host): *E_tot, *E_per_e = E_tot / n_elec, *stderr_tot.
 * Errors: GF2_E_ARG (n_elec <= 0, ns < 2 with e_samples), GF2_E_NUMERIC. */
gf2_status gf2_energy(gf2_ctx* ctx, int64_t n, int64_t ntau, const double* w,
                      const double* Sigma, const double* Gbar,
                      const double* e_samples, int64_t ns, double n_elec,
                      double* E_tot, double* E_per_e, double* stderr_tot);

/* gf2_energy_noalloc: gf2_energy for callers that cannot allocate device
 * memory -- code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same kernels and arithmetic as gf2_energy, with
 * every argument on the DEVICE: w [ntau], Sigma and Gbar [ntau][n][n],
 * e_samples [ns][ntau] or NULL, out [3] = {E_tot, E_tot / n_elec, stderr}.
 * It allocates nothing and does not synchronise: it only enqueues kernels on
 * the context's stream.  Its scratch (per-tau traces and result slots) is a
 * fixed library array of 520 doubles per GPU, resolved by gf2_create and
 * held until the process ends, so ntau is limited to 512.  Every call on a
 * GPU shares that array: calls that overlap on one GPU (other streams, other
 * threads, other contexts) race and must be ordered by the caller.
 * Errors: GF2_E_ARG (ntau > 512, n_elec <= 0, ns < 2 with e_samples, null
 * pointers).  Non-finite results are written through, not reported (a check
 * would need a host synchronisation). */
gf2_status gf2_energy_noalloc(gf2_ctx* ctx, int64_t n, int64_t ntau, const double* w,
                              const double* Sigma, const double* Gbar,
                              const double* e_samples, int64_t ns, double n_elec,
                              double* out);

/* ------------------------------------------------------------ SCF (f1)
 * The steps on either side of the self-energy that make GF2 self-consistent
 * (Section III).  Common arguments: F and S host [n][n] (S NULL = the
 * identity; S must be positive definite), beta > 0, tau and w host [ntau]
 * (the quadrature of the self-energy's tau grid, tau in [0, beta]), Sigma
 * device [ntau][n][n] FP64 (e.g. from gf2_sigma_finalize), nw >= 1 odd
 * Matsubara frequencies w_k = (2k + 1) pi / beta, k < nw.
 *
 * Numerics (the paper leaves them open; these are the readings):
 *   Sigma(i w_k) = sum_t w_t e^{i w_k tau_t} Sigma(tau_t)      (eq:GFT)
 *   G(i w_k) = [(mu + i w_k) S - F - Sigma(i w_k)]^{-1}       (eq:dyson, eq:G0)
 *   G(tau) = G0(tau) + (2/beta) sum_{k<nw} Re[e^{-i w_k tau} (G - G0)(i w_k)]
 *                                                             (eq:Ginverse)
 * with G0 the non-interacting function of the same (F, S, mu), whose tau
 * form is closed.  The work runs in the orthonormal eigenbasis of (F, S)
 * (there G0(i w) is diagonal), frequency chunk by chunk: the quadrature and
 * the back-transform as FP64 kernels, the per-frequency inversion as
 * blocked complex Gauss-Jordan on FP64 MFMAs without pivoting (the Dyson
 * matrix is complex symmetric with a positive definite imaginary part for a
 * causal self-energy).  A vanishing or non-finite pivot: GF2_E_NUMERIC.
 *
 * gf2_dyson: G(tau_t), Gbar = G(beta - tau_t) (device [ntau][n][n]) and
 *   G(beta-) (device [n][n]) at the given mu; any output may be NULL (not
 *   all).  Symmetrised ((X + X^T) / 2) like gf2_green_tau.  Synchronous.
 * gf2_electron_count: *n_e = N_e(mu) = -2 sum_ij G_ij(beta-) S_ij (host).
 * gf2_tune_mu: the mu in [mu_lo, mu_hi] with N_e(mu) = n_elec at fixed
 *   Sigma (N_e grows with mu): Newton steps from the middle of the bracket,
 *   with dN_e/dmu from the same inverses (dG/dmu = -G^2), bisection where a
 *   step leaves the narrowed bracket, to |N_e - n_elec| <= 1e-11
 *   max(1, n_elec) or a bracket of 1e-15 relative.  *mu_out, and *n_e (may
 *   be NULL) the count reached.  GF2_E_ARG if the bracket does not contain
 *   the root.
 * gf2_fock: eq:F with the RI factors of eq:vKQKQ, F = h + J[P] - K[P]/2,
 *   J_ij = sum_Q B^Q_ij Tr(B^Q P), K = sum_Q B^Q P B^Q, P = -2 G(beta-).
 *   B device [naux][n][n] (dtype), h host [n][n], Gbeta device [n][n];
 *   F_out host [n][n].  FP64 throughout.
 * gf2_scf_step: one update of the loop around the self-energy: mu tuned
 *   to n_elec (gf2_tune_mu), G, Gbar, G(beta-) at that mu (gf2_dyson), and
 *   the new Fock matrix (gf2_fock).  Outputs as above; *mu_out host. */
/* gf2_qp_energies: quasiparticle energies in the diagonal approximation
 *   (the Conclusions' excited-state direction; the method is this library's
 *   reading).  For every orbital k of (F, S): the orbital self-energy
 *   s_k(i w_f) = c_k^T Sigma(i w_f) c_k on the first n_pade Matsubara
 *   frequencies (the quadrature above), its n_pade-point Pade continuation
 *   (Thiele continued fraction, Vidberg-Serene recursion), and the fixed
 *   point of E = eps_k + Re s_k(E - mu + i eta) from E = eps_k, stopped at
 *   |dE| <= 1e-13 or after max_iter steps.  E host [n] (ascending eps
 *   order); converged host [n] (1 where the tolerance was met) or NULL.
 *   Errors: GF2_E_ARG (n_pade outside [1, 4096], max_iter < 1),
 *   GF2_E_NUMERIC (a non-finite energy). */
gf2_status gf2_qp_energies(gf2_ctx* ctx, int64_t n, const double* F, const double* S,
                           double mu, double beta, int64_t ntau, const double* tau,
                           const double* w, const double* Sigma, int32_t n_pade, double eta,
                           int32_t max_iter, double* E, int32_t* converged);
gf2_status gf2_dyson(gf2_ctx* ctx, int64_t n, const double* F, const double* S, double mu,
                     double beta, int64_t ntau, const double* tau, const double* w,
                     const double* Sigma, int64_t nw, double* G, double* Gbar,
                     double* Gbeta);
gf2_status gf2_electron_count(gf2_ctx* ctx, int64_t n, const double* F, const double* S,
                              double mu, double beta, int64_t ntau, const double* tau,
                              const double* w, const double* Sigma, int64_t nw,
                              double* n_e);
gf2_status gf2_tune_mu(gf2_ctx* ctx, int64_t n, const double* F, const double* S,
                       double beta, int64_t ntau, const double* tau, const double* w,
                       const double* Sigma, int64_t nw, double n_elec, double mu_lo,
                       double mu_hi, double* mu_out, double* n_e);
gf2_status gf2_fock(gf2_ctx* ctx, int64_t n, int64_t naux, const void* B, gf2_dtype dtype,
                    const double* h, const double* Gbeta, double* F_out);
gf2_status gf2_scf_step(gf2_ctx* ctx, int64_t n, int64_t naux, const void* B,
                        gf2_dtype dtype, const double* h, const double* F, const double* S,
                        double beta, int64_t ntau, const double* tau, const double* w,
                        const double* Sigma, int64_t nw, double n_elec, double mu_lo,
                        double mu_hi, double* mu_out, double* G, double* Gbar,
                        double* Gbeta, double* F_out);

/* ------------------------------------------------------------ RNG ---------
 * word(seed, stream, s, q) = mix(seed * 0x9E3779B97F4A7C15
 *                                + ((stream << 62) | (s << 32) | q) + 1),
 * mix = SplitMix64 finaliser (Steele, Lea, Flood 2014).  Fills out[count]
 * (host) with the words for q = q0 .. q0+count-1, computed on the device. */
gf2_status gf2_rng_words(gf2_ctx* ctx, uint64_t seed, uint32_t stream, uint32_t s,
                         uint32_t q0, int64_t count, uint64_t* out);

/* ------------------------------------------------------------ profiling ---
 * Optional timing of the library's launches with HIP events on the
 * context's stream (off by default).  gf2_profile_read synchronises the
 * stream, then reports up to `cap` kernel classes: names (host array of
 * `cap` char[32]), launch counts, summed durations (ms), and the algorithmic
 * flops and bytes the launches were charged with; *count receives the
 * number of classes.  It clears the record.  */
gf2_status gf2_set_profiling(gf2_ctx* ctx, int on);
gf2_status gf2_profile_read(gf2_ctx* ctx, int32_t cap, char* names, int64_t* launches,
                            double* total_ms, double* flops, double* bytes, int32_t* count);

/* ------------------------------------------------------------ GEMM tiles --
 * Tile choice of the BF16 chain products where a 160-wide tile pads an
 * N x N product less than the 128 x 128 tile (N = 400, 800, ...):
 * mode 2 (default): the deep-K stage (exchange and cross terms) on 160 x 160
 *   tiles of 16x16x32 MFMAs with 64-wide k tiles, and the dual-A product
 *   launches (U and V^T, W and Z^T, T) on 320 x 160 tiles (two 160 x 160
 *   products sharing the B tile) with 32-wide k tiles, both fed by direct
 *   global -> LDS loads;
 * mode 1: only the deep-K stage on the 160 tile (and gf2_debug_gemm);
 * mode 0: the 128 x 128 tile everywhere.
 * All modes give the same results up to the FP32 rounding of the
 * accumulation order.  Setting a mode discards the tile modes the batch
 * autotuner chose (below), so the setting applies to every size again.
 * GF2_E_ARG for other modes. */
gf2_status gf2_set_gemm_tiles(gf2_ctx* ctx, int32_t mode);

/* Tile mode (0, 1 or 2, as gf2_set_gemm_tiles) that GF2_BATCH_AUTOTUNE chose
 * for chains of size n at precision prec (FP64, FP32, BF16 or BF16X3), or
 * -1 in *mode if it chose none (it tunes BF16 sizes where the 160-wide tile
 * pads less than 128, i.e. where the mode changes the launch).  A chosen
 * mode applies to every later call of the context on chains of that size,
 * single-chain calls included.  GF2_E_ARG for a null mode, n <= 0 or an
 * adaptive-only precision. */
gf2_status gf2_tuned_tiles(gf2_ctx* ctx, gf2_precision prec, int64_t n, int32_t* mode);

/* ------------------------------------------------------------ batch -------
 * Many chains of uneven size in one schedule: every instance's (tau, pair)
 * units go through the same grouped product launches (each unit carries its
 * instance; tiles beyond an instance's size are skipped), so small instances
 * fill the GPU together.  Per instance the result equals gf2_sigma_tau:
 *   Sigma = Sigma[D,D] + (1/N_s) sum_s (Sigma_s + Sigma_s^T)/2  (eq:sigma_2)
 * and e_samples [ns][ntau] (may be NULL).
 * flags: GF2_BATCH_GRAPH records the chunk loop of the call into one HIP
 * graph and launches it; GF2_BATCH_AUTOTUNE first picks the tile mode of
 * every chain size where it matters (each mode timed on one chain of that
 * size; the fastest kept per (precision, N) in ctx, see gf2_tuned_tiles),
 * then times candidate launch shapes (pairs x tau points per chunk,
 * persistent grid or not) on the first chunks of the whole batch and keeps
 * the fastest for this batch signature (cached in ctx).
 * The library allocates per-instance workspace (freed by gf2_destroy).
 * Errors: as gf2_sigma_tau for any item; GF2_E_ARG for nitem < 1. */
typedef struct {
  const gf2_split_h* split;
  const void* B;
  const double* G;          /* device [ntau][n][n]                              */
  const double* Gbar;       /* device [ntau][n][n]                              */
  int64_t ntau;
  gf2_sampling sampling;    /* ns pairs from s0, seed, mode, k, p               */
  double* Sigma;            /* out, device [ntau][n][n]                         */
  double* e_samples;        /* out, device [ns][ntau] or NULL                   */
} gf2_batch_item;

#define GF2_BATCH_GRAPH 1
#define GF2_BATCH_AUTOTUNE 2

gf2_status gf2_sigma_batch(gf2_ctx* ctx, int32_t nitem, const gf2_batch_item* items,
                           gf2_precision prec, int32_t flags);

/* ------------------------------------------------------------ adaptive ---
 * Sampling until a target standard error (the accuracy criterion of the
 * results section: statistical error of the total E_corr of eq:corr).
 * Pairs are drawn in batches of sampling->ns (sampling->s0 is ignored; pair
 * indices run 0, 1, ...) until the standard error of the total E_corr is
 * below `target` (Eh) with 95% confidence, or `max_pairs` is reached; at
 * least two pairs.  The stopping test uses the one-sided 95% upper bound of
 * the standard error estimated from the pairs so far (chi-square with
 * pairs - 1 degrees of freedom; 1.80x the estimate at 8 pairs, 1.26x at 32),
 * so a small first batch cannot stop on a lucky low estimate.
 *
 * prec GF2_PREC_AUTO: the two-level estimator.  Pairs 0 .. k-1 (the
 * probe, first k = min(2, max_pairs)) run in BF16 and in BF16X3, the rest
 * in BF16 (the first batch filled up to sampling->ns pairs); at the end
 * Sigma and the per-pair traces are moved by the mean BF16X3 - BF16
 * difference d of the k probe pairs (scaled to all pairs), which removes
 * the BF16 rounding bias in expectation.  The correction is accepted when
 * twice the standard error of that mean, std(d_E)/sqrt(k), is below 0.1 x
 * the standard error reached and, for every tau, twice the standard error
 * of the mean trace difference is below the larger of 0.1 x the standard
 * error of that tau's mean trace and 1e-5 x the trace Tr(Sigma(tau)
 * Gbar(tau)).  If it is not, the probe grows to min(8, pairs) pairs (their
 * BF16X3 runs added); if it still is not, every pair is taken in BF16X3
 * (same theta: the probe pairs from the probe, the others recomputed) and
 * sampling continues in BF16X3.  When the first probe already puts twice
 * std(d_E) above 3 x 0.1 x the spread std(E) of its own BF16X3 pair
 * energies (the two standard errors fall together while the probe holds
 * every pair, so a larger probe would not help), sampling goes on in BF16X3
 * from there without the BF16 batch.  res->precision reports BF16C or
 * BF16X3; res->bias_probe the |mean d_E| removed.  batch must be >= 2.
 *
 * Inputs as gf2_sigma_stoch; w host [ntau] quadrature weights; Sigma_det
 * device [ntau][n][n] (gf2_sigma_det).  Outputs: Sigma device [ntau][n][n]
 * FP64 (= Sigma_det + symmetrised mean); e_samples device [max_pairs][ntau]
 * (rows 0 .. pairs-1 written); *res host.  The library keeps the running
 * sum in its own workspace.
 * Errors: as gf2_sigma_stoch; GF2_E_ARG for target <= 0, max_pairs < 2,
 * ntau > 512. */
typedef struct {
  double e_corr;          /* total E_corr (Eh)                               */
  double e_corr_per_e;    /* E_corr / n_elec                                 */
  double stderr_tot;      /* standard error of the total E_corr              */
  int64_t pairs;          /* pairs used                                      */
  int32_t precision;      /* gf2_precision the final pairs were computed in  */
  double bias_probe;      /* AUTO: b above (0 otherwise)                     */
} gf2_adaptive_result;

gf2_status gf2_energy_adaptive(gf2_ctx* ctx, const gf2_split_h* split, const void* B,
                               const double* G, const double* Gbar, int64_t ntau,
                               const double* w, const double* Sigma_det, double n_elec,
                               const gf2_sampling* sampling, gf2_precision prec, double target,
                               int64_t max_pairs, double* Sigma, double* e_samples,
                               gf2_adaptive_result* res);

/* gf2_energy_adaptive with the deterministic block computed inside:
 * Sigma_det (device [ntau][n][n] FP64, output) is formed as by gf2_sigma_det
 * on a second stream of the context while the first batch of pairs runs,
 * and the energy statistics wait for it.  Results are those of
 * gf2_sigma_det followed by gf2_energy_adaptive.  The call returns after
 * both streams have finished.  Errors: as gf2_energy_adaptive. */
gf2_status gf2_energy_adaptive_det(gf2_ctx* ctx, const gf2_split_h* split, const void* B,
                                   const double* G, const double* Gbar, int64_t ntau,
                                   const double* w, double n_elec, const gf2_sampling* sampling,
                                   gf2_precision prec, double target, int64_t max_pairs,
                                   double* Sigma_det, double* Sigma, double* e_samples,
                                   gf2_adaptive_result* res);

/* ------------------------------------------------------------ test hook ---
 * The chain's GEMM kernel on its own: C[b] = A[b] B[b]^T for b < batch,
 * square n x n operands (row-major, leading dimension ld = n rounded up to a
 * multiple of 32, zero padded, device).  prec FP64: double operands and
 * output; FP32: float; BF16: bf16 operands, float output; BF16X3: each
 * operand is two bf16 planes (hi, lo) of ld*ld elements each.  For tests and
 * benchmarks of the kernel itself. */
gf2_status gf2_debug_gemm(gf2_ctx* ctx, gf2_precision prec, int64_t n, int64_t batch,
                          const void* A, const void* Bt, void* C);

#ifdef __cplusplus
}
#endif
#endif /* GF2_H */
