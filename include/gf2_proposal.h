/*
 * gf2_proposal.h -- learned importance proposal over the auxiliary index.
 *
 * Stochastic orbitals theta = (1/sqrt k) sum_j e_j u_{Q_j} / sqrt(p_{Q_j})
 * (gf2_sampling mode GF2_SAMPLE_IMPORTANCE) keep every identity the paper's
 * +-1 orbitals satisfy (E[theta theta^T] = I, Section II), so the RS-SRI
 * estimator of eq:sigma_2 stays unbiased for any p > 0.  This header builds p
 * from a small network trained on per-Q contribution magnitudes that the
 * method itself produces.  Conventions as in gf2.h.
 *
 * Network: z_Q = w2 . tanh(W1 x_Q + b1), x_Q = (phi_Q - mean) / std,
 * hidden width GF2_MLP_HIDDEN, p = (1 - alpha) softmax(z) + alpha / N_aux.
 */
#ifndef GF2_PROPOSAL_H
#define GF2_PROPOSAL_H

#include "gf2.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GF2_MLP_IN 4
#define GF2_MLP_HIDDEN 128

/* Device buffers of one network (FP32), owned by the caller:
 * w1[HIDDEN][IN], b1[HIDDEN], w2[HIDDEN], mean[IN], std[IN], and the Adam
 * moments m[P], v[P] over the P = HIDDEN*IN + 2*HIDDEN parameters in the
 * order (w1, b1, w2); step counts Adam updates taken so far (host). */
typedef struct gf2_mlp {
  float* w1;
  float* b1;
  float* w2;
  float* mean;
  float* std;
  float* adam_m;
  float* adam_v;
  int64_t step;
} gf2_mlp;

/* Per-Q features phi[naux][4] (device FP64):
 *   phi0 = tanh(d / 4), d = distance of x_Q to the nearer chain end
 *          (min(xq - x[0], x[n-1] - xq)),
 *   phi1 = ln(||B_Q||_F + 1e-30),
 *   phi2 = ln(||B_Q - K^L_Q||_F + 1e-30)  (K^L from the split),
 *   phi3 = -2 sum_ij B_Q,ij Gbeta_ij      (density P = -2 G(beta-)).
 * x host [n], xq host [naux]; Gbeta device [n][n] FP64 (G at beta-, e.g.
 * gf2_green_tau's Gbar at a tau just above 0).  Deterministic reductions. */
gf2_status gf2_proposal_features(gf2_ctx* ctx, const gf2_split_h* split, const void* B,
                                 const double* x, const double* xq, const double* Gbeta,
                                 double* phi);

/* Per-Q contribution magnitudes (training targets).  With B_Q truncated to
 * |B| >= rel * max|B| (supports of at most 32 orbitals) and K_Q = K^L_Q,
 *   P(a, b) = sum_t w_t [2 Tr(a G b Gb)^2 - Tr((a G b Gb)^2)]   (eq:sigma,
 *   energy of one bilinear piece per vertex, tau quadrature with w),
 *   d_QQ' = P(B_Q,B_Q') - P(B_Q,K_Q') - P(K_Q,B_Q') + P(K_Q,K_Q'),
 *   cL_Q = sum_R [P(K_R,B_Q) - P(K_R,K_Q)], cR_Q = sum_R [P(B_Q,K_R) - P(K_Q,K_R)],
 *   t_Q = |cL_Q| + |cR_Q| + sum_Q' |d_QQ'|.
 * G, Gbar device [ntau][n][n]; w host [ntau]; t device [naux] FP64;
 * tables (device [4][naux][naux] FP64, order BB, BK, KB, KK) may be NULL. */
gf2_status gf2_proposal_targets(gf2_ctx* ctx, const gf2_split_h* split, const void* B,
                                const double* G, const double* Gbar, int64_t ntau,
                                const double* w, double rel, double* t, double* tables);

/* Standardisation (mean, std of phi over the training set, FP64 reductions)
 * and initial weights: uniform(-1, 1)/sqrt(fan_in) from counter words
 * word(seed, 2, 0, q), q over w1 (row-major), then b1, then w2.  Clears the
 * Adam state. phi device [ntotal][4]. */
gf2_status gf2_proposal_init(gf2_ctx* ctx, gf2_mlp* mlp, const double* phi, int64_t ntotal,
                             uint64_t seed);

/* Loss sum over chains of KL(t_hat || softmax(z)) and its exact gradient
 * (backpropagation, dL/dz = softmax(z) - t_hat per chain).  chain_off host
 * [nchains+1] sample offsets; phi device [ntotal][4]; t_hat device [ntotal]
 * (each chain's targets sum to 1).  grad host [P] in the order (w1, b1, w2)
 * (may be NULL); *loss host. */
gf2_status gf2_proposal_grad(gf2_ctx* ctx, const gf2_mlp* mlp, int32_t nchains,
                             const int64_t* chain_off, const double* phi, const double* t_hat,
                             double* loss, double* grad);

/* `steps` full-batch Adam steps (lr, beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
 * bias corrected), all on the device in one launch.  loss_hist host [steps]
 * (loss before each step) may be NULL.  Deterministic. */
gf2_status gf2_proposal_train(gf2_ctx* ctx, gf2_mlp* mlp, int32_t nchains, const int64_t* chain_off,
                              const double* phi, const double* t_hat, int32_t steps, double lr,
                              double* loss_hist);

/* p[naux] (device FP64) = (1 - alpha) softmax(z) + alpha / naux with z from
 * the network; bf16 != 0 evaluates the network with BF16 weights and inputs
 * (FP32 accumulation), else in FP32.  phi device [naux][4]. */
gf2_status gf2_proposal_infer(gf2_ctx* ctx, const gf2_mlp* mlp, const double* phi, int64_t naux,
                              double alpha, int32_t bf16, double* p);

#ifdef __cplusplus
}
#endif
#endif /* GF2_PROPOSAL_H */
