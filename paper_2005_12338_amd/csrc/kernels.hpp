// Launchers of the libgf2 kernels (host-callable, defined in the .hip files).
#pragma once

#include <algorithm>

#include "gf2_internal.hpp"

void launch_rng_words(uint64_t seed, uint32_t stream, uint32_t s, uint32_t q0, int64_t count,
                      uint64_t* out, hipStream_t st);
void launch_theta(uint64_t seed, int64_t ns, int64_t s0, int64_t naux, int8_t* theta, hipStream_t st);
void launch_draws(uint64_t seed, int64_t ns, int64_t s0, int32_t k, const double* cdf, int64_t naux,
                  const double* p, int32_t* q, double* w, hipStream_t st);
void launch_synth_b(int64_t n, int64_t naux, const double* x, const double* xq, double amp, double a,
                    double c, void* out, bool f64, hipStream_t st);
void launch_maxabs(const void* b, bool f64, int64_t total, double* part, int nblk, hipStream_t st);
void launch_rowflags(const void* b, bool f64, int64_t n, int64_t naux, double thr, uint8_t* flags,
                     unsigned long long* nnz, hipStream_t st);
void launch_extract_blocks(const void* b, bool f64, int64_t n, int64_t naux, double thr,
                           const int32_t* w, const int32_t* idx, double* blk, float* blk32,
                           hipStream_t st);
void launch_rbuild(const void* b, bool f64, int64_t n, int64_t naux, double thr, const int8_t* theta,
                   int64_t nvec, Prec prec, void* xl, void* xs, int64_t np, int64_t plane,
                   int64_t mstride, hipStream_t st, const double* vscale = nullptr, const void* lsrc = nullptr);
void launch_theta_strat(uint64_t seed, int64_t ns, int64_t s0, int64_t naux, int32_t nclass, const double* cdf,
                        const double* pi, int8_t* theta, double* vscale, hipStream_t st);
void launch_rimportance(const void* b, bool f64, int64_t n, double thr, const int32_t* q,
                        const double* w, int32_t k, int64_t nvec, Prec prec, void* xl, void* xs,
                        int64_t np, int64_t plane, int64_t mstride, hipStream_t st, const void* lsrc = nullptr);
void launch_scale_cols(const double* c, const double* lw, int64_t n, int64_t np, int64_t ntau,
                       double* out, hipStream_t st);
void launch_unpad_sym(const double* p, int64_t n, int64_t np, int64_t ntau, double sign, double* out,
                      hipStream_t st);
void launch_pad_convert(const double* g, int64_t n, int64_t np, int64_t ntau, Prec prec, void* stbuf,
                        int64_t plane, int64_t mstride, double* f64pad, hipStream_t st);
void launch_jk_blocks(bool f64, const void* wbase, int64_t w_st_slot, int64_t w_st_m, int64_t np,
                      int64_t naux, int32_t nslot, int32_t wmax, const int32_t* wq, const int32_t* idx,
                      const void* blk, void* jout, hipStream_t st);
// bytes of the J blocks of nslot slots (block pitch from the widest block)
size_t jk_block_bytes(bool f64, int64_t nslot, int64_t naux, int32_t wmax);
void launch_jk_scatter(bool f64, const void* jblk, int64_t naux, int32_t nslot, int32_t wmax, int64_t npat,
                       const int32_t* pat_ij, const int32_t* pat_off, const int32_t* pat_q, int64_t np,
                       Prec prec, int64_t plane, void* jw_l, void* jw_s, void* jz_st, void* jz_sum_t,
                       int64_t out_st_slot, hipStream_t st);
// mode 0: the L/S-resolved direct-term coefficients; 1: the control-variate form's.
void launch_trace_coef(const double* part, int64_t ntiles, int32_t nslot, double* coef, int mode,
                       hipStream_t st);
// E and the U-statistic standard error of the double average (ns <= 256).
void launch_double_stats(const double* tr, const double* w, int64_t ntau, const double* es, int64_t ns, double gm,
                         double* out, hipStream_t st);
// xt = xl + xs for count storage elements (matrices of mstride elements).
void launch_vec_sum(const void* xl, const void* xs, void* xt, int64_t count, Prec prec, int64_t plane,
                    int64_t mstride, hipStream_t st);
// Per-slot direct-term record written by launch_trace_coef: coef[0..3] for
// M_LL, M_LS, M_SL, M_SS, then Tr(T_h) for h = 0..3.
constexpr int kCoefStride = 8;
void launch_accumulate(const Unit* units, int32_t nunit, const void* sig, bool f64, int64_t sig_st_slot,
                       int64_t n, int64_t np, double* sum, int32_t tau_lo, int32_t tau_hi, const void* mst,
                       Prec prec, int64_t m_st_slot, int64_t m_st_m, int64_t plane, const double* coef,
                       hipStream_t st);
void launch_esamples(const Unit* units, int32_t nunit, const double* part, int64_t ntiles, int64_t s0,
                     int64_t ntau, double* es, const double* coef, hipStream_t st);
void launch_finalize(const double* det, const double* sum, int64_t n, int64_t ntau, double inv2ns,
                     double* out, hipStream_t st);
// Two-level (BF16 / BF16X3) correction: sum += lo + c (hi - lo); and the
// per-tau mean of hi - es over the first k sample rows added to all ns rows.
void launch_level_correct(double* sum, const double* hi, const double* lo, int64_t count, double c,
                          hipStream_t st);
void launch_level_shift(double* es, const double* hi, int64_t k, int64_t ns, int64_t ntau, hipStream_t st);
void launch_trace_prod(const double* sig, const double* gb, int64_t n, int64_t ntau, double* tr,
                       hipStream_t st);
void launch_energy_stats(const double* tr, const double* w, int64_t ntau, const double* es, int64_t ns,
                         double gm, double* out, hipStream_t st, bool add_mean = false);
void launch_transpose(const void* src, bool f64, int64_t rows, int64_t cols, double* dst, int64_t ld,
                      hipStream_t st);
void launch_untranspose(const double* src, int64_t rows, int64_t cols, int64_t ld, void* dst, bool f64,
                        hipStream_t st);
void launch_count_nonfinite(const double* x, int64_t count, unsigned long long* bad, hipStream_t st);
int dblock_tile();
void launch_dblock(const double* G, const double* Gb, int64_t n, int64_t ntau, int32_t wmax,
                   const int32_t* wq, const int32_t* idx, const double* blk, const int32_t* tq_off,
                   const int32_t* tq, double* out, hipStream_t st);

int64_t dd_strip_bytes(int64_t n, int64_t naux, int32_t wmax, int64_t ntau_batch);
// Register form of the deterministic block for supports of at most 8
// orbitals (returns false, launching nothing, for wider supports).
bool launch_dd_strips(const double* G, const double* Gb, int64_t n, int64_t naux, int64_t ntau, int32_t wmax,
                      int32_t span128,
                      const int32_t* wq, const int32_t* idx, const double* blk, const int32_t* idx_t,
                      const double* blk_t, const int32_t* col_off,
                      const int32_t* col_q, const int32_t* col_cs, int32_t ncs, double* strip,
                      int64_t ntau_batch, double* out, hipStream_t st);
// By-column tables of the supports and blocks for the register form:
// idx_t [kDdW][naux], blk_t [kDdW * kDdW][naux].
void launch_dd_tables(const int32_t* idx, const double* blk, int64_t naux, int32_t* idx_t, double* blk_t,
                      hipStream_t st);

// eq:V_ijA screening (front.hip); mbits [n] and kept must be zeroed.
void launch_screen_ija(const void* x, bool f64, int64_t n, int64_t naux, double eps_over_n,
                       unsigned long long* mbits, void* out, unsigned long long* kept, hipStream_t st);

// Self-consistent GF2 steps (scf.hip).  Frequencies per chunk are padded to
// a multiple of scf_freq_group(), output times to scf_time_group().
int scf_freq_group();
int scf_time_group();
int scf_panel();
void launch_sig_iw(const double* sig, int64_t ntau, int64_t np, int64_t n, const double* ph, int32_t nc, int32_t ncp,
                   const double* shift, const double* om, double* a, hipStream_t st);
void launch_gj_invert(double* a, int32_t nmat, int64_t np, double* colbuf, double* pbuf, int* err, hipStream_t st);
void launch_iw_back(const double* a, int32_t nc, int64_t np, int64_t n, const double* shift, const double* om,
                    const double* cs, int32_t nto, int32_t ntop, double* pc, double* ps, hipStream_t st);
void launch_iw_diag(const double* a, int32_t nc, int64_t np, int64_t n, const double* shift, const double* om,
                    double* tr, hipStream_t st);
void launch_g_mo(const double* pc, const double* ps, int64_t np, int64_t n, int64_t ntau, const double* tau,
                 const double* emu, double beta, double* out, hipStream_t st);
void launch_pad_bq(const void* b, bool f64, int64_t n, int64_t naux, int64_t np, int64_t q0, int64_t qc, double* out,
                   hipStream_t st);
void launch_bq_dot(const void* b, bool f64, int64_t n, int64_t naux, const double* p, double* c, hipStream_t st);
void launch_fock_final(const void* b, bool f64, int64_t n, int64_t naux, const double* c, const double* h,
                       const double* kp, int64_t ng, int64_t np, double* f, hipStream_t st);
void launch_density(const double* gbeta, int64_t nn, double* p, hipStream_t st);
// Quasiparticle energies: work holds 2 m complex (32 bytes) per orbital.
void launch_qp(const double* sig, int64_t ntau, int64_t np, int64_t n, const double* ph, int32_t m, int32_t ncp,
               const double* om, const double* eps, double mu, double eta, int32_t iters, void* work, double* e_out,
               int32_t* conv, hipStream_t st);

struct gf2_mlp;
int mlp_nparam();
void launch_features(const void* b, bool f64, int64_t n, int64_t naux, double thr, const double* x,
                     const double* xq, const double* gbeta, double* phi, hipStream_t st);
void launch_pair_tables(int wmax, const double* G, const double* Gb, int64_t n, int64_t ntau, const double* w,
                        int64_t naux, const int32_t* wb, const int32_t* ib, const double* bb, const int32_t* wk,
                        const int32_t* ik, const double* kb, double* tab, hipStream_t st);
void launch_targets(const double* tab, int64_t naux, double* t, hipStream_t st);

#include "host_numerics.hpp"
