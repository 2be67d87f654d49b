/*
 * ht_rise_testing.h - kernel-level entry points of the batch hierarchical Tucker
 * library, for verification against independent references.  Each wraps one
 * device step of the path on caller-owned device buffers; none allocates.
 *
 * Unfolding views: a C-order tensor viewed as (P, m, S), element (p, a, s) at
 * (p * m + a) * S + s; its mode unfolding is the m x (P*S) matrix with column
 * (p, s) (Sec. 2.1 "matricization").  dtype arguments are ht_dtype values.
 * All matrices are float64; U matrices are column-major (m x R).  Calls are
 * enqueued on hip_stream and return without synchronising.  Invalid sizes or
 * NULL pointers return HT_EINVAL before anything is enqueued.
 */
#ifndef HT_RISE_TESTING_H
#define HT_RISE_TESTING_H

#include "ht_rise.h"

#ifdef __cplusplus
extern "C" {
#endif

/* sum of squares of n elements into out[0] (float64); scratch >= 1024 doubles */
ht_status ht_test_sumsq(const void* x, int32_t dtype, int64_t n, double* out, double* scratch, void* hip_stream);

/* Gram of the mode unfolding: G (m x m row-major) = X_(k) X_(k)^T (the matrix
 * whose eigen-decomposition gives the SVD of Eq. ht_leaf_svd).  scratch must hold
 * ht_test_gram_scratch_doubles(P, m, S) doubles. */
size_t ht_test_gram_scratch_doubles(int64_t P, int64_t m, int64_t S);
ht_status ht_test_gram(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, double* G, double* scratch,
                       void* hip_stream);

/* Gram of the explicit residual R = X_(k) - U (U^T X_(k)) (Eq. compute_residual) for
 * m <= 128 and 1 <= R <= 64, U column-major (m x R); the scratch of ht_test_gram. */
ht_status ht_test_resid_gram(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U, int32_t R,
                             double* G, double* scratch, void* hip_stream);

/* Mode contraction with U^T (Eq. multi_index_contraction): Z[p, r, s] = sum_a U[a, r] X[p, a, s], 1 <= R <= 64. */
ht_status ht_test_ttm_contract(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                               int32_t R, double* Z, void* hip_stream);

/* The contraction above for modes of more than 128 rows (Z FP64), with the energies
 * sq[0] = ||X||^2 and sq[1] = ||Z||^2, and with scratch_doubles of device scratch lent
 * to it: a contraction of fewer than 256 column blocks of 16 is then split into row
 * chunks whose partial products are summed in chunk order.  sq holds 2 + 2048
 * doubles (the sums, then the workgroup partials).  HT_EINVAL for m <= 128. */
ht_status ht_test_ttm_contract_split(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                                     int32_t R, double* Z, double* scratch, size_t scratch_doubles, double* sq,
                                     void* hip_stream);

/* Mixed form (HT_FP32): the residual Gram above with every product on FP32 matrix
 * cores and the workgroup partials summed in FP64.  Same arguments and scratch. */
ht_status ht_test_resid_gram_f32(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                                 int32_t R, double* G, double* scratch, void* hip_stream);

/* Mixed form: the residual Gram above as (I - U U^T) G (I - U U^T) from the FP64 Gram
 * G = X_(k) X_(k)^T, no residual formed (the identity R R^T = (I - U U^T) G (I - U U^T)
 * of Eq. compute_residual).  m <= 4096, 1 <= R <= 64 (else HT_EINVAL); FP32 or FP64
 * x.  Same arguments and scratch as ht_test_resid_gram. */
ht_status ht_test_resid_gram_proj(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                                  int32_t R, double* G, double* scratch, void* hip_stream);

/* Mixed form contraction: Z (float32, [P][R][S]) = U^T X on FP32 matrix cores, with
 * norm2[0] = ||X||^2 and resid2[0] = ||X - U U^T X||^2 (the explicit residual of
 * Eq. compute_residual, summed in FP64).  m <= 128, 1 <= R <= 64; scratch holds
 * 2 * ht_test_ttm_partials_doubles() doubles. */
size_t ht_test_ttm_partials_doubles(void);
ht_status ht_test_ttm_contract_f32(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                                   int32_t R, float* Z, double* norm2, double* resid2, double* scratch,
                                   void* hip_stream);

/* Mode expansion: out[p, a, s] = sum_t U[a, t] Z[p, t, s], or M[p, a, s] minus that when M
 * is not NULL (the residual of Eq. compute_residual).  1 <= R <= 64. */
ht_status ht_test_ttm_expand(const double* Z, int64_t P, int32_t R, int64_t S, const double* U, int64_t m,
                             const void* M, int32_t m_dtype, void* out, int32_t out_dtype, void* hip_stream);

/* Eigen-decomposition of the symmetric k x k G (row-major) and the truncation rule:
 * the minimal rank r in [rmin, rmax] whose discarded energy (the clipped eigenvalues
 * beyond the r leading ones) is <= thr, written to rank[0], that energy to tail[0],
 * and the r leading sign-normalised eigenvectors to vecs (k x r column-major).
 * evals receives the leading eigenvalues in descending order, as many as the rule
 * needed (at least r); the remaining entries are left untouched.  When rmin = 0 and
 * trace(G) <= thr the rule keeps nothing and the decomposition is skipped: rank 0,
 * tail = trace(G), evals and vecs untouched.
 * scratch holds ht_test_eig_scratch_doubles(k, rmax). */
size_t ht_test_eig_scratch_doubles(int32_t k, int32_t rmax);
ht_status ht_test_eig(const double* G, int32_t k, int32_t rmin, int32_t rmax, double thr, double* evals,
                      double* vecs, int32_t* rank, double* tail, double* scratch, void* hip_stream);
/* The same with the solver chosen: method 0 as ht_test_eig (a Lanczos decision where
 * it can be proven, else Householder tridiagonalisation), 1 Householder only, 2
 * Lanczos only (rank[0] = -1 when the decision could not be proven).  After the call
 * scratch[ht_test_eig_scratch_doubles(k, rmax) - 56] holds the Lanczos steps taken
 * (negative when the decision was not proven, 0 when the fast path was not tried). */
ht_status ht_test_eig_method(const double* G, int32_t k, int32_t rmin, int32_t rmax, double thr, int32_t method,
                             double* evals, double* vecs, int32_t* rank, double* tail, double* scratch,
                             void* hip_stream);

/* Basis expansion (Eq. concatenating_orthonormal_vectors): V (alpha x rR) is made
 * orthogonal to U_old (alpha x r_old) twice, orthonormalised by CholeskyQR twice,
 * sign-normalised, and [U_old, V] is written to core (alpha x (r_old + rR)). */
ht_status ht_test_orth_expand(const double* U_old, int64_t alpha, int32_t r_old, double* V, int32_t rR, double* core,
                              void* hip_stream);

/* Host-only: the mixed form's certificate of one rank decision.  The rule chose rank
 * r in [rmin, room] with discarded energy t_r and smallest kept eigenvalue lam_r on a
 * Gram whose tail sums may be off by 2 sqrt(t) dR + dR^2 + gerr; returns 1 when every
 * Gram within that error leads to the same decision (within thr on the kept side,
 * above it one rank lower; a decision cut short by the capacity, r == room with
 * t_r > thr, must stay above thr), else 0. */
int32_t ht_test_decision_certified(int32_t r, int32_t rmin, int32_t room, double t_r, double lam_r, double thr,
                                   double dR, double gerr);

#ifdef __cplusplus
}
#endif

#endif /* HT_RISE_TESTING_H */
