// Internal interface between the host driver (ht_abi.hip) and the device
// kernels (ht_kernels.hip, ht_eig.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace ht {

// A mode-k view of a C-order level tensor [N][m_1]...[m_q]: P = N * prod_{i<k} m_i,
// m = m_k, S = prod_{i>k} m_i.  Element (p, a, s) sits at (p * m + a) * S + s.  The
// mode-k unfolding is the m x (P*S) matrix whose column c is (p, s) = divmod(c, S).
struct ModeView {
  int64_t P;
  int64_t m;
  int64_t S;
};

enum class Elem : int { F32 = 0, F64 = 1 };

// ---- reductions -------------------------------------------------------------
// Sum of squares of n elements into *out (FP64), deterministic two-level reduction.
// partials must hold kSumsqBlocks doubles.
constexpr int kSumsqBlocks = 1024;
void sumsq(const void* x, Elem t, int64_t n, double* partials, double* out, hipStream_t s);
// Sum of squares of each of nseg consecutive segments of len elements into out[g];
// partials must hold nseg * kSegBlocks doubles.  nseg < 65536.
constexpr int kSegBlocks = 64;
void sumsq_segments(const void* x, Elem t, int64_t nseg, int64_t len, double* partials, double* out,
                    hipStream_t s);

// The second level of every split reduction (workgroup partials -> one FP64 sum,
// in a fixed order).  Between sums_defer_begin and sums_defer_end the launchers of
// this thread queue these final sums in *list instead of launching one kernel
// each; reduce_batch then sums them all in one launch (the same order, so the same
// bits).  While deferring, every queued sum must own its partial array.
struct SumJob {
  const double* part;
  int n;
  double* out;
};
void sums_defer_begin(std::vector<SumJob>* list);
void sums_defer_end();
void reduce_batch(const std::vector<SumJob>& jobs, hipStream_t s);

// ---- Gram of a mode unfolding (FP64 MFMA) -----------------------------------
// G (m x m, row-major, both triangles) = X_(k) X_(k)^T.  part is scratch of
// gram_partial_doubles(view) doubles.
size_t gram_partial_doubles(const ModeView& v);
// upper bound of gram_partial_doubles over every view with m rows
size_t gram_partial_bound(int64_t m);
void gram(const void* x, Elem t, const ModeView& v, double* part, double* G, hipStream_t s);
// Gram of the explicit residual R = X_(k) - U (U^T X_(k)) for m <= 128 (U m x R column-major,
// R <= 64), reading X once; the same partial scratch as gram().
constexpr int kResidGramMaxM = 128;
void resid_gram(const void* x, Elem t, const ModeView& v, const double* U, int R, double* part, double* G,
                hipStream_t s);

// ---- tensor-times-matrix ------------------------------------------------------
// Z[p, r, s] = sum_a U[a, r] X[p, a, s]: mode contraction with U^T (U m x R, column-major).
void ttm_contract(const void* x, Elem t, const ModeView& v, const double* U, int R, double* Z,
                  hipStream_t s);
// The same, also writing ||X||^2 (FP64) to norm_out; norm_part holds ttm_norm_partials() doubles.
size_t ttm_norm_partials();
void ttm_contract_norm(const void* x, Elem t, const ModeView& v, const double* U, int R, double* Z, double* norm_part,
                       double* norm_out, hipStream_t s);
// For modes of more than 128 rows: the contraction together with ||X||^2 and
// ||Z||^2 (FP64) from its own workgroup partials (in_part and out_part hold at least
// max_parts doubles each).  Returns false, launching nothing, for other shapes or
// when more than max_parts workgroups would be needed.
bool ttm_contract_sq(const void* x, Elem t, const ModeView& v, const double* U, int R, double* Z, double* in_part,
                     double* in_out, double* out_part, double* out_out, int max_parts, hipStream_t s);
// ---- mixed form: FP32 matrix cores, FP64 sums (m <= kResidGramMaxM) --------------
// Z (FP32) = U^T X; optionally ||X||^2 and the explicit residual energy
// ||X - U (U^T X)||^2 (the part this contraction discards), both FP64; the partial
// arrays hold ttm_norm_partials() doubles each.
void ttm_contract_f32(const void* x, Elem t, const ModeView& v, const double* U, int R, float* Z, double* norm_part,
                      double* norm_out, double* res_part, double* res_out, hipStream_t s);

// ---- grouped contractions -----------------------------------------------------
// Independent contractions Z = U^T X of small level tensors (one step of the
// projection chains of many streams) through the LDS-panel kernel, one launch per
// input / output type combination for up to 24 jobs.  A job computes what the panel
// kernel computes for it alone, so the result does not depend on the group: an FP32
// output (zt) takes FP32 products, with res_part (ttm_norm_partials() doubles) the
// explicit residual energy ||X - U Z||^2 as well (into res_out); with norm_part the
// sum of squares of X (into norm_out).  The final sums go through the deferred-sum
// mechanism when it is active.  ttm_groupable says which contractions qualify: modes
// of at most 128 rows, 1 <= R <= 64, at most kGroupMaxElems input elements.
constexpr int64_t kGroupMaxElems = int64_t(1) << 20;
struct TtmJob {
  const void* x;
  Elem t;
  ModeView v;
  const double* U;
  int R;
  void* Z;
  Elem zt;
  double* norm_part;
  double* norm_out;
  double* res_part;
  double* res_out;
};
bool ttm_groupable(const ModeView& v, int R);
void ttm_group(const std::vector<TtmJob>& jobs, hipStream_t s);
// The residual Gram (I - U U^T) G (I - U U^T) from the FP64 Gram G = M M^T of an
// unfolding of at least kGramProjMinElems elements and at most kGramProjMaxM rows
// (register-direct blocks for FP32 data in their shapes, else the LDS-panel or
// large-mode Gram), no residual formed: FP64 products, G's rounding relative to
// ||M||^2.  Modes of more than 128 rows need work of resid_gram_proj_work_doubles(m, R)
// doubles.
constexpr double kGramProjMinElems = 4194304.0;
constexpr int64_t kGramProjMaxM = 4096;
bool resid_gram_proj_applies(Elem t, const ModeView& v, int R);
size_t resid_gram_proj_work_doubles(int64_t m, int R);
// Device scratch (doubles) that the direct contractions of modes above 128 rows may
// use while the scope lives (one host thread), to split a contraction of few column
// blocks into row chunks; without it they run unsplit.
struct SplitScratch {
  SplitScratch(double* p, size_t n);
  ~SplitScratch();
  SplitScratch(const SplitScratch&) = delete;
  SplitScratch& operator=(const SplitScratch&) = delete;
};

// The projection of an m <= 128 Gram, in place; with defer, resid_gram_proj queues it
// there instead of launching it, and gram_project_batch launches a layer's (of every
// handle) together, one workgroup each.
struct ProjJob {
  double* G;
  const double* U;
  int m, R;
};
constexpr int kMaxProjJobs = 32;
void resid_gram_proj(const void* x, Elem t, const ModeView& v, const double* U, int R, double* part, double* G,
                     double* work, hipStream_t s, std::vector<ProjJob>* defer = nullptr);
void gram_project_batch(const ProjJob* jobs, int count, hipStream_t s);
// Gram of the explicit residual with the products on FP32 matrix cores and the
// workgroup partials summed in FP64.
void resid_gram_f32(const void* x, Elem t, const ModeView& v, const double* U, int R, double* part, double* G,
                    hipStream_t s);

// out[p, a, s] = sum_t U[a, t] Z[p, t, s] (mode expansion, U m x R column-major), or with
// M given: out = M - that (the explicit residual of a projection).  out is FP64 unless
// out_t says F32.
void ttm_expand(const double* Z, int64_t P, int R, int64_t S, const double* U, int64_t m,
                const void* M, Elem mt, void* out, Elem out_t, hipStream_t s);

// ---- symmetric eigen-decomposition and truncation (FP64) -----------------------
struct EigJob {
  const double* G;     // k x k symmetric, row-major
  double* scratch;     // eig_scratch_doubles(k, rmax) doubles
  double* evals;       // out: the leading eigenvalues, descending (as many as the rule needed, >= rank)
  double* vecs;        // out: k x r eigenvectors (column-major, sign-normalised)
  int* rank;           // out: chosen rank r
  double* tail;        // out: discarded energy sum_{i>=r} max(lambda_i, 0)
  double thr;          // eps_nw^2
  int k;
  int rmin;
  int rmax;
  int method;          // kEigAuto, or (testing) kEigHouseholder / kEigLanczos alone
};
// kEigAuto: the certified Lanczos decision where it can be proven, else the
// Householder path; kEigLanczos reports an unproven decision as rank -1.
constexpr int kEigAuto = 0, kEigHouseholder = 1, kEigLanczos = 2;
constexpr int kMaxEigJobs = 32;
size_t eig_scratch_doubles(int k, int rmax);
// Runs up to kMaxEigJobs independent problems in one launch (one workgroup each).
void eig_trunc(const EigJob* jobs, int count, hipStream_t s);

// Inputs of the mixed form's decision certificate, gathered after an eigen launch:
// out[0] = trace(G), out[1] = the smallest kept eigenvalue lambda_r (0 when the rule
// kept nothing), so that the discarded energy one rank lower is tail + lambda_r.
struct AuxJob {
  const double* G;
  const int* rank;
  const double* evals;
  double* out;
  int k;
};
void decision_aux(const AuxJob* jobs, int count, hipStream_t s);

// ---- basis expansion (FP64) -----------------------------------------------------
// Orthogonalises the rR columns of V (alpha x rR) against U_old (alpha x r_old) twice
// (classical Gram-Schmidt), orthonormalises them by CholeskyQR twice, normalises signs
// and writes [U_old, V] into core (alpha x (r_old + rR)).  core may alias U_old.
void orth_expand(const double* U_old, int64_t alpha, int r_old, double* V, int rR, double* core,
                 double* scratch, hipStream_t s);
size_t orth_scratch_doubles(int rR);
// Several independent expansions (the growing nodes of a layer, of one or many
// handles) in one launch per kMaxOrthJobs, one workgroup each.
struct OrthJob {
  const double* U_old;
  double* V;
  double* core;
  int64_t alpha;
  int r_old;
  int rR;
};
constexpr int kMaxOrthJobs = 32;
void orth_expand_batch(const OrthJob* jobs, int count, hipStream_t s);

// ---- layout helpers ---------------------------------------------------------------
// Zero-padding of a transfer core when a successor grows (padWithZeros): src is
// (ra*rb) x rp column-major with row i_a*rb + i_b, dst is (ra2*rb2) x rp.
void pad_core(const double* src, int ra, int rb, int rp, double* dst, int ra2, int rb2, hipStream_t s);
// root[(n_acc + n) * rcap * rcap + i * rcap + j] = C1[n][i][j] for n < N, i < r11, j < r12
// (C1 FP32 or FP64, the root FP64).
void root_append(const void* C1, Elem t, int64_t N, int r11, int r12, double* root, int64_t n_acc, int rcap,
                 hipStream_t s);
// latent[n][i][j] = root[(first + n)][i][j] (packed r11 x r12), zero for i >= r11 etc.
void root_extract(const double* root, int64_t first, int64_t count, int r11, int r12, int rcap,
                  double* latent, hipStream_t s);
void copy_f64(const double* src, double* dst, int64_t n, hipStream_t s);
void fill_f64(double* dst, double v, int64_t n, hipStream_t s);

}  // namespace ht

namespace ht {
// ---- optional per-kernel timing (include/ht_rise_profile.h) -----------------------
enum class KKind : int {
  Sumsq = 0, Gram, TtmContract, TtmExpand, Eig, Orth, Layout, Gram32, TtmContract32,
  Gram32Reg, TtmContract32Reg, GramReg64, TtmContractReg64, Count
};
extern bool g_prof_on;
void prof_begin(KKind k, hipStream_t s, double flops, double bytes);
void prof_end(hipStream_t s);
struct ProfScope {
  bool on;
  hipStream_t s;
  ProfScope(KKind k, hipStream_t s_, double flops, double bytes) : on(g_prof_on), s(s_) {
    if (on) prof_begin(k, s, flops, bytes);
  }
  ~ProfScope() {
    if (on) prof_end(s);
  }
};
}  // namespace ht
