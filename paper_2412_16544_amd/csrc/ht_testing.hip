// Kernel-level entry points declared in ht_rise_testing.h: argument checks, then
// the same launchers the BHT-l2r / HT-RISE driver uses.
#include <hip/hip_runtime.h>

#include "ht_internal.h"
#include "ht_rise_testing.h"

namespace {
ht::Elem elem(int32_t t) { return t == HT_F32 ? ht::Elem::F32 : ht::Elem::F64; }
bool ok_dtype(int32_t t) { return t == HT_F32 || t == HT_F64; }
hipStream_t st(void* s) { return static_cast<hipStream_t>(s); }
}  // namespace

extern "C" {

ht_status ht_test_sumsq(const void* x, int32_t dtype, int64_t n, double* out, double* scratch, void* s) {
  if (!x || !out || !scratch || n < 1 || !ok_dtype(dtype)) return HT_EINVAL;
  ht::sumsq(x, elem(dtype), n, scratch, out, st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

size_t ht_test_gram_scratch_doubles(int64_t P, int64_t m, int64_t S) {
  if (P < 1 || m < 1 || S < 1) return 0;
  return ht::gram_partial_doubles(ht::ModeView{P, m, S}) + ht::resid_gram_proj_work_doubles(m, 64);
}

ht_status ht_test_gram(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, double* G, double* scratch,
                       void* s) {
  if (!x || !G || !scratch || P < 1 || m < 1 || S < 1 || !ok_dtype(dtype)) return HT_EINVAL;
  ht::gram(x, elem(dtype), ht::ModeView{P, m, S}, scratch, G, st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

ht_status ht_test_resid_gram(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U, int32_t R,
                             double* G, double* scratch, void* s) {
  if (!x || !U || !G || !scratch || P < 1 || m < 1 || m > ht::kResidGramMaxM || S < 1 || R < 1 || R > 64 ||
      !ok_dtype(dtype))
    return HT_EINVAL;
  ht::resid_gram(x, elem(dtype), ht::ModeView{P, m, S}, U, R, scratch, G, st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

ht_status ht_test_ttm_contract(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                               int32_t R, double* Z, void* s) {
  if (!x || !U || !Z || P < 1 || m < 1 || S < 1 || R < 1 || R > 64 || !ok_dtype(dtype)) return HT_EINVAL;
  ht::ttm_contract(x, elem(dtype), ht::ModeView{P, m, S}, U, R, Z, st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

ht_status ht_test_ttm_contract_split(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                                     int32_t R, double* Z, double* scratch, size_t scratch_doubles, double* sq,
                                     void* s) {
  if (!x || !U || !Z || !scratch || !sq || P < 1 || m < 1 || S < 1 || R < 1 || R > 64 || !ok_dtype(dtype))
    return HT_EINVAL;
  // partials of ||X||^2 and ||Z||^2 (sq[0], sq[1]) follow the two sums in sq
  const ht::SplitScratch split(scratch, scratch_doubles);
  if (!ht::ttm_contract_sq(x, elem(dtype), ht::ModeView{P, m, S}, U, R, Z, sq + 2, sq, sq + 2 + 1024, sq + 1, 1024,
                           st(s)))
    return HT_EINVAL;
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

ht_status ht_test_resid_gram_f32(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                                 int32_t R, double* G, double* scratch, void* s) {
  if (!x || !U || !G || !scratch || P < 1 || m < 1 || m > ht::kResidGramMaxM || S < 1 || R < 1 || R > 64 ||
      !ok_dtype(dtype))
    return HT_EINVAL;
  ht::resid_gram_f32(x, elem(dtype), ht::ModeView{P, m, S}, U, R, scratch, G, st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

ht_status ht_test_resid_gram_proj(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                                  int32_t R, double* G, double* scratch, void* s) {
  const ht::ModeView v{P, m, S};
  if (!x || !U || !G || !scratch || P < 1 || m < 1 || S < 1 || R < 1 || R > 64 || !ok_dtype(dtype) ||
      m > ht::kGramProjMaxM)
    return HT_EINVAL;
  // the projection's work follows the partials in the scratch
  ht::resid_gram_proj(x, elem(dtype), v, U, R, scratch, G, scratch + ht::gram_partial_doubles(v), st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

size_t ht_test_ttm_partials_doubles(void) { return ht::ttm_norm_partials(); }

ht_status ht_test_ttm_contract_f32(const void* x, int32_t dtype, int64_t P, int64_t m, int64_t S, const double* U,
                                   int32_t R, float* Z, double* norm2, double* resid2, double* scratch, void* s) {
  if (!x || !U || !Z || !norm2 || !resid2 || !scratch || P < 1 || m < 1 || m > ht::kResidGramMaxM || S < 1 ||
      R < 1 || R > 64 || !ok_dtype(dtype))
    return HT_EINVAL;
  const size_t np = ht::ttm_norm_partials();
  ht::ttm_contract_f32(x, elem(dtype), ht::ModeView{P, m, S}, U, R, Z, scratch, norm2, scratch + np, resid2, st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

ht_status ht_test_ttm_expand(const double* Z, int64_t P, int32_t R, int64_t S, const double* U, int64_t m,
                             const void* M, int32_t m_dtype, void* out, int32_t out_dtype, void* s) {
  if (!Z || !U || !out || P < 1 || m < 1 || S < 1 || R < 1 || R > 64 || !ok_dtype(m_dtype) || !ok_dtype(out_dtype))
    return HT_EINVAL;
  if (M != nullptr && out_dtype != HT_F64) return HT_EINVAL;
  ht::ttm_expand(Z, P, R, S, U, m, M, elem(m_dtype), out, elem(out_dtype), st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

size_t ht_test_eig_scratch_doubles(int32_t k, int32_t rmax) {
  if (k < 1 || rmax < 0) return 0;
  return ht::eig_scratch_doubles(k, rmax > 0 ? rmax : 1);
}

ht_status ht_test_eig_method(const double* G, int32_t k, int32_t rmin, int32_t rmax, double thr, int32_t method,
                             double* evals, double* vecs, int32_t* rank, double* tail, double* scratch, void* s) {
  if (!G || !evals || !vecs || !rank || !tail || !scratch || k < 1 || k > 4096 || rmin < 0 || rmax < rmin ||
      rmax > k || method < ht::kEigAuto || method > ht::kEigLanczos)
    return HT_EINVAL;
  ht::EigJob j;
  j.G = G;
  j.scratch = scratch;
  j.evals = evals;
  j.vecs = vecs;
  j.rank = rank;
  j.tail = tail;
  j.thr = thr;
  j.k = k;
  j.rmin = rmin;
  j.rmax = rmax;
  j.method = method;
  ht::eig_trunc(&j, 1, st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

ht_status ht_test_eig(const double* G, int32_t k, int32_t rmin, int32_t rmax, double thr, double* evals, double* vecs,
                      int32_t* rank, double* tail, double* scratch, void* s) {
  return ht_test_eig_method(G, k, rmin, rmax, thr, ht::kEigAuto, evals, vecs, rank, tail, scratch, s);
}

ht_status ht_test_orth_expand(const double* U_old, int64_t alpha, int32_t r_old, double* V, int32_t rR, double* core,
                              void* s) {
  if (!V || !core || alpha < 1 || r_old < 0 || rR < 1 || r_old > 64 || rR > 64 || r_old + rR > alpha ||
      (r_old > 0 && !U_old))
    return HT_EINVAL;
  ht::orth_expand(U_old, alpha, r_old, V, rR, core, nullptr, st(s));
  return hipGetLastError() == hipSuccess ? HT_OK : HT_EDEVICE;
}

}  // extern "C"
