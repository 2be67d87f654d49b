// FP64 symmetric eigen-decomposition with the error-truncation rule, on gfx950.
//
// The truncated SVD of an unfolding M (Eq. ht_leaf_svd, Eq. svd_on_residual) is
// taken from the Gram matrix G = M M^T: sigma_i^2 = lambda_i(G) and the left
// singular vectors are G's eigenvectors.  One workgroup solves one k x k problem.
// It first runs Lanczos with full re-orthogonalisation and takes the decision
// from the Krylov space when a certificate proves it equal to the rule on the
// exact spectrum (the Ritz vectors are then the kept vectors); otherwise:
//
//   1. Householder reduction G = Q T Q^T to tridiagonal T.  Up to k = 224 the
//      matrix stays in registers (lower 32 x 32 tiles, one entry per thread per
//      tile); beyond, its lower triangle is packed in LDS or global memory;
//   2. every eigenvalue of T by multisection on Sturm counts (several lanes of a
//      wave per eigenvalue; signs of the leading principal minors);
//   3. the minimal rank r in [rmin, rmax] whose discarded energy, summed from the
//      smallest eigenvalue up, is <= thr = eps_nw^2 (clipping lambda at 0);
//   4. the r leading eigenvectors of T by inverse iteration (the partial-pivoting
//      LU of T - lambda I recomputed in each sweep, chains carried in registers),
//      re-orthogonalised twice, mapped back with Q and sign-normalised (largest
//      magnitude entry positive, lowest index on ties).
//
// Several independent problems (the nodes of one tree layer) run in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "ht_internal.h"

namespace ht {
namespace {

constexpr int ET = 512;
constexpr int NW = ET / 64;
constexpr int kLdsDoubles = 19968;  // 156 KiB of dynamic LDS per workgroup
constexpr int kSmallMax = 1024;     // the 6k work vectors live in LDS up to this k

// global-memory view of a pointer (stores through it wait on the vector counter only)
typedef __attribute__((address_space(1))) double gdouble;

// a value that every lane holds alike, moved to scalar registers
__device__ __forceinline__ double uniform(double x) {
  const uint64_t b = __double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b), hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

struct EigBatch {
  EigJob j[kMaxEigJobs];
};

// Cross-lane sums of doubles through DPP (row shifts and row broadcasts of the
// two 32-bit halves) instead of ds_bpermute-based shuffles.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

// sum over the 64 lanes, returned to every lane
__device__ __forceinline__ double dpp_wave_sum(double v) {
  v += dpp_mov<0x111, 0xf>(v);  // row_shr:1
  v += dpp_mov<0x112, 0xf>(v);  // row_shr:2
  v += dpp_mov<0x114, 0xf>(v);  // row_shr:4
  v += dpp_mov<0x118, 0xf>(v);  // row_shr:8  -> lane 15 of each row holds its row sum
  v += dpp_mov<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3 -> lane 63 holds the total
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// sum over each half-wave, left in lanes 31 and 63
__device__ __forceinline__ double dpp_half_sum(double v) {
  v += dpp_mov<0x111, 0xf>(v);  // row_shr:1
  v += dpp_mov<0x112, 0xf>(v);  // row_shr:2
  v += dpp_mov<0x114, 0xf>(v);  // row_shr:4
  v += dpp_mov<0x118, 0xf>(v);  // row_shr:8  -> lane 15 of each row holds its row sum
  v += dpp_mov<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  return v;
}

// sum over each aligned group of 4 lanes, returned to the 4 lanes
__device__ __forceinline__ double dpp_quad_sum(double v) {
  v += dpp_mov<0xB1, 0xf>(v);  // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E, 0xf>(v);  // quad_perm [2,3,0,1]
  return v;
}

__device__ __forceinline__ double wsum(double v) { return dpp_wave_sum(v); }

// DPP move that keeps the lane's own value where the source lane is invalid
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_self(double x) {
  const int xl = __double2loint(x), xh = __double2hiint(x);
  const int lo = __builtin_amdgcn_update_dpp(xl, xl, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(xh, xh, CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

template <bool MAX>
__device__ __forceinline__ double dpp_wave_minmax(double v) {
#define HT_MM(a, b) (MAX ? fmax((a), (b)) : fmin((a), (b)))
  v = HT_MM(v, (dpp_self<0x111, 0xf>(v)));
  v = HT_MM(v, (dpp_self<0x112, 0xf>(v)));
  v = HT_MM(v, (dpp_self<0x114, 0xf>(v)));
  v = HT_MM(v, (dpp_self<0x118, 0xf>(v)));
  v = HT_MM(v, (dpp_self<0x142, 0xa>(v)));
  v = HT_MM(v, (dpp_self<0x143, 0xc>(v)));
#undef HT_MM
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}


__device__ __forceinline__ double bsum(double v, double* red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ size_t eig_scratch_doubles_dev(int k, int rmax) {
  const size_t K = (size_t)k;
  return K * (K + 1) / 2 + K * K + 6 * K + K + K + (K + 1) + 4 * K * (size_t)(rmax > 1 ? rmax : 1) + 64;
}

__device__ __forceinline__ int pk(int a, int b) { return a * (a + 1) / 2 + b; }  // a >= b, k <= 4096

// row index of entry q of a packed lower triangle
__device__ __forceinline__ int prow(int q) {
  int a = (int)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) / 2 > q) --a;
  while ((a + 1) * (a + 2) / 2 <= q) ++a;
  return a;
}

// Number of eigenvalues of T below x from the signs of the leading principal
// minors p_i = det(T_i - x I) = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}: the pivot
// p_i / p_{i-1} of T - x I is negative exactly when the two signs differ
// (Sylvester's law of inertia).  dn and e2n are T scaled by a power of two so
// that |T| <= 1; the pair (p_{i-1}, p_{i-2}) is rescaled by a power of two every
// four steps, which keeps it in range without touching the signs.  As in the
// pivot form, a pivot of magnitude below the floor DBL_MIN is replaced by
// -DBL_MIN (the pair is then re-expressed at a large scale so that it cannot
// underflow).  The recurrence has one dependent FMA per step, against a division
// or a refined reciprocal per step in the pivot form.
__device__ __forceinline__ int sturm_scaled(const double* __restrict__ dn, const double* __restrict__ e2n, int k,
                                            double x) {
  double p1 = 1.0, p2 = 0.0;
  int cnt = 0;
#define HT_STURM_STEP(dd, ff)                                    \
  {                                                              \
    const double fl = DBL_MIN * fabs(p1);                        \
    double p = fma((dd) - x, p1, -((ff) * p2));                  \
    if (fabs(p) < fl) {                                          \
      p1 = copysign(0x1p960, p1);                                \
      p = -DBL_MIN * p1;                                         \
    }                                                            \
    cnt += (__double2hiint(p) ^ __double2hiint(p1)) < 0 ? 1 : 0; \
    p2 = p1;                                                     \
    p1 = p;                                                      \
  }
  HT_STURM_STEP(dn[0], 0.0)
  int i = 1;
  for (; i + 4 <= k; i += 4) {
    const double d0 = dn[i], d1 = dn[i + 1], d2 = dn[i + 2], d3 = dn[i + 3];
    const double f0 = e2n[i - 1], f1 = e2n[i], f2 = e2n[i + 1], f3 = e2n[i + 2];
    HT_STURM_STEP(d0, f0)
    HT_STURM_STEP(d1, f1)
    HT_STURM_STEP(d2, f2)
    HT_STURM_STEP(d3, f3)
    const int ex = __builtin_amdgcn_frexp_exp(p1);
    p1 = __builtin_amdgcn_ldexp(p1, -ex);
    p2 = __builtin_amdgcn_ldexp(p2, -ex);
  }
  for (; i < k; ++i) HT_STURM_STEP(dn[i], e2n[i - 1])
#undef HT_STURM_STEP
  return cnt;
}

// The same count without the pivot floor on the dependent chain: each step is
// one FMA (the e^2 p_{i-2} product and the sign test hang off the chain), the pair
// is rescaled every eight steps, and the dn / e2n loads run one block ahead.  A
// pivot below the floor only raises a flag, and the caller then repeats the count
// with sturm_scaled.
__device__ __forceinline__ int sturm_fast(const double* __restrict__ dn, const double* __restrict__ e2n, int k,
                                          double x, bool& tiny) {
  double p1 = 1.0, p2 = 0.0;
  int cnt = 0;
  bool t = false;
#define HT_FAST_STEP(dd, ff)                                         \
  {                                                                  \
    const double fl = DBL_MIN * fabs(p1);                            \
    const double p = fma((dd) - x, p1, -((ff) * p2));                \
    t |= !(fabs(p) >= fl) | (p == 0.0);                              \
    cnt += (__double2hiint(p) ^ __double2hiint(p1)) < 0 ? 1 : 0;     \
    p2 = p1;                                                         \
    p1 = p;                                                          \
  }
  HT_FAST_STEP(dn[0], 0.0)
  int i = 1;
  if (i + 8 <= k) {
    double d[8], f[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      d[q] = dn[i + q];
      f[q] = e2n[i + q - 1];
    }
    for (; i + 16 <= k; i += 8) {
      double dn8[8], f8[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        dn8[q] = dn[i + 8 + q];
        f8[q] = e2n[i + 7 + q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) HT_FAST_STEP(d[q], f[q])
      const int ex = __builtin_amdgcn_frexp_exp(p1);
      p1 = __builtin_amdgcn_ldexp(p1, -ex);
      p2 = __builtin_amdgcn_ldexp(p2, -ex);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        d[q] = dn8[q];
        f[q] = f8[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) HT_FAST_STEP(d[q], f[q])
    i += 8;
    const int ex = __builtin_amdgcn_frexp_exp(p1);
    p1 = __builtin_amdgcn_ldexp(p1, -ex);
    p2 = __builtin_amdgcn_ldexp(p2, -ex);
  }
  for (; i < k; ++i) HT_FAST_STEP(dn[i], e2n[i - 1])
#undef HT_FAST_STEP
  tiny = t;
  return cnt;
}

__device__ __forceinline__ double start_entry(int j, int i) {
  unsigned h = (unsigned)(j * 0x9E3779B1u) ^ (unsigned)(i * 0x85EBCA77u) ^ 0xC2B2AE3Du;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return 0.5 + (double)(h & 0xFFFFFF) * (1.0 / 16777216.0);
}

// One Householder step on the packed lower triangle P (entry (a, b), a >= b, at
// pk(a, b)): column j is annihilated below the subdiagonal, the reflector goes to
// row j of hv.
__device__ __forceinline__ void house_step(double* P, int k, int j, double* vb, double* pb, double* wb, double* red,
                                           double* d, double* e, double* tau, double* hv) {
  const int tid = threadIdx.x;
  const int r0 = j + 1, n2 = k - r0;
  double loc = 0.0;
  for (int i = 1 + tid; i < n2; i += ET) {
    const double x = P[pk(r0 + i, j)];
    loc = fma(x, x, loc);
  }
  const double xn2 = bsum(loc, red);
  const double alpha = P[pk(r0, j)];
  double beta, tj, scale;
  if (xn2 == 0.0) {
    beta = alpha;
    tj = 0.0;
    scale = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    tj = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  for (int i = tid; i < n2; i += ET) {
    const double v = (i == 0) ? 1.0 : P[pk(r0 + i, j)] * scale;
    vb[i] = v;
    hv[(int64_t)j * k + r0 + i] = v;
  }
  if (tid == 0) {
    d[j] = P[pk(j, j)];
    e[j] = beta;
    tau[j] = tj;
  }
  __syncthreads();
  if (tj != 0.0) {
    // p = tau A22 v: four lanes per row, each summing every fourth entry, joined by shuffles
    for (int base = 0; base < n2; base += ET / 4) {
      const int i = base + (tid >> 2), u = tid & 3;
      double s = 0.0;
      if (i < n2) {
        const int a = r0 + i;
        const double* row = P + pk(a, r0);
        // independent partial sums keep several LDS loads in flight
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int l = u;
        for (; l + 12 <= i; l += 16) {
          s = fma(row[l], vb[l], s);
          s1 = fma(row[l + 4], vb[l + 4], s1);
          s2 = fma(row[l + 8], vb[l + 8], s2);
          s3 = fma(row[l + 12], vb[l + 12], s3);
        }
        for (; l <= i; l += 4) s = fma(row[l], vb[l], s);  // entries (a, b <= a)
        int l2 = i + 1 + u;
        int idx = pk(r0 + l2, a);
        int step = r0 + l2 + 1;  // pk(c + 1, a) - pk(c, a) = c + 1
        for (; l2 + 12 < n2; l2 += 16) {
          const int i1 = idx + step + (step + 1) + (step + 2) + (step + 3);
          const int i2 = i1 + (step + 4) + (step + 5) + (step + 6) + (step + 7);
          const int i3 = i2 + (step + 8) + (step + 9) + (step + 10) + (step + 11);
          s = fma(P[idx], vb[l2], s);
          s1 = fma(P[i1], vb[l2 + 4], s1);
          s2 = fma(P[i2], vb[l2 + 8], s2);
          s3 = fma(P[i3], vb[l2 + 12], s3);
          idx = i3 + (step + 12) + (step + 13) + (step + 14) + (step + 15);
          step += 16;
        }
        for (; l2 < n2; l2 += 4) {  // entries (b > a, a)
          s = fma(P[idx], vb[l2], s);
          idx += step + (step + 1) + (step + 2) + (step + 3);
          step += 4;
        }
        s += (s1 + s2) + s3;
      }
      s = dpp_quad_sum(s);
      if (i < n2 && u == 0) pb[i] = tj * s;
    }
    __syncthreads();
    double loc2 = 0.0;
    for (int i = tid; i < n2; i += ET) loc2 = fma(pb[i], vb[i], loc2);
    const double kk = -0.5 * tj * bsum(loc2, red);
    for (int i = tid; i < n2; i += ET) wb[i] = fma(kk, vb[i], pb[i]);
    __syncthreads();
    // rank-2 update of the trailing packed triangle; (a, b) advanced incrementally
    const int nq = n2 * (n2 + 1) / 2;
    if (tid < nq) {
      int a = prow(tid);
      int b = tid - a * (a + 1) / 2;
      const int o = pk(r0, r0);
      for (int q = tid; q < nq; q += ET) {
        // entry (r0 + a, r0 + b) sits at pk(r0 + a, r0 + b) = o + pk(a, b) + r0 * a
        P[o + pk(a, b) + r0 * a] -= vb[a] * wb[b] + wb[a] * vb[b];
        b += ET;
        while (b > a) {
          b -= a + 1;
          ++a;
        }
      }
    }
  }
  __syncthreads();
}

// ---- phase 1, packed path (k > 16 kRegRowTiles): lower triangle packed in LDS or
//      global memory, one Householder step at a time over the whole workgroup
__device__ __forceinline__ void tridiagonalise_packed(double* P, const double* __restrict__ G, int k, double* vb,
                                                      double* pb, double* wb, double* red, double* d, double* e,
                                                      double* tau, double* hv) {
  const int tid = threadIdx.x;
  const int npk = k * (k + 1) / 2;
  for (int q = tid; q < npk; q += ET) {
    const int a = prow(q);
    const int b = q - a * (a + 1) / 2;
    P[q] = G[(int64_t)a * k + b];
  }
  __syncthreads();
  for (int j = 0; j + 2 < k; ++j) house_step(P, k, j, vb, pb, wb, red, d, e, tau, hv);
  if (tid == 0) {
    if (k >= 2) {
      d[k - 2] = P[pk(k - 2, k - 2)];
      e[k - 2] = P[pk(k - 1, k - 2)];
      tau[k - 2] = 0.0;
    }
    d[k - 1] = P[pk(k - 1, k - 1)];
    e[k - 1] = 0.0;
    tau[k - 1] = 0.0;
  }
  __syncthreads();
}

// ---- phase 1, register path (k <= 16 kRegRowTiles) ---------------------------------
// The symmetric matrix lives in registers: thread (tr, tc) = (tid / 32, tid % 32)
// holds entry (16 a + tr, 32 b + tc) of every stored tile (a, b), the 16 x 32 tiles
// that meet the lower triangle (b <= a / 2), so the 32 x 32 diagonal blocks are
// stored in full.  Step j annihilates column j below the subdiagonal with the
// reflector H = I - tau v v^T, v = e_{j+1} + s x' (x' the column below row j + 1,
// s its scale), and costs three workgroup barriers:
//   A. the owners of columns j and j + 1 publish them in LDS;
//   B. every thread forms its partial sums of y = A x' (row partials of each
//      active tile, transposed partials of the strictly lower ones), while wave 0
//      computes tau and s from the column -- the reflector is not needed yet since
//      A v = s y + A e_{j+1};
//   C. p = tau A v and v are assembled in LDS;
// then every wave forms p^T v redundantly and applies A -= v w^T + w v^T,
// w = p - (tau / 2)(p^T v) v, to its registers.  LDS loads of a phase are issued
// before their first use, and tiles outside the active trailing block are skipped.
constexpr int kRegRowTiles = 14;  // k <= 224

__host__ __device__ constexpr int tile_base(int a) {
  int s = 0;
  for (int q = 0; q < a; ++q) s += q / 2 + 1;
  return s;
}

// The owners of column c (lanes with tc == c % 32, in column tile c / 32) copy the
// column's stored rows into buf.  Rows below c come out of stale tiles and are
// never read; rows >= k are zero.  Straight-line stores, no per-row branches.
template <int TA>
__device__ __forceinline__ void put_column(const double (&A)[tile_base(TA)], int c, int tr, int tc, double* buf) {
  if (tc != (c & 31)) return;
  const int bc = c >> 5;
#pragma unroll
  for (int b = 0; b < (TA + 1) / 2; ++b) {
    if (b == bc) {
#pragma unroll
      for (int a = 2 * b; a < TA; ++a) {
        double val = A[tile_base(a) + b];
        asm volatile("" : "+v"(val));  // keeps the case blocks apart, so A stays in registers
        buf[16 * a + tr] = val;
      }
    }
  }
}

// The owners of column c publish the part below the diagonal that the next
// reflector annihilates: rows c + 2 .. of buf get the column, rows 32 (c / 32) ..
// c + 1 get zero (rows above were zeroed by earlier steps, rows >= k hold zeros of
// A), the diagonal entry goes to *dg and the subdiagonal one to *sd.
template <int TA>
__device__ __forceinline__ void put_lower(const double (&A)[tile_base(TA)], int c, int tr, int tc, double* buf,
                                          double* dg, double* sd) {
  if (tc != (c & 31)) return;
  const int bc = c >> 5;
#pragma unroll
  for (int b = 0; b < (TA + 1) / 2; ++b) {
    if (b == bc) {
      double dgv = 0.0, sdv = 0.0;
#pragma unroll
      for (int a = 2 * b; a < TA; ++a) {
        const int i = 16 * a + tr;
        double val = A[tile_base(a) + b];
        asm volatile("" : "+v"(val));
        buf[i] = i > c + 1 ? val : 0.0;
        dgv = i == c ? val : dgv;
        sdv = i == c + 1 ? val : sdv;
      }
      // row c sits in this lane's tile c / 16 >= 2 b, row c + 1 in tile (c + 1) / 16
      if (tr == (c & 15)) *dg = dgv;
      if (tr == ((c + 1) & 15)) *sd = sdv;
    }
  }
}

template <int TA>
__device__ __forceinline__ void tridiag_reg(const double* __restrict__ G, int k, double* xb, double* cb,
                                            double* vbuf, double* pbuf, double* rowpart, double* colpart, double* d,
                                            double* e, double* tau, double* __restrict__ hv, double* s_red) {
  constexpr int TB = (TA + 1) / 2;
  constexpr int NT = tile_base(TA);
  constexpr int RP = 16 * TA + 1;  // row strides of the partials (odd: spreads the LDS banks)
  constexpr int CP = 32 * TB + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, tr = tid >> 5, tc = tid & 31;
  // the size and the reflector store are the same for every lane: keep them scalar,
  // so the step loop runs on scalar branches
  k = __builtin_amdgcn_readfirstlane(k);
  gdouble* hvg = reinterpret_cast<gdouble*>(reinterpret_cast<uintptr_t>(hv));
  double A[NT];
#pragma unroll
  for (int a = 0; a < TA; ++a) {
#pragma unroll
    for (int b = 0; b <= a / 2; ++b) {
      const int i = 16 * a + tr, l = 32 * b + tc;
      A[tile_base(a) + b] = (i < k && l < k) ? G[(int64_t)i * k + l] : 0.0;
    }
  }
  // xb, vbuf and pbuf hold exact zeros outside the entries a step defines, so the
  // loads below need no masks
  for (int i = tid; i < 256; i += ET) {
    xb[i] = 0.0;
    vbuf[i] = 0.0;
    pbuf[i] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j + 2 < k; ++j) {
    const int r0 = j + 1;
    const int a0 = r0 >> 4, b0 = r0 >> 5;  // first row / column tiles that meet the trailing block
    // ---- A: x' (column j below row r0) into xb, column r0 into cb
    put_lower<TA>(A, j, tr, tc, xb, s_red + 2, s_red + 3);
    put_column<TA>(A, r0, tr, tc, cb);
    __syncthreads();
    // ---- B: partial sums of y = A x', and the reflector on wave 0
    {
      double xr[TA], xc[TB];
#pragma unroll
      for (int a = 0; a < TA; ++a) xr[a] = xb[16 * a + tr];
#pragma unroll
      for (int b = 0; b < TB; ++b) xc[b] = xb[32 * b + tc];
      double colacc[TB];
#pragma unroll
      for (int b = 0; b < TB; ++b) colacc[b] = 0.0;
#pragma unroll
      for (int a = 0; a < TA; ++a) {
        if (a >= a0) {
          double racc = 0.0;
#pragma unroll
          for (int b = 0; b <= a / 2; ++b) {
            racc = fma(A[tile_base(a) + b], xc[b], racc);
            if (b < a / 2) colacc[b] = fma(A[tile_base(a) + b], xr[a], colacc[b]);
          }
          rowpart[tc * RP + 16 * a + tr] = racc;
        }
      }
#pragma unroll
      for (int b = 0; b < TB; ++b)
        if (b >= b0) colpart[tr * CP + 32 * b + tc] = colacc[b];
      if (wave == 0) {
        double sq = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const double x = xb[lane + 64 * m];
          sq = fma(x, x, sq);
        }
        const double xn2 = dpp_wave_sum(sq);
        const double alpha = s_red[3], dj = s_red[2];
        double beta, tj, scale;
        if (xn2 == 0.0) {
          beta = alpha;
          tj = 0.0;
          scale = 0.0;
        } else {
          beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
          tj = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        if (lane == 0) {
          d[j] = dj;
          e[j] = beta;
          tau[j] = tj;
          s_red[0] = tj;
          s_red[1] = scale;
        }
      }
    }
    __syncthreads();
    const double tj = uniform(s_red[0]), scale = s_red[1];
    if (tj == 0.0) continue;  // the column is already reduced
    // ---- C: v and p = tau (s y + A[:, r0]) for every index; two threads per entry
    {
      const int i = tid >> 1, h = tid & 1;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int m = 0; m < 16; m += 4) {
        s0 += rowpart[(h + 2 * m) * RP + i];
        s1 += rowpart[(h + 2 * m + 2) * RP + i];
        s2 += rowpart[(h + 2 * m + 4) * RP + i];
        s3 += rowpart[(h + 2 * m + 6) * RP + i];
      }
#pragma unroll
      for (int m = 0; m < 8; m += 2) {
        s0 += colpart[(h + 2 * m) * CP + i];
        s1 += colpart[(h + 2 * m + 2) * CP + i];
      }
      const double x = xb[i], c = cb[i];
      double y = (s0 + s1) + (s2 + s3);
      y += dpp_mov<0xB1, 0xf>(y);  // quad_perm [1,0,3,2]: the pair's sum
      if (h == 0 && i < 32 * TB) {
        const bool live = i >= r0 && i < k;
        const double v = (i == r0) ? 1.0 : x * scale;
        vbuf[i] = v;
        pbuf[i] = live ? tj * fma(scale, y, c) : 0.0;
        if (live) hvg[(int64_t)j * k + i] = v;
      }
    }
    __syncthreads();
    // ---- w = p - (tau / 2)(p^T v) v and A -= v w^T + w v^T on the active tiles
    {
      double vr[TA], pr[TA], vc[TB], pc[TB], dv[4], dp[4];
#pragma unroll
      for (int a = 0; a < TA; ++a) {
        vr[a] = vbuf[16 * a + tr];
        pr[a] = pbuf[16 * a + tr];
      }
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        vc[b] = vbuf[32 * b + tc];
        pc[b] = pbuf[32 * b + tc];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        dv[m] = vbuf[lane + 64 * m];
        dp[m] = pbuf[lane + 64 * m];
      }
      double dl = 0.0;
#pragma unroll
      for (int m = 0; m < 4; ++m) dl = fma(dp[m], dv[m], dl);
      const double kk = -0.5 * tj * dpp_wave_sum(dl);
      double wc[TB];
#pragma unroll
      for (int b = 0; b < TB; ++b) wc[b] = fma(kk, vc[b], pc[b]);
#pragma unroll
      for (int a = 0; a < TA; ++a) {
        if (a >= a0) {
          const double wr = fma(kk, vr[a], pr[a]);
#pragma unroll
          for (int b = 0; b <= a / 2; ++b)
            A[tile_base(a) + b] = fma(-wr, vc[b], fma(-vr[a], wc[b], A[tile_base(a) + b]));
        }
      }
    }
  }
  // the trailing 2 x 2 (or 1 x 1) block
  __syncthreads();
  if (k >= 2) put_column<TA>(A, k - 2, tr, tc, xb);
  put_column<TA>(A, k - 1, tr, tc, cb);
  __syncthreads();
  if (tid == 0) {
    if (k >= 2) {
      d[k - 2] = xb[k - 2];
      e[k - 2] = xb[k - 1];
      tau[k - 2] = 0.0;
    }
    d[k - 1] = cb[k - 1];
    e[k - 1] = 0.0;
    tau[k - 1] = 0.0;
  }
  __syncthreads();
}

// ---- end of phase 1 (both paths): squared off-diagonal, Gershgorin interval, |T|
//      and the power-of-two scaled copy used by the Sturm counts.
//      sh = {lower bound, upper bound, |T|, scale}
__device__ __forceinline__ void finish_tridiag(int k, const double* d, const double* e, double* e2, double* dn,
                                               double* e2n, double* sh) {
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    double gl = DBL_MAX, gu = -DBL_MAX, em = 0.0;
    for (int i = lane; i < k; i += 64) {
      const double off = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < k ? fabs(e[i]) : 0.0);
      gl = fmin(gl, d[i] - off);
      gu = fmax(gu, d[i] + off);
      const double ee = (i + 1 < k) ? e[i] * e[i] : 0.0;
      e2[i] = ee;
      em = fmax(em, ee);
    }
    gl = dpp_wave_minmax<false>(gl);
    gu = dpp_wave_minmax<true>(gu);
    em = dpp_wave_minmax<true>(em);
    if (lane == 0) {
      const double tn = fmax(fabs(gl), fabs(gu));
      const double pivmin = DBL_MIN * fmax(1.0, em);
      sh[0] = gl - 2.2e-16 * tn - pivmin;
      sh[1] = gu + 2.2e-16 * tn + pivmin;
      sh[2] = tn;
      sh[3] = tn > 0.0 ? __builtin_amdgcn_ldexp(1.0, -__builtin_amdgcn_frexp_exp(tn)) : 1.0;
    }
  }
  __syncthreads();
  const double sc = sh[3];
  for (int i = tid; i < k; i += ET) {
    dn[i] = d[i] * sc;
    const double es = (i + 1 < k) ? e[i] * sc : 0.0;
    e2n[i] = es * es;
  }
  __syncthreads();
}

// Isolates eigenvalue idx (ascending index) of the scaled tridiagonal by
// multisection: the T lanes of a group evaluate Sturm counts at T interior points
// of its interval and keep the sub-interval that holds it.  u is the lane's place
// in its group, gbase the group's first lane in the wave; fast(x, tiny) counts
// (raising tiny when a pivot fell below the floor) and scaled(x) is the careful
// count that then replaces it.
template <int T, class Fast, class Scaled>
__device__ __forceinline__ double multisect_by(Fast fast, Scaled scaled, const double* sh, int idx, int u,
                                               int gbase) {
  const double atol = 2.2e-16 * sh[2], sc = sh[3];
  double lo = sh[0], hi = sh[1];  // invariant: count(lo) <= idx < count(hi)
  for (int it = 0; it < 160; ++it) {
    const bool done = hi - lo <= fmax(2.2e-16 * fmax(fabs(lo), fabs(hi)), atol);
    if (__all(done)) break;
    const double w = (hi - lo) / (double)(T + 1);
    const double x = lo + w * (double)(u + 1);
    bool above = false;
    if (!done && x < hi && x > lo) {
      bool tiny;
      int cnt = fast(x * sc, tiny);
      if (tiny) cnt = scaled(x * sc);
      above = cnt > idx;
    } else {
      above = !done && x >= hi;
    }
    const unsigned long long msk = __ballot(above);
    if (!done) {
      const unsigned long long gm = (msk >> gbase) & ((1ull << T) - 1);
      double nlo, nhi;
      if (gm == 0) {
        nlo = lo + w * (double)T;
        nhi = hi;
      } else {
        const int us = __builtin_ctzll(gm);
        nhi = lo + w * (double)(us + 1);
        nlo = us > 0 ? lo + w * (double)us : lo;
      }
      if (nhi > hi) nhi = hi;
      if (nlo < lo) nlo = lo;
      lo = nlo;
      hi = nhi;
    }
  }
  return 0.5 * (lo + hi);
}

template <int T>
__device__ __forceinline__ double multisect(const double* dn, const double* e2n, int k, const double* sh, int idx,
                                            int u, int gbase) {
  return multisect_by<T>([&](double x, bool& tiny) { return sturm_fast(dn, e2n, k, x, tiny); },
                         [&](double x) { return sturm_scaled(dn, e2n, k, x); }, sh, idx, u, gbase);
}

// ---- phases 2 and 3: the leading eigenvalues and the truncation rule.  The
//      discarded energy of rank c is trace(T) minus the sum of the c leading
//      eigenvalues (clipped at 0); eigenvalues are found in descending chunks (8,
//      then 32 at a time) only until the rule is decided, each by multisection
//      over 16 lanes.  top[m] receives the m-th largest eigenvalue; returns how
//      many were found.
__device__ __forceinline__ int top_eigen_rank(const double* dn, const double* e2n, const double* d, int k,
                                              const double* sh, int rmin, int rmax, double thr, double* top,
                                              int* rank_out, double* tail_out, int* s_rank, double* s_acc) {
  constexpr int T = 16;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    double t = 0.0;
    for (int i = lane; i < k; i += 64) t += d[i];
    t = dpp_wave_sum(t);
    if (lane == 0) {
      s_acc[0] = t;    // trace(T)
      s_acc[1] = 0.0;  // sum of the clipped eigenvalues found so far
    }
  }
  __syncthreads();
  const int kmax = min(k, rmax);
  const int slot = tid / T, u = tid % T, gbase = lane - (lane % T);
  int m0 = 0, chunk = 8;
  for (;;) {
    const int m = m0 + slot;
    if (slot < chunk && m < k) {
      const double v = multisect<T>(dn, e2n, k, sh, k - 1 - m, u, gbase);
      if (u == 0) top[m] = v;
    }
    __syncthreads();
    if (tid == 0) {
      const double tr = s_acc[0];
      double S = s_acc[1];
      const int cend = min(min(kmax, m0 + chunk), k);
      int r = -1;
      double tl = 0.0;
      int c = m0;
      for (; c <= cend; ++c) {
        if (c >= rmin && tr - S <= thr) {
          r = c;
          tl = tr - S;
          break;
        }
        if (c < cend) S += fmax(top[c], 0.0);
      }
      if (r < 0 && cend == kmax) {
        r = kmax;
        tl = tr - S;
      }
      if (r >= 0) {
        *rank_out = r;
        *tail_out = fmax(tl, 0.0);
      }
      *s_rank = r;
      s_acc[1] = S;
    }
    __syncthreads();
    const int found = min(m0 + chunk, k);
    if (*s_rank >= 0 || found >= k) {
      if (*s_rank < 0 && tid == 0) *s_rank = kmax;  // not reached: found == k implies cend == kmax
      __syncthreads();
      return found;
    }
    m0 += chunk;
    chunk = ET / T;
  }
}

// reciprocal of a nonzero double: the hardware estimate and two Newton steps
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double t = fma(-x, y, 1.0);
  y = fma(y, t, y);
  t = fma(-x, y, 1.0);
  return fma(y, t, y);
}

// ---- phase 4a: inverse iteration (two sweeps from a fixed pseudo-random start),
//      one thread per vector, for the r leading eigenvalues (top, descending).  W
//      holds 4 k r doubles: the iterate Z and the three rows of U of the
//      partial-pivoting LU of T - lambda I (the pivot stored as its reciprocal);
//      entry (i, j) of each at i * r + j.  Row choices are selects, so vectors
//      that pivot differently do not split the wave.
__device__ __forceinline__ void inverse_iteration(double* W, int k, int r, const double* top, const double* d,
                                                  const double* e, double tnorm) {
  const int tid = threadIdx.x;
  double* Z = W;
  double* U0 = Z + (size_t)k * r;
  double* U1 = U0 + (size_t)k * r;
  double* U2 = U1 + (size_t)k * r;
  const double tiny = fmax(2.2e-16 * tnorm, DBL_MIN);
  for (int j = tid; j < r; j += ET) {
    const double lm = top[j];
    for (int i = 0; i < k; ++i) Z[(size_t)i * r + j] = start_entry(j, i);
    for (int it = 0; it < 2; ++it) {
      // forward: factor T - lm I row by row with partial pivoting, apply to the rhs
      double u0 = d[0] - lm, u1 = (k > 1) ? e[0] : 0.0, u2 = 0.0;
      double bi = Z[j];
      for (int i = 0; i + 1 < k; ++i) {
        const double l0 = e[i], l1 = d[i + 1] - lm, l2 = (i + 2 < k) ? e[i + 1] : 0.0;
        const double bn = Z[(size_t)(i + 1) * r + j];
        const bool sw = fabs(u0) < fabs(l0);  // the next row becomes the pivot row
        double p0 = sw ? l0 : u0;
        const double p1 = sw ? l1 : u1, p2 = sw ? l2 : u2, bp = sw ? bn : bi;
        const double o0 = sw ? u0 : l0, o1 = sw ? u1 : l1, o2 = sw ? u2 : l2, bo = sw ? bi : bn;
        if (p0 == 0.0) p0 = tiny;  // both candidates zero
        const double ip = recip(p0);
        const double mlt = o0 * ip;
        // the back substitution divides by the pivot held away from zero
        U0[(size_t)i * r + j] = fabs(p0) < tiny ? recip(p0 < 0.0 ? -tiny : tiny) : ip;
        U1[(size_t)i * r + j] = p1;
        U2[(size_t)i * r + j] = p2;
        Z[(size_t)i * r + j] = bp;
        u0 = fma(-mlt, p1, o1);
        u1 = fma(-mlt, p2, o2);
        u2 = 0.0;
        bi = fma(-mlt, bp, bo);
      }
      if (fabs(u0) < tiny) u0 = (u0 < 0.0) ? -tiny : tiny;
      // backward substitution, the two previous unknowns kept in registers and the
      // next rows' factors loaded one step ahead
      double x1 = bi / u0, x2 = 0.0, mx = fabs(x1);
      Z[(size_t)(k - 1) * r + j] = x1;
      if (k >= 2) {
        size_t o = (size_t)(k - 2) * r + j;
        double q0 = U0[o], q1 = U1[o], q2 = U2[o], qz = Z[o];
        for (int i = k - 2; i >= 0; --i) {
          const size_t on = (i > 0) ? o - r : o;
          const double n0 = U0[on], n1 = U1[on], n2 = U2[on], nz = Z[on];
          const double x = (qz - q1 * x1 - q2 * x2) * q0;
          Z[o] = x;
          x2 = x1;
          x1 = x;
          mx = fmax(mx, fabs(x));
          q0 = n0;
          q1 = n1;
          q2 = n2;
          qz = nz;
          o = on;
        }
      }
      const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
      for (int i = 0; i < k; ++i) Z[(size_t)i * r + j] *= inv;
    }
  }
  __syncthreads();
}

// ---- phase 4b: orthonormalise the r columns of Z in order (classical
//      Gram-Schmidt, two passes)
__device__ __forceinline__ void cgs2_columns(double* Z, int k, int r, double* pb, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < r; ++j) {
      for (int t = wave; t < j; t += NW) {
        double s = 0.0;
        for (int i = lane; i < k; i += 64) s = fma(Z[(size_t)i * r + t], Z[(size_t)i * r + j], s);
        s = wsum(s);
        if (lane == 0) pb[t] = s;
      }
      __syncthreads();
      double loc = 0.0;
      for (int i = tid; i < k; i += ET) {
        double v = Z[(size_t)i * r + j];
        for (int t = 0; t < j; ++t) v -= pb[t] * Z[(size_t)i * r + t];
        Z[(size_t)i * r + j] = v;
        loc = fma(v, v, loc);
      }
      const double nrm = sqrt(bsum(loc, red));
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int i = tid; i < k; i += ET) Z[(size_t)i * r + j] *= inv;
      __syncthreads();
    }
  }
}

// sign rule on a wave-held vector: the largest-magnitude entry (lowest index on ties)
// is made positive; returns the factor
__device__ __forceinline__ double sign_factor(double best, int bidx, double at_best) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o);
    const int oi = __shfl_xor(bidx, o);
    const double ov = __shfl_xor(at_best, o);
    if (ob > best || (ob == best && oi < bidx)) {
      best = ob;
      bidx = oi;
      at_best = ov;
    }
  }
  return at_best < 0.0 ? -1.0 : 1.0;
}

// ---- phase 4c, packed path: x = Q z with each wave applying every reflector
//      (global hv rows) to its own vectors, then the sign rule
__device__ __forceinline__ void back_transform_wave(double* Z, int k, int r, const double* tau,
                                                    const double* __restrict__ hv, double* vecs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = wave; j < r; j += NW) {
    for (int jj = k - 3; jj >= 0; --jj) {
      const double tj = tau[jj];
      if (tj == 0.0) continue;
      const int r0 = jj + 1, n2 = k - r0;
      const double* v = hv + (int64_t)jj * k + r0;
      double s = 0.0;
      for (int i = lane; i < n2; i += 64) s = fma(v[i], Z[(size_t)(r0 + i) * r + j], s);
      s = wsum(s) * tj;
      for (int i = lane; i < n2; i += 64) Z[(size_t)(r0 + i) * r + j] -= s * v[i];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int j = wave; j < r; j += NW) {
    double best = -1.0, at = 0.0;
    int bidx = 0;
    for (int i = lane; i < k; i += 64) {
      const double z = Z[(size_t)i * r + j];
      if (fabs(z) > best) {
        best = fabs(z);
        bidx = i;
        at = z;
      }
    }
    const double sg = sign_factor(best, bidx, at);
    for (int i = lane; i < k; i += 64) vecs[(size_t)j * k + i] = sg * Z[(size_t)i * r + j];
  }
}

// ---- phase 4c, register path (k <= 64 ZR, r <= kStagedVectors): the vectors stay in the
//      registers of their wave (vector wave + NW t); the reflectors are staged
//      through LDS 32 at a time by the whole workgroup, so each is read from
//      global memory once.
constexpr int kStagedVectors = 64;  // vectors kept in registers by the staged back-transformation

template <int ZR>
__device__ __forceinline__ void back_transform_staged(const double* Z, int k, int r, const double* tau,
                                                      const double* __restrict__ hv, double* stage, double* vecs) {
  constexpr int MV = kStagedVectors / NW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nv = (r - wave + NW - 1) / NW;  // vectors of this wave
  double z[MV][ZR];
#pragma unroll
  for (int t = 0; t < MV; ++t) {
    const int j = wave + NW * t;
#pragma unroll
    for (int m = 0; m < ZR; ++m) {
      const int i = lane + 64 * m;
      z[t][m] = (j < r && i < k) ? Z[(size_t)i * r + j] : 0.0;
    }
  }
  __syncthreads();  // Z may share the staging area
  for (int top = k - 3; top >= 0; top -= 32) {
    const int lo = top >= 31 ? top - 31 : 0;
    for (int q = wave; q <= top - lo; q += NW) {
      const int jj = lo + q;
      for (int i = lane; i < k; i += 64) stage[q * k + i] = (i > jj) ? hv[(int64_t)jj * k + i] : 0.0;
    }
    __syncthreads();
    if (nv > 0) {
      for (int jj = top; jj >= lo; --jj) {
        const double tj = tau[jj];
        if (tj == 0.0) continue;
        const double* vr = stage + (jj - lo) * k;
        double v[ZR];
#pragma unroll
        for (int m = 0; m < ZR; ++m) {
          const int i = lane + 64 * m;
          v[m] = i < k ? vr[i] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < MV; ++t) {
          if (t < nv) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < ZR; ++m) s = fma(v[m], z[t][m], s);
            s = dpp_wave_sum(s) * tj;
#pragma unroll
            for (int m = 0; m < ZR; ++m) z[t][m] = fma(-s, v[m], z[t][m]);
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < MV; ++t) {
    if (t < nv) {
      const int j = wave + NW * t;
      double best = -1.0, at = 0.0;
      int bidx = 0;
#pragma unroll
      for (int m = 0; m < ZR; ++m) {
        const int i = lane + 64 * m;
        if (i < k && fabs(z[t][m]) > best) {
          best = fabs(z[t][m]);
          bidx = i;
          at = z[t][m];
        }
      }
      const double sg = sign_factor(best, bidx, at);
#pragma unroll
      for (int m = 0; m < ZR; ++m) {
        const int i = lane + 64 * m;
        if (i < k) vecs[(size_t)j * k + i] = sg * z[t][m];
      }
    }
  }
}

// Global scratch of one problem (doubles): packed triangle (packed path), the
// Householder vectors (row j = reflector j), 6 k small vectors (packed path),
// tau, ascending eigenvalues, tail sums, the inverse-iteration arrays when they do
// not fit in LDS, 64 doubles of phase clocks.
struct EigScratch {
  double* P;
  double* hv;
  double* small;
  double* tau;
  double* lam;
  double* tail;
  double* gz;
  double* clk;
};

__device__ __forceinline__ EigScratch carve(const EigJob& J) {
  const size_t K = (size_t)J.k;
  EigScratch c;
  double* sc = J.scratch;
  c.P = sc;
  sc += K * (K + 1) / 2;
  c.hv = sc;
  sc += K * K;
  c.small = sc;
  sc += 6 * K;
  c.tau = sc;
  sc += K;
  c.lam = sc;
  sc += K;
  c.tail = sc;
  sc += K + 1;
  c.gz = sc;
  c.clk = J.scratch + (eig_scratch_doubles_dev(J.k, J.rmax) - 64);
  return c;
}

#define HT_EIG_MARK(i) \
  if (threadIdx.x == 0) c.clk[i] = (double)wall_clock64();

// ---- fast path: Lanczos with a certified truncation decision ------------------------
// The leading eigenpairs are taken from a Krylov space of G (fully
// re-orthogonalised: two classical Gram-Schmidt passes per step) whenever the rank
// decision can be proven from it; otherwise the Householder path above runs.  With
// T_m = Q^T G Q (m x m tridiagonal, Ritz values theta_1 >= ... >= theta_m, s the
// last row of its eigenvector matrix) and beta the norm of the next Krylov
// direction:
//   * tail(r) = trace(G) - (lambda_1 + ... + lambda_r) is at most
//     trace(G) - (theta_1 + ... + theta_r), since Ritz sums bound eigenvalue sums
//     from below (Ky Fan); this gives the smallest r that surely meets the budget;
//   * the first j = r - 1 Ritz pairs couple to the rest of the space only through
//     beta, with norm E = beta |s_{1..j}|, and the rest has eigenvalues below
//     max(theta_{j+1}, trace(G) - trace(T_m)) + beta |s_{j+1..m}| (G is positive
//     semidefinite, so the unexplored part's largest eigenvalue is at most its
//     trace); with delta = theta_j minus that bound, lambda_i <= theta_i + E^2 /
//     delta for i <= j (quadratic residual bound of a 2 x 2 block partition), so
//     tail(j) > thr is proven when trace(G) - sum_{i<=j} theta_i - j E^2 / delta
//     exceeds it.
// Both comparisons keep a margin of 64 k eps trace(G) for rounding (E is taken
// twice as large), the kept Ritz values must be separated by more than
// 1e-10 theta_1 and each kept pair's residual beta |s_i| must stay below
// 1e-13 theta_1; otherwise the decision is left to the Householder path.
constexpr int kLzSteps = 64;   // Krylov dimension limit
constexpr int kLzMinK = 40;    // smaller problems go straight to the Householder path
constexpr int kLzLdsK = 224;   // the Krylov basis sits in LDS up to this k, beyond in global scratch
constexpr int kLzMaxK = 1024;  // larger problems go straight to the Householder path

typedef __attribute__((address_space(1))) const double cgdouble;

// steps at which the decision is checked (and at an invariant Krylov space)
__device__ __forceinline__ bool lz_check_at(int m) { return m >= 6 && (m - 6) % 4 == 0; }

constexpr int kLzPad = 72;  // length of the padded scaled copy of T_m

// The Sturm count of sturm_fast on a copy of the (padded) tridiagonal held in
// registers: d[i] the scaled diagonal, f[i] the squared scaled off-diagonal
// entry above row i (f[0] = 0); the pair is rescaled every eight steps.
template <int N>
__device__ __forceinline__ int sturm_regs(const double (&d)[N], const double (&f)[N], double x, bool& tiny) {
  double p1 = 1.0, p2 = 0.0;
  int cnt = 0;
  bool t = false;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double fl = DBL_MIN * fabs(p1);
    const double p = fma(d[i] - x, p1, -(f[i] * p2));
    t |= !(fabs(p) >= fl) | (p == 0.0);
    cnt += (__double2hiint(p) ^ __double2hiint(p1)) < 0 ? 1 : 0;
    p2 = p1;
    p1 = p;
    if ((i & 7) == 0) {
      const int ex = __builtin_amdgcn_frexp_exp(p1);
      p1 = __builtin_amdgcn_ldexp(p1, -ex);
      p2 = __builtin_amdgcn_ldexp(p2, -ex);
    }
  }
  tiny = t;
  return cnt;
}

// every eigenvalue of the (padded, length N) scaled tridiagonal, descending, the
// counts on register copies
template <int N>
__device__ __forceinline__ void tridiag_values_regs(const double* dn, const double* e2n, int m, const double* sh,
                                                    double* top) {
  constexpr int T = 16;
  const int tid = threadIdx.x, lane = tid & 63, slot = tid / T, u = tid % T, gbase = lane - (lane % T);
  double d[N], f[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    d[i] = dn[i];
    f[i] = i ? e2n[i - 1] : 0.0;
  }
  for (int m0 = 0; m0 < m; m0 += ET / T) {
    const int q = m0 + slot;
    if (q < m) {
      const double v = multisect_by<T>([&](double x, bool& tiny) { return sturm_regs<N>(d, f, x, tiny); },
                                       [&](double x) { return sturm_scaled(dn, e2n, N, x); }, sh, m - 1 - q, u,
                                       gbase);
      if (u == 0) top[q] = v;
    }
  }
}

// every eigenvalue of an m x m tridiagonal (m <= 64), descending.  The scaled copy
// (dn, e2n) is padded to M entries with decoupled diagonal entries 4 > |T| /
// scale, which add no Sturm count below any point of the search interval; up to
// 33 entries the counts run on register copies, beyond in the prefetching blocks
// of eight of sturm_fast (M = 1 + 8 ceil((m - 1) / 8)).
__device__ __forceinline__ void tridiag_values(double* dn, double* e2n, int m, const double* sh, double* top) {
  constexpr int T = 16;
  const int tid = threadIdx.x, lane = tid & 63, slot = tid / T, u = tid % T, gbase = lane - (lane % T);
  const int M = m <= 17 ? 17 : m <= 33 ? 33 : 1 + 8 * ((m + 6) / 8);
  for (int i = m + tid; i < M; i += ET) {
    dn[i] = 4.0;
    e2n[i] = 0.0;
  }
  __syncthreads();
  if (m <= 17) {
    tridiag_values_regs<17>(dn, e2n, m, sh, top);
  } else if (m <= 33) {
    tridiag_values_regs<33>(dn, e2n, m, sh, top);
  } else {
    for (int m0 = 0; m0 < m; m0 += ET / T) {
      const int q = m0 + slot;
      if (q < m) {
        const double v = multisect<T>(dn, e2n, M, sh, m - 1 - q, u, gbase);
        if (u == 0) top[q] = v;
      }
    }
  }
  __syncthreads();
}

// Orthonormalises the r columns of the m x r block Z (Z[i r + j], m <= 64) in
// order with two classical Gram-Schmidt passes, on one wave (lane = row).
__device__ __forceinline__ void cgs2_wave(double* Z, int m, int r) {
  const int lane = threadIdx.x & 63;
  const bool row = lane < m;
  for (int j = 0; j < r; ++j) {
    double z = row ? Z[(size_t)lane * r + j] : 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      double acc = 0.0;
      for (int t = 0; t < j; ++t) {
        const double zt = row ? Z[(size_t)lane * r + t] : 0.0;
        acc = fma(zt, dpp_wave_sum(zt * z), acc);
      }
      z -= acc;
    }
    const double nrm = sqrt(dpp_wave_sum(z * z));
    z = nrm > 0.0 ? z / nrm : 0.0;
    if (row) Z[(size_t)lane * r + j] = z;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Buffers of the Lanczos solve used by the certification.
struct LzView {
  double* Q;
  double* al;
  double* be;
  double* e2;
  double* dn;
  double* e2n;
  double* top;
  double* pb;
  double* free_lds;
  int64_t free_cap;
};

// The check at step m (kept out of line, so the solve's own registers need not
// survive its code): returns true when the decision is proven and written.
__device__ __noinline__ bool lz_certify(const EigJob& J, const LzView& v, int m, double beta, double tr, double guard,
                                        double* sh, double* red, int* ctl) {
  const EigScratch c = carve(J);
  const int k = J.k, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Q = v.Q;
  double* al = v.al;
  double* be = v.be;
  double* e2 = v.e2;
  double* dn = v.dn;
  double* e2n = v.e2n;
  double* top = v.top;
  double* pb = v.pb;
  double* free_lds = v.free_lds;
  const int64_t free_cap = v.free_cap;
  // T_m: diagonal al, off-diagonal be[0 .. m-2]; be[m-1] is the coupling beta
  finish_tridiag(m, al, be, e2, dn, e2n, sh);
  tridiag_values(dn, e2n, m, sh, top);
  if (tid == 0) {
    double tsum = 0.0;
    for (int i = 0; i < m; ++i) tsum += al[i];
    const int rlim = min(J.rmax, m);
    double S = 0.0;
    int rh = -1;
    for (int r = 0; r <= rlim; ++r) {
      if (r >= J.rmin && tr - S <= J.thr - guard) {
        rh = r;
        break;
      }
      if (r < rlim) S += top[r];
    }
    ctl[0] = rh;
    sh[4] = tsum;
  }
  __syncthreads();
  const int rh = ctl[0];
  bool done = false;
  if (rh > 0 && tid == 0) {
    // the certificate without the eigenvector components, with E = 0: when even
    // this fails (or the kept values are not separated) the check stops here
    const double th1 = top[0];
    bool ok = th1 > 0.0;
    const int nv = min(rh + 1, m);
    for (int i = 0; i + 1 < nv; ++i) ok = ok && (top[i] - top[i + 1] > 1e-10 * th1);
    const int jj = rh - 1;
    if (ok && jj >= J.rmin && jj > 0) {
      double sj = 0.0;
      for (int i = 0; i < jj; ++i) sj += top[i];
      const double tperp = fmax(tr - sh[4], 0.0);
      ok = top[jj - 1] > fmax(jj < m ? top[jj] : 0.0, tperp) && tr - sj > J.thr + guard;
    }
    ctl[1] = ok ? 1 : 0;
  }
  __syncthreads();
  if (rh > 0 && !ctl[1]) return false;
  if (rh == 0) {
    if (tid == 0) {
      *J.rank = 0;
      *J.tail = tr;
    }
    done = true;
  } else if (rh > 0) {
    double* Z = (int64_t)4 * m * rh <= free_cap ? free_lds : c.gz;
    inverse_iteration(Z, m, rh, top, al, be, sh[2]);  // Z[i rh + j], ends with a barrier
    if (tid < 64 && lane < rh) {
      double n2 = 0.0;
      for (int i = 0; i < m; ++i) n2 = fma(Z[(size_t)i * rh + lane], Z[(size_t)i * rh + lane], n2);
      pb[lane] = Z[(size_t)(m - 1) * rh + lane] / sqrt(n2);
    }
    __syncthreads();
    if (tid == 0) {
      const double th1 = top[0];
      bool ok = th1 > 0.0;
      const int nv = min(rh + 1, m);
      for (int i = 0; i + 1 < nv; ++i) ok = ok && (top[i] - top[i + 1] > 1e-10 * th1);
      for (int i = 0; i < rh; ++i) ok = ok && (beta * fabs(pb[i]) <= 1e-13 * th1);
      const int jj = rh - 1;
      if (ok && jj >= J.rmin) {
        double lb = tr;
        if (jj > 0) {
          double s2 = 0.0, sj = 0.0;
          for (int i = 0; i < jj; ++i) {
            s2 = fma(pb[i], pb[i], s2);
            sj += top[i];
          }
          const double e2b = 4.0 * beta * beta * s2;
          const double tperp = fmax(tr - sh[4], 0.0);
          const double lam_c = fmax(jj < m ? top[jj] : 0.0, tperp) + beta * sqrt(fmax(0.0, 1.0 - s2));
          const double dl = top[jj - 1] - lam_c;
          lb = dl > 0.0 ? tr - sj - (double)jj * e2b / dl : -DBL_MAX;
        }
        ok = lb > J.thr + guard;
      }
      ctl[1] = ok ? 1 : 0;
    }
    __syncthreads();
    if (ctl[1]) {
      if (wave == 0) cgs2_wave(Z, m, rh);
      __syncthreads();
      // Ritz vectors Q z_j, one wave per vector, then the sign rule
      for (int j = wave; j < rh; j += NW) {
        double best = -1.0, at = 0.0;
        int bidx = 0;
        for (int i = lane; i < k; i += 64) {
          double y = 0.0;
          for (int q = 0; q < m; ++q) y = fma(Q[(size_t)q * k + i], Z[(size_t)q * rh + j], y);
          J.vecs[(size_t)j * k + i] = y;
          if (fabs(y) > best) {
            best = fabs(y);
            bidx = i;
            at = y;
          }
        }
        const double sg = sign_factor(best, bidx, at);
        if (sg < 0.0)
          for (int i = lane; i < k; i += 64) J.vecs[(size_t)j * k + i] = -J.vecs[(size_t)j * k + i];
      }
      for (int i = tid; i < rh; i += ET) J.evals[i] = top[i];
      if (tid == 0) {
        double S = 0.0;
        for (int i = 0; i < rh; ++i) S += top[i];
        *J.rank = rh;
        *J.tail = fmax(tr - S, 0.0);
      }
      done = true;
    }
  }
  return done;
}

// Returns true when the decision and its eigenpairs are written; false leaves the
// outputs untouched.  The last 64 doubles of the scratch record the attempt:
// [8] = steps (negative when the decision was not proven), [9] = checks.
// MV selects the product G q: 0 (k <= 128) G stays in registers, thread (i, h)
// holding column i's rows 32 h .. 32 h + 31 (G is symmetric, so column i serves
// row i); 1 (k <= kLzLdsK) the tiles of the register Householder path that meet
// the lower triangle stay in registers, row sums over each half-wave by DPP and
// the transposed sums of the strictly lower tiles per wave through LDS; 2
// (k <= kLzMaxK) whole columns streamed from the cache (coalesced), the Krylov
// basis in global scratch.
template <int MV>
__device__ __noinline__ bool lanczos_solve(const EigJob& J, double* lds, double* sh, double* red, int* ctl) {
  constexpr bool QL = MV < 2;
  constexpr int WS = QL ? 4 : 16;  // entries of w per lane in the projections (k <= 64 WS)
  const EigScratch c = carve(J);
  const int k = J.k, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  cgdouble* G = reinterpret_cast<cgdouble*>(reinterpret_cast<uintptr_t>(J.G));
  const int mlim = min(k, kLzSteps);
  double* Q = QL ? lds : c.hv;  // Krylov vector v at Q + v k
  double* wv = lds + (QL ? (kLzSteps + 1) * k : 0);
  double* qv = wv + k;      // the scaled vector the product reads (MV == 2)
  double* part = qv + k;    // partial sums of the product (2048 >= 16 TA + NW 32 TB)
  double* hc = part + 2048;  // projection coefficients
  double* al = hc + kLzSteps;
  double* be = al + kLzSteps;
  double* e2 = be + kLzSteps;
  double* dn = e2 + kLzSteps;
  double* e2n = dn + kLzPad;
  double* top = e2n + kLzPad;
  double* pb = top + kLzSteps;
  double* lzred = pb + kLzSteps;  // two alternating NW-entry reduction buffers
  double* free_lds = lzred + 2 * NW;
  const int64_t free_cap = kLdsDoubles - (int64_t)(free_lds - lds);

  double t = 0.0;
  for (int i = tid; i < k; i += ET) t += G[(size_t)i * k + i];
  const double tr = bsum(t, red);
  if (!(tr > 0.0) || !(tr < DBL_MAX)) return false;
  const double guard = 64.0 * k * DBL_EPSILON * tr;

  // MV == 0: rows 32 h .. 32 h + 31 of column i; MV == 1: entry (16 a + trow,
  // 32 b + tc) of every stored tile (a, b), b <= a / 2; kept for the whole solve
  constexpr int TA = kRegRowTiles, TB = (TA + 1) / 2;
  double g[MV == 0 ? 32 : MV == 1 ? tile_base(TA) : 1];
  const int trow = tid >> 5, tc = tid & 31;
  if constexpr (MV == 0) {
    const int i = tid & 127, h = tid >> 7;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int l = 32 * h + q;
      g[q] = (i < k && l < k) ? G[(size_t)l * k + i] : 0.0;
    }
  } else if constexpr (MV == 1) {
#pragma unroll
    for (int a = 0; a < TA; ++a) {
#pragma unroll
      for (int b = 0; b <= a / 2; ++b) {
        const int i = 16 * a + trow, l = 32 * b + tc;
        g[tile_base(a) + b] = (i < k && l < k) ? G[(size_t)i * k + l] : 0.0;
      }
    }
  }

  // fixed pseudo-random start
  double loc = 0.0;
  for (int i = tid; i < k; i += ET) {
    const double v = start_entry(kMaxEigJobs + 7, i) - 1.0;
    wv[i] = v;
    loc = fma(v, v, loc);
  }
  double scl = 1.0 / sqrt(bsum(loc, red));  // q_{m-1} = scl w at the top of step m

  int checks = 0;
  for (int m = 1; m <= mlim; ++m) {
    // ---- w <- G q_{m-1}, and q_{m-1} into the basis
    if constexpr (MV == 2) {
      for (int i = tid; i < k; i += ET) {
        const double v = wv[i] * scl;
        qv[i] = v;
        Q[(size_t)(m - 1) * k + i] = v;
      }
      __syncthreads();
      for (int i = tid; i < k; i += ET) {
        double a0 = 0.0, a1 = 0.0;
        int l = 0;
        for (; l + 16 <= k; l += 16) {
          double gv[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) gv[q] = G[(size_t)(l + q) * k + i];
#pragma unroll
          for (int q = 0; q < 16; q += 2) {
            a0 = fma(gv[q], qv[l + q], a0);
            a1 = fma(gv[q + 1], qv[l + q + 1], a1);
          }
        }
        for (; l < k; ++l) a0 = fma(G[(size_t)l * k + i], qv[l], a0);
        wv[i] = a0 + a1;
      }
      __syncthreads();
    } else {
      if constexpr (MV == 0) {
        const int h = tid >> 7;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int q = 0; q < 32; q += 2) {
          a0 = fma(g[q], wv[min(32 * h + q, k - 1)], a0);
          a1 = fma(g[q + 1], wv[min(32 * h + q + 1, k - 1)], a1);
        }
        part[tid] = (a0 + a1) * scl;
      } else {
        // row sums of the stored tiles (each row's lanes are one half-wave) and the
        // transposed sums of the strictly lower tiles (b < a / 2), per wave
        double xr[TA], xc[TB];
#pragma unroll
        for (int a = 0; a < TA; ++a) xr[a] = 16 * a + trow < k ? wv[16 * a + trow] : 0.0;
#pragma unroll
        for (int b = 0; b < TB; ++b) xc[b] = 32 * b + tc < k ? wv[32 * b + tc] : 0.0;
        double colacc[TB];
#pragma unroll
        for (int b = 0; b < TB; ++b) colacc[b] = 0.0;
#pragma unroll
        for (int a = 0; a < TA; ++a) {
          double racc = 0.0;
#pragma unroll
          for (int b = 0; b <= a / 2; ++b) {
            racc = fma(g[tile_base(a) + b], xc[b], racc);
            if (b < a / 2) colacc[b] = fma(g[tile_base(a) + b], xr[a], colacc[b]);
          }
          racc = dpp_half_sum(racc);
          if ((lane & 31) == 31) part[16 * a + trow] = racc * scl;
        }
#pragma unroll
        for (int b = 0; b < TB; ++b) {
          const double cv = colacc[b] + __shfl_xor(colacc[b], 32);
          if (lane < 32) part[16 * TA + wave * (32 * TB) + 32 * b + tc] = cv * scl;
        }
      }
      for (int i = tid; i < k; i += ET) Q[(size_t)(m - 1) * k + i] = wv[i] * scl;
      __syncthreads();
      if (tid < k) {
        if (MV == 0) {
          wv[tid] = (part[tid] + part[128 + tid]) + (part[256 + tid] + part[384 + tid]);
        } else {
          double c = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) c += part[16 * TA + w * (32 * TB) + tid];
          wv[tid] = part[tid] + c;
        }
      }
      __syncthreads();
    }
    // ---- two classical Gram-Schmidt passes against q_0 .. q_{m-1}, one wave per
    //      basis vector; the coefficients on q_{m-1} add up to T's diagonal entry
    double beta = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      double wr[WS];
#pragma unroll
      for (int s = 0; s < WS; ++s) {
        const int i = lane + 64 * s;
        wr[s] = i < k ? wv[i] : 0.0;
      }
      for (int cc = wave; cc < m; cc += NW) {
        const double* qc = Q + (size_t)cc * k;
        double a = 0.0;
#pragma unroll
        for (int s = 0; s < WS; ++s) {
          const int i = lane + 64 * s;
          if (i < k) a = fma(qc[i], wr[s], a);
        }
        a = dpp_wave_sum(a);
        if (lane == 0) hc[cc] = a;
      }
      __syncthreads();
      if (tid == 0) al[m - 1] = pass ? al[m - 1] + hc[m - 1] : hc[m - 1];
      double l2 = 0.0;
      for (int i = tid; i < k; i += ET) {
        double v0 = wv[i], v1 = 0.0;
        int cc = 0;
        for (; cc + 2 <= m; cc += 2) {
          v0 = fma(-Q[(size_t)cc * k + i], hc[cc], v0);
          v1 = fma(-Q[(size_t)(cc + 1) * k + i], hc[cc + 1], v1);
        }
        if (cc < m) v0 = fma(-Q[(size_t)cc * k + i], hc[cc], v0);
        const double v = v0 + v1;
        wv[i] = v;
        l2 = fma(v, v, l2);
      }
      if (pass == 0) {
        __syncthreads();
      } else {
        // ||w||: each step alternates between two buffers, so the barriers of the
        // step in between keep them apart
        const double ws = dpp_wave_sum(l2);
        double* rb = lzred + (m & 1) * NW;
        if (lane == 0) rb[wave] = ws;
        __syncthreads();
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) tot += rb[w];
        beta = sqrt(tot);
      }
    }
    const bool brk = !(beta > 1e-14 * tr);  // the Krylov space is (numerically) invariant
    if (tid == 0) be[m - 1] = beta;
    if (brk || m == mlim || lz_check_at(m)) {
      __syncthreads();
      ++checks;
      const LzView v{Q, al, be, e2, dn, e2n, top, pb, free_lds, free_cap};
      const bool done = lz_certify(J, v, m, beta, tr, guard, sh, red, ctl);
      if (done || brk || m == mlim) {
        if (tid == 0) {
          c.clk[8] = done ? m : -m;
          c.clk[9] = checks;
        }
        return done;
      }
    }
    scl = 1.0 / beta;
  }
  return false;
}

// LDS of the register path (doubles): d, e, e2, tau, dn, e2n, top, xb, cb, vbuf,
// pbuf (256 each), then one region shared by the row and column partials (phase
// 1), the inverse-iteration arrays (4a, 4b) and the reflector staging (4c).
constexpr int kRegSmall = 11 * 256;

// Phase 1 of the register path, the only part that depends on the tile count: one
// instantiation per tile count, each a compact loop (the code of all phases
// together would not fit the instruction cache).
template <int TA>
__device__ __noinline__ void phase1_reg(const EigJob& J, double* lds, double* sh) {
  double* d = lds;
  double* e = d + 256;
  double* tau = e + 512;
  double* xb = lds + 7 * 256;
  double* cb = xb + 256;
  double* vbuf = cb + 256;
  double* pbuf = vbuf + 256;
  double* region = lds + kRegSmall;
  const EigScratch c = carve(J);
  tridiag_reg<TA>(J.G, J.k, xb, cb, vbuf, pbuf, region, region + 32 * (16 * TA + 1), d, e, tau, c.hv, sh + 4);
}

// Phases 2 - 4 of the register path (k <= 16 kRegRowTiles), after phase1_reg.
__device__ __forceinline__ void solve_reg_tail(const EigJob& J, double* lds, double* sh, int* s_rank, double* red) {
  constexpr int ZR = (16 * kRegRowTiles + 63) / 64;
  const EigScratch c = carve(J);
  const int k = J.k, tid = threadIdx.x;
  double* d = lds;
  double* e = d + 256;
  double* e2 = e + 256;
  double* tau = e2 + 256;
  double* dn = tau + 256;
  double* e2n = dn + 256;
  double* top = e2n + 256;
  double* pbuf = lds + 10 * 256;
  double* region = lds + kRegSmall;
  const int64_t region_cap = kLdsDoubles - kRegSmall;

  finish_tridiag(k, d, e, e2, dn, e2n, sh);
  HT_EIG_MARK(1)
  const int found = top_eigen_rank(dn, e2n, d, k, sh, J.rmin, J.rmax, J.thr, top, J.rank, J.tail, s_rank, sh + 6);
  for (int i = tid; i < found; i += ET) J.evals[i] = top[i];
  const int r = *s_rank;
  HT_EIG_MARK(2)
  if (r == 0) return;
  if ((int64_t)4 * k * r <= region_cap) {
    inverse_iteration(region, k, r, top, d, e, sh[2]);
    HT_EIG_MARK(3)
    cgs2_columns(region, k, r, pbuf, red);
    HT_EIG_MARK(4)
    if (r <= kStagedVectors)
      back_transform_staged<ZR>(region, k, r, tau, c.hv, region, J.vecs);
    else
      back_transform_wave(region, k, r, tau, c.hv, J.vecs);
  } else {
    inverse_iteration(c.gz, k, r, top, d, e, sh[2]);
    HT_EIG_MARK(3)
    cgs2_columns(c.gz, k, r, pbuf, red);
    HT_EIG_MARK(4)
    if (r <= kStagedVectors)
      back_transform_staged<ZR>(c.gz, k, r, tau, c.hv, region, J.vecs);
    else
      back_transform_wave(c.gz, k, r, tau, c.hv, J.vecs);
  }
  HT_EIG_MARK(6)
}

// One problem on the packed path.  SMALL_LDS: the 6 k vectors (d, e, e2 and three
// work vectors) live in LDS (k <= kSmallMax), else in global scratch; the storage
// choice is a compile-time one so every access keeps a single address space.
template <bool SMALL_LDS>
__device__ __forceinline__ void solve_packed(const EigJob& J, double* lds, double* sh, int* s_rank, double* red) {
  const EigScratch c = carve(J);
  const int k = J.k, tid = threadIdx.x;
  double* small = SMALL_LDS ? lds : c.small;
  double* d = small;
  double* e = d + k;
  double* e2 = e + k;
  double* vb = e2 + k;
  double* pb = vb + k;
  double* wb = pb + k;
  double* work = lds + (SMALL_LDS ? 6 * k : 0);
  const int64_t work_cap = kLdsDoubles - (SMALL_LDS ? 6 * k : 0);
  const int64_t npk = (int64_t)k * (k + 1) / 2;

  if (npk <= work_cap)
    tridiagonalise_packed(work, J.G, k, vb, pb, wb, red, d, e, c.tau, c.hv);
  else
    tridiagonalise_packed(c.P, J.G, k, vb, pb, wb, red, d, e, c.tau, c.hv);
  // vb and wb are free again: they hold the scaled copy for the Sturm counts
  finish_tridiag(k, d, e, e2, vb, wb, sh);
  HT_EIG_MARK(1)
  const int found = top_eigen_rank(vb, wb, d, k, sh, J.rmin, J.rmax, J.thr, c.lam, J.rank, J.tail, s_rank, sh + 6);
  for (int i = tid; i < found; i += ET) J.evals[i] = c.lam[i];
  const int r = *s_rank;
  HT_EIG_MARK(2)
  if (r == 0) return;
  if ((int64_t)4 * k * r <= work_cap) {
    inverse_iteration(work, k, r, c.lam, d, e, sh[2]);
    HT_EIG_MARK(3)
    cgs2_columns(work, k, r, pb, red);
    HT_EIG_MARK(4)
    back_transform_wave(work, k, r, c.tau, c.hv, J.vecs);
  } else {
    inverse_iteration(c.gz, k, r, c.lam, d, e, sh[2]);
    HT_EIG_MARK(3)
    cgs2_columns(c.gz, k, r, pb, red);
    HT_EIG_MARK(4)
    back_transform_wave(c.gz, k, r, c.tau, c.hv, J.vecs);
  }
  HT_EIG_MARK(6)
}

template <bool SMALL_LDS>
__global__ __launch_bounds__(ET) void eig_trunc_kernel(EigBatch batch) {
  const EigJob J = batch.j[blockIdx.x];
  const EigScratch c = carve(J);
  HT_EIG_MARK(0)
  extern __shared__ double lds[];
  __shared__ double red[NW];
  __shared__ double sh[8];
  __shared__ int s_rank;
  __shared__ int lz_ctl[2];
  const int k = J.k, tid = threadIdx.x;
  if (tid == 0) c.clk[8] = 0.0;

  // all the energy already within the budget and no rank floor: the rule keeps
  // nothing (tail(0) = trace <= thr), so the decomposition is not needed
  if (J.rmin == 0) {
    double tr = 0.0;
    for (int i = tid; i < k; i += ET) tr += J.G[(int64_t)i * k + i];
    tr = bsum(tr, red);
    if (tr <= J.thr) {
      if (tid == 0) {
        *J.rank = 0;
        *J.tail = tr;
      }
      return;
    }
  }
  if (J.method != kEigHouseholder && k >= kLzMinK && k <= kLzMaxK && J.rmax > 0) {
    const bool done = k <= 128       ? lanczos_solve<0>(J, lds, sh, red, lz_ctl)
                      : k <= kLzLdsK ? lanczos_solve<1>(J, lds, sh, red, lz_ctl)
                                     : lanczos_solve<2>(J, lds, sh, red, lz_ctl);
    if (done) return;
    if (J.method == kEigLanczos) {
      if (tid == 0) *J.rank = -1;
      return;
    }
    __syncthreads();
  }
  if constexpr (SMALL_LDS) {
    if (k <= 16 * kRegRowTiles) {
      switch ((k + 15) >> 4) {
        case 1: phase1_reg<1>(J, lds, sh); break;
        case 2: phase1_reg<2>(J, lds, sh); break;
        case 3: phase1_reg<3>(J, lds, sh); break;
        case 4: phase1_reg<4>(J, lds, sh); break;
        case 5: phase1_reg<5>(J, lds, sh); break;
        case 6: phase1_reg<6>(J, lds, sh); break;
        case 7: phase1_reg<7>(J, lds, sh); break;
        case 8: phase1_reg<8>(J, lds, sh); break;
        case 9: phase1_reg<9>(J, lds, sh); break;
        case 10: phase1_reg<10>(J, lds, sh); break;
        case 11: phase1_reg<11>(J, lds, sh); break;
        case 12: phase1_reg<12>(J, lds, sh); break;
        case 13: phase1_reg<13>(J, lds, sh); break;
        case 14: phase1_reg<14>(J, lds, sh); break;
        default: break;
      }
      solve_reg_tail(J, lds, sh, &s_rank, red);
      return;
    }
  }
  solve_packed<SMALL_LDS>(J, lds, sh, &s_rank, red);
}
#undef HT_EIG_MARK

}  // namespace

namespace {

struct AuxBatch {
  AuxJob j[kMaxEigJobs];
};

// trace(G) in a fixed order (strided partial sums, DPP-free wave tree, then the
// four waves in order) and the smallest kept eigenvalue of one decision.
__global__ __launch_bounds__(256) void decision_aux_kernel(AuxBatch b) {
  const AuxJob J = b.j[blockIdx.x];
  __shared__ double red[4];
  double tr = 0.0;
  for (int i = threadIdx.x; i < J.k; i += 256) tr += J.G[(int64_t)i * J.k + i];
  for (int off = 32; off > 0; off >>= 1) tr += __shfl_down(tr, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tr;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int r = *J.rank;
    J.out[0] = (red[0] + red[1]) + (red[2] + red[3]);
    J.out[1] = r >= 1 ? J.evals[r - 1] : 0.0;
  }
}

}  // namespace

void decision_aux(const AuxJob* jobs, int count, hipStream_t s) {
  for (int b0 = 0; b0 < count; b0 += kMaxEigJobs) {
    const int n = std::min(kMaxEigJobs, count - b0);
    AuxBatch b;
    for (int i = 0; i < n; ++i) b.j[i] = jobs[b0 + i];
    ProfScope prof(KKind::Layout, s, 0.0, 0.0);
    decision_aux_kernel<<<n, 256, 0, s>>>(b);
  }
}

size_t eig_scratch_doubles(int k, int rmax) {
  const size_t K = (size_t)k;
  return K * (K + 1) / 2 + K * K + 6 * K + K + K + (K + 1) + 4 * K * (size_t)std::max(rmax, 1) + 64;
}

void eig_trunc(const EigJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return;
  EigBatch b;
  for (int i = 0; i < count; ++i) b.j[i] = jobs[i];
  int kmax = 0;
  for (int i = 0; i < count; ++i) kmax = std::max(kmax, jobs[i].k);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&eig_trunc_kernel<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsDoubles * (int)sizeof(double));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&eig_trunc_kernel<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsDoubles * (int)sizeof(double));
    attr_set = true;
  }
  ProfScope prof(KKind::Eig, s, 0.0, 0.0);
  if (kmax <= kSmallMax)
    eig_trunc_kernel<true><<<count, ET, kLdsDoubles * sizeof(double), s>>>(b);
  else
    eig_trunc_kernel<false><<<count, ET, kLdsDoubles * sizeof(double), s>>>(b);
}

}  // namespace ht
