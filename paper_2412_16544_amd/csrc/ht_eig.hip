// FP64 symmetric eigen-decomposition with the error-truncation rule, on gfx950.
//
// The truncated SVD of an unfolding M (Eq. ht_leaf_svd, Eq. svd_on_residual) is
// taken from the Gram matrix G = M M^T: sigma_i^2 = lambda_i(G) and the left
// singular vectors are G's eigenvectors.  One workgroup solves one k x k problem:
//
//   1. Householder reduction G = Q T Q^T to tridiagonal T.  The lower triangle
//      is kept packed in LDS when it fits (k <= ~190), else in global memory;
//   2. every eigenvalue of T by multisection on Sturm counts (several lanes of a
//      wave per eigenvalue);
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

constexpr int ET = 1024;
constexpr int NW = ET / 64;
constexpr int kLdsDoubles = 19968;  // 156 KiB of dynamic LDS per workgroup
constexpr int kSmallMax = 1024;     // the 6k work vectors live in LDS up to this k

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

// sum over each aligned group of 4 lanes, returned to the 4 lanes
__device__ __forceinline__ double dpp_quad_sum(double v) {
  v += dpp_mov<0xB1, 0xf>(v);  // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E, 0xf>(v);  // quad_perm [2,3,0,1]
  return v;
}

__device__ __forceinline__ double wsum(double v) { return dpp_wave_sum(v); }

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

// 1/q to full double precision: hardware reciprocal refined by two Newton steps
__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// number of eigenvalues of T (diag d, squared off-diagonal e2) below x
__device__ int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int k, double x,
                           double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < k; ++i) {
    q = (d[i] - x) - e2[i - 1] * recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
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
                                           double* d, double* e, double* tau, double* hv, double* clk) {
  const int tid = threadIdx.x;
#define HT_STEP_MARK(i) \
  if (j == 10 && tid == 0) clk[8 + (i)] = (double)wall_clock64();
  HT_STEP_MARK(0)
  const int r0 = j + 1, n2 = k - r0;
  double loc = 0.0;
  for (int i = 1 + tid; i < n2; i += ET) {
    const double x = P[pk(r0 + i, j)];
    loc = fma(x, x, loc);
  }
  const double xn2 = bsum(loc, red);
  HT_STEP_MARK(1)
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
  HT_STEP_MARK(2)
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
    HT_STEP_MARK(3)
    double loc2 = 0.0;
    for (int i = tid; i < n2; i += ET) loc2 = fma(pb[i], vb[i], loc2);
    const double kk = -0.5 * tj * bsum(loc2, red);
    for (int i = tid; i < n2; i += ET) wb[i] = fma(kk, vb[i], pb[i]);
    __syncthreads();
    HT_STEP_MARK(4)
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
  HT_STEP_MARK(5)
#undef HT_STEP_MARK
}

// Phase 1: packed copy of G's lower triangle into P, Householder steps, then the
// tridiagonal (d, e, e2), its Gershgorin interval and the pivot floor.
__device__ __forceinline__ void tridiagonalise(double* P, const double* __restrict__ G, int k, double* vb, double* pb,
                                               double* wb, double* red, double* d, double* e, double* e2,
                                               double* tau, double* hv, double* s_gl, double* s_gu,
                                               double* s_pivmin, double* s_tnorm, double* clk) {
  const int tid = threadIdx.x;
  const int npk = k * (k + 1) / 2;
  for (int q = tid; q < npk; q += ET) {
    const int a = prow(q);
    const int b = q - a * (a + 1) / 2;
    P[q] = G[(int64_t)a * k + b];
  }
  __syncthreads();
  for (int j = 0; j + 2 < k; ++j) house_step(P, k, j, vb, pb, wb, red, d, e, tau, hv, clk);
  if (tid == 0) {
    if (k >= 2) {
      d[k - 2] = P[pk(k - 2, k - 2)];
      e[k - 2] = P[pk(k - 1, k - 2)];
      tau[k - 2] = 0.0;
    }
    d[k - 1] = P[pk(k - 1, k - 1)];
    e[k - 1] = 0.0;
    tau[k - 1] = 0.0;
    double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
    for (int i = 0; i < k; ++i) {
      const double off = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < k ? fabs(e[i]) : 0.0);
      gl = fmin(gl, d[i] - off);
      gu = fmax(gu, d[i] + off);
      e2[i] = (i + 1 < k) ? e[i] * e[i] : 0.0;
      emax2 = fmax(emax2, e2[i]);
    }
    const double tn = fmax(fabs(gl), fabs(gu));
    *s_tnorm = tn;
    *s_pivmin = DBL_MIN * fmax(1.0, emax2);
    *s_gl = gl - 2.2e-16 * tn - *s_pivmin;
    *s_gu = gu + 2.2e-16 * tn + *s_pivmin;
  }
  __syncthreads();
}

// Phase 4: the r leading eigenvectors of T (ascending eigenvalues lam), mapped
// back with the reflectors in hv and sign-normalised into vecs (k x r).  Z holds
// 4 k r doubles; entry (i, j) of a work array at i * r + j.
__device__ __forceinline__ void eigenvectors(double* Z, int k, int r, const double* lam, const double* d,
                                             const double* e, double* pb, double* red, const double* tau,
                                             const double* hv, double* vecs, double tnorm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ---- 4a. inverse iteration, one thread per vector; entry (i, j) at i * r + j
  double* U0 = Z + (size_t)k * r;
  double* U1 = U0 + (size_t)k * r;
  double* U2 = U1 + (size_t)k * r;
  {
    const double tiny = fmax(2.2e-16 * tnorm, DBL_MIN);
    for (int j = tid; j < r; j += ET) {
      const double lm = lam[k - 1 - j];
      for (int i = 0; i < k; ++i) Z[(size_t)i * r + j] = start_entry(j, i);
      for (int it = 0; it < 3; ++it) {
        // forward: factor T - lm I row by row with partial pivoting, apply to the rhs
        double u0 = d[0] - lm, u1 = (k > 1) ? e[0] : 0.0, u2 = 0.0;
        double bi = Z[j];
        for (int i = 0; i + 1 < k; ++i) {
          const double l0 = e[i], l1 = d[i + 1] - lm, l2 = (i + 2 < k) ? e[i + 1] : 0.0;
          double bn = Z[(size_t)(i + 1) * r + j];
          double nu0, nu1;
          if (fabs(u0) >= fabs(l0)) {
            if (u0 == 0.0) u0 = tiny;
            const double mlt = l0 / u0;
            U0[(size_t)i * r + j] = u0;
            U1[(size_t)i * r + j] = u1;
            U2[(size_t)i * r + j] = u2;
            Z[(size_t)i * r + j] = bi;
            nu0 = l1 - mlt * u1;
            nu1 = l2 - mlt * u2;
            bn = bn - mlt * bi;
          } else {
            const double mlt = u0 / l0;
            U0[(size_t)i * r + j] = l0;
            U1[(size_t)i * r + j] = l1;
            U2[(size_t)i * r + j] = l2;
            Z[(size_t)i * r + j] = bn;
            nu0 = u1 - mlt * l1;
            nu1 = u2 - mlt * l2;
            bn = bi - mlt * bn;
          }
          u0 = nu0;
          u1 = nu1;
          u2 = 0.0;
          bi = bn;
        }
        if (fabs(u0) < tiny) u0 = (u0 < 0.0) ? -tiny : tiny;
        // backward substitution, the two previous unknowns kept in registers
        double x1 = bi / u0, x2 = 0.0, mx = fabs(x1);
        Z[(size_t)(k - 1) * r + j] = x1;
        for (int i = k - 2; i >= 0; --i) {
          double piv = U0[(size_t)i * r + j];
          if (fabs(piv) < tiny) piv = (piv < 0.0) ? -tiny : tiny;
          const double x = (Z[(size_t)i * r + j] - U1[(size_t)i * r + j] * x1 - U2[(size_t)i * r + j] * x2) / piv;
          Z[(size_t)i * r + j] = x;
          x2 = x1;
          x1 = x;
          mx = fmax(mx, fabs(x));
        }
        const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
        for (int i = 0; i < k; ++i) Z[(size_t)i * r + j] *= inv;
      }
    }
  }
  __syncthreads();

  // ---- 4b. orthonormalise the r vectors in order (classical Gram-Schmidt, twice)
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

  // ---- 4c. back-transformation x = Q z: each wave applies every reflector to its
  //          own vectors, so no block barrier is needed between reflectors
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
    double best = -1.0;
    int bidx = 0;
    for (int i = lane; i < k; i += 64) {
      const double a = fabs(Z[(size_t)i * r + j]);
      if (a > best) {
        best = a;
        bidx = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bidx, o);
      if (ob > best || (ob == best && oi < bidx)) {
        best = ob;
        bidx = oi;
      }
    }
    const double sg = Z[(size_t)bidx * r + j] < 0.0 ? -1.0 : 1.0;
    for (int i = lane; i < k; i += 64) vecs[(size_t)j * k + i] = sg * Z[(size_t)i * r + j];
  }
}

template <bool SMALL_LDS>
__global__ __launch_bounds__(ET) void eig_trunc_kernel(EigBatch batch) {
  const EigJob J = batch.j[blockIdx.x];
  // phase clocks (wall_clock64 ticks) in the 64 spare doubles at the end of the scratch
  double* clk = J.scratch + (eig_scratch_doubles_dev(J.k, J.rmax) - 64);
#define HT_EIG_MARK(i) \
  if (threadIdx.x == 0) clk[i] = (double)wall_clock64();
  HT_EIG_MARK(0)
  extern __shared__ double lds[];
  __shared__ double red[NW];
  __shared__ double s_gl, s_gu, s_pivmin, s_tnorm;
  __shared__ int s_rank;
  const int k = J.k;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // ---- carve scratch (global) and LDS
  double* sc = J.scratch;
  double* gP = sc;  // packed lower triangle when it does not fit in LDS
  sc += (size_t)k * (k + 1) / 2;
  double* hv = sc;  // Householder vectors, reflector j in row j
  sc += (size_t)k * k;
  double* gsmall = sc;
  sc += (size_t)6 * k;
  double* tau = sc;
  sc += k;
  double* lam = sc;  // ascending eigenvalues
  sc += k;
  double* tail = sc;
  sc += k + 1;
  double* gz = sc;  // 4 k rmax, used when the inverse-iteration arrays do not fit in LDS

  // the storage choice is a compile-time one so that every access keeps a single
  // address space (LDS accesses through a generic pointer would be flat loads)
  double* small = SMALL_LDS ? lds : gsmall;
  double* d = small;
  double* e = d + k;
  double* e2 = e + k;
  double* vb = e2 + k;
  double* pb = vb + k;
  double* wb = pb + k;
  double* work = lds + (SMALL_LDS ? 6 * k : 0);
  const int64_t work_cap = kLdsDoubles - (SMALL_LDS ? 6 * k : 0);
  const int64_t npk = (int64_t)k * (k + 1) / 2;
  const bool packed_lds = npk <= work_cap;

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

  // ---- 1. tridiagonalisation
  if (packed_lds)
    tridiagonalise(work, J.G, k, vb, pb, wb, red, d, e, e2, tau, hv, &s_gl, &s_gu, &s_pivmin, &s_tnorm, clk);
  else
    tridiagonalise(gP, J.G, k, vb, pb, wb, red, d, e, e2, tau, hv, &s_gl, &s_gu, &s_pivmin, &s_tnorm, clk);

  HT_EIG_MARK(1)
  // ---- 2. all eigenvalues by multisection: T lanes of one wave share an eigenvalue,
  //         evaluate Sturm counts at T interior points and keep the sub-interval.
  {
    const double tn = s_tnorm, pivmin = s_pivmin;
    const double atol = 2.2e-16 * tn;
    int T = 1;
    while (T < 64 && 2 * T * k <= ET) T *= 2;
    const int groups = ET / T;
    const int u = tid % T;
    const int gbase = lane - (lane % T);
    // a group's lanes share idx, so every group runs a uniform number of rounds
    for (int idx = tid / T; idx < k; idx += groups) {
      double lo = s_gl, hi = s_gu;  // invariant: count(lo) <= idx < count(hi)
      for (int it = 0; it < 160; ++it) {
        const bool done = hi - lo <= fmax(2.2e-16 * fmax(fabs(lo), fabs(hi)), atol);
        if (__all(done)) break;
        const double w = (hi - lo) / (double)(T + 1);
        const double x = lo + w * (double)(u + 1);
        bool above = false;
        if (!done) above = (x >= hi) ? true : (x <= lo) ? false : (sturm_count(d, e2, k, x, pivmin) > idx);
        const unsigned long long m = __ballot(above);
        if (!done) {
          const unsigned long long gm = (m >> gbase) & ((T == 64) ? ~0ull : ((1ull << T) - 1));
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
      if (u == 0) lam[idx] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();

  HT_EIG_MARK(2)
  // ---- 3. truncation rule
  if (tid == 0) {
    double acc = 0.0;
    tail[k] = 0.0;
    for (int i = 0; i < k; ++i) {
      const double l = lam[i];
      acc += l > 0.0 ? l : 0.0;
      tail[k - 1 - i] = acc;
    }
    const int kmax = min(k, J.rmax);
    int r = kmax;
    for (int cand = J.rmin; cand <= kmax; ++cand) {
      if (tail[cand] <= J.thr) {
        r = cand;
        break;
      }
    }
    s_rank = r;
    *J.rank = r;
    *J.tail = tail[r];
  }
  for (int i = tid; i < k; i += ET) J.evals[i] = lam[k - 1 - i];
  __syncthreads();
  const int r = s_rank;
  if (r == 0) return;

  HT_EIG_MARK(3)
  // ---- 4. eigenvectors, in LDS when the 4 k r work arrays fit
  if ((int64_t)4 * k * r <= work_cap)
    eigenvectors(work, k, r, lam, d, e, pb, red, tau, hv, J.vecs, s_tnorm);
  else
    eigenvectors(gz, k, r, lam, d, e, pb, red, tau, hv, J.vecs, s_tnorm);
  HT_EIG_MARK(6)
#undef HT_EIG_MARK
}

}  // namespace

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
