// FP64 symmetric eigen-decomposition with the error-truncation rule, on gfx950.
//
// The truncated SVD of an unfolding M (Eq. ht_leaf_svd, Eq. svd_on_residual) is
// taken from the Gram matrix G = M M^T: sigma_i^2 = lambda_i(G) and the left
// singular vectors are G's eigenvectors.  One workgroup solves one k x k problem:
//
//   1. Householder reduction G = Q T Q^T to tridiagonal T (LDS-resident for k <= 132);
//   2. every eigenvalue of T by bisection on Sturm counts, in parallel;
//   3. the minimal rank r in [rmin, rmax] whose discarded energy, summed from the
//      smallest eigenvalue up, is <= thr = eps_nw^2 (clipping lambda at 0);
//   4. the r leading eigenvectors of T by inverse iteration (partial-pivoting LU
//      of T - lambda I), re-orthogonalised twice, mapped back with Q, and
//      sign-normalised (largest-magnitude entry positive, lowest index on ties).
//
// Several independent problems (the nodes of one tree layer) run in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "ht_internal.h"

namespace ht {
namespace {

constexpr int ET = 256;
constexpr int kLdsA = 132;       // k <= kLdsA: the matrix itself lives in LDS
constexpr int kLdsSmall = 1024;  // k <= kLdsSmall: the O(k) work vectors live in LDS

struct EigBatch {
  EigJob j[kMaxEigJobs];
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ double bsum(double v, double* red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// number of eigenvalues of T (diag d, squared off-diagonal e2) below x
__device__ int sturm_count(const double* d, const double* e2, int k, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < k; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

__device__ __forceinline__ double start_entry(int j, int i) {
  // deterministic pseudo-random start vector for inverse iteration
  unsigned h = (unsigned)(j * 0x9E3779B1u) ^ (unsigned)(i * 0x85EBCA77u) ^ 0xC2B2AE3Du;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return 0.5 + (double)(h & 0xFFFFFF) * (1.0 / 16777216.0);
}

__global__ __launch_bounds__(ET) void eig_trunc_kernel(EigBatch batch) {
  const EigJob J = batch.j[blockIdx.x];
  extern __shared__ double lds[];
  __shared__ double red[4];
  __shared__ double s_gl, s_gu, s_pivmin, s_tnorm;
  __shared__ int s_rank;
  const int k = J.k;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rmax = J.rmax;

  // ---- carve scratch
  double* sc = J.scratch;
  double* A = (k <= kLdsA) ? lds : sc;
  sc += (size_t)k * k;
  double* small = (k <= kLdsSmall) ? lds + ((k <= kLdsA) ? (size_t)k * k : 0) : sc;
  sc += (size_t)6 * k;
  double* d = small;
  double* e = d + k;
  double* e2 = e + k;
  double* vb = e2 + k;
  double* pb = vb + k;
  double* wb = pb + k;
  double* tau = sc;
  sc += k;
  double* lam = sc;  // ascending eigenvalues
  sc += k;
  double* tail = sc;  // tail[r] = sum of the k - r smallest (clipped) eigenvalues
  sc += k + 1;
  double* lu = sc;  // 5 bands x k x rmax, entry (band, i, j) at (band * k + i) * rmax + j
  sc += (size_t)5 * k * rmax;
  double* z = sc;  // r vectors of length k, vector j at j * k

  for (int64_t q = tid; q < (int64_t)k * k; q += ET) A[q] = J.G[q];
  __syncthreads();

  // ---- 1. Householder tridiagonalisation (lower), reflector j stored in row j
  for (int j = 0; j + 2 < k; ++j) {
    const int r0 = j + 1, n2 = k - r0;
    double loc = 0.0;
    for (int i = 1 + tid; i < n2; i += ET) {
      const double x = A[(int64_t)(r0 + i) * k + j];
      loc = fma(x, x, loc);
    }
    const double xn2 = bsum(loc, red);
    const double alpha = A[(int64_t)r0 * k + j];
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
    for (int i = tid; i < n2; i += ET) vb[i] = (i == 0) ? 1.0 : A[(int64_t)(r0 + i) * k + j] * scale;
    __syncthreads();
    if (tj != 0.0) {
      for (int i = tid; i < n2; i += ET) {
        double s = 0.0;
        for (int l = 0; l < n2; ++l) s = fma(A[(int64_t)(r0 + l) * k + r0 + i], vb[l], s);
        pb[i] = tj * s;
      }
      __syncthreads();
      double loc2 = 0.0;
      for (int i = tid; i < n2; i += ET) loc2 = fma(pb[i], vb[i], loc2);
      const double pv = bsum(loc2, red);
      const double kk = -0.5 * tj * pv;
      for (int i = tid; i < n2; i += ET) wb[i] = fma(kk, vb[i], pb[i]);
      __syncthreads();
      for (int64_t q = tid; q < (int64_t)n2 * n2; q += ET) {
        const int i = (int)(q / n2), l = (int)(q - (q / n2) * n2);
        A[(int64_t)(r0 + i) * k + r0 + l] -= vb[i] * wb[l] + wb[i] * vb[l];
      }
    }
    if (tid == 0) {
      d[j] = A[(int64_t)j * k + j];
      e[j] = beta;
      tau[j] = tj;
    }
    for (int i = 1 + tid; i < n2; i += ET) A[(int64_t)j * k + r0 + i] = vb[i];
    __syncthreads();
  }
  if (tid == 0) {
    if (k >= 2) {
      d[k - 2] = A[(int64_t)(k - 2) * k + (k - 2)];
      e[k - 2] = A[(int64_t)(k - 1) * k + (k - 2)];
      tau[k - 2] = 0.0;
    }
    d[k - 1] = A[(int64_t)(k - 1) * k + (k - 1)];
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
    s_tnorm = tn;
    s_pivmin = DBL_MIN * fmax(1.0, emax2);
    s_gl = gl - 2.2e-16 * tn - s_pivmin;
    s_gu = gu + 2.2e-16 * tn + s_pivmin;
  }
  __syncthreads();

  // ---- 2. all eigenvalues by bisection (ascending index)
  {
    const double tn = s_tnorm, pivmin = s_pivmin;
    const double atol = 2.2e-16 * tn;
    for (int idx = tid; idx < k; idx += ET) {
      double lo = s_gl, hi = s_gu;
      for (int it = 0; it < 128; ++it) {
        const double width = hi - lo;
        if (width <= fmax(2.2e-16 * fmax(fabs(lo), fabs(hi)), atol)) break;
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(d, e2, k, mid, pivmin) > idx)
          hi = mid;
        else
          lo = mid;
      }
      lam[idx] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();

  // ---- 3. truncation rule
  if (tid == 0) {
    double acc = 0.0;
    tail[k] = 0.0;
    for (int i = 0; i < k; ++i) {
      const double l = lam[i];
      acc += l > 0.0 ? l : 0.0;
      tail[k - 1 - i] = acc;
    }
    const int kmax = min(k, rmax);
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

  // ---- 4a. inverse iteration for the r leading eigenvectors of T (one thread each)
  {
    const double tn = s_tnorm;
    const double tiny = fmax(2.2e-16 * tn, DBL_MIN);
    for (int j = tid; j < r; j += ET) {
      const double lm = lam[k - 1 - j];
      double* U0 = lu;
      double* U1 = lu + (size_t)k * rmax;
      double* U2 = lu + (size_t)2 * k * rmax;
      double* ML = lu + (size_t)3 * k * rmax;
      double* PV = lu + (size_t)4 * k * rmax;
#define LU(arr, i) arr[(size_t)(i) * rmax + j]
      // partial-pivoting LU of T - lm I, row by row
      double u0 = d[0] - lm, u1 = (k > 1) ? e[0] : 0.0, u2 = 0.0;
      for (int i = 0; i + 1 < k; ++i) {
        const double l0 = e[i], l1 = d[i + 1] - lm, l2 = (i + 2 < k) ? e[i + 1] : 0.0;
        if (fabs(u0) >= fabs(l0)) {
          if (u0 == 0.0) u0 = tiny;
          const double mlt = l0 / u0;
          LU(U0, i) = u0;
          LU(U1, i) = u1;
          LU(U2, i) = u2;
          LU(ML, i) = mlt;
          LU(PV, i) = 0.0;
          u0 = l1 - mlt * u1;
          u1 = l2 - mlt * u2;
          u2 = 0.0;
        } else {
          const double mlt = u0 / l0;
          LU(U0, i) = l0;
          LU(U1, i) = l1;
          LU(U2, i) = l2;
          LU(ML, i) = mlt;
          LU(PV, i) = 1.0;
          const double n0 = u1 - mlt * l1, n1 = u2 - mlt * l2;
          u0 = n0;
          u1 = n1;
          u2 = 0.0;
        }
      }
      if (u0 == 0.0) u0 = tiny;
      LU(U0, k - 1) = u0;
      LU(U1, k - 1) = 0.0;
      LU(U2, k - 1) = 0.0;
      double* zj = z + (size_t)j * k;
      for (int i = 0; i < k; ++i) zj[i] = start_entry(j, i);
      for (int it = 0; it < 3; ++it) {
        for (int i = 0; i + 1 < k; ++i) {
          if (LU(PV, i) != 0.0) {
            const double t = zj[i];
            zj[i] = zj[i + 1];
            zj[i + 1] = t;
          }
          zj[i + 1] -= LU(ML, i) * zj[i];
        }
        for (int i = k - 1; i >= 0; --i) {
          double s = zj[i];
          if (i + 1 < k) s -= LU(U1, i) * zj[i + 1];
          if (i + 2 < k) s -= LU(U2, i) * zj[i + 2];
          double piv = LU(U0, i);
          if (fabs(piv) < tiny) piv = copysign(tiny, piv);
          zj[i] = s / piv;
        }
        double mx = 0.0;
        for (int i = 0; i < k; ++i) mx = fmax(mx, fabs(zj[i]));
        const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
        for (int i = 0; i < k; ++i) zj[i] *= inv;
      }
#undef LU
    }
  }
  __syncthreads();

  // ---- 4b. orthonormalise the r vectors in order (classical Gram-Schmidt, twice)
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < r; ++j) {
      double* zj = z + (size_t)j * k;
      // coefficients against earlier vectors, one wave per coefficient
      for (int t = wave; t < j; t += ET / 64) {
        const double* zt = z + (size_t)t * k;
        double s = 0.0;
        for (int i = lane; i < k; i += 64) s = fma(zt[i], zj[i], s);
        s = wsum(s);
        if (lane == 0) pb[t] = s;
      }
      __syncthreads();
      for (int i = tid; i < k; i += ET) {
        double v = zj[i];
        for (int t = 0; t < j; ++t) v -= pb[t] * z[(size_t)t * k + i];
        zj[i] = v;
      }
      __syncthreads();
      double loc = 0.0;
      for (int i = tid; i < k; i += ET) loc = fma(zj[i], zj[i], loc);
      const double nrm = sqrt(bsum(loc, red));
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int i = tid; i < k; i += ET) zj[i] *= inv;
      __syncthreads();
    }
  }

  // ---- 4c. back-transformation x = Q z, one wave per vector; then signs
  for (int j = wave; j < r; j += ET / 64) {
    double* zj = z + (size_t)j * k;
    for (int jj = k - 3; jj >= 0; --jj) {
      const double tj = tau[jj];
      if (tj == 0.0) continue;
      const int r0 = jj + 1, n2 = k - r0;
      double s = 0.0;
      for (int i = lane; i < n2; i += 64) s = fma(i == 0 ? 1.0 : A[(int64_t)jj * k + r0 + i], zj[r0 + i], s);
      s = wsum(s) * tj;
      for (int i = lane; i < n2; i += 64) zj[r0 + i] -= s * (i == 0 ? 1.0 : A[(int64_t)jj * k + r0 + i]);
      __threadfence_block();
    }
    double best = -1.0;
    int bidx = 0;
    for (int i = lane; i < k; i += 64) {
      const double v = fabs(zj[i]);
      if (v > best) {
        best = v;
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
    const double sg = zj[bidx] < 0.0 ? -1.0 : 1.0;
    for (int i = lane; i < k; i += 64) J.vecs[(size_t)j * k + i] = sg * zj[i];
  }
}

size_t lds_bytes_for(int k) {
  size_t n = 0;
  if (k <= kLdsA) n += (size_t)k * k;
  if (k <= kLdsSmall) n += (size_t)6 * k;
  return n * sizeof(double);
}

}  // namespace

size_t eig_scratch_doubles(int k, int rmax) {
  return (size_t)k * k + (size_t)6 * k + (size_t)k + (size_t)k + (size_t)(k + 1) + (size_t)5 * k * rmax +
         (size_t)k * rmax + 64;
}

void eig_trunc(const EigJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return;
  EigBatch b;
  size_t lds = 0;
  for (int i = 0; i < count; ++i) {
    b.j[i] = jobs[i];
    lds = std::max(lds, lds_bytes_for(jobs[i].k));
  }
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&eig_trunc_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
    attr_set = true;
  }
  ProfScope prof(KKind::Eig, s, 0.0, 0.0);
  eig_trunc_kernel<<<count, ET, lds, s>>>(b);
}

}  // namespace ht
