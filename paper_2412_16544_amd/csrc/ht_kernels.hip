// Device kernels of the batch hierarchical Tucker path on gfx950 (MI355X).
//
// Contractions (the TTM projections of Alg. 1/2 and Eq. multi_index_contraction)
// and Gram products of mode unfoldings (the SVDs of Eq. ht_leaf_svd and
// svd_on_residual, taken as eigen-decompositions of the Gram matrix) run on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64).  Unfoldings are never copied: a
// kernel reads the level tensor through its (P, m, S) mode view.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ht_internal.h"

namespace ht {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 operand layout (lane l of a wave64):
//   A (16x4): A[l % 16][l / 16];  B (4x16): B[l / 16][l % 16];
//   D (16x16): register v of lane l holds D[l / 16 + 4 v][l % 16].

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ double ld(const T* __restrict__ p, int64_t i) {
  return static_cast<double>(p[i]);
}

// address of element (c, a=0) of the unfolding, column c = (p, s)
__device__ __forceinline__ int64_t col_base(int64_t c, int64_t m, int64_t S) {
  const int64_t p = c / S;
  const int64_t s = c - p * S;
  return p * m * S + s;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// --------------------------------------------------------------------------
// Sum of squares (FP64 accumulation), two fixed-order levels
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void sumsq_partial_kernel(const T* __restrict__ x, int64_t n,
                                                            double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = ld(x, i);
    acc = fma(v, v, acc);
  }
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

// --------------------------------------------------------------------------
// Gram of a mode unfolding: G = X_(k) X_(k)^T, FP64 MFMA.
// Grid (pair, split): pair enumerates 128x128 blocks (bi <= bj) of G, split a
// contiguous range of 32-column tiles of the unfolding.  Each workgroup stages
// the two 128-row panels of its columns in LDS and accumulates its block's
// 16x16 tiles (upper ones only on the diagonal) round-robin over 4 waves.
// --------------------------------------------------------------------------
constexpr int GB = 128;
constexpr int GBK = 32;
constexpr int GLD = GB + 1;  // odd stride in doubles: conflict-free column writes
constexpr int GMAXT = 16;

__device__ __forceinline__ void tile_of(int t, bool diag, int tI, int tJ, int& ti, int& tj) {
  if (!diag) {
    ti = t / tJ;
    tj = t - ti * tJ;
    return;
  }
  int row = 0, rem = t;
  while (rem >= tI - row) {
    rem -= tI - row;
    ++row;
  }
  ti = row;
  tj = row + rem;
}

template <typename T>
__global__ __launch_bounds__(256) void gram_partial_kernel(const T* __restrict__ X, int64_t P, int64_t m, int64_t S,
                                                           int nb, int npairs, int64_t ktiles, int64_t kt_per_split,
                                                           int64_t blk, double* __restrict__ part) {
  __shared__ double sI[GBK * GLD];
  __shared__ double sJ[GBK * GLD];
  const int pair = blockIdx.x;
  const int split = blockIdx.y;
  int bi = 0, rem = pair;
  while (rem >= nb - bi) {
    rem -= nb - bi;
    ++bi;
  }
  const int bj = bi + rem;
  const bool diag = (bi == bj);
  const int rowsI = (int)min<int64_t>(GB, m - (int64_t)bi * GB);
  const int rowsJ = (int)min<int64_t>(GB, m - (int64_t)bj * GB);
  const int tI = (rowsI + 15) >> 4, tJ = (rowsJ + 15) >> 4;
  const int ntiles = diag ? tI * (tI + 1) / 2 : tI * tJ;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  int myti[GMAXT], mytj[GMAXT];
#pragma unroll
  for (int q = 0; q < GMAXT; ++q) {
    const int t = wave + 4 * q;
    int a = 0, b = 0;
    if (t < ntiles) tile_of(t, diag, tI, tJ, a, b);
    myti[q] = a;
    mytj[q] = b;
  }
  d4 acc[GMAXT];
#pragma unroll
  for (int q = 0; q < GMAXT; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t K = P * S;
  const int64_t kt0 = (int64_t)split * kt_per_split;
  const int64_t kt1 = min(ktiles, kt0 + kt_per_split);
  const int64_t rowI0 = (int64_t)bi * GB, rowJ0 = (int64_t)bj * GB;
  const double* sB = diag ? sI : sJ;

  for (int64_t kt = kt0; kt < kt1; ++kt) {
    const int64_t c0 = kt * GBK;
    for (int e = threadIdx.x; e < GBK * GB; e += 256) {
      int kk, row;
      if (S == 1) {
        row = e % GB;
        kk = e / GB;
      } else {
        kk = e % GBK;
        row = e / GBK;
      }
      const int64_t c = c0 + kk;
      double vi = 0.0, vj = 0.0;
      if (c < K) {
        const int64_t base = col_base(c, m, S);
        if (row < rowsI) vi = ld(X, base + (rowI0 + row) * S);
        if (!diag && row < rowsJ) vj = ld(X, base + (rowJ0 + row) * S);
      }
      sI[kk * GLD + row] = vi;
      if (!diag) sJ[kk * GLD + row] = vj;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 4) {
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int q = 0; q < GMAXT; ++q) {
        if (wave + 4 * q < ntiles) {
          const double a = sI[kr * GLD + myti[q] * 16 + (lane & 15)];
          const double b = sB[kr * GLD + mytj[q] * 16 + (lane & 15)];
          acc[q] = mfma16(a, b, acc[q]);
        }
      }
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)split * npairs + pair) * blk;
  const int ld_out = (int)min<int64_t>(GB, m);
#pragma unroll
  for (int q = 0; q < GMAXT; ++q) {
    if (wave + 4 * q < ntiles) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = myti[q] * 16 + (lane >> 4) + 4 * v;
        const int j = mytj[q] * 16 + (lane & 15);
        if (i < rowsI && j < rowsJ) out[i * ld_out + j] = acc[q][v];
      }
    }
  }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ part, int64_t m, int nb,
                                                          int npairs, int nsplit, int64_t blk,
                                                          double* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * m) return;
  int64_t i = e / m, j = e - (e / m) * m;
  int bi = (int)(i / GB), bj = (int)(j / GB);
  int li = (int)(i - (int64_t)bi * GB), lj = (int)(j - (int64_t)bj * GB);
  if (bi > bj || (bi == bj && (li >> 4) > (lj >> 4))) {
    int t = bi; bi = bj; bj = t;
    t = li; li = lj; lj = t;
  }
  const int pair = bi * nb - bi * (bi - 1) / 2 + (bj - bi);
  const int ld_out = (int)min<int64_t>(GB, m);
  double acc = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) acc += part[((int64_t)sp * npairs + pair) * blk + li * ld_out + lj];
  G[e] = acc;
}

struct GramPlan {
  int nb, npairs, nsplit;
  int64_t ktiles, kt_per_split, blk;
};

GramPlan gram_plan(const ModeView& v) {
  GramPlan g;
  g.nb = (int)((v.m + GB - 1) / GB);
  g.npairs = g.nb * (g.nb + 1) / 2;
  const int64_t K = v.P * v.S;
  g.ktiles = (K + GBK - 1) / GBK;
  int64_t want = std::max<int64_t>(1, 512 / g.npairs);
  want = std::min<int64_t>(want, std::max<int64_t>(1, g.ktiles));
  g.kt_per_split = (g.ktiles + want - 1) / want;
  if (g.kt_per_split < 1) g.kt_per_split = 1;
  g.nsplit = (int)((g.ktiles + g.kt_per_split - 1) / g.kt_per_split);
  if (g.nsplit < 1) g.nsplit = 1;
  const int64_t side = std::min<int64_t>(GB, v.m);
  g.blk = side * side;
  return g;
}

// --------------------------------------------------------------------------
// TTM contraction Z[p, r, s] = sum_a U[a, r] X[p, a, s]  (FP64 MFMA)
// Each wave owns 64 columns (p, s) and every output row r < R (<= 64); U^T
// is staged in LDS in chunks of 64 rows of a; X is read once, straight into
// the B operand registers.
// --------------------------------------------------------------------------
constexpr int TAC = 64;
constexpr int TUS = 65;  // LDS row stride (doubles) of the staged U chunk

template <typename T>
__global__ __launch_bounds__(256) void ttm_contract_kernel(const T* __restrict__ X, int64_t P, int64_t m, int64_t S,
                                                           const double* __restrict__ U, int R,
                                                           double* __restrict__ Z) {
  __shared__ double sU[TAC * TUS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t K = P * S;
  const int64_t colw = ((int64_t)blockIdx.x * 4 + wave) * 64;
  const int rt = (R + 15) >> 4;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  int64_t base[4];
  bool valid[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t c = colw + ct * 16 + (lane & 15);
    valid[ct] = c < K;
    base[ct] = valid[ct] ? col_base(c, m, S) : 0;
  }
  for (int64_t a0 = 0; a0 < m; a0 += TAC) {
    const int ac = (int)min<int64_t>(TAC, m - a0);
    __syncthreads();
    for (int e = threadIdx.x; e < TAC * 64; e += 256) {
      const int a = e >> 6, r = e & 63;
      sU[a * TUS + r] = (a < ac && r < R) ? U[(a0 + a) + (int64_t)r * m] : 0.0;
    }
    __syncthreads();
    for (int ks = 0; ks < ac; ks += 4) {
      const int a = ks + (lane >> 4);
      double b[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) b[ct] = (valid[ct] && a < ac) ? ld(X, base[ct] + (a0 + a) * S) : 0.0;
#pragma unroll
      for (int rti = 0; rti < 4; ++rti) {
        if (rti < rt) {
          const double av = sU[a * TUS + rti * 16 + (lane & 15)];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) acc[rti][ct] = mfma16(av, b[ct], acc[rti][ct]);
        }
      }
    }
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t c = colw + ct * 16 + (lane & 15);
    if (c >= K) continue;
    const int64_t p = c / S, s = c - (c / S) * S;
#pragma unroll
    for (int rti = 0; rti < 4; ++rti) {
      if (rti < rt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = rti * 16 + (lane >> 4) + 4 * v;
          if (r < R) Z[(p * R + r) * S + s] = acc[rti][ct][v];
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// TTM expansion out[p, a, s] = (M[p,a,s] -) sum_t U[a, t] Z[p, t, s]  (FP64 MFMA)
// Block = 4 waves x 64 columns, blockIdx.y selects 64 rows of a.
// --------------------------------------------------------------------------
template <typename TM, typename TO>
__global__ __launch_bounds__(256) void ttm_expand_kernel(const double* __restrict__ Z, int64_t P, int R, int64_t S,
                                                         const double* __restrict__ U, int64_t m,
                                                         const TM* __restrict__ M, TO* __restrict__ out) {
  __shared__ double sU[64 * TUS];  // sU[t][a_local]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t K = P * S;
  const int64_t a0 = (int64_t)blockIdx.y * 64;
  const int64_t colw = ((int64_t)blockIdx.x * 4 + wave) * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int t = e >> 6, al = e & 63;
    sU[t * TUS + al] = (t < R && a0 + al < m) ? U[(a0 + al) + (int64_t)t * m] : 0.0;
  }
  __syncthreads();
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  int64_t zb[4];
  bool valid[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t c = colw + ct * 16 + (lane & 15);
    valid[ct] = c < K;
    const int64_t p = valid[ct] ? c / S : 0;
    const int64_t s = valid[ct] ? c - p * S : 0;
    zb[ct] = p * R * S + s;
  }
  const int at_n = (int)min<int64_t>(4, (m - a0 + 15) >> 4);
  for (int t0 = 0; t0 < R; t0 += 4) {
    const int t = t0 + (lane >> 4);
    double b[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) b[ct] = (valid[ct] && t < R) ? Z[zb[ct] + (int64_t)t * S] : 0.0;
#pragma unroll
    for (int at = 0; at < 4; ++at) {
      if (at < at_n) {
        const double av = sU[t * TUS + at * 16 + (lane & 15)];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[at][ct] = mfma16(av, b[ct], acc[at][ct]);
      }
    }
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t c = colw + ct * 16 + (lane & 15);
    if (c >= K) continue;
    const int64_t p = c / S, s = c - (c / S) * S;
#pragma unroll
    for (int at = 0; at < 4; ++at) {
      if (at < at_n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t a = a0 + at * 16 + (lane >> 4) + 4 * v;
          if (a < m) {
            const int64_t idx = (p * m + a) * S + s;
            double val = acc[at][ct][v];
            if (M != nullptr) val = ld(M, idx) - val;
            out[idx] = static_cast<TO>(val);
          }
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// Basis expansion: CGS2 against U_old, CholeskyQR2, sign normalisation.
// One workgroup of 256 threads; alpha rows, r_old + rR <= 2 * 64 columns.
// --------------------------------------------------------------------------
__device__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void orth_expand_kernel(const double* __restrict__ Uold, int64_t alpha, int r_old,
                                                          double* __restrict__ V, int rR, double* __restrict__ core,
                                                          double* __restrict__ scratch) {
  __shared__ double red[4];
  __shared__ double Cs[64 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // ---- two passes of classical Gram-Schmidt against the old basis
  for (int pass = 0; pass < 2 && r_old > 0; ++pass) {
    for (int e = wave; e < r_old * rR; e += 4) {
      const int i = e / rR, j = e - (e / rR) * rR;
      double acc = 0.0;
      for (int64_t a = lane; a < alpha; a += 64) acc = fma(Uold[a + (int64_t)i * alpha], V[a + (int64_t)j * alpha], acc);
      acc = wave_sum(acc);
      if (lane == 0) Cs[i * rR + j] = acc;
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < alpha * rR; e += 256) {
      const int64_t a = e % alpha;
      const int j = (int)(e / alpha);
      double acc = V[a + (int64_t)j * alpha];
      for (int i = 0; i < r_old; ++i) acc = fma(-Uold[a + (int64_t)i * alpha], Cs[i * rR + j], acc);
      V[a + (int64_t)j * alpha] = acc;
    }
    __syncthreads();
  }
  // ---- CholeskyQR, twice: V <- V L^{-T} with L L^T = V^T V
  for (int pass = 0; pass < 2; ++pass) {
    for (int e = wave; e < rR * rR; e += 4) {
      const int i = e / rR, j = e - (e / rR) * rR;
      double acc = 0.0;
      if (j <= i)
        for (int64_t a = lane; a < alpha; a += 64) acc = fma(V[a + (int64_t)i * alpha], V[a + (int64_t)j * alpha], acc);
      acc = wave_sum(acc);
      if (lane == 0) Cs[i * rR + j] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      // in-place lower Cholesky of Cs (rR x rR)
      for (int j = 0; j < rR; ++j) {
        double d = Cs[j * rR + j];
        for (int k = 0; k < j; ++k) d -= Cs[j * rR + k] * Cs[j * rR + k];
        d = sqrt(d > 0.0 ? d : 1e-300);
        Cs[j * rR + j] = d;
        for (int i = j + 1; i < rR; ++i) {
          double s = Cs[i * rR + j];
          for (int k = 0; k < j; ++k) s -= Cs[i * rR + k] * Cs[j * rR + k];
          Cs[i * rR + j] = s / d;
        }
      }
    }
    __syncthreads();
    // each row x of V solves x_new L^T = x  (forward substitution over columns)
    for (int64_t a = threadIdx.x; a < alpha; a += 256) {
      for (int j = 0; j < rR; ++j) {
        double s = V[a + (int64_t)j * alpha];
        for (int k = 0; k < j; ++k) s -= V[a + (int64_t)k * alpha] * Cs[j * rR + k];
        V[a + (int64_t)j * alpha] = s / Cs[j * rR + j];
      }
    }
    __syncthreads();
  }
  // ---- sign: the largest-magnitude entry (lowest index on ties) is positive
  for (int j = wave; j < rR; j += 4) {
    double best = -1.0;
    int64_t bidx = 0;
    for (int64_t a = lane; a < alpha; a += 64) {
      const double v = fabs(V[a + (int64_t)j * alpha]);
      if (v > best) {
        best = v;
        bidx = a;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int64_t oi = __shfl_xor(bidx, o);
      if (ob > best || (ob == best && oi < bidx)) {
        best = ob;
        bidx = oi;
      }
    }
    const double sg = V[bidx + (int64_t)j * alpha] < 0.0 ? -1.0 : 1.0;
    for (int64_t a = lane; a < alpha; a += 64) core[a + (int64_t)(r_old + j) * alpha] = sg * V[a + (int64_t)j * alpha];
  }
  if (core != Uold)
    for (int64_t e = threadIdx.x; e < alpha * r_old; e += 256) core[e] = Uold[e];
}

// --------------------------------------------------------------------------
// layout helpers
// --------------------------------------------------------------------------
__global__ void pad_core_kernel(const double* __restrict__ src, int ra, int rb, int rp, double* __restrict__ dst,
                                int ra2, int rb2) {
  const int64_t n = (int64_t)ra2 * rb2 * rp;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t rows2 = (int64_t)ra2 * rb2;
    const int64_t col = e / rows2;
    const int64_t row = e - col * rows2;
    const int ia = (int)(row / rb2), ib = (int)(row - (row / rb2) * rb2);
    dst[e] = (ia < ra && ib < rb) ? src[(int64_t)ia * rb + ib + col * (int64_t)ra * rb] : 0.0;
  }
}

__global__ void root_append_kernel(const double* __restrict__ C1, int64_t N, int r11, int r12,
                                   double* __restrict__ root, int64_t n_acc, int rcap) {
  const int64_t n = N * rcap * rcap;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t s = e / ((int64_t)rcap * rcap);
    const int64_t rem = e - s * rcap * rcap;
    const int i = (int)(rem / rcap), j = (int)(rem - (rem / rcap) * rcap);
    root[(n_acc + s) * rcap * rcap + rem] = (i < r11 && j < r12) ? C1[(s * r11 + i) * r12 + j] : 0.0;
  }
}

__global__ void root_extract_kernel(const double* __restrict__ root, int64_t first, int64_t count, int r11, int r12,
                                    int rcap, double* __restrict__ lat) {
  const int64_t n = count * r11 * r12;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t s = e / ((int64_t)r11 * r12);
    const int64_t rem = e - s * r11 * r12;
    const int i = (int)(rem / r12), j = (int)(rem - (rem / r12) * r12);
    lat[e] = root[(first + s) * rcap * rcap + (int64_t)i * rcap + j];
  }
}

__global__ void copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = src[e];
}

__global__ void fill_kernel(double* __restrict__ dst, double v, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = v;
}

inline unsigned grid_for(int64_t n, int64_t cap = 4096) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

// ============================================================================
// host launchers
// ============================================================================
void sumsq(const void* x, Elem t, int64_t n, double* partials, double* out, hipStream_t s) {
  ProfScope prof(KKind::Sumsq, s, 2.0 * n, (double)n * (t == Elem::F32 ? 4 : 8));
  if (t == Elem::F32)
    sumsq_partial_kernel<float><<<kSumsqBlocks, 256, 0, s>>>(static_cast<const float*>(x), n, partials);
  else
    sumsq_partial_kernel<double><<<kSumsqBlocks, 256, 0, s>>>(static_cast<const double*>(x), n, partials);
  reduce_kernel<<<1, 256, 0, s>>>(partials, kSumsqBlocks, out);
}

size_t gram_partial_doubles(const ModeView& v) {
  const GramPlan g = gram_plan(v);
  return (size_t)g.nsplit * g.npairs * g.blk;
}

void gram(const void* x, Elem t, const ModeView& v, double* part, double* G, hipStream_t s) {
  const GramPlan g = gram_plan(v);
  // algorithmic work of the symmetric product: m^2 K flops, the m x K unfolding read once
  const double K = (double)v.P * v.S, md = (double)v.m;
  dim3 grid(g.npairs, g.nsplit);
  {
    ProfScope prof(KKind::Gram, s, md * md * K, md * K * (t == Elem::F32 ? 4 : 8));
    if (t == Elem::F32)
      gram_partial_kernel<float><<<grid, 256, 0, s>>>(static_cast<const float*>(x), v.P, v.m, v.S, g.nb, g.npairs,
                                                      g.ktiles, g.kt_per_split, g.blk, part);
    else
      gram_partial_kernel<double><<<grid, 256, 0, s>>>(static_cast<const double*>(x), v.P, v.m, v.S, g.nb,
                                                       g.npairs, g.ktiles, g.kt_per_split, g.blk, part);
  }
  const int64_t mm = v.m * v.m;
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  gram_reduce_kernel<<<(unsigned)((mm + 255) / 256), 256, 0, s>>>(part, v.m, g.nb, g.npairs, g.nsplit, g.blk, G);
}

void ttm_contract(const void* x, Elem t, const ModeView& v, const double* U, int R, double* Z, hipStream_t s) {
  const int64_t K = v.P * v.S;
  ProfScope prof(KKind::TtmContract, s, 2.0 * R * v.m * (double)K,
                 (double)v.m * K * (t == Elem::F32 ? 4 : 8) + (double)R * K * 8 + (double)v.m * R * 8);
  const unsigned blocks = (unsigned)((K + 255) / 256);
  if (t == Elem::F32)
    ttm_contract_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const float*>(x), v.P, v.m, v.S, U, R, Z);
  else
    ttm_contract_kernel<double><<<blocks, 256, 0, s>>>(static_cast<const double*>(x), v.P, v.m, v.S, U, R, Z);
}

void ttm_expand(const double* Z, int64_t P, int R, int64_t S, const double* U, int64_t m, const void* M, Elem mt,
                void* out, Elem out_t, hipStream_t s) {
  const int64_t K = P * S;
  ProfScope prof(KKind::TtmExpand, s, 2.0 * R * m * (double)K,
                 (double)R * K * 8 + (double)m * K * (out_t == Elem::F32 ? 4 : 8) +
                     (M ? (double)m * K * (mt == Elem::F32 ? 4 : 8) : 0.0));
  dim3 grid((unsigned)((K + 255) / 256), (unsigned)((m + 63) / 64));
  if (out_t == Elem::F32) {
    ttm_expand_kernel<double, float><<<grid, 256, 0, s>>>(Z, P, R, S, U, m, nullptr, static_cast<float*>(out));
  } else if (M == nullptr) {
    ttm_expand_kernel<double, double><<<grid, 256, 0, s>>>(Z, P, R, S, U, m, nullptr, static_cast<double*>(out));
  } else if (mt == Elem::F32) {
    ttm_expand_kernel<float, double><<<grid, 256, 0, s>>>(Z, P, R, S, U, m, static_cast<const float*>(M),
                                                          static_cast<double*>(out));
  } else {
    ttm_expand_kernel<double, double><<<grid, 256, 0, s>>>(Z, P, R, S, U, m, static_cast<const double*>(M),
                                                           static_cast<double*>(out));
  }
}

size_t orth_scratch_doubles(int rR) { return (size_t)64 * 64 + (size_t)rR; }

void orth_expand(const double* U_old, int64_t alpha, int r_old, double* V, int rR, double* core, double* scratch,
                 hipStream_t s) {
  if (rR <= 0) return;
  ProfScope prof(KKind::Orth, s, 0.0, 0.0);
  orth_expand_kernel<<<1, 256, 0, s>>>(U_old, alpha, r_old, V, rR, core, scratch);
}

void pad_core(const double* src, int ra, int rb, int rp, double* dst, int ra2, int rb2, hipStream_t s) {
  const int64_t n = (int64_t)ra2 * rb2 * rp;
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  pad_core_kernel<<<grid_for(n), 256, 0, s>>>(src, ra, rb, rp, dst, ra2, rb2);
}

void root_append(const double* C1, int64_t N, int r11, int r12, double* root, int64_t n_acc, int rcap, hipStream_t s) {
  const int64_t n = N * rcap * rcap;
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  root_append_kernel<<<grid_for(n), 256, 0, s>>>(C1, N, r11, r12, root, n_acc, rcap);
}

void root_extract(const double* root, int64_t first, int64_t count, int r11, int r12, int rcap, double* latent,
                  hipStream_t s) {
  const int64_t n = count * r11 * r12;
  root_extract_kernel<<<grid_for(n), 256, 0, s>>>(root, first, count, r11, r12, rcap, latent);
}

void copy_f64(const double* src, double* dst, int64_t n, hipStream_t s) {
  if (n > 0) copy_kernel<<<grid_for(n), 256, 0, s>>>(src, dst, n);
}

void fill_f64(double* dst, double v, int64_t n, hipStream_t s) {
  if (n > 0) fill_kernel<<<grid_for(n), 256, 0, s>>>(dst, v, n);
}

}  // namespace ht
