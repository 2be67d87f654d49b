// Device kernels of the batch hierarchical Tucker path on gfx950 (MI355X).
//
// Contractions (the TTM projections of Alg. 1/2 and Eq. multi_index_contraction)
// and Gram products of mode unfoldings (the SVDs of Eq. ht_leaf_svd and
// svd_on_residual, taken as eigen-decompositions of the Gram matrix) run on the
// matrix cores: FP64 (v_mfma_f64_16x16x4f64) in the plain form, FP32
// (v_mfma_f32_16x16x4f32, FP64 partial sums) in the mixed form.  Unfoldings are
// never copied: a kernel reads the level tensor through its (P, m, S) mode view.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "ht_internal.h"

namespace ht {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix-core products, operand layout (lane l of a wave64):
//   A (16x4): A[l % 16][l / 16];  B (4x16): B[l / 16][l % 16];
//   D (16x16), register v of lane l:  FP64: D[l / 16 + 4 v][l % 16],
//                                      FP32: D[4 (l / 16) + v][l % 16].
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// accumulator type and output row of register v for a compute type
template <typename CT>
struct MA;
template <>
struct MA<double> {
  typedef d4 acc;
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct MA<float> {
  typedef f4 acc;
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

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

__device__ __forceinline__ double wave_sum(double v) { return dpp_wave_sum(v); }

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

__device__ __forceinline__ void reduce_body(const double* __restrict__ part, int n, double* __restrict__ out) {
  double acc = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * 256 < n; i += 4 * 256)  // four loads in flight, fixed order
    acc += (part[i] + part[i + 256]) + (part[i + 512] + part[i + 768]);
  for (; i < n; i += 256) acc += part[i];
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  reduce_body(part, n, out);
}

constexpr int kMaxSumJobs = 64;
struct SumBatch {
  SumJob j[kMaxSumJobs];
};

// one workgroup per queued sum
__global__ __launch_bounds__(256) void reduce_many_kernel(SumBatch b) {
  const SumJob J = b.j[blockIdx.x];
  reduce_body(J.part, J.n, J.out);
}

thread_local std::vector<SumJob>* t_defer = nullptr;

// the final sum of a split reduction: queued while this thread defers, else launched
void finish_sum(const double* part, int n, double* out, hipStream_t s) {
  if (t_defer != nullptr)
    t_defer->push_back(SumJob{part, n, out});
  else
    reduce_kernel<<<1, 256, 0, s>>>(part, n, out);
}

// --------------------------------------------------------------------------
// Gram of a mode unfolding: G = X_(k) X_(k)^T, FP64 MFMA.
// Grid (pair, split): pair enumerates 128x128 blocks (bi <= bj) of G, split a
// contiguous range of column tiles of the unfolding (BK columns each).  Each
// workgroup stages the two 128-row panels of its columns in LDS and accumulates its
// block's 16x16 tiles (upper ones only on the diagonal), each wave two tile rows.
// --------------------------------------------------------------------------
constexpr int GB = 128;
constexpr int GBK = 32;
constexpr int GLD = GB + 1;  // odd stride in doubles: conflict-free column writes
constexpr int GMAXT = 16;
// Column tile of the Gram of modes above 128 rows for FP32 data: 64 columns, so that
// a wave's load of one row is 256 contiguous bytes and each barrier pair covers 16
// k steps (FP64 data keeps 32: its prefetched tile would not fit the registers).
constexpr int GPK = 64;

// A basis U (column-major, m rows, R columns, FP64) staged transposed into LDS:
// dst[a * ld + r] = U[a0 + a, r] for a < na, r < nr, zero where a >= na_valid or
// r >= R.  The workgroup walks the entries column by column (consecutive threads read
// consecutive rows of one column) and keeps eight loads in flight per thread before
// the LDS stores, so the staging costs a few cache round trips, not one per entry.
template <typename CT>
__device__ __forceinline__ void stage_ut(const double* __restrict__ U, int64_t m, int R, int64_t a0, int na,
                                         int nr, int na_valid, CT* dst, int ld) {
  const int tot = na * nr;
  for (int e0 = threadIdx.x; e0 < tot; e0 += 256 * 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      const int r = e / na, a = e - (e / na) * na;
      v[q] = (e < tot && a < na_valid && r < R) ? U[(a0 + a) + (int64_t)r * m] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      const int r = e / na, a = e - (e / na) * na;
      if (e < tot) dst[a * ld + r] = static_cast<CT>(v[q]);
    }
  }
}

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

// Column tiles: when S >= BK a tile is BK consecutive columns (rows strided by
// S, each row segment contiguous), loaded by this helper into registers one tile
// ahead; when S < BK it is floor(BK/S) whole slices p, one contiguous block of
// memory, scattered straight into LDS by the kernel.
// The values stay in the data type until they are stored to LDS: a conversion right
// after the load would make the wave wait for it there, and the tile ahead would no
// longer overlap the products of the current one.
template <typename T, int BK>
__device__ __forceinline__ void gram_load_tile(const T* __restrict__ X, int64_t m, int64_t S, int64_t K, int64_t kt,
                                               int tw, int64_t rowI0, int rowsI, int64_t rowJ0, int rowsJ, bool diag,
                                               T (&ri)[BK * GB / 256], T (&rj)[BK * GB / 256]) {
  constexpr int PER = BK * GB / 256;
  // thread owns column kk = tid % BK of the tile and rows tid / BK + (256 / BK) q
  const int kk = threadIdx.x % BK;
  const int64_t c = kt * tw + kk;
  const bool cv = c < K;
  const int64_t base = cv ? col_base(c, m, S) : 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int row = threadIdx.x / BK + q * (256 / BK);
    ri[q] = (cv && row < rowsI) ? X[base + (rowI0 + row) * S] : T(0);
    rj[q] = (!diag && cv && row < rowsJ) ? X[base + (rowJ0 + row) * S] : T(0);
  }
}

template <typename T, int BK>
__global__ __launch_bounds__(256) void gram_partial_kernel(const T* __restrict__ X, int64_t P, int64_t m, int64_t S,
                                                           int nb, int npairs, int64_t ktiles, int64_t kt_per_split,
                                                           int64_t blk, int tw, double* __restrict__ part) {
  __shared__ double sI[BK * GLD];
  __shared__ double sJ[BK * GLD];
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
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // A wave owns two tile rows and every tile of them in the pair's block: off the
  // diagonal rows 2w and 2w + 1 (16 tiles); on it rows w and tI - 1 - w, whose upper
  // tiles add up to tI + 1 (9 of the 36).  A k step then reads 2 A and 8 B operands
  // from LDS for up to 16 products; the bit 8 i + j of `act` (uniform) says whether
  // the tile of row slot i, tile column j is the wave's.
  int rowA, rowB;
  if (diag) {
    rowA = wave < (tI + 1) / 2 ? wave : tI;
    rowB = tI - 1 - wave > rowA ? tI - 1 - wave : tI;
  } else {
    rowA = 2 * wave;
    rowB = 2 * wave + 1;
  }
  unsigned act = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (rowA < tI && j < tJ && (!diag || j >= rowA)) act |= 1u << j;
    if (rowB < tI && j < tJ && (!diag || j >= rowB)) act |= 1u << (8 + j);
  }
  const int offA = (rowA < tI ? rowA : 0) * 16 + (lane & 15);
  const int offB = (rowB < tI ? rowB : 0) * 16 + (lane & 15);
  d4 acc[GMAXT];
#pragma unroll
  for (int q = 0; q < GMAXT; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t K = P * S;
  const int64_t kt0 = (int64_t)split * kt_per_split;
  const int64_t kt1 = min(ktiles, kt0 + kt_per_split);
  const int64_t rowI0 = (int64_t)bi * GB, rowJ0 = (int64_t)bj * GB;
  const double* sB = diag ? sI : sJ;
  constexpr int PER = BK * GB / 256;
  const bool slab = S < BK;
  const int ms = (int)(m * S);

  T ri[PER], rj[PER];
  if (kt0 < kt1 && !slab)
    gram_load_tile<T, BK>(X, m, S, K, kt0, tw, rowI0, rowsI, rowJ0, rowsJ, diag, ri, rj);
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    if (slab) {
      // contiguous region of whole slices, scattered to (column, row) in LDS
      for (int e = threadIdx.x; e < BK * GB; e += 256) {
        sI[(e % BK) * GLD + e / BK] = 0.0;
        if (!diag) sJ[(e % BK) * GLD + e / BK] = 0.0;
      }
      __syncthreads();
      const int64_t p0 = kt * tw / S;
      const int64_t np = min<int64_t>(tw / S, P - p0);
      const int64_t nvalid = np * ms;
      const T* src = X + p0 * m * S;
      for (int64_t q = threadIdx.x; q < nvalid; q += 256) {
        const int pp = (int)(q / ms);
        const int remq = (int)(q - (int64_t)pp * ms);
        const int a = remq / (int)S;
        const int sidx = remq - a * (int)S;
        const int kk = pp * (int)S + sidx;
        const double v = ld(src, q);
        const int64_t li = a - rowI0, lj = a - rowJ0;
        if (li >= 0 && li < rowsI) sI[kk * GLD + li] = v;
        if (!diag && lj >= 0 && lj < rowsJ) sJ[kk * GLD + lj] = v;
      }
    } else {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int kk = threadIdx.x % BK;
        const int row = threadIdx.x / BK + q * (256 / BK);
        sI[kk * GLD + row] = static_cast<double>(ri[q]);
        if (!diag) sJ[kk * GLD + row] = static_cast<double>(rj[q]);
      }
      // prefetch the next tile while this one is multiplied
      if (kt + 1 < kt1) gram_load_tile<T, BK>(X, m, S, K, kt + 1, tw, rowI0, rowsI, rowJ0, rowsJ, diag, ri, rj);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      // every operand of the step first (all in the staged panels), then the products
      const double a0 = sI[kr * GLD + offA], a1 = sI[kr * GLD + offB];
      double b[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = sB[kr * GLD + j * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (act & (1u << j)) acc[j] = mfma16(a0, b[j], acc[j]);
        if (act & (1u << (8 + j))) acc[8 + j] = mfma16(a1, b[j], acc[8 + j]);
      }
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)split * npairs + pair) * blk;
  const int ld_out = (int)min<int64_t>(GB, m);
#pragma unroll
  for (int q = 0; q < GMAXT; ++q) {
    if (act & (1u << q)) {
      const int ti = q < 8 ? rowA : rowB, tj = q & 7;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ti * 16 + (lane >> 4) + 4 * v;
        const int j = tj * 16 + (lane & 15);
        if (i < rowsI && j < rowsJ) out[i * ld_out + j] = acc[q][v];
      }
    }
  }
}

// Gram of a unfolding with few rows (m <= kSmallM) on the vector ALUs: every
// thread accumulates the m(m+1)/2 products of its columns, the block sums them.
constexpr int kSmallM = 8;
constexpr int kSmallBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void gram_small_kernel(const T* __restrict__ X, int64_t m64, int64_t S, int64_t K,
                                                         double* __restrict__ part) {
  const int m = (int)m64;
  double acc[kSmallM * (kSmallM + 1) / 2];
#pragma unroll
  for (int q = 0; q < kSmallM * (kSmallM + 1) / 2; ++q) acc[q] = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < K; c += (int64_t)gridDim.x * 256) {
    const int64_t base = (S == 1) ? c * m : col_base(c, m, S);
    double x[kSmallM];
#pragma unroll
    for (int a = 0; a < kSmallM; ++a) x[a] = a < m ? ld(X, base + (int64_t)a * S) : 0.0;
    int q = 0;
#pragma unroll
    for (int a = 0; a < kSmallM; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b, ++q) acc[q] = fma(x[a], x[b], acc[q]);
  }
  __shared__ double red[4][kSmallM * (kSmallM + 1) / 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kSmallM * (kSmallM + 1) / 2; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kSmallM * (kSmallM + 1) / 2; q += 256)
    part[(int64_t)blockIdx.x * (kSmallM * (kSmallM + 1) / 2) + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
}

// One workgroup per entry of the small Gram: 256 threads sum the block partials in
// a fixed order (strided, then a fixed tree), so the result does not depend on
// timing.
__global__ __launch_bounds__(256) void gram_small_reduce_kernel(const double* __restrict__ part, int m, int nblk,
                                                                double* __restrict__ G) {
  __shared__ double red[4];
  const int e = blockIdx.x;
  int a = e / m, b = e % m;
  if (b > a) {
    const int t = a;
    a = b;
    b = t;
  }
  const int q = a * (a + 1) / 2 + b;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += part[(int64_t)i * (kSmallM * (kSmallM + 1) / 2) + q];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) G[e] = (red[0] + red[1]) + (red[2] + red[3]);
}

// --------------------------------------------------------------------------
// Single-panel Gram for m <= 128, optionally of the explicit residual.
// Each workgroup walks its column tiles; a tile (all m rows x 32 columns) is
// prefetched into registers one step ahead and stored to LDS as sM[column][row]
// in the compute type CT (double: FP64 matrix cores; float: FP32 ones).
// With RESID the tile is first replaced, in LDS, by R = M - U (U^T M) (both
// products on the matrix cores, Z = U^T M staged in LDS), so only the data is
// read.  The workgroup's partial Gram is written in FP64.
// --------------------------------------------------------------------------
constexpr int PER_PANEL = GBK * GB / 256;     // prefetched values per thread (16)
constexpr int ZLD = GBK + 1;
constexpr int kTtmMaxBlocks = 4096;
// The register-direct contractions run one resident round of workgroups (256
// compute units x 4 workgroups of four waves), each looping over its blocks, so
// the U staging of a workgroup is spread over several blocks.
constexpr int kRegMaxBlocks = 1024;

template <typename T>
struct PanelLoader {
  // S >= GBK: thread owns column kk = tid % GBK, rows tid / GBK + 8 q.
  // S <  GBK: whole slices, entry q = tid + 256 t of the contiguous slab; its
  //           destination (column, row) is fixed for every tile.
  bool slab;
  int dst[PER_PANEL];
  __device__ void init(int64_t m, int64_t S, int tw) {
    slab = S < GBK;
    const int ms = (int)(m * S);
#pragma unroll
    for (int t = 0; t < PER_PANEL; ++t) {
      if (slab) {
        const int q = threadIdx.x + 256 * t;
        const int pp = q / ms, rq = q - pp * ms;
        const int a = rq / (int)S, sidx = rq - a * (int)S;
        dst[t] = (q < tw * (int)m) ? (pp * (int)S + sidx) * GLD + a : -1;
      } else {
        const int kk = threadIdx.x % GBK, row = threadIdx.x / GBK + t * (256 / GBK);
        dst[t] = (row < m) ? kk * GLD + row : -1;
      }
    }
  }
  // raw elements stay in registers; the conversion to FP64 happens at the LDS store,
  // so the loads of the next tile overlap the products of the current one
  __device__ void load(const T* __restrict__ X, int64_t P, int64_t m, int64_t S, int64_t K, int64_t kt, int tw,
                       T (&r)[PER_PANEL]) const {
    if (slab) {
      const int64_t p0 = kt * tw / S;
      const int64_t nvalid = min<int64_t>(tw / S, P - p0) * m * S;
      const T* src = X + p0 * m * S;
#pragma unroll
      for (int t = 0; t < PER_PANEL; ++t) {
        const int q = threadIdx.x + 256 * t;
        r[t] = (dst[t] >= 0 && q < nvalid) ? src[q] : T(0);
      }
    } else {
      const int kk = threadIdx.x % GBK;
      const int64_t c = kt * tw + kk;
      const bool cv = c < K;
      const int64_t base = cv ? col_base(c, m, S) : 0;
#pragma unroll
      for (int t = 0; t < PER_PANEL; ++t) {
        const int row = threadIdx.x / GBK + t * (256 / GBK);
        r[t] = (cv && dst[t] >= 0) ? X[base + (int64_t)row * S] : T(0);
      }
    }
  }
  template <typename CT>
  __device__ void store(CT* sM, const T (&r)[PER_PANEL]) const {
#pragma unroll
    for (int t = 0; t < PER_PANEL; ++t)
      if (dst[t] >= 0) sM[dst[t]] = static_cast<CT>(r[t]);
  }
};

template <typename T, typename CT, bool RESID, int MT>
__global__ __launch_bounds__(256) void gram_panel_kernel(const T* __restrict__ X, int64_t P, int64_t m, int64_t S,
                                                         int64_t ktiles, int64_t kt_per_split, int tw,
                                                         const double* __restrict__ U, int R,
                                                         double* __restrict__ part) {
  typedef typename MA<CT>::acc AT;
  extern __shared__ double dsm[];
  CT* sM = reinterpret_cast<CT*>(dsm);   // [GBK][GLD]
  const int RP = (R + 15) & ~15;         // rank padded to the MFMA tile
  const int ULD = RP + 1;
  CT* sU = sM + GBK * GLD;               // [128][ULD]   (RESID)
  CT* sZ = sU + GB * ULD;                // [RP][ZLD]    (RESID)
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int mi = (int)m;
  const int tI = (mi + 15) >> 4;
  const int ntiles = tI * (tI + 1) / 2;
  // MT upper tiles per wave, round-robin; a wave's surplus slots recompute tile (0,0)
  int offa[MT], offb[MT];
  bool live[MT];
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    const int t = wave + 4 * q;
    int a = 0, b = 0;
    live[q] = t < ntiles;
    if (live[q]) tile_of(t, true, tI, tI, a, b);
    offa[q] = a * 16 + (lane & 15);
    offb[q] = b * 16 + (lane & 15);
  }
  AT acc[MT];
#pragma unroll
  for (int q = 0; q < MT; ++q) acc[q] = AT{0, 0, 0, 0};

  // zero the panel once: entries never written by a tile stay zero
  for (int e = threadIdx.x; e < GBK * GLD; e += 256) sM[e] = CT(0);
  if (RESID) stage_ut(U, m, R, 0, GB, ULD, mi, sU, ULD);
  PanelLoader<T> L;
  L.init(m, S, tw);
  const int64_t K = P * S;
  const int64_t kt0 = (int64_t)blockIdx.x * kt_per_split;
  const int64_t kt1 = min(ktiles, kt0 + kt_per_split);
  T rg[PER_PANEL];
  if (kt0 < kt1) L.load(X, P, m, S, K, kt0, tw, rg);
  __syncthreads();
  const int nzt = (RP >> 4) * 2;  // Z tiles: (RP/16) x (GBK/16)
  const int nrt = tI * 2;         // R tiles: (m/16) x (GBK/16)
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    L.store(sM, rg);
    if (kt + 1 < kt1) L.load(X, P, m, S, K, kt + 1, tw, rg);
    __syncthreads();
    if (RESID) {
      // Z = U^T M (RP x GBK)
      for (int zt = wave; zt < nzt; zt += 4) {
        const int zi = zt >> 1, zc = zt & 1;
        AT z = AT{0, 0, 0, 0};
        const CT* pa = sU + (lane >> 4) * ULD + zi * 16 + (lane & 15);
        const CT* pb = sM + (zc * 16 + (lane & 15)) * GLD + (lane >> 4);
        for (int ks = 0; ks < tI * 16; ks += 16) {
          CT a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a[u] = pa[(ks + 4 * u) * ULD];
            b[u] = pb[ks + 4 * u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) z = mfma16(a[u], b[u], z);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) sZ[(zi * 16 + MA<CT>::row(lane, v)) * ZLD + zc * 16 + (lane & 15)] = z[v];
      }
      __syncthreads();
      // M <- M - U Z (m x GBK), in place
      for (int rt = wave; rt < nrt; rt += 4) {
        const int ri = rt >> 1, rc = rt & 1;
        AT y = AT{0, 0, 0, 0};
        const CT* pa = sU + (ri * 16 + (lane & 15)) * ULD + (lane >> 4);
        const CT* pb = sZ + (lane >> 4) * ZLD + rc * 16 + (lane & 15);
        for (int ks = 0; ks < RP; ks += 16) {
          CT a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a[u] = pa[ks + 4 * u];
            b[u] = pb[(ks + 4 * u) * ZLD];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) y = mfma16(a[u], b[u], y);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) sM[(rc * 16 + (lane & 15)) * GLD + ri * 16 + MA<CT>::row(lane, v)] -= y[v];
      }
      __syncthreads();
    }
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 4) {
      const int kr = (ks + (lane >> 4)) * GLD;
      CT a[MT], b[MT];
#pragma unroll
      for (int q = 0; q < MT; ++q) {
        a[q] = sM[kr + offa[q]];
        b[q] = sM[kr + offb[q]];
      }
#pragma unroll
      for (int q = 0; q < MT; ++q) acc[q] = mfma16(a[q], b[q], acc[q]);
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.x * m * m;
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    if (live[q]) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (offa[q] - (lane & 15)) + MA<CT>::row(lane, v);
        const int j = offb[q];
        if (i < mi && j < mi) out[i * m + j] = static_cast<double>(acc[q][v]);
      }
    }
  }
}

// Fixed-order sum of the split partials: 16 groups of 64 lanes split the partial
// range for 64 consecutive entries, then add their sums in group order.  Only the
// entries of the stored (upper) tiles are summed, so a wave's reads are
// consecutive; an entry of a strictly upper tile is also written to its mirror.
__global__ __launch_bounds__(1024) void gram_reduce2_kernel(const double* __restrict__ part, int64_t m, int nb,
                                                            int npairs, int nsplit, int64_t blk,
                                                            double* __restrict__ G) {
  __shared__ double red[16][64];
  const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + l;
  double acc = 0.0;
  bool stored = false, mirror = false;
  int64_t i = 0, j = 0;
  if (e < m * m) {
    i = e / m;
    j = e - (e / m) * m;
    const int bi = (int)(i / GB), bj = (int)(j / GB);
    const int li = (int)(i - (int64_t)bi * GB), lj = (int)(j - (int64_t)bj * GB);
    stored = bi < bj || (bi == bj && (li >> 4) <= (lj >> 4));
    mirror = bi < bj || (bi == bj && (li >> 4) < (lj >> 4));
    if (stored) {
      const int pair = bi * nb - bi * (bi - 1) / 2 + (bj - bi);
      const int ld_out = (int)min<int64_t>(GB, m);
      const int64_t off = (int64_t)pair * blk + li * ld_out + lj;
      const int64_t stride = (int64_t)npairs * blk;
      // eight independent loads in flight per thread, summed in a fixed order
      int sp = g;
      for (; sp + 7 * 16 < nsplit; sp += 8 * 16) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = part[(int64_t)(sp + 16 * q) * stride + off];
        acc += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
      }
      for (; sp < nsplit; sp += 16) acc += part[(int64_t)sp * stride + off];
    }
  }
  red[g][l] = acc;
  __syncthreads();
  if (g == 0 && stored) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += red[q][l];
    G[e] = s;
    if (mirror) G[j * m + i] = s;
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

// --------------------------------------------------------------------------
// Residual Gram from the Gram of the data: for R = M - U U^T M,
//   R R^T = (I - U U^T) G (I - U U^T),  G = M M^T,
// for any U (I - U U^T is symmetric).  With B = U^T G, V = B U (= U^T G U) and
// E = B - V U^T / 2 it is G - U E - E^T U^T, which is symmetric by construction
// and written so.  G is m x m row-major and symmetric, U is m x R column-major;
// one workgroup (m <= 128, R <= 64), the result in place.  E and V sit in LDS, and
// U and G too when STAGE (then every inner loop reads LDS only).
// --------------------------------------------------------------------------
constexpr int kProjThreads = 512;
constexpr int kProjLdsDoubles = 19456;  // 152 KiB

__host__ __device__ constexpr int proj_lds_doubles(int m, int R, bool stage) {
  return R * m + R * R + (stage ? m * m + R * m : 0);
}

struct ProjBatch {
  ProjJob j[kMaxProjJobs];
};

// one workgroup per job; a job stages G and U when its layout fits lds_cap doubles
__global__ __launch_bounds__(kProjThreads) void gram_project_kernel(ProjBatch b, int lds_cap) {
  const ProjJob J = b.j[blockIdx.x];
  double* __restrict__ G = J.G;
  const double* __restrict__ U = J.U;
  const int m = J.m, R = J.R;
  const bool STAGE = proj_lds_doubles(m, R, true) <= lds_cap;
  extern __shared__ double gpL[];
  double* E = gpL;               // R x m: B, then E
  double* V = E + R * m;         // R x R
  double* Gs = V + R * R;        // G (STAGE)
  double* Ul = Gs + m * m;       // U, m x R column-major (STAGE)
  const double* Gr = STAGE ? Gs : G;
  const double* Us = STAGE ? Ul : U;
  const int tid = threadIdx.x;
  if (STAGE) {
    for (int e = tid; e < R * m; e += kProjThreads) Ul[e] = U[e];
    for (int e = tid; e < m * m; e += kProjThreads) Gs[e] = G[e];
    __syncthreads();
  }
  for (int e = tid; e < R * m; e += kProjThreads) {  // B = U^T G
    const int r = e / m, j = e - r * m;
    const double* u = Us + r * m;
    double a0 = 0.0, a1 = 0.0;
    int i = 0;
    for (; i + 1 < m; i += 2) {
      a0 = fma(u[i], Gr[i * m + j], a0);
      a1 = fma(u[i + 1], Gr[(i + 1) * m + j], a1);
    }
    if (i < m) a0 = fma(u[i], Gr[i * m + j], a0);
    E[e] = a0 + a1;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += kProjThreads) {  // V = B U
    const int r = e / R, q = e - r * R;
    const double* u = Us + q * m;
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc = fma(E[r * m + j], u[j], acc);
    V[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < R * m; e += kProjThreads) {  // E = B - V U^T / 2 (reads V and U only)
    const int r = e / m, j = e - r * m;
    double acc = 0.0;
    for (int q = 0; q < R; ++q) acc = fma(V[r * R + q], Us[j + q * m], acc);
    E[e] -= 0.5 * acc;
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += kProjThreads) {  // upper triangle: G - U E - E^T U^T, mirrored
    const int i = e / m, j = e - i * m;
    if (i > j) continue;
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc = fma(Us[i + r * m], E[r * m + j], fma(E[r * m + i], Us[j + r * m], acc));
    const double g = Gr[e] - acc;
    G[e] = g;
    G[(int64_t)j * m + i] = g;
  }
}

// The same projection for modes of more than 128 rows, in four launches over global
// memory (G in L2): B = U^T G, V = B U, E = B - V U^T / 2, then the upper triangle
// of G - U E - E^T U^T, mirrored.  Reads of G, U and E are coalesced along the
// thread index or broadcast over a wave.
// B = U^T G: a workgroup per (r, 32 columns j); eight threads per column split the
// rows i (i = ic mod 8) and add their sums in a fixed order.
__global__ __launch_bounds__(256) void gram_proj_b_kernel(const double* __restrict__ G, int m,
                                                          const double* __restrict__ U, int R, double* __restrict__ B) {
  __shared__ double red[8][33];
  const int nj = (m + 31) / 32;
  const int r = blockIdx.x / nj, j = (blockIdx.x - r * nj) * 32 + (threadIdx.x & 31);
  const int ic = threadIdx.x >> 5;
  const double* u = U + (int64_t)r * m;
  double acc = 0.0;
  if (j < m)
    for (int i = ic; i < m; i += 8) acc = fma(u[i], G[(int64_t)i * m + j], acc);
  red[ic][threadIdx.x & 31] = acc;
  __syncthreads();
  if (ic == 0 && j < m) {
    const int l = threadIdx.x & 31;
    B[(int64_t)r * m + j] = ((red[0][l] + red[1][l]) + (red[2][l] + red[3][l])) +
                            ((red[4][l] + red[5][l]) + (red[6][l] + red[7][l]));
  }
}

// V = B U: one wave per entry, lanes over j, the wave's sum in a fixed order.
__global__ __launch_bounds__(64) void gram_proj_v_kernel(const double* __restrict__ B, int m,
                                                         const double* __restrict__ U, int R, double* __restrict__ V) {
  const int r = blockIdx.x / R, q = blockIdx.x - r * R;
  const double* b = B + (int64_t)r * m;
  const double* u = U + (int64_t)q * m;
  double acc = 0.0;
  for (int j = threadIdx.x; j < m; j += 64) acc = fma(b[j], u[j], acc);
  acc = wave_sum(acc);
  if (threadIdx.x == 0) V[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void gram_proj_e_kernel(const double* __restrict__ B, int m,
                                                          const double* __restrict__ U, int R,
                                                          const double* __restrict__ V, double* __restrict__ E) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)R * m) return;
  const int r = (int)(e / m), j = (int)(e - (int64_t)r * m);
  double acc = 0.0;
  for (int q = 0; q < R; ++q) acc = fma(V[r * R + q], U[j + (int64_t)q * m], acc);
  E[e] = B[e] - 0.5 * acc;
}

__global__ __launch_bounds__(256) void gram_proj_g_kernel(double* __restrict__ G, int m, const double* __restrict__ U,
                                                          int R, const double* __restrict__ E) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int i = (int)(e / m), j = (int)(e - (int64_t)i * m);
  if (i > j) return;
  double acc = 0.0;
  for (int r = 0; r < R; ++r)
    acc = fma(U[i + (int64_t)r * m], E[(int64_t)r * m + j], fma(E[(int64_t)r * m + i], U[j + (int64_t)r * m], acc));
  const double g = G[e] - acc;
  G[e] = g;
  G[(int64_t)j * m + i] = g;
}

struct GramPlan {
  int nb, npairs, nsplit, tw;
  int64_t ktiles, kt_per_split, blk;
};

GramPlan gram_plan(const ModeView& v, int bk = GBK) {
  GramPlan g;
  g.nb = (int)((v.m + GB - 1) / GB);
  g.npairs = g.nb * (g.nb + 1) / 2;
  const int64_t K = v.P * v.S;
  g.tw = v.S >= bk ? bk : (int)(v.S * (bk / v.S));
  g.ktiles = (K + g.tw - 1) / g.tw;
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
// --------------------------------------------------------------------------
// TTM contraction for m <= 128: Z[p, r, s] = sum_a U[a, r] X[p, a, s].  Tiles of
// 32 unfolding columns go through the same prefetching panel loader as the Gram;
// U^T (R <= 64 rows) sits in LDS; each wave computes 16 x 16 blocks of Z and
// writes them straight from its accumulators, in the compute type CT.  With NORM
// the workgroup also sums the squares of every element it reads (the ||Y||^2 of
// the skip test); with RESE it also forms the explicit residual X - U Z of each
// tile in registers and sums its squares (the energy one contraction discards,
// Eq. compute_residual).  Both sums are FP64.
// --------------------------------------------------------------------------
// The work of workgroup bid of one panel contraction (the kernel below, and one job of
// the grouped launch).
template <typename T, typename CT, bool NORM, bool RESE>
__device__ __forceinline__ void ttm_panel_body(const T* __restrict__ X, int64_t P, int64_t m, int64_t S,
                                               int64_t ktiles, int64_t kt_per_split, int tw,
                                               const double* __restrict__ U, int R, CT* __restrict__ Z,
                                               double* __restrict__ norm_part, double* __restrict__ res_part,
                                               int bid) {
  typedef typename MA<CT>::acc AT;
  extern __shared__ double dsm[];
  CT* sM = reinterpret_cast<CT*>(dsm);  // [GBK][GLD]
  const int RP = (R + 15) & ~15;
  const int ULD = RP + 1;
  CT* sU = sM + GBK * GLD;              // [128][ULD]
  CT* sZ = sU + GB * ULD;               // [RP][ZLD]  (RESE)
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int mi = (int)m;
  const int tI = (mi + 15) >> 4;
  for (int e = threadIdx.x; e < GBK * GLD; e += 256) sM[e] = CT(0);
  stage_ut(U, m, R, 0, GB, ULD, mi, sU, ULD);
  PanelLoader<T> L;
  L.init(m, S, tw);
  const int64_t K = P * S;
  const int64_t kt0 = (int64_t)bid * kt_per_split;
  const int64_t kt1 = min(ktiles, kt0 + kt_per_split);
  T rg[PER_PANEL];
  if (kt0 < kt1) L.load(X, P, m, S, K, kt0, tw, rg);
  double nrm = 0.0, res = 0.0;
  __syncthreads();
  const int nzt = (RP >> 4) * 2;
  const int nrt = tI * 2;
  const bool slab = S < GBK;
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    if (NORM) {
#pragma unroll
      for (int t = 0; t < PER_PANEL; ++t) {
        const double v = static_cast<double>(rg[t]);
        nrm = fma(v, v, nrm);
      }
    }
    L.store(sM, rg);
    if (kt + 1 < kt1) L.load(X, P, m, S, K, kt + 1, tw, rg);
    __syncthreads();
    for (int zt = wave; zt < nzt; zt += 4) {
      const int zi = zt >> 1, zc = zt & 1;
      AT z = AT{0, 0, 0, 0};
      const CT* pa = sU + (lane >> 4) * ULD + zi * 16 + (lane & 15);
      const CT* pb = sM + (zc * 16 + (lane & 15)) * GLD + (lane >> 4);
      for (int ks = 0; ks < tI * 16; ks += 16) {
        CT a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = pa[(ks + 4 * u) * ULD];
          b[u] = pb[ks + 4 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) z = mfma16(a[u], b[u], z);
      }
      if (RESE) {
#pragma unroll
        for (int v = 0; v < 4; ++v) sZ[(zi * 16 + MA<CT>::row(lane, v)) * ZLD + zc * 16 + (lane & 15)] = z[v];
      }
      // column j of the tile is unfolding column kt * tw + zc * 16 + j
      const int64_t c = kt * tw + zc * 16 + (lane & 15);
      const bool cv = slab ? (zc * 16 + (lane & 15)) < tw && c < K : c < K;
      if (cv) {
        const int64_t p = c / S, sidx = c - (c / S) * S;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = zi * 16 + MA<CT>::row(lane, v);
          if (r < R) Z[(p * R + r) * S + sidx] = z[v];
        }
      }
    }
    if (RESE) {
      __syncthreads();
      // X - U Z over the tile's m rows; padding rows and columns hold zeros on both sides
      for (int rt = wave; rt < nrt; rt += 4) {
        const int ri = rt >> 1, rc = rt & 1;
        AT y = AT{0, 0, 0, 0};
        const CT* pa = sU + (ri * 16 + (lane & 15)) * ULD + (lane >> 4);
        const CT* pb = sZ + (lane >> 4) * ZLD + rc * 16 + (lane & 15);
        for (int ks = 0; ks < RP; ks += 16) {
          CT a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a[u] = pa[ks + 4 * u];
            b[u] = pb[(ks + 4 * u) * ZLD];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) y = mfma16(a[u], b[u], y);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double dl =
              static_cast<double>(sM[(rc * 16 + (lane & 15)) * GLD + ri * 16 + MA<CT>::row(lane, v)]) -
              static_cast<double>(y[v]);
          res = fma(dl, dl, res);
        }
      }
    }
    __syncthreads();
  }
  if (NORM || RESE) {
    __shared__ double red[8];
    if (NORM) nrm = wave_sum(nrm);
    if (RESE) res = wave_sum(res);
    if (lane == 0) {
      red[threadIdx.x >> 6] = nrm;
      red[4 + (threadIdx.x >> 6)] = res;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (NORM) norm_part[bid] = (red[0] + red[1]) + (red[2] + red[3]);
      if (RESE) res_part[bid] = (red[4] + red[5]) + (red[6] + red[7]);
    }
  }
}

template <typename T, typename CT, bool NORM, bool RESE>
__global__ __launch_bounds__(256) void ttm_panel_kernel(const T* __restrict__ X, int64_t P, int64_t m, int64_t S,
                                                        int64_t ktiles, int64_t kt_per_split, int tw,
                                                        const double* __restrict__ U, int R, CT* __restrict__ Z,
                                                        double* __restrict__ norm_part,
                                                        double* __restrict__ res_part) {
  ttm_panel_body<T, CT, NORM, RESE>(X, P, m, S, ktiles, kt_per_split, tw, U, R, Z, norm_part, res_part,
                                    (int)blockIdx.x);
}

// Many independent panel contractions of one input and output type in one launch
// (the same step of the projection chains of many streams): job q owns workgroups
// [blk0_q, blk0_{q+1}); whether a job also sums the squares of its input (NORM) is
// per job.  Each job computes exactly what its own ttm_panel_kernel launch would.
struct PanelJob {
  const void* X;
  int64_t P, m, S, ktiles, kt_per_split;
  const double* U;
  void* Z;
  double* norm_part;  // NULL: no sum of squares of the input
  double* res_part;
  int tw, R, blk0;
};
constexpr int kMaxPanelJobs = 24;
struct PanelBatch {
  PanelJob j[kMaxPanelJobs];
  int n;
};

template <typename T, typename CT, bool RESE>
__global__ __launch_bounds__(256) void ttm_panel_group_kernel(PanelBatch b) {
  int q = 0;
  while (q + 1 < b.n && (int)blockIdx.x >= b.j[q + 1].blk0) ++q;
  const PanelJob& J = b.j[q];
  const int bid = (int)blockIdx.x - J.blk0;
  if (J.norm_part != nullptr)
    ttm_panel_body<T, CT, true, RESE>(static_cast<const T*>(J.X), J.P, J.m, J.S, J.ktiles, J.kt_per_split, J.tw,
                                      J.U, J.R, static_cast<CT*>(J.Z), J.norm_part, J.res_part, bid);
  else
    ttm_panel_body<T, CT, false, RESE>(static_cast<const T*>(J.X), J.P, J.m, J.S, J.ktiles, J.kt_per_split, J.tw,
                                       J.U, J.R, static_cast<CT*>(J.Z), nullptr, J.res_part, bid);
}

// --------------------------------------------------------------------------
// Register-direct FP32 blocks.  A wave takes a block of unfolding columns and
// loads rows 4 t + l / 16 (t < 4 TI) of 16 columns per "half" straight into the
// B-operand layout of the 16 x 16 x 4 matrix cores (row on l / 16, column on
// l % 16), NH halves per block:
//   SL = 0, column runs in whole blocks of 32 (S % 32 == 0): one p, 32
//     consecutive s; lane l loads columns 2 (l % 16) and 2 (l % 16) + 1 as one
//     float2, so the halves are the even and the odd columns (NH = 2);
//   SL = S <= 4 (short runs): 16 consecutive p, all S values of s; lane l loads
//     the S entries of row a of slab p0 + l % 16 in one load, half h = s (NH = S).
// Loads are buffer loads with the row step as a scalar offset; lanes past the
// last slab fall outside the buffer's extent and read zeros.
// --------------------------------------------------------------------------
// The register-direct kernels keep two sets of block registers: a wave's next block
// is loaded into one set while it works on the other.  The two copies of the block
// code must stay separate (merged, they would need a copy between the sets, which
// waits for the loads); the marker differs per set, and as a memory clobber it also
// keeps U^T re-read from LDS per block instead of held in registers.
template <int SET>
__device__ __forceinline__ void reg_set_mark() {
  if (SET == 0)
    asm volatile("; register set 0" ::: "memory");
  else
    asm volatile("; register set 1" ::: "memory");
}
constexpr std::integral_constant<int, 0> kSet0{};
constexpr std::integral_constant<int, 1> kSet1{};

// Cache policy of the block loads: non-temporal (the data is read once per pass; a
// level tensor written by the previous contraction keeps more of the last-level
// cache for its reader): 2-8 % faster contractions on the 48^4 x 4 stream.
constexpr int kNonTemporal = 2;

template <int SL>
struct RegBlock {
  static constexpr int NH = SL == 0 ? 2 : SL;
  __amdgpu_buffer_rsrc_t rs;
  int lane_off, step;
  int64_t p;   // SL = 0: the block's p; else the lane's slab
  int s0;      // SL = 0: first s of the block
  bool live;   // the lane's columns exist

  // valid = false: a buffer of extent 0, whose loads read zeros without touching memory
  __device__ __forceinline__ void setup(const float* X, int64_t P, int m, int64_t S, int blk, int g4, int c16,
                                        bool valid = true) {
    if (SL == 0) {
      const int S32 = (int)S;
      const int c0 = blk * 32;
      p = c0 / S32;
      s0 = c0 - (int)p * S32;
      rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X) + p * m * S + s0, (short)0,
                                             valid ? (m * S32 - s0) * 4 : 0, 0x00020000);
      lane_off = (2 * c16 + g4 * S32) * 4;
      step = 16 * S32;
      live = true;
    } else {
      const int64_t p0 = (int64_t)blk * 16;
      p = p0 + c16;
      s0 = 0;
      const int64_t left = P - p0 < 16 ? P - p0 : 16;
      rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X) + p0 * m * SL, (short)0,
                                             valid ? (int)(left * m * SL * 4) : 0, 0x00020000);
      lane_off = (c16 * m * SL + g4 * SL) * 4;
      step = 16 * SL;
      live = p < P;
    }
  }
  template <int NT>
  __device__ __forceinline__ void load(float (&x)[NT][NH], int m) const {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    typedef unsigned int u3 __attribute__((ext_vector_type(3)));
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      // SL = 0: rows past m lie past the extent, which ends with the block's slab, and
      // read zeros; the loads go out unconditionally, so the compiler can count the
      // loads in flight (a wave's next block is loaded while it works on the current)
      if (SL == 0 || 4 * t < m) {
        if (SL == 1) {
          x[t][0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, lane_off, t * step, kNonTemporal));
        } else if (SL == 0 || SL == 2) {
          const u2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, lane_off, t * step, kNonTemporal);
          x[t][0] = __uint_as_float(v.x);
          x[t][1] = __uint_as_float(v.y);
        } else if (SL == 3) {
          const u3 v = __builtin_amdgcn_raw_buffer_load_b96(rs, lane_off, t * step, kNonTemporal);
          x[t][0] = __uint_as_float(v.x);
          x[t][1] = __uint_as_float(v.y);
          x[t][NH > 2 ? 2 : 0] = __uint_as_float(v.z);
        } else {
          const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off, t * step, kNonTemporal);
          x[t][0] = __uint_as_float(v.x);
          x[t][1] = __uint_as_float(v.y);
          x[t][NH > 2 ? 2 : 0] = __uint_as_float(v.z);
          x[t][NH > 3 ? 3 : 0] = __uint_as_float(v.w);
        }
      } else {
#pragma unroll
        for (int h = 0; h < NH; ++h) x[t][h] = 0.f;
      }
    }
  }
  // address of (row r, half h) of the lane's column in the (P, R, S) output
  __device__ __forceinline__ int64_t out_index(int R, int64_t S, int r, int h, int c16) const {
    return SL == 0 ? (p * R + r) * S + s0 + 2 * c16 + h : (p * R + r) * SL + h;
  }
  __device__ __forceinline__ static int64_t blocks(int64_t P, int64_t S) {
    return SL == 0 ? P * S / 32 : (P + 15) / 16;
  }
};

// --------------------------------------------------------------------------
// FP32 contraction Z = U^T X for a mode with m <= 16 TI rows (m % 4 == 0) on
// register-direct blocks.  U^T (RT row tiles of 16) sits in LDS.  With RESE the
// residual X - U Z is formed in registers as well: register v of the Z
// accumulators is a valid B operand for the step whose k index l / 16 stands for
// row 16 rt + 4 (l / 16) + v of Z, and reading the rows of U in the order
// pi(q) = 4 (q % 4) + q / 4 makes row q of the product the row that the lane
// holds in its X registers.  Many waves per SIMD and a whole block of loads per
// wave keep the HBM pipe full without LDS staging.
// --------------------------------------------------------------------------
template <int TI, int RT, bool NORM, bool RESE, int SL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SL == 0 && TI * RT <= 6 ? 4 : 1))) void ttm_reg_kernel(
    const float* __restrict__ X, int64_t P, int m, int64_t S, const double* __restrict__ U, int R,
    float* __restrict__ Z, double* __restrict__ norm_part, double* __restrict__ res_part) {
  constexpr int NT = 4 * TI;
  constexpr int ULD = 16 * RT + 1;
  constexpr int NH = RegBlock<SL>::NH;
  extern __shared__ float sUr[];  // sUr[a * ULD + r]: U in FP32, zero outside m x R
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g4 = lane >> 4, c16 = lane & 15;
  stage_ut(U, m, R, 0, 16 * TI, ULD, m, sUr, ULD);
  __syncthreads();
  const int nblk = (int)RegBlock<SL>::blocks(P, S);
  const int pr = 4 * (c16 & 3) + (c16 >> 2);  // permuted row of U read by this lane
  double nrm = 0.0, res = 0.0;
  // one block on loaded registers
  auto block = [&](const RegBlock<SL>& B, float (&x)[NT][NH], auto set) {
    reg_set_mark<decltype(set)::value>();  // U^T is re-read from LDS per block, not held in registers
    if (NORM) {
      double n0 = 0.0, n1 = 0.0;  // two chains: the sums are not latency-bound
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          if (h & 1) n1 = fma((double)x[t][h], (double)x[t][h], n1);
          else n0 = fma((double)x[t][h], (double)x[t][h], n0);
        }
      }
      nrm += n0 + n1;
    }
    f4 zz[RT][NH];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      f4 c0[NH], c1[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) c0[h] = c1[h] = f4{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < NT; t += 2) {
        const float a0 = sUr[(4 * t + g4) * ULD + 16 * rt + c16];
        const float a1 = sUr[(4 * t + 4 + g4) * ULD + 16 * rt + c16];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          c0[h] = mfma16(a0, x[t][h], c0[h]);
          c1[h] = mfma16(a1, x[t + 1][h], c1[h]);
        }
      }
#pragma unroll
      for (int h = 0; h < NH; ++h) zz[rt][h] = c0[h] + c1[h];
      // register v: row 16 rt + 4 (l / 16) + v of Z
      if (B.live) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * rt + 4 * g4 + v;
          if (r < R) {
            if constexpr (SL == 0) {
              *reinterpret_cast<float2*>(Z + B.out_index(R, S, r, 0, c16)) = make_float2(zz[rt][0][v], zz[rt][1][v]);
            } else {
#pragma unroll
              for (int h = 0; h < NH; ++h) Z[B.out_index(R, S, r, h, c16)] = zz[rt][h][v];
            }
          }
        }
      }
    }
    if (RESE) {
      // the block's residual energy is summed in FP32 (relative error ~1e-5, far
      // below what the skip test resolves) and added to an FP64 total
      float e0 = 0.f, e1 = 0.f;
#pragma unroll
      for (int it = 0; it < TI; ++it) {
        f4 y[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) y[h] = f4{0, 0, 0, 0};
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float a = sUr[(16 * it + pr) * ULD + 16 * rt + 4 * g4 + v];
#pragma unroll
            for (int h = 0; h < NH; ++h) y[h] = mfma16(a, zz[rt][h][v], y[h]);
          }
        }
        // register v of the product: row 16 it + 4 v + l / 16 = the row of x[4 it + v]
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            const float d = x[4 * it + v][h] - y[h][v];
            if (h & 1) e1 = fmaf(d, d, e1);
            else e0 = fmaf(d, d, e0);
          }
        }
      }
      res += (double)e0 + (double)e1;
    }
  };
  // two register sets: the loads of a wave's next block are in flight while it
  // works on the current one (a copy between the sets would wait for them)
  const int step = gridDim.x * 4;
  RegBlock<SL> B0, B1;
  float x0[NT][NH], x1[NT][NH];
  // (past the last block the loads go to an empty buffer: no branch around them)
  int blk = blockIdx.x * 4 + wave;
  if (blk < nblk) {
    B0.setup(X, P, m, S, blk, g4, c16);
    B0.load(x0, m);
    for (;;) {
      const int b1 = blk + step;
      B1.setup(X, P, m, S, b1 < nblk ? b1 : blk, g4, c16, b1 < nblk);
      B1.load(x1, m);
      block(B0, x0, kSet0);
      if (b1 >= nblk) break;
      blk = b1 + step;
      B0.setup(X, P, m, S, blk < nblk ? blk : b1, g4, c16, blk < nblk);
      B0.load(x0, m);
      block(B1, x1, kSet1);
      if (blk >= nblk) break;
    }
  }
  if (NORM || RESE) {
    __shared__ double red[8];
    if (NORM) nrm = wave_sum(nrm);
    if (RESE) res = wave_sum(res);
    if (lane == 0) {
      red[wave] = nrm;
      red[4 + wave] = res;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (NORM) norm_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
      if (RESE) res_part[blockIdx.x] = (red[4] + red[5]) + (red[6] + red[7]);
    }
  }
}

// --------------------------------------------------------------------------
// FP32 residual Gram R R^T, R = M - U U^T M, on register-direct blocks (the
// shapes of ttm_reg_kernel).  A wave forms Z = U^T M and the residual of its block
// in registers, then feeds the matrix cores through a wave-private LDS transpose,
// one 16-column half at a time: the Gram operands want the row index on l % 16,
// the loaded layout has the column there.  Every wave accumulates all
// TI (TI + 1) / 2 upper 16 x 16 tiles; the four waves of a workgroup add theirs
// in wave order and the workgroup writes one FP64 partial (upper tiles of an
// m x m array), summed over the workgroups in a fixed order afterwards.
// --------------------------------------------------------------------------
constexpr int kGramRegLd = 17;  // row stride (floats) of a wave's 16-column transpose buffer

template <int TI, int RT, int SL>
__global__ __launch_bounds__(256) void gram_reg_kernel(const float* __restrict__ X, int64_t P, int m, int64_t S,
                                                       const double* __restrict__ U, int R,
                                                       double* __restrict__ part) {
  constexpr int NT = 4 * TI;
  constexpr int ULD = 16 * RT + 1;
  constexpr int NTILE = TI * (TI + 1) / 2;
  constexpr int WREG = 16 * TI * kGramRegLd;  // floats of one wave's transpose buffer
  constexpr int NH = RegBlock<SL>::NH;
  extern __shared__ float sgr[];
  float* sUr = sgr;                  // U, 16 TI x ULD
  float* sT = sgr + 16 * TI * ULD;   // 4 transpose buffers, later the tile sums
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g4 = lane >> 4, c16 = lane & 15;
  stage_ut(U, m, R, 0, 16 * TI, ULD, m, sUr, ULD);
  __syncthreads();
  float* myT = sT + wave * WREG;
  const int nblk = (int)RegBlock<SL>::blocks(P, S);
  const int pr = 4 * (c16 & 3) + (c16 >> 2);
  f4 acc[NTILE];
#pragma unroll
  for (int q = 0; q < NTILE; ++q) acc[q] = f4{0, 0, 0, 0};
  // one block on loaded registers
  auto block = [&](float (&x)[NT][NH], auto set) {
    reg_set_mark<decltype(set)::value>();
    {
      f4 zz[RT][NH];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        f4 c0[NH], c1[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) c0[h] = c1[h] = f4{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < NT; t += 2) {
          const float a0 = sUr[(4 * t + g4) * ULD + 16 * rt + c16];
          const float a1 = sUr[(4 * t + 4 + g4) * ULD + 16 * rt + c16];
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            c0[h] = mfma16(a0, x[t][h], c0[h]);
            c1[h] = mfma16(a1, x[t + 1][h], c1[h]);
          }
        }
#pragma unroll
        for (int h = 0; h < NH; ++h) zz[rt][h] = c0[h] + c1[h];
      }
#pragma unroll
      for (int it = 0; it < TI; ++it) {
        f4 y[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) y[h] = f4{0, 0, 0, 0};
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float a = sUr[(16 * it + pr) * ULD + 16 * rt + 4 * g4 + v];
#pragma unroll
            for (int h = 0; h < NH; ++h) y[h] = mfma16(a, zz[rt][h][v], y[h]);
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
          for (int h = 0; h < NH; ++h) x[4 * it + v][h] -= y[h][v];
        }
      }
    }
    // Gram of the block, one 16-column half at a time
#pragma unroll
    for (int h = 0; h < NH; ++h) {
#pragma unroll
      for (int t = 0; t < NT; ++t) myT[(4 * t + g4) * kGramRegLd + c16] = x[t][h];
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        float op[TI];
#pragma unroll
        for (int i = 0; i < TI; ++i) op[i] = myT[(16 * i + c16) * kGramRegLd + 4 * k4 + g4];
        int q = 0;
#pragma unroll
        for (int i = 0; i < TI; ++i) {
#pragma unroll
          for (int j = i; j < TI; ++j) {
            acc[q] = mfma16(op[i], op[j], acc[q]);
            ++q;
          }
        }
      }
    }
  };
  // two register sets, the next block's loads in flight during the current one.  The
  // loop runs whole pairs of blocks with no branch between a load and its use (the
  // compiler would sink the loads to their use); a block past the last is read from an
  // empty buffer as zeros, which add nothing to the Gram.
  const int step = gridDim.x * 4;
  const int first = blockIdx.x * 4 + wave;
  const int pairs = first < nblk ? ((nblk - 1 - first) / step + 2) / 2 : 0;
  RegBlock<SL> B0, B1;
  float x0[NT][NH], x1[NT][NH];
  if (pairs > 0) {
    B0.setup(X, P, m, S, first, g4, c16);
    B0.load(x0, m);
  }
  for (int q = 0; q < pairs; ++q) {
    const int b1 = first + (2 * q + 1) * step, b2 = b1 + step;
    B1.setup(X, P, m, S, b1 < nblk ? b1 : first, g4, c16, b1 < nblk);
    B1.load(x1, m);
    block(x0, kSet0);
    B0.setup(X, P, m, S, b2 < nblk ? b2 : first, g4, c16, b2 < nblk);
    B0.load(x0, m);
    block(x1, kSet1);
  }
  // the workgroup's sum in wave order, then one FP64 partial: tile (i, j), register
  // v of lane l is G[16 i + 4 (l / 16) + v][16 j + l % 16]
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int q = 0; q < NTILE; ++q) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float* d = sT + (q * 256 + v * 64 + lane);
          *d = (w == 0) ? acc[q][v] : *d + acc[q][v];
        }
      }
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.x * m * m;
  for (int e = threadIdx.x; e < NTILE * 256; e += 256) {
    const int q = e >> 8, v = (e >> 6) & 3, l = e & 63;
    int i = 0, qq = q;
    while (qq >= TI - i) {
      qq -= TI - i;
      ++i;
    }
    const int j = i + qq;
    const int row = 16 * i + 4 * (l >> 4) + v, col = 16 * j + (l & 15);
    if (row < m && col < m) out[row * m + col] = static_cast<double>(sT[e]);
  }
}

// --------------------------------------------------------------------------
// FP64 Gram of an FP32 mode unfolding on register-direct blocks: G = M M^T, or
// with RESID the residual Gram R R^T, R = M - U U^T M, the residual formed in
// FP64 registers (FP64 accumulator register v of lane l is row l / 16 + 4 v of a
// tile, so the rows of U are read in their natural order).  FP64 accumulators
// for every upper tile would not fit a wave's registers, so the four waves of a
// workgroup cooperate: each loads and projects one block, writes the residual of
// one half (16 columns) to its LDS region, and after a barrier every wave
// accumulates its own rows of upper tiles over all four regions.  The waves' tile
// sets are disjoint, so each writes its tiles of the workgroup's FP64 partial
// directly.
// --------------------------------------------------------------------------
constexpr int kGram64Ld = 17;  // row stride (doubles) of a wave's residual half in LDS

// Owner wave of upper tile (i, j) of a TI x TI tile grid.  Up to four tile rows the
// tiles go round robin in row-major order (TI = 3: two tiles for waves 0-1, one for
// waves 2-3, against three for wave 0 with whole rows); for 6 and 8 rows whole rows,
// paired so the waves get near-equal tile counts (8 rows: i with 7 - i, 9 tiles
// each; 6 rows: 6 | 5 + 1 | 4 + 2 | 3) and a wave reads each operand row once per
// k step.
__host__ __device__ constexpr int gram64_owner(int TI, int i, int j) {
  if (TI <= 4) {
    int q = j - i;
    for (int a = 0; a < i; ++a) q += TI - a;
    return q % 4;
  }
  return TI == 8 ? (i < 7 - i ? i : 7 - i) : (i < 4 ? i : TI - i);
}
__host__ __device__ constexpr int gram64_tiles(int TI, int W) {
  int n = 0;
  for (int i = 0; i < TI; ++i)
    for (int j = i; j < TI; ++j)
      if (gram64_owner(TI, i, j) == W) ++n;
  return n;
}
__host__ __device__ constexpr int gram64_max_tiles(int TI) {
  int n = 0;
  for (int w = 0; w < 4; ++w) n = gram64_tiles(TI, w) > n ? gram64_tiles(TI, w) : n;
  return n;
}
// true when wave W owns a tile in tile row or tile column i (it needs operand row i)
__host__ __device__ constexpr bool gram64_uses(int TI, int W, int i) {
  for (int k = 0; k < TI; ++k)
    if (gram64_owner(TI, k < i ? k : i, k < i ? i : k) == W) return true;
  return false;
}

// wave W's tiles, accumulated over the four waves' residual halves in LDS
template <int TI, int W, int NA>
__device__ __forceinline__ void gram64_accumulate(const double* sRw, int wreg, int c16, int g4, d4 (&acc)[NA]) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const double* rw = sRw + w * wreg;
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      double op[TI];
#pragma unroll
      for (int i = 0; i < TI; ++i)
        op[i] = gram64_uses(TI, W, i) ? rw[(16 * i + c16) * kGram64Ld + 4 * k4 + g4] : 0.0;
      int q = 0;
#pragma unroll
      for (int i = 0; i < TI; ++i) {
#pragma unroll
        for (int j = i; j < TI; ++j) {
          if (gram64_owner(TI, i, j) == W) {
            acc[q] = mfma16(op[i], op[j], acc[q]);
            ++q;
          }
        }
      }
    }
  }
}

template <int TI, int W, int NA>
__device__ __forceinline__ void gram64_store(const d4 (&acc)[NA], int m, int c16, int g4, double* out) {
  int q = 0;
#pragma unroll
  for (int i = 0; i < TI; ++i) {
#pragma unroll
    for (int j = i; j < TI; ++j) {
      if (gram64_owner(TI, i, j) == W) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * i + g4 + 4 * v, col = 16 * j + c16;
          if (row < m && col < m) out[row * m + col] = acc[q][v];
        }
        ++q;
      }
    }
  }
}

template <int TI, int RT, bool RESID, int SL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SL == 0 && TI * RT <= 6 ? 2 : 1))) void gram_reg64_kernel(const float* __restrict__ X, int64_t P, int m, int64_t S,
                                                         const double* __restrict__ U, int R,
                                                         double* __restrict__ part) {
  constexpr int NT = 4 * TI;
  constexpr int ULD = 16 * RT + 1;
  constexpr int NH = RegBlock<SL>::NH;
  constexpr int WREG = 16 * TI * kGram64Ld;
  extern __shared__ double sg64[];
  double* sUd = sg64;                                  // U (RESID), 16 TI x ULD
  double* sRw = sg64 + (RESID ? 16 * TI * ULD : 0);    // four residual halves
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g4 = lane >> 4, c16 = lane & 15;
  if (RESID) stage_ut(U, m, R, 0, 16 * TI, ULD, m, sUd, ULD);
  // Up to four row tiles every wave accumulates every upper tile over its own blocks
  // (the accumulators fit), so the waves never wait for each other; the four sets are
  // added in wave order at the end.  Larger modes share the tiles out as above.
  constexpr bool ALL = TI <= 4;
  constexpr int NA = ALL ? TI * (TI + 1) / 2 : gram64_max_tiles(TI);
  d4 acc[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) acc[u] = d4{0, 0, 0, 0};
  double* myR = sRw + wave * WREG;
  const int nblk = (int)RegBlock<SL>::blocks(P, S);
  __syncthreads();
  // one step of the workgroup (block g0 + wave of every wave; zeros past the last)
  auto block = [&](float (&x)[NT][NH], auto set) {
    reg_set_mark<decltype(set)::value>();
    d4 zz[RESID ? RT : 1][NH];
    if (RESID) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        d4 c0[NH], c1[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) c0[h] = c1[h] = d4{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < NT; t += 2) {
          const double a0 = sUd[(4 * t + g4) * ULD + 16 * rt + c16];
          const double a1 = sUd[(4 * t + 4 + g4) * ULD + 16 * rt + c16];
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            c0[h] = mfma16(a0, (double)x[t][h], c0[h]);
            c1[h] = mfma16(a1, (double)x[t + 1][h], c1[h]);
          }
        }
#pragma unroll
        for (int h = 0; h < NH; ++h) zz[rt][h] = c0[h] + c1[h];
      }
    }
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      // this wave's residual half into its region: row 4 t + l / 16, column l % 16
#pragma unroll
      for (int it = 0; it < TI; ++it) {
        d4 y = d4{0, 0, 0, 0};
        if (RESID) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const double a = sUd[(16 * it + c16) * ULD + 16 * rt + 4 * v + g4];
              y = mfma16(a, zz[rt][h][v], y);
            }
          }
        }
        // register v of the product is row 16 it + l / 16 + 4 v = the row of x[4 it + v]
#pragma unroll
        for (int v = 0; v < 4; ++v)
          myR[(16 * it + 4 * v + g4) * kGram64Ld + c16] = (double)x[4 * it + v][h] - y[v];
      }
      if constexpr (ALL) {
        // the wave's own half only: it reads back its own LDS writes, no barrier
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4) {
          double op[TI];
#pragma unroll
          for (int i = 0; i < TI; ++i) op[i] = myR[(16 * i + c16) * kGram64Ld + 4 * k4 + g4];
          int q = 0;
#pragma unroll
          for (int i = 0; i < TI; ++i) {
#pragma unroll
            for (int j = i; j < TI; ++j) {
              acc[q] = mfma16(op[i], op[j], acc[q]);
              ++q;
            }
          }
        }
      } else {
        __syncthreads();
        switch (wave) {
          case 0: gram64_accumulate<TI, 0>(sRw, WREG, c16, g4, acc); break;
          case 1: gram64_accumulate<TI, 1>(sRw, WREG, c16, g4, acc); break;
          case 2: gram64_accumulate<TI, 2>(sRw, WREG, c16, g4, acc); break;
          default: gram64_accumulate<TI, 3>(sRw, WREG, c16, g4, acc); break;
        }
        __syncthreads();
      }
    }
  };
  // two register sets, the next step's loads in flight during the current one.  The
  // loop runs whole pairs of steps with no branch between a load and its use (the
  // compiler would sink the loads to their use); a wave past the last block reads an
  // empty buffer as zeros (no memory access), which add nothing to the Gram.
  const int step = gridDim.x * 4;
  const int g0 = blockIdx.x * 4;  // uniform over the workgroup
  const int pairs = g0 < nblk ? ((nblk - 1 - g0) / step + 2) / 2 : 0;
  RegBlock<SL> B0, B1;
  float x0[NT][NH], x1[NT][NH];
  auto setup = [&](RegBlock<SL>& B, int g) {
    const bool ok = g + wave < nblk;
    B.setup(X, P, m, S, ok ? g + wave : 0, g4, c16, ok);
  };
  if (pairs > 0) {
    setup(B0, g0);
    B0.load(x0, m);
  }
  for (int q = 0; q < pairs; ++q) {
    setup(B1, g0 + (2 * q + 1) * step);
    B1.load(x1, m);
    block(x0, kSet0);
    setup(B0, g0 + (2 * q + 2) * step);
    B0.load(x0, m);
    block(x1, kSet1);
  }
  double* out = part + (int64_t)blockIdx.x * m * m;
  if constexpr (ALL) {
    // the four waves' tiles added in wave order through LDS (the residual regions,
    // free now), then one FP64 partial: tile (i, j), register v of lane l is
    // G[16 i + l / 16 + 4 v][16 j + l % 16]
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
      if (wave == w) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double* d = sRw + (q * 256 + v * 64 + lane);
            *d = (w == 0) ? acc[q][v] : *d + acc[q][v];
          }
        }
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < NA * 256; e += 256) {
      const int q = e >> 8, v = (e >> 6) & 3, l = e & 63;
      int i = 0, qq = q;
      while (qq >= TI - i) {
        qq -= TI - i;
        ++i;
      }
      const int j = i + qq;
      const int row = 16 * i + (l >> 4) + 4 * v, col = 16 * j + (l & 15);
      if (row < m && col < m) out[row * m + col] = sRw[e];
    }
  } else {
    switch (wave) {
      case 0: gram64_store<TI, 0>(acc, m, c16, g4, out); break;
      case 1: gram64_store<TI, 1>(acc, m, c16, g4, out); break;
      case 2: gram64_store<TI, 2>(acc, m, c16, g4, out); break;
      default: gram64_store<TI, 3>(acc, m, c16, g4, out); break;
    }
  }
}

// --------------------------------------------------------------------------
// FP64 contraction Z = U^T X (FP32 or FP64 X) for the shapes of ttm_reg_kernel, on
// FP64 matrix cores with operands straight from registers: the same blocks of 32
// columns and the same loads (two adjacent columns per lane and row), U^T in LDS,
// the R / 16 output row tiles one after another.  FP64 accumulator register v of
// lane l is row l / 16 + 4 v of the tile.
// --------------------------------------------------------------------------
template <typename T, int TI, bool NORM>
__global__ __launch_bounds__(256) void ttm_reg64_kernel(const T* __restrict__ X, int64_t P, int m, int64_t S,
                                                        const double* __restrict__ U, int R, double* __restrict__ Z,
                                                        double* __restrict__ norm_part) {
  constexpr int NT = 4 * TI;
  extern __shared__ double sUd[];  // sUd[a * uld + r]: U, zero outside m x R
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g4 = lane >> 4, c16 = lane & 15;
  const int nrt = (R + 15) >> 4, uld = 16 * nrt + 1;
  stage_ut(U, m, R, 0, 16 * TI, uld, m, sUd, uld);
  __syncthreads();
  constexpr int esz = (int)sizeof(T);
  const int lane_off = (2 * c16 + g4 * (int)S) * esz;
  const int step = 4 * (int)S * esz;
  const int S32 = (int)S;
  const int nblk = (int)(P * S / 32);
  double nrm = 0.0;
  for (int blk = blockIdx.x * 4 + wave; blk < nblk; blk += gridDim.x * 4) {
    asm volatile("" ::: "memory");  // U^T is re-read from LDS per block, not held in registers
    const int c0 = blk * 32;
    const int p = c0 / S32, s0 = c0 - p * S32;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(X) + (int64_t)p * m * S + s0, (short)0, (m * S32 - s0) * esz, 0x00020000);
    T x0[NT], x1[NT];  // converted to FP64 where they feed the matrix cores
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (4 * t < m) {
        if constexpr (esz == 4) {
          typedef unsigned int u2 __attribute__((ext_vector_type(2)));
          const u2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, lane_off, t * step, 0);
          x0[t] = __uint_as_float(v.x);
          x1[t] = __uint_as_float(v.y);
        } else {
          typedef unsigned int u4 __attribute__((ext_vector_type(4)));
          const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off, t * step, 0);
          x0[t] = __hiloint2double((int)v.y, (int)v.x);
          x1[t] = __hiloint2double((int)v.w, (int)v.z);
        }
      } else {
        x0[t] = T(0);
        x1[t] = T(0);
      }
    }
    if (NORM) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        nrm = fma((double)x0[t], (double)x0[t], nrm);
        nrm = fma((double)x1[t], (double)x1[t], nrm);
      }
    }
    for (int rt = 0; rt < nrt; ++rt) {
      d4 e0 = d4{0, 0, 0, 0}, e1 = e0, o0 = e0, o1 = e0;
#pragma unroll
      for (int t = 0; t < NT; t += 2) {
        const double a0 = sUd[(4 * t + g4) * uld + 16 * rt + c16];
        const double a1 = sUd[(4 * t + 4 + g4) * uld + 16 * rt + c16];
        T b0 = x0[t], b1 = x1[t], b2 = x0[t + 1], b3 = x1[t + 1];
        if constexpr (esz == 4) asm volatile("" : "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3));  // convert here
        e0 = mfma16(a0, (double)b0, e0);
        o0 = mfma16(a0, (double)b1, o0);
        e1 = mfma16(a1, (double)b2, e1);
        o1 = mfma16(a1, (double)b3, o1);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rt + g4 + 4 * v;
        if (r < R)
          *reinterpret_cast<double2*>(Z + (p * R + r) * S + s0 + 2 * c16) =
              make_double2(e0[v] + e1[v], o0[v] + o1[v]);
      }
    }
  }
  if (NORM) {
    __shared__ double red[4];
    nrm = wave_sum(nrm);
    if (lane == 0) red[wave] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) norm_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

constexpr int TUS = 65;  // LDS row stride (doubles) of the staged U chunk of the expansion

// --------------------------------------------------------------------------
// TTM contraction for modes with more than 128 rows (transfer nodes, large
// leaves): Z[p, r, s] = sum_a U[a, r] X[p, a, s] on FP64 matrix cores.  A
// workgroup owns 16 unfolding columns and every output row (R <= 64); its four
// waves split the row steps of a (step q of a chunk goes to wave q % 4), so small
// column counts (the level tensors of transfer nodes) still spread over many
// waves.  U^T is staged in dynamic LDS (reads coalesced along a), whole up to
// kDirectLdsDoubles and otherwise in chunks of rows of a; each wave keeps the X
// operands of its next eight steps in flight.  The four partial products are
// added in wave order through LDS.
// --------------------------------------------------------------------------
constexpr int kDirectLdsDoubles = 19968;  // U chunk: chunk x (RP + 1) doubles of dynamic LDS
constexpr unsigned kDirectColsMinBlocks = 512;  // column blocks from which whole blocks go to waves

// SQ: also the workgroup partials of ||X||^2 (in_part) and ||Z||^2 (out_part)
// With gridDim.y > 1 workgroup (x, y) takes rows [y rows, (y + 1) rows) only and writes
// its partial product to Zp + y P R S (summed by split_sum_kernel), and ||X||^2 of its
// rows to in_part[y gridDim.x + x].
template <typename T, bool SQ>
__global__ __launch_bounds__(256) void ttm_direct_kernel(const T* __restrict__ X, int64_t P, int64_t m, int64_t S,
                                                         const double* __restrict__ U, int R, int chunk,
                                                         double* __restrict__ Z, double* __restrict__ in_part,
                                                         double* __restrict__ out_part, int64_t rows,
                                                         double* __restrict__ Zp) {
  extern __shared__ double sU[];  // sU[a][r] (chunk rows of ULD), then the wave partials
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int RP = (R + 15) & ~15, ULD = RP + 1, rt = RP >> 4;
  const int64_t K = P * S;
  const int64_t c = (int64_t)blockIdx.x * 16 + (lane & 15);
  const bool cv = c < K;
  const int64_t base = cv ? col_base(c, m, S) : 0;
  const int kr = lane >> 4;  // row of the 4-row step this lane feeds
  d4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  double xsq = 0.0;
  const bool split = gridDim.y > 1;
  const int64_t lo = (int64_t)blockIdx.y * rows, hi = min(m, lo + rows);
  for (int64_t a0 = lo; a0 < hi; a0 += chunk) {
    const int ac = (int)min<int64_t>(chunk, hi - a0);
    const int ac4 = (ac + 3) & ~3;
    __syncthreads();
    stage_ut(U, m, R, a0, ac4, RP, ac, sU, ULD);
    __syncthreads();
    const int nst = ac4 >> 2;
    const T* xp = X + base + a0 * S;
    T b[8];  // in the data type until used: a conversion at the load would wait for it
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int a = 4 * (wave + 4 * q) + kr;
      b[q] = (cv && a < ac) ? xp[(int64_t)a * S] : T(0);
    }
    for (int j = 0; wave + 4 * j < nst; j += 8) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int st = wave + 4 * (j + q);
        if (st < nst) {
          const double bv = static_cast<double>(b[q]);
          if (SQ) xsq = fma(bv, bv, xsq);
          const int an = 4 * (st + 32) + kr;
          b[q] = (cv && an < ac) ? xp[(int64_t)an * S] : T(0);
          const double* ua = sU + (4 * st + kr) * ULD + (lane & 15);
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (t < rt) acc[t] = mfma16(ua[t * 16], bv, acc[t]);
        }
      }
    }
  }
  // partials of waves 1-3 through LDS, added to wave 0's in wave order
  __syncthreads();
  if (wave > 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < rt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) sU[(((wave - 1) * 4 + t) * 4 + v) * 64 + lane] = acc[t][v];
      }
  }
  __syncthreads();
  double zsq = 0.0;
  if (wave == 0 && cv) {
    const int64_t p = c / S, sidx = c - (c / S) * S;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < rt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double z = acc[t][v];
#pragma unroll
          for (int w = 0; w < 3; ++w) z += sU[((w * 4 + t) * 4 + v) * 64 + lane];
          const int r = t * 16 + MA<double>::row(lane, v);
          if (r < R) {
            if (split) {
              Zp[(int64_t)blockIdx.y * P * R * S + (p * R + r) * S + sidx] = z;
            } else {
              Z[(p * R + r) * S + sidx] = z;
              if (SQ) zsq = fma(z, z, zsq);
            }
          }
        }
      }
    }
  }
  if (SQ) {
    __shared__ double red[4];
    xsq = wave_sum(xsq);
    zsq = wave_sum(zsq);
    if (lane == 0) red[wave] = xsq;
    __syncthreads();
    if (threadIdx.x == 0) {
      in_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
      if (!split) out_part[blockIdx.x] = zsq;
    }
  }
}

// Z = the sum of the nsplit partial products (in split order); with SQ the
// workgroup partials of ||Z||^2
template <bool SQ>
__global__ __launch_bounds__(256) void split_sum_kernel(const double* __restrict__ Zp, int nsplit, int64_t n,
                                                        double* __restrict__ Z, double* __restrict__ out_part) {
  double zsq = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double z = Zp[e];
    for (int k = 1; k < nsplit; ++k) z += Zp[(int64_t)k * n + e];
    Z[e] = z;
    if (SQ) zsq = fma(z, z, zsq);
  }
  if (SQ) {
    __shared__ double red[4];
    zsq = wave_sum(zsq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = zsq;
    __syncthreads();
    if (threadIdx.x == 0) out_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// The same contraction for many columns: each wave owns whole 16-column blocks (two
// at a time) and runs every row of them, so no partial sum crosses waves; the
// workgroup's eight column blocks share each staged chunk of U, and workgroups loop
// over tiles of eight blocks.  With SQ the workgroup partials of ||X||^2 and ||Z||^2.
template <typename T, bool SQ>
__global__ __launch_bounds__(256) void ttm_direct_cols_kernel(const T* __restrict__ X, int64_t P, int64_t m,
                                                              int64_t S, const double* __restrict__ U, int R,
                                                              int chunk, double* __restrict__ Z,
                                                              double* __restrict__ in_part,
                                                              double* __restrict__ out_part, int64_t rows,
                                                              double* __restrict__ Zp) {
  extern __shared__ double sU[];  // sU[a][r], chunk rows of ULD
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int RP = (R + 15) & ~15, ULD = RP + 1, rt = RP >> 4;
  const int64_t K = P * S;
  const int64_t ncb = (K + 15) / 16;
  const int kr = lane >> 4;
  double xsq = 0.0, zsq = 0.0;
  const bool split = gridDim.y > 1;  // rows [y rows, (y + 1) rows) into Zp + y P R S
  const int64_t lo = (int64_t)blockIdx.y * rows, hi = min(m, lo + rows);
  for (int64_t cb0 = (int64_t)blockIdx.x * 8; cb0 < ncb; cb0 += (int64_t)gridDim.x * 8) {  // uniform
    int64_t c[2], base[2];
    bool cv[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      c[j] = (cb0 + 2 * wave + j) * 16 + (lane & 15);
      cv[j] = c[j] < K;
      base[j] = cv[j] ? col_base(c[j], m, S) : 0;
    }
    d4 acc[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[j][t] = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t a0 = lo; a0 < hi; a0 += chunk) {
      const int ac = (int)min<int64_t>(chunk, hi - a0);
      const int ac4 = (ac + 3) & ~3;
      __syncthreads();
      stage_ut(U, m, R, a0, ac4, RP, ac, sU, ULD);
      __syncthreads();
      const int nst = ac4 >> 2;
      for (int st = 0; st < nst; st += 4) {  // four row steps of both blocks: eight loads in flight
        T b[2][4];  // converted at use: all eight loads go out first
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int a = 4 * (st + q) + kr;
#pragma unroll
          for (int j = 0; j < 2; ++j) b[j][q] = (cv[j] && a < ac) ? X[base[j] + (a0 + a) * S] : T(0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (st + q < nst) {
            const double* ua = sU + (4 * (st + q) + kr) * ULD + (lane & 15);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              const double bv = static_cast<double>(b[j][q]);
              if (SQ) xsq = fma(bv, bv, xsq);
#pragma unroll
              for (int t = 0; t < 4; ++t)
                if (t < rt) acc[j][t] = mfma16(ua[t * 16], bv, acc[j][t]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!cv[j]) continue;
      const int64_t p = c[j] / S, sidx = c[j] - (c[j] / S) * S;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < rt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = t * 16 + MA<double>::row(lane, v);
            if (r < R) {
              const double z = acc[j][t][v];
              if (split) {
                Zp[(int64_t)blockIdx.y * P * R * S + (p * R + r) * S + sidx] = z;
              } else {
                Z[(p * R + r) * S + sidx] = z;
                if (SQ) zsq = fma(z, z, zsq);
              }
            }
          }
        }
      }
    }
  }
  if (SQ) {
    __shared__ double red[8];
    xsq = wave_sum(xsq);
    zsq = wave_sum(zsq);
    if (lane == 0) {
      red[wave] = xsq;
      red[4 + wave] = zsq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      in_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
      if (!split) out_part[blockIdx.x] = (red[4] + red[5]) + (red[6] + red[7]);
    }
  }
}

// --------------------------------------------------------------------------
// Contraction of a mode of at most kSmallModeM rows (such as a channel mode), one
// unfolding column per thread in FP64: z = U^T x (stored as CT), optionally
// ||x||^2 and the residual energy ||x - U z||^2 of the column, summed per
// workgroup in a fixed order.  Such modes have many columns of a few values each,
// which the panel kernel's 128-row tiles would mostly leave empty.
// --------------------------------------------------------------------------
constexpr int kSmallModeM = 8;

template <typename T, typename CT, bool NORM, bool RESE>
__global__ __launch_bounds__(256) void ttm_small_kernel(const T* __restrict__ X, int64_t P, int m, int64_t S,
                                                        const double* __restrict__ U, int R, CT* __restrict__ Z,
                                                        double* __restrict__ norm_part,
                                                        double* __restrict__ res_part) {
  __shared__ double sUs[kSmallModeM * kSmallModeM];  // sUs[a * R + r]
  for (int e = threadIdx.x; e < m * R; e += 256) {
    const int a = e / R, r = e - (e / R) * R;
    sUs[e] = U[a + (int64_t)r * m];
  }
  __syncthreads();
  const int64_t K = P * S;
  double nrm = 0.0, res = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < K; c += (int64_t)gridDim.x * 256) {
    const int64_t p = c / S, sx = c - (c / S) * S;
    const T* xp = X + p * m * S + sx;
    double x[kSmallModeM], y[kSmallModeM];
#pragma unroll
    for (int a = 0; a < kSmallModeM; ++a) {
      x[a] = a < m ? static_cast<double>(xp[(int64_t)a * S]) : 0.0;
      y[a] = 0.0;
    }
    if (NORM) {
#pragma unroll
      for (int a = 0; a < kSmallModeM; ++a) nrm = fma(x[a], x[a], nrm);
    }
#pragma unroll
    for (int r = 0; r < kSmallModeM; ++r) {
      if (r < R) {
        double z = 0.0;
#pragma unroll
        for (int a = 0; a < kSmallModeM; ++a)
          if (a < m) z = fma(sUs[a * R + r], x[a], z);
        Z[(p * R + r) * S + sx] = static_cast<CT>(z);
        if (RESE) {
#pragma unroll
          for (int a = 0; a < kSmallModeM; ++a)
            if (a < m) y[a] = fma(sUs[a * R + r], z, y[a]);
        }
      }
    }
    if (RESE) {
#pragma unroll
      for (int a = 0; a < kSmallModeM; ++a) {
        const double d = x[a] - y[a];
        res = fma(d, d, res);
      }
    }
  }
  if (NORM || RESE) {
    __shared__ double red[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (NORM) nrm = wave_sum(nrm);
    if (RESE) res = wave_sum(res);
    if (lane == 0) {
      red[wave] = nrm;
      red[4 + wave] = res;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (NORM) norm_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
      if (RESE) res_part[blockIdx.x] = (red[4] + red[5]) + (red[6] + red[7]);
    }
  }
}

// --------------------------------------------------------------------------
// TTM expansion out[p, a, s] = (M[p,a,s] -) sum_t U[a, t] Z[p, t, s]  (FP64 MFMA)
// One wave per 16 columns and 64 rows of a (blockIdx.y); all of the wave's Z
// operands (R <= 64: at most 16 steps of 4) are loaded before the first product.
// --------------------------------------------------------------------------
template <typename TM, typename TO>
__global__ __launch_bounds__(256) void ttm_expand_kernel(const double* __restrict__ Z, int64_t P, int R, int64_t S,
                                                         const double* __restrict__ U, int64_t m,
                                                         const TM* __restrict__ M, TO* __restrict__ out) {
  __shared__ double sU[64 * TUS];  // sU[t][a_local]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t K = P * S;
  const int64_t a0 = (int64_t)blockIdx.y * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int t = e >> 6, al = e & 63;
    sU[t * TUS + al] = (t < R && a0 + al < m) ? U[(a0 + al) + (int64_t)t * m] : 0.0;
  }
  const int64_t c = ((int64_t)blockIdx.x * 4 + wave) * 16 + (lane & 15);
  const bool cv = c < K;
  const int64_t p = cv ? c / S : 0;
  const int64_t sidx = cv ? c - p * S : 0;
  const int64_t zb = p * R * S + sidx;
  const int kr = lane >> 4;
  const int nst = (R + 3) >> 2;
  double b[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int t = 4 * q + kr;
    b[q] = (cv && t < R) ? Z[zb + (int64_t)t * S] : 0.0;
  }
  __syncthreads();
  d4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  const int at_n = (int)min<int64_t>(4, (m - a0 + 15) >> 4);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (q < nst) {
      const int t = 4 * q + kr;
#pragma unroll
      for (int at = 0; at < 4; ++at)
        if (at < at_n) acc[at] = mfma16(sU[t * TUS + at * 16 + (lane & 15)], b[q], acc[at]);
    }
  }
  if (!cv) return;
#pragma unroll
  for (int at = 0; at < 4; ++at) {
    if (at < at_n) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t a = a0 + at * 16 + MA<double>::row(lane, v);
        if (a < m) {
          const int64_t idx = (p * m + a) * S + sidx;
          double val = acc[at][v];
          if (M != nullptr) val = ld(M, idx) - val;
          out[idx] = static_cast<TO>(val);
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

// U (alpha x r_old) and V (alpha x rR), column-major with leading dimension alpha,
// live in LDS or in global memory (a compile-time choice through the inlined
// pointers); Cs is rR x max(r_old, rR) of LDS.
__device__ __forceinline__ void orth_body(const double* U, int64_t alpha, int r_old, double* V, int rR, double* Cs,
                                          double* core, const double* Uold_g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // ---- two passes of classical Gram-Schmidt against the old basis
  for (int pass = 0; pass < 2 && r_old > 0; ++pass) {
    for (int e = wave; e < r_old * rR; e += 4) {
      const int i = e / rR, j = e - (e / rR) * rR;
      double acc = 0.0;
      for (int64_t a = lane; a < alpha; a += 64) acc = fma(U[a + (int64_t)i * alpha], V[a + (int64_t)j * alpha], acc);
      acc = wave_sum(acc);
      if (lane == 0) Cs[i * rR + j] = acc;
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < alpha * rR; e += 256) {
      const int64_t a = e % alpha;
      const int j = (int)(e / alpha);
      double acc = V[a + (int64_t)j * alpha];
      for (int i = 0; i < r_old; ++i) acc = fma(-U[a + (int64_t)i * alpha], Cs[i * rR + j], acc);
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
          double sum = Cs[i * rR + j];
          for (int k = 0; k < j; ++k) sum -= Cs[i * rR + k] * Cs[j * rR + k];
          Cs[i * rR + j] = sum / d;
        }
      }
    }
    __syncthreads();
    // each row x of V solves x_new L^T = x  (forward substitution over columns)
    for (int64_t a = threadIdx.x; a < alpha; a += 256) {
      for (int j = 0; j < rR; ++j) {
        double sum = V[a + (int64_t)j * alpha];
        for (int k = 0; k < j; ++k) sum -= V[a + (int64_t)k * alpha] * Cs[j * rR + k];
        V[a + (int64_t)j * alpha] = sum / Cs[j * rR + j];
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
  if (core != Uold_g)
    for (int64_t e = threadIdx.x; e < alpha * r_old; e += 256) core[e] = Uold_g[e];
}

constexpr int kOrthLdsDoubles = 12288;  // U_old and V staged in LDS up to this size (96 KiB)

struct OrthBatch {
  OrthJob j[kMaxOrthJobs];
};

__global__ __launch_bounds__(256) void orth_expand_kernel(OrthBatch b) {
  const OrthJob J = b.j[blockIdx.x];
  extern __shared__ double osm[];
  double* Cs = osm;  // 64 x 64
  const int64_t alpha = J.alpha;
  const int r_old = J.r_old, rR = J.rR;
  const int64_t need = alpha * (int64_t)(r_old + rR);
  if (need <= kOrthLdsDoubles) {
    double* sU = osm + 64 * 64;
    double* sV = sU + alpha * r_old;
    for (int64_t e = threadIdx.x; e < alpha * r_old; e += 256) sU[e] = J.U_old[e];
    for (int64_t e = threadIdx.x; e < alpha * rR; e += 256) sV[e] = J.V[e];
    __syncthreads();
    orth_body(sU, alpha, r_old, sV, rR, Cs, J.core, J.U_old);
  } else {
    orth_body(J.U_old, alpha, r_old, J.V, rR, Cs, J.core, J.U_old);
  }
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

template <typename T>
__global__ void root_append_kernel(const T* __restrict__ C1, int64_t N, int r11, int r12,
                                   double* __restrict__ root, int64_t n_acc, int rcap) {
  const int64_t n = N * rcap * rcap;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t s = e / ((int64_t)rcap * rcap);
    const int64_t rem = e - s * rcap * rcap;
    const int i = (int)(rem / rcap), j = (int)(rem - (rem / rcap) * rcap);
    root[(n_acc + s) * rcap * rcap + rem] =
        (i < r11 && j < r12) ? static_cast<double>(C1[(s * r11 + i) * r12 + j]) : 0.0;
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
void sums_defer_begin(std::vector<SumJob>* list) { t_defer = list; }
void sums_defer_end() { t_defer = nullptr; }

void reduce_batch(const std::vector<SumJob>& jobs, hipStream_t s) {
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  for (size_t b0 = 0; b0 < jobs.size(); b0 += kMaxSumJobs) {
    const int n = (int)std::min<size_t>(kMaxSumJobs, jobs.size() - b0);
    SumBatch b;
    for (int i = 0; i < n; ++i) b.j[i] = jobs[b0 + i];
    reduce_many_kernel<<<n, 256, 0, s>>>(b);
  }
}

void sumsq(const void* x, Elem t, int64_t n, double* partials, double* out, hipStream_t s) {
  ProfScope prof(KKind::Sumsq, s, 2.0 * n, (double)n * (t == Elem::F32 ? 4 : 8));
  if (t == Elem::F32)
    sumsq_partial_kernel<float><<<kSumsqBlocks, 256, 0, s>>>(static_cast<const float*>(x), n, partials);
  else
    sumsq_partial_kernel<double><<<kSumsqBlocks, 256, 0, s>>>(static_cast<const double*>(x), n, partials);
  finish_sum(partials, kSumsqBlocks, out, s);
}

// Per-segment sums of squares: segment g is x[g * len, (g + 1) * len).  Grid
// (blocks, segments) of partials, then one workgroup per segment sums its partials
// in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void sumsq_seg_kernel(const T* __restrict__ x, int64_t len,
                                                        double* __restrict__ part) {
  const T* xs = x + (int64_t)blockIdx.y * len;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    const double v = ld(xs, i);
    acc = fma(v, v, acc);
  }
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void reduce_seg_kernel(const double* __restrict__ part, int n,
                                                         double* __restrict__ out) {
  reduce_body(part + (int64_t)blockIdx.x * n, n, out + blockIdx.x);
}

void sumsq_segments(const void* x, Elem t, int64_t nseg, int64_t len, double* partials, double* out,
                    hipStream_t s) {
  if (nseg <= 0 || len <= 0) return;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kSegBlocks, len / 4096));
  ProfScope prof(KKind::Sumsq, s, 2.0 * nseg * len, (double)nseg * len * (t == Elem::F32 ? 4 : 8));
  const dim3 grid((unsigned)blocks, (unsigned)nseg);
  if (t == Elem::F32)
    sumsq_seg_kernel<float><<<grid, 256, 0, s>>>(static_cast<const float*>(x), len, partials);
  else
    sumsq_seg_kernel<double><<<grid, 256, 0, s>>>(static_cast<const double*>(x), len, partials);
  reduce_seg_kernel<<<(unsigned)nseg, 256, 0, s>>>(partials, blocks, out);
}

size_t panel_lds_bytes(bool resid, int R, size_t esz) {
  const int RP = (R + 15) & ~15;
  size_t n = (size_t)GBK * GLD;
  if (resid) n += (size_t)GB * (RP + 1) + (size_t)RP * ZLD;
  return n * esz;
}

template <typename T, typename CT, bool RESID, int MT>
void launch_panel_t(const void* x, const ModeView& v, const GramPlan& g, const double* U, int R, double* part,
                    hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_panel_kernel<T, CT, RESID, MT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    attr = true;
  }
  gram_panel_kernel<T, CT, RESID, MT><<<g.nsplit, 256, panel_lds_bytes(RESID, R, sizeof(CT)), s>>>(
      static_cast<const T*>(x), v.P, v.m, v.S, g.ktiles, g.kt_per_split, g.tw, U, R, part);
}

template <typename T, typename CT, bool RESID>
void launch_panel_mt(const void* x, const ModeView& v, const GramPlan& g, const double* U, int R, double* part,
                     hipStream_t s) {
  const int tI = (int)((v.m + 15) / 16);
  const int mt = (tI * (tI + 1) / 2 + 3) / 4;  // upper 16x16 tiles per wave
  switch (mt) {
    case 1: launch_panel_t<T, CT, RESID, 1>(x, v, g, U, R, part, s); break;
    case 2: launch_panel_t<T, CT, RESID, 2>(x, v, g, U, R, part, s); break;
    case 3: launch_panel_t<T, CT, RESID, 3>(x, v, g, U, R, part, s); break;
    case 4: launch_panel_t<T, CT, RESID, 4>(x, v, g, U, R, part, s); break;
    case 6: launch_panel_t<T, CT, RESID, 6>(x, v, g, U, R, part, s); break;
    case 7: launch_panel_t<T, CT, RESID, 7>(x, v, g, U, R, part, s); break;
    default: launch_panel_t<T, CT, RESID, 9>(x, v, g, U, R, part, s); break;
  }
}

template <typename CT, bool RESID>
void launch_panel(const void* x, Elem t, const ModeView& v, const GramPlan& g, const double* U, int R, double* part,
                  hipStream_t s) {
  if (t == Elem::F32)
    launch_panel_mt<float, CT, RESID>(x, v, g, U, R, part, s);
  else
    launch_panel_mt<double, CT, RESID>(x, v, g, U, R, part, s);
}

void gram_finish(const GramPlan& g, const ModeView& v, const double* part, double* G, hipStream_t s) {
  const int64_t mm = v.m * v.m;
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  gram_reduce2_kernel<<<(unsigned)((mm + 63) / 64), 1024, 0, s>>>(part, v.m, g.nb, g.npairs, g.nsplit, g.blk, G);
}

size_t gram_partial_bound(int64_t m) {
  if (m <= kSmallM) return (size_t)kSmallBlocks * (kSmallM * (kSmallM + 1) / 2);
  const size_t nb = (size_t)((m + GB - 1) / GB), npairs = nb * (nb + 1) / 2, side = (size_t)std::min<int64_t>(GB, m);
  return std::max<size_t>(512, npairs) * side * side;
}

size_t gram_partial_doubles(const ModeView& v) {
  if (v.m <= kSmallM) return (size_t)kSmallBlocks * (kSmallM * (kSmallM + 1) / 2);
  const GramPlan g = gram_plan(v), w = gram_plan(v, GPK);  // (the latter for modes above 128 rows)
  // (the register-direct Grams write up to 512 partials of m x m)
  const size_t reg = v.m <= kResidGramMaxM ? (size_t)512 * v.m * v.m : 0;
  return std::max<size_t>(std::max<size_t>((size_t)g.nsplit * g.npairs, (size_t)w.nsplit * w.npairs) * g.blk, reg);
}

// Register-direct block mode of an FP32 mode view: 0 for column runs in blocks of
// 32, S for runs of 1-4 (with at most 32 rows of U and 36 to 96 rows), -1 when
// neither applies; offsets must fit 32 bits.
int reg_mode(Elem t, const ModeView& v, int R) {
  if (t != Elem::F32 || v.m % 4 != 0 || v.m > 128 || R < 1 || R > 64) return -1;
  if (v.m * v.S >= (int64_t(1) << 29) || v.P * v.S >= (int64_t(1) << 31)) return -1;
  if (v.S % 32 == 0) return 0;
  if (v.S <= 4 && R <= 32 && v.m > 32 && v.m <= 96) return (int)v.S;
  return -1;
}

#define HT_REG_CASES(X)                                                                                \
  X(2, 1, 0) X(2, 2, 0) X(2, 3, 0) X(2, 4, 0) X(4, 1, 0) X(4, 2, 0) X(4, 3, 0) X(4, 4, 0)                 \
  X(3, 1, 0) X(3, 2, 0) X(3, 3, 0) X(3, 4, 0) X(3, 1, 1) X(3, 2, 1) X(3, 1, 2) X(3, 2, 2)                 \
  X(3, 1, 3) X(3, 2, 3) X(3, 1, 4) X(3, 2, 4)                                                             \
  X(6, 1, 0) X(6, 2, 0) X(6, 3, 0) X(6, 4, 0) X(8, 1, 0) X(8, 2, 0) X(8, 3, 0) X(8, 4, 0)                 \
  X(4, 1, 1) X(4, 2, 1) X(6, 1, 1) X(6, 2, 1) X(4, 1, 2) X(4, 2, 2) X(6, 1, 2) X(6, 2, 2)                 \
  X(4, 1, 3) X(4, 2, 3) X(6, 1, 3) X(6, 2, 3) X(4, 1, 4) X(4, 2, 4) X(6, 1, 4) X(6, 2, 4)
#define HT_REG_KEY(TI, RT, SL) ((TI) * 64 + (RT) * 8 + (SL))
// the FP64 Gram's cases: without 128 rows and more than 32 basis columns
#define HT_REG64_CASES(X)                                                                              \
  X(2, 1, 0) X(2, 2, 0) X(2, 3, 0) X(2, 4, 0) X(4, 1, 0) X(4, 2, 0) X(4, 3, 0) X(4, 4, 0)                 \
  X(3, 1, 0) X(3, 2, 0) X(3, 3, 0) X(3, 4, 0) X(3, 1, 1) X(3, 2, 1) X(3, 1, 2) X(3, 2, 2)                 \
  X(3, 1, 3) X(3, 2, 3) X(3, 1, 4) X(3, 2, 4)                                                             \
  X(6, 1, 0) X(6, 2, 0) X(6, 3, 0) X(6, 4, 0) X(8, 1, 0) X(8, 2, 0)                                       \
  X(4, 1, 1) X(4, 2, 1) X(6, 1, 1) X(6, 2, 1) X(4, 1, 2) X(4, 2, 2) X(6, 1, 2) X(6, 2, 2)                 \
  X(4, 1, 3) X(4, 2, 3) X(6, 1, 3) X(6, 2, 3) X(4, 1, 4) X(4, 2, 4) X(6, 1, 4) X(6, 2, 4)

// the FP64 Gram of the data on register-direct blocks (no basis): one instantiation
// per row-tile count and block mode
#define HT_GRAM64M_CASES(X)                                                                            \
  X(2, 0) X(3, 0) X(4, 0) X(6, 0) X(8, 0) X(3, 1) X(3, 2) X(3, 3) X(3, 4) X(4, 1) X(4, 2) X(4, 3) X(4, 4) \
  X(6, 1) X(6, 2) X(6, 3) X(6, 4)

// row tiles of 16 of a register-direct kernel for an m-row mode: 2, 3, 4, 6 or 8 (an
// odd count other than 3 is rounded up; three tiles cover the 33-48 row modes without
// a padding tile)
int reg_tiles(int64_t m) {
  const int t = (int)((m + 15) / 16);
  return t == 3 ? 3 : (t + 1) & ~1;
}

int64_t reg_blocks(const ModeView& v, int mode) { return mode == 0 ? v.P * v.S / 32 : (v.P + 15) / 16; }

// residual Gram through gram_reg_kernel; at most 512 workgroup partials, the
// bound the partial buffer is sized for
void gram_reg(const float* x, const ModeView& v, int mode, const double* U, int R, double* part, double* G,
              hipStream_t s) {
  const int ti = reg_tiles(v.m);
  const int rt = (R + 15) / 16;
  const int64_t nblk = reg_blocks(v, mode);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(512, (nblk + 3) / 4));
  const size_t lds = ((size_t)16 * ti * (16 * rt + 1) +
                      std::max<size_t>((size_t)4 * 16 * ti * kGramRegLd, (size_t)(ti * (ti + 1) / 2) * 256)) *
                     sizeof(float);
  static bool attr = false;
  if (!attr) {
#define HT_GA(TI, RT, SL)                                                                  \
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_reg_kernel<TI, RT, SL>), \
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    HT_REG_CASES(HT_GA)
#undef HT_GA
    attr = true;
  }
  const double K = (double)v.P * v.S, md = (double)v.m;
  {
    ProfScope prof(KKind::Gram32Reg, s, md * md * K + 4.0 * R * md * K, md * K * 4);
#define HT_GR(TI, RT, SL)                                                                \
  case HT_REG_KEY(TI, RT, SL):                                                           \
    gram_reg_kernel<TI, RT, SL><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, U, R, part); \
    break;
    switch (HT_REG_KEY(ti, rt, mode)) {
      HT_REG_CASES(HT_GR)
      default: break;
    }
#undef HT_GR
  }
  GramPlan g;
  g.nb = 1;
  g.npairs = 1;
  g.nsplit = blocks;
  g.blk = v.m * v.m;
  gram_finish(g, v, part, G, s);
}

// FP64 residual Gram through gram_reg64_kernel (R >= 1); at most 512 workgroup
// partials.  The plain Gram keeps the panel kernel, which is faster without the
// projection.
void gram_reg64(const float* x, const ModeView& v, int mode, const double* U, int R, double* part, double* G,
                hipStream_t s) {
  const int ti = reg_tiles(v.m);
  const int rt = R > 0 ? (R + 15) / 16 : 1;
  const int64_t nblk = reg_blocks(v, mode);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(512, (nblk + 3) / 4));
  const size_t lds = ((R > 0 ? (size_t)16 * ti * (16 * rt + 1) : 0) + (size_t)4 * 16 * ti * kGram64Ld) * sizeof(double);
  static bool attr = false;
  if (!attr) {
#define HT_GA(TI, RT, SL)                                                                           \
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_reg64_kernel<TI, RT, true, SL>),  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    HT_REG64_CASES(HT_GA)
#undef HT_GA
    attr = true;
  }
  const double K = (double)v.P * v.S, md = (double)v.m;
  {
    ProfScope prof(KKind::GramReg64, s, md * md * K + 4.0 * R * md * K, md * K * 4);
#define HT_GR(TI, RT, SL)                                                                                  \
  case HT_REG_KEY(TI, RT, SL):                                                                             \
    gram_reg64_kernel<TI, RT, true, SL><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, U, R, part);       \
    break;
    switch (HT_REG_KEY(ti, rt, mode)) {
      HT_REG64_CASES(HT_GR)
      default: break;
    }
#undef HT_GR
  }
  GramPlan g;
  g.nb = 1;
  g.npairs = 1;
  g.nsplit = blocks;
  g.blk = v.m * v.m;
  gram_finish(g, v, part, G, s);
}

// FP64 Gram M M^T of an FP32 unfolding on register-direct blocks (block mode from
// reg_mode): gram_reg64_kernel without a basis, at most 512 workgroup partials
void gram_m64(const float* x, const ModeView& v, int mode, double* part, double* G, hipStream_t s) {
  const int ti = reg_tiles(v.m);
  const int64_t nblk = reg_blocks(v, mode);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(512, (nblk + 3) / 4));
  const size_t lds = (size_t)4 * 16 * ti * kGram64Ld * sizeof(double);
  static bool attr = false;
  if (!attr) {
#define HT_GMA(TI, SL)                                                                              \
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_reg64_kernel<TI, 1, false, SL>),  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    HT_GRAM64M_CASES(HT_GMA)
#undef HT_GMA
    attr = true;
  }
  const double K = (double)v.P * v.S, md = (double)v.m;
  {
    ProfScope prof(KKind::GramReg64, s, md * md * K, md * K * 4);
#define HT_GM(TI, SL)                                                                                     \
  case HT_REG_KEY(TI, 1, SL):                                                                             \
    gram_reg64_kernel<TI, 1, false, SL><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, nullptr, 0, part); \
    break;
    switch (HT_REG_KEY(ti, 1, mode)) {
      HT_GRAM64M_CASES(HT_GM)
      default: break;
    }
#undef HT_GM
  }
  GramPlan g;
  g.nb = 1;
  g.npairs = 1;
  g.nsplit = blocks;
  g.blk = v.m * v.m;
  gram_finish(g, v, part, G, s);
}

bool resid_gram_proj_applies(Elem t, const ModeView& v, int R) {
  if ((double)v.P * v.m * v.S < kGramProjMinElems) return false;
  return R >= 1 && R <= 64 && v.m <= kGramProjMaxM;
}

size_t resid_gram_proj_work_doubles(int64_t m, int R) {
  return m <= kResidGramMaxM ? 0 : (size_t)2 * R * m + (size_t)R * R;
}

void gram_project_batch(const ProjJob* jobs, int count, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_project_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kProjLdsDoubles * (int)sizeof(double));
    attr = true;
  }
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  for (int b0 = 0; b0 < count; b0 += kMaxProjJobs) {
    const int n = std::min(kMaxProjJobs, count - b0);
    ProjBatch b;
    int cap = 0;
    for (int i = 0; i < n; ++i) {
      b.j[i] = jobs[b0 + i];
      const int st = proj_lds_doubles(b.j[i].m, b.j[i].R, true);
      cap = std::max(cap, st <= kProjLdsDoubles ? st : proj_lds_doubles(b.j[i].m, b.j[i].R, false));
    }
    gram_project_kernel<<<n, kProjThreads, (size_t)cap * sizeof(double), s>>>(b, cap);
  }
}

void resid_gram_proj(const void* x, Elem t, const ModeView& v, const double* U, int R, double* part, double* G,
                     double* work, hipStream_t s, std::vector<ProjJob>* defer) {
  if (v.m > kResidGramMaxM) {
    gram(x, t, v, part, G, s);
    ProfScope prof(KKind::Layout, s, 0.0, 0.0);
    const int m = (int)v.m;
    double* B = work;
    double* E = work + (size_t)R * m;
    double* V = E + (size_t)R * m;
    const unsigned nrm = (unsigned)(((int64_t)R * m + 255) / 256);
    gram_proj_b_kernel<<<(unsigned)(R * ((m + 31) / 32)), 256, 0, s>>>(G, m, U, R, B);
    gram_proj_v_kernel<<<(unsigned)(R * R), 64, 0, s>>>(B, m, U, R, V);
    gram_proj_e_kernel<<<nrm, 256, 0, s>>>(B, m, U, R, V, E);
    gram_proj_g_kernel<<<(unsigned)(((int64_t)m * m + 255) / 256), 256, 0, s>>>(G, m, U, R, E);
    return;
  }
  const int mode = reg_mode(t, v, R);
  if (mode >= 0)
    gram_m64(static_cast<const float*>(x), v, mode, part, G, s);
  else
    gram(x, t, v, part, G, s);  // LDS-panel FP64 Gram of the data (other shapes)
  const ProjJob job{G, U, (int)v.m, R};
  if (defer)
    defer->push_back(job);
  else
    gram_project_batch(&job, 1, s);
}

void gram(const void* x, Elem t, const ModeView& v, double* part, double* G, hipStream_t s) {
  const double K = (double)v.P * v.S, md = (double)v.m;
  if (v.m <= kSmallM) {
    {
      ProfScope prof(KKind::Gram, s, md * md * K, md * K * (t == Elem::F32 ? 4 : 8));
      const int64_t Ki = v.P * v.S;
      if (t == Elem::F32)
        gram_small_kernel<float><<<kSmallBlocks, 256, 0, s>>>(static_cast<const float*>(x), v.m, v.S, Ki, part);
      else
        gram_small_kernel<double><<<kSmallBlocks, 256, 0, s>>>(static_cast<const double*>(x), v.m, v.S, Ki, part);
    }
    ProfScope prof(KKind::Layout, s, 0.0, 0.0);
    gram_small_reduce_kernel<<<(unsigned)(v.m * v.m), 256, 0, s>>>(part, (int)v.m, kSmallBlocks, G);
    return;
  }
  const int mode = reg_mode(t, v, 1);
  if (mode >= 0) {  // FP32 data in register-direct blocks
    gram_m64(static_cast<const float*>(x), v, mode, part, G, s);
    return;
  }
  const GramPlan g = v.m <= GB || t != Elem::F32 ? gram_plan(v) : gram_plan(v, GPK);
  if (v.m <= GB) {
    ProfScope prof(KKind::Gram, s, md * md * K, md * K * (t == Elem::F32 ? 4 : 8));
    launch_panel<double, false>(x, t, v, g, nullptr, 0, part, s);
  } else {
    dim3 grid(g.npairs, g.nsplit);
    ProfScope prof(KKind::Gram, s, md * md * K, md * K * (t == Elem::F32 ? 4 : 8));
    if (t == Elem::F32)
      gram_partial_kernel<float, GPK><<<grid, 256, 0, s>>>(static_cast<const float*>(x), v.P, v.m, v.S, g.nb, g.npairs,
                                                      g.ktiles, g.kt_per_split, g.blk, g.tw, part);
    else
      gram_partial_kernel<double, GBK><<<grid, 256, 0, s>>>(static_cast<const double*>(x), v.P, v.m, v.S, g.nb,
                                                       g.npairs, g.ktiles, g.kt_per_split, g.blk, g.tw, part);
  }
  gram_finish(g, v, part, G, s);
}

void resid_gram(const void* x, Elem t, const ModeView& v, const double* U, int R, double* part, double* G,
                hipStream_t s) {
  const int mode = reg_mode(t, v, R);
  if (mode >= 0 && (v.m <= 96 || R <= 32)) {  // (128 rows with 48+ basis columns spill)
    gram_reg64(static_cast<const float*>(x), v, mode, U, R, part, G, s);
    return;
  }
  const GramPlan g = gram_plan(v);
  const double K = (double)v.P * v.S, md = (double)v.m;
  // residual formation (4 R m flops per column) plus the symmetric product
  {
    ProfScope prof(KKind::Gram, s, md * md * K + 4.0 * R * md * K, md * K * (t == Elem::F32 ? 4 : 8));
    launch_panel<double, true>(x, t, v, g, U, R, part, s);
  }
  gram_finish(g, v, part, G, s);
}

void resid_gram_f32(const void* x, Elem t, const ModeView& v, const double* U, int R, double* part, double* G,
                    hipStream_t s) {
  const int mode = reg_mode(t, v, R);
  if (mode >= 0) {
    gram_reg(static_cast<const float*>(x), v, mode, U, R, part, G, s);
    return;
  }
  const GramPlan g = gram_plan(v);
  const double K = (double)v.P * v.S, md = (double)v.m;
  {
    ProfScope prof(KKind::Gram32, s, md * md * K + 4.0 * R * md * K, md * K * (t == Elem::F32 ? 4 : 8));
    launch_panel<float, true>(x, t, v, g, U, R, part, s);
  }
  gram_finish(g, v, part, G, s);
}

void ttm_contract(const void* x, Elem t, const ModeView& v, const double* U, int R, double* Z, hipStream_t s) {
  ttm_contract_norm(x, t, v, U, R, Z, nullptr, nullptr, s);
}

// ---- row splits of the direct contraction ------------------------------------
// A contraction of few column blocks runs on few workgroups, each over all m rows;
// with device scratch lent by SplitScratch it is split into row chunks (one
// workgroup per block and chunk) whose partial products a second launch sums in
// chunk order.
thread_local double* t_split_ws = nullptr;
thread_local size_t t_split_elems = 0;
SplitScratch::SplitScratch(double* p, size_t n) {
  t_split_ws = p;
  t_split_elems = n;
}
SplitScratch::~SplitScratch() {
  t_split_ws = nullptr;
  t_split_elems = 0;
}

int split_sum_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, (n + 255) / 256)); }

// row chunks of a per-block direct contraction: about 512 workgroups in all, chunks of
// at least 64 rows, at most 8, and the partial products within the lent scratch
int direct_split(const ModeView& v, int R, int64_t blocks) {
  if (t_split_ws == nullptr || blocks >= 256 || v.m < 128) return 1;
  int n = (int)std::min<int64_t>({8, (512 + blocks - 1) / blocks, v.m / 64});
  while (n > 1 && (size_t)n * v.P * R * v.S > t_split_elems) --n;
  if (n < 2) return 1;
  // whole chunks of rows in steps of four
  const int64_t rows = ((v.m + n - 1) / n + 3) & ~int64_t(3);
  return (int)((v.m + rows - 1) / rows);
}

// one launch of the direct contraction (modes of more than 128 rows); with SQ also
// ||X||^2 and ||Z||^2 from the workgroup partials
template <bool SQ>
void launch_ttm_direct(const void* x, Elem t, const ModeView& v, const double* U, int R, double* Z, double* in_part,
                       double* in_out, double* out_part, double* out_out, hipStream_t s) {
  const int64_t K = v.P * v.S;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ttm_direct_kernel<float, SQ>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kDirectLdsDoubles * (int)sizeof(double));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ttm_direct_kernel<double, SQ>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kDirectLdsDoubles * (int)sizeof(double));
    attr = true;
  }
  const unsigned blocks = (unsigned)((K + 15) / 16);
  const int RP = (R + 15) & ~15;
  if (blocks >= kDirectColsMinBlocks) {
    // many column blocks: whole blocks per wave, U in chunks of at most 64 KiB (two
    // workgroups per compute unit), tiles of eight blocks spread evenly over at most
    // 512 workgroups
    static bool cattr = false;
    if (!cattr) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ttm_direct_cols_kernel<float, SQ>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 8192 * (int)sizeof(double));
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ttm_direct_cols_kernel<double, SQ>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 8192 * (int)sizeof(double));
      cattr = true;
    }
    const int64_t tiles = ((int64_t)blocks + 7) / 8;
    const int64_t per = (tiles + 511) / 512;
    const unsigned grid = (unsigned)((tiles + per - 1) / per);
    const int nsplit = direct_split(v, R, grid);
    const int64_t rows = nsplit > 1 ? ((v.m + nsplit - 1) / nsplit + 3) & ~int64_t(3) : v.m;
    const int chunk = (int)std::min<int64_t>(((8192 / (RP + 1)) / 4) * 4, (rows + 3) & ~3);
    const size_t lds = (size_t)chunk * (RP + 1) * sizeof(double);
    const dim3 g2(grid, (unsigned)nsplit);
    double* Zp = nsplit > 1 ? t_split_ws : nullptr;
    {
      ProfScope prof(KKind::TtmContract, s, 2.0 * R * v.m * (double)K,
                     (double)v.m * K * (t == Elem::F32 ? 4 : 8) + (double)R * K * 8 + (double)v.m * R * 8);
      if (t == Elem::F32)
        ttm_direct_cols_kernel<float, SQ><<<g2, 256, lds, s>>>(static_cast<const float*>(x), v.P, v.m, v.S, U, R,
                                                               chunk, Z, in_part, out_part, rows, Zp);
      else
        ttm_direct_cols_kernel<double, SQ><<<g2, 256, lds, s>>>(static_cast<const double*>(x), v.P, v.m, v.S, U,
                                                                R, chunk, Z, in_part, out_part, rows, Zp);
      if (nsplit > 1) {
        const int64_t n = v.P * R * v.S;
        split_sum_kernel<SQ><<<split_sum_blocks(n), 256, 0, s>>>(Zp, nsplit, n, Z, out_part);
      }
    }
    if (SQ) {
      ProfScope prof(KKind::Layout, s, 0.0, 0.0);
      finish_sum(in_part, (int)grid * nsplit, in_out, s);
      finish_sum(out_part, nsplit > 1 ? split_sum_blocks(v.P * R * v.S) : (int)grid, out_out, s);
    }
    return;
  }
  // few column blocks (transfer nodes): all of U (or of the rows of a split) in one
  // chunk; many: at most 64 KiB, two workgroups per compute unit
  const int nsplit = direct_split(v, R, blocks);
  const int64_t rows = nsplit > 1 ? ((v.m + nsplit - 1) / nsplit + 3) & ~int64_t(3) : v.m;
  const int cap = blocks >= 512 ? 8192 : kDirectLdsDoubles;
  const int chunk = (int)std::min<int64_t>(((cap / (RP + 1)) / 4) * 4, (rows + 3) & ~3);
  // the wave partials (3 x 4 x 4 x 64 doubles) reuse the same space at the end
  const size_t lds = (size_t)std::max<int64_t>((int64_t)chunk * (RP + 1), 3 * 4 * 4 * 64) * sizeof(double);
  const dim3 grid(blocks, (unsigned)nsplit);
  double* Zp = nsplit > 1 ? t_split_ws : nullptr;
  {
    ProfScope prof(KKind::TtmContract, s, 2.0 * R * v.m * (double)K,
                   (double)v.m * K * (t == Elem::F32 ? 4 : 8) + (double)R * K * 8 + (double)v.m * R * 8);
    if (t == Elem::F32)
      ttm_direct_kernel<float, SQ><<<grid, 256, lds, s>>>(static_cast<const float*>(x), v.P, v.m, v.S, U, R, chunk, Z,
                                                          in_part, out_part, rows, Zp);
    else
      ttm_direct_kernel<double, SQ><<<grid, 256, lds, s>>>(static_cast<const double*>(x), v.P, v.m, v.S, U, R, chunk,
                                                           Z, in_part, out_part, rows, Zp);
    if (nsplit > 1) {
      const int64_t n = v.P * R * v.S;
      split_sum_kernel<SQ><<<split_sum_blocks(n), 256, 0, s>>>(Zp, nsplit, n, Z, out_part);
    }
  }
  if (SQ) {
    ProfScope prof(KKind::Layout, s, 0.0, 0.0);
    finish_sum(in_part, (int)blocks * nsplit, in_out, s);
    finish_sum(out_part, nsplit > 1 ? split_sum_blocks(v.P * R * v.S) : (int)blocks, out_out, s);
  }
}

// one launch of the small-mode contraction (m <= kSmallModeM), at most kTtmMaxBlocks
// workgroup partials
template <typename T, typename CT, bool NORM, bool RESE>
void launch_ttm_small(const void* x, const ModeView& v, const double* U, int R, CT* Z, double* norm_part,
                      double* norm_out, double* res_part, double* res_out, KKind kind, double flops, double bytes,
                      hipStream_t s) {
  const int64_t K = v.P * v.S;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kTtmMaxBlocks, (K + 255) / 256));
  {
    ProfScope prof(kind, s, flops, bytes);
    ttm_small_kernel<T, CT, NORM, RESE><<<blocks, 256, 0, s>>>(static_cast<const T*>(x), v.P, (int)v.m, v.S, U, R, Z,
                                                               norm_part, res_part);
  }
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  if (NORM) finish_sum(norm_part, blocks, norm_out, s);
  if (RESE) finish_sum(res_part, blocks, res_out, s);
}

size_t ttm_norm_partials() { return kTtmMaxBlocks; }

// one launch of the panel contraction: blocks over column tiles, optional norm and
// residual-energy partials (one per block), reduced in fixed order
template <typename T, typename CT, bool NORM, bool RESE>
void launch_ttm_panel(const void* x, const ModeView& v, const double* U, int R, CT* Z, double* norm_part,
                      double* norm_out, double* res_part, double* res_out, KKind kind, double flops, double bytes,
                      hipStream_t s) {
  const int64_t K = v.P * v.S;
  GramPlan g;
  g.tw = v.S >= GBK ? GBK : (int)(v.S * (GBK / v.S));
  g.ktiles = (K + g.tw - 1) / g.tw;
  const int64_t want = std::min<int64_t>(kTtmMaxBlocks, std::max<int64_t>(1, g.ktiles));
  g.kt_per_split = (g.ktiles + want - 1) / want;
  const int blocks = (int)((g.ktiles + g.kt_per_split - 1) / g.kt_per_split);
  const int RP = (R + 15) & ~15;
  const size_t lds = ((size_t)GBK * GLD + (size_t)GB * (RP + 1) + (RESE ? (size_t)RP * ZLD : 0)) * sizeof(CT);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ttm_panel_kernel<T, CT, NORM, RESE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    attr = true;
  }
  {
    ProfScope prof(kind, s, flops, bytes);
    ttm_panel_kernel<T, CT, NORM, RESE><<<blocks, 256, lds, s>>>(static_cast<const T*>(x), v.P, v.m, v.S, g.ktiles,
                                                                 g.kt_per_split, g.tw, U, R, Z, norm_part, res_part);
  }
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  if (NORM) finish_sum(norm_part, blocks, norm_out, s);
  if (RESE) finish_sum(res_part, blocks, res_out, s);
}

bool ttm_groupable(const ModeView& v, int R) {
  return v.m <= GB && R >= 1 && R <= 64 && v.P * v.m * v.S <= kGroupMaxElems;
}

// one launch of up to kMaxPanelJobs jobs of one type combination
template <typename T, typename CT, bool RESE>
void launch_panel_group(const TtmJob* jobs, int n, hipStream_t s) {
  PanelBatch b;
  b.n = n;
  int blocks = 0, rpmax = 16;
  double fl = 0.0, by = 0.0;
  for (int q = 0; q < n; ++q) {
    const TtmJob& J = jobs[q];
    const int64_t K = J.v.P * J.v.S;
    PanelJob& P = b.j[q];
    P.X = J.x;
    P.P = J.v.P;
    P.m = J.v.m;
    P.S = J.v.S;
    P.tw = J.v.S >= GBK ? GBK : (int)(J.v.S * (GBK / J.v.S));
    P.ktiles = (K + P.tw - 1) / P.tw;
    const int64_t want = std::min<int64_t>(kTtmMaxBlocks, std::max<int64_t>(1, P.ktiles));
    P.kt_per_split = (P.ktiles + want - 1) / want;
    const int nb = (int)((P.ktiles + P.kt_per_split - 1) / P.kt_per_split);
    P.U = J.U;
    P.R = J.R;
    P.Z = J.Z;
    P.norm_part = J.norm_part;
    P.res_part = J.res_part;
    P.blk0 = blocks;
    blocks += nb;
    rpmax = std::max(rpmax, (J.R + 15) & ~15);
    fl += (RESE ? 4.0 : 2.0) * J.R * J.v.m * (double)K;
    by += (double)J.v.m * K * sizeof(T) + (double)J.R * K * sizeof(CT) + (double)J.v.m * J.R * 8;
  }
  const size_t lds = ((size_t)GBK * GLD + (size_t)GB * (rpmax + 1) + (RESE ? (size_t)rpmax * ZLD : 0)) * sizeof(CT);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ttm_panel_group_kernel<T, CT, RESE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    attr = true;
  }
  {
    ProfScope prof(std::is_same<CT, float>::value ? KKind::TtmContract32 : KKind::TtmContract, s, fl, by);
    ttm_panel_group_kernel<T, CT, RESE><<<blocks, 256, lds, s>>>(b);
  }
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  for (int q = 0; q < n; ++q) {
    const PanelJob& P = b.j[q];
    const int nb = (q + 1 < n ? b.j[q + 1].blk0 : blocks) - P.blk0;
    if (P.norm_part != nullptr) finish_sum(P.norm_part, nb, jobs[q].norm_out, s);
    if (RESE) finish_sum(P.res_part, nb, jobs[q].res_out, s);
  }
}

void ttm_group(const std::vector<TtmJob>& jobs, hipStream_t s) {
  // the jobs of each type combination, in list order, up to kMaxPanelJobs per launch
  for (int combo = 0; combo < 8; ++combo) {
    std::vector<TtmJob> sel;
    for (const TtmJob& J : jobs) {
      const int c = (J.t == Elem::F64 ? 4 : 0) + (J.zt == Elem::F64 ? 2 : 0) + (J.res_part != nullptr ? 1 : 0);
      if (c == combo) sel.push_back(J);
    }
    for (size_t b0 = 0; b0 < sel.size(); b0 += kMaxPanelJobs) {
      const int n = (int)std::min<size_t>(kMaxPanelJobs, sel.size() - b0);
      const TtmJob* js = sel.data() + b0;
      switch (combo) {
        case 0: launch_panel_group<float, float, false>(js, n, s); break;
        case 1: launch_panel_group<float, float, true>(js, n, s); break;
        case 2: launch_panel_group<float, double, false>(js, n, s); break;
        case 3: launch_panel_group<float, double, true>(js, n, s); break;
        case 4: launch_panel_group<double, float, false>(js, n, s); break;
        case 5: launch_panel_group<double, float, true>(js, n, s); break;
        case 6: launch_panel_group<double, double, false>(js, n, s); break;
        default: launch_panel_group<double, double, true>(js, n, s); break;
      }
    }
  }
}

bool ttm_reg64_applies(Elem t, const ModeView& v, int R) {
  const int64_t esz = t == Elem::F32 ? 4 : 8;
  return v.S % 32 == 0 && v.m % 4 == 0 && v.m <= 128 && v.m * v.S * esz < (int64_t(1) << 31) &&
         v.P * v.S < (int64_t(1) << 31) && R >= 1 && R <= 64;
}

template <typename T, bool NN>
void launch_ttm_reg64(const T* x, const ModeView& v, const double* U, int R, double* Z, double* norm_part,
                      double* norm_out, double fl, double by, hipStream_t s) {
  const int ti = reg_tiles(v.m);
  const int nrt = (R + 15) / 16;
  const int64_t nblk = v.P * v.S / 32;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kTtmMaxBlocks, (nblk + 3) / 4));
  const size_t lds = (size_t)16 * ti * (16 * nrt + 1) * sizeof(double);
  {
    ProfScope prof(KKind::TtmContractReg64, s, fl, by);
    switch (ti) {
      case 2: ttm_reg64_kernel<T, 2, NN><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, U, R, Z, norm_part); break;
      case 3: ttm_reg64_kernel<T, 3, NN><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, U, R, Z, norm_part); break;
      case 4: ttm_reg64_kernel<T, 4, NN><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, U, R, Z, norm_part); break;
      case 6: ttm_reg64_kernel<T, 6, NN><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, U, R, Z, norm_part); break;
      default: ttm_reg64_kernel<T, 8, NN><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, U, R, Z, norm_part); break;
    }
  }
  if (NN) {
    ProfScope prof(KKind::Layout, s, 0.0, 0.0);
    finish_sum(norm_part, blocks, norm_out, s);
  }
}

void ttm_contract_norm(const void* x, Elem t, const ModeView& v, const double* U, int R, double* Z, double* norm_part,
                       double* norm_out, hipStream_t s) {
  const int64_t K = v.P * v.S;
  if (v.m <= GB) {
    const double fl = 2.0 * R * v.m * (double)K,
                 by = (double)v.m * K * (t == Elem::F32 ? 4 : 8) + (double)R * K * 8 + (double)v.m * R * 8;
    const KKind kd = KKind::TtmContract;
    const bool nrm = norm_part != nullptr;
    if (ttm_reg64_applies(t, v, R)) {
      if (t == Elem::F32) {
        const float* xf = static_cast<const float*>(x);
        if (nrm) launch_ttm_reg64<float, true>(xf, v, U, R, Z, norm_part, norm_out, fl, by, s);
        else launch_ttm_reg64<float, false>(xf, v, U, R, Z, nullptr, nullptr, fl, by, s);
      } else {
        const double* xd = static_cast<const double*>(x);
        if (nrm) launch_ttm_reg64<double, true>(xd, v, U, R, Z, norm_part, norm_out, fl, by, s);
        else launch_ttm_reg64<double, false>(xd, v, U, R, Z, nullptr, nullptr, fl, by, s);
      }
      return;
    }
    if (v.m <= kSmallModeM && R <= kSmallModeM) {
      if (t == Elem::F32) {
        if (nrm)
          launch_ttm_small<float, double, true, false>(x, v, U, R, Z, norm_part, norm_out, nullptr, nullptr, kd, fl,
                                                       by, s);
        else
          launch_ttm_small<float, double, false, false>(x, v, U, R, Z, nullptr, nullptr, nullptr, nullptr, kd, fl, by,
                                                        s);
      } else {
        if (nrm)
          launch_ttm_small<double, double, true, false>(x, v, U, R, Z, norm_part, norm_out, nullptr, nullptr, kd, fl,
                                                        by, s);
        else
          launch_ttm_small<double, double, false, false>(x, v, U, R, Z, nullptr, nullptr, nullptr, nullptr, kd, fl,
                                                         by, s);
      }
      return;
    }
    if (t == Elem::F32) {
      if (nrm)
        launch_ttm_panel<float, double, true, false>(x, v, U, R, Z, norm_part, norm_out, nullptr, nullptr, kd, fl, by,
                                                     s);
      else
        launch_ttm_panel<float, double, false, false>(x, v, U, R, Z, nullptr, nullptr, nullptr, nullptr, kd, fl, by,
                                                      s);
    } else {
      if (nrm)
        launch_ttm_panel<double, double, true, false>(x, v, U, R, Z, norm_part, norm_out, nullptr, nullptr, kd, fl,
                                                      by, s);
      else
        launch_ttm_panel<double, double, false, false>(x, v, U, R, Z, nullptr, nullptr, nullptr, nullptr, kd, fl,
                                                       by, s);
    }
    return;
  }
  if (norm_part != nullptr) sumsq(x, t, v.P * v.m * v.S, norm_part, norm_out, s);
  launch_ttm_direct<false>(x, t, v, U, R, Z, nullptr, nullptr, nullptr, nullptr, s);
}

bool ttm_contract_sq(const void* x, Elem t, const ModeView& v, const double* U, int R, double* Z, double* in_part,
                     double* in_out, double* out_part, double* out_out, int max_parts, hipStream_t s) {
  const int64_t K = v.P * v.S;
  const int64_t blocks = (K + 15) / 16;
  // workgroup partials: one per column block (and row chunk), or at most 512 with
  // whole blocks per wave
  const int64_t tiles = (blocks + 7) / 8, grid = (tiles + (tiles + 511) / 512 - 1) / ((tiles + 511) / 512);
  const int64_t parts = blocks >= kDirectColsMinBlocks ? grid * direct_split(v, R, grid)
                                                       : blocks * direct_split(v, R, blocks);
  if (v.m <= GB || parts > max_parts) return false;
  launch_ttm_direct<true>(x, t, v, U, R, Z, in_part, in_out, out_part, out_out, s);
  return true;
}

// the register-direct FP32 contraction applies to FP32 level tensors whose column
// runs split into whole blocks of 32 (S % 32 == 0), modes of at most 128 rows in
// steps of four, and sizes with 32-bit offsets
template <bool NN, bool RR>
void launch_ttm_reg(const float* x, const ModeView& v, int mode, const double* U, int R, float* Z,
                    double* norm_part, double* norm_out, double* res_part, double* res_out, double fl, double by,
                    hipStream_t s) {
  const int ti = reg_tiles(v.m);
  const int rt = (R + 15) / 16;
  const int64_t nblk = reg_blocks(v, mode);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kRegMaxBlocks, (nblk + 3) / 4));
  const size_t lds = (size_t)16 * ti * (16 * rt + 1) * sizeof(float);
  {
    ProfScope prof(KKind::TtmContract32Reg, s, fl, by);
#define HT_TR(TI, RT, SL)                                                                                    \
  case HT_REG_KEY(TI, RT, SL):                                                                               \
    ttm_reg_kernel<TI, RT, NN, RR, SL><<<blocks, 256, lds, s>>>(x, v.P, (int)v.m, v.S, U, R, Z, norm_part, \
                                                                res_part);                                 \
    break;
    switch (HT_REG_KEY(ti, rt, mode)) {
      HT_REG_CASES(HT_TR)
      default: break;
    }
#undef HT_TR
  }
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  if (NN) finish_sum(norm_part, blocks, norm_out, s);
  if (RR) finish_sum(res_part, blocks, res_out, s);
}

void ttm_contract_f32(const void* x, Elem t, const ModeView& v, const double* U, int R, float* Z, double* norm_part,
                      double* norm_out, double* res_part, double* res_out, hipStream_t s) {
  const int64_t K = v.P * v.S;
  const bool nrm = norm_part != nullptr, rese = res_part != nullptr;
  const double fl = (rese ? 4.0 : 2.0) * R * v.m * (double)K,
               by = (double)v.m * K * (t == Elem::F32 ? 4 : 8) + (double)R * K * 4 + (double)v.m * R * 8;
#define HT_TTM32(TT, NN, RR)                                                                                  \
  launch_ttm_panel<TT, float, NN, RR>(x, v, U, R, Z, NN ? norm_part : nullptr, NN ? norm_out : nullptr,       \
                                      RR ? res_part : nullptr, RR ? res_out : nullptr, KKind::TtmContract32, fl, \
                                      by, s)
  const int mode = reg_mode(t, v, R);
  if (mode >= 0 && (rese || !nrm)) {
    const float* xf = static_cast<const float*>(x);
    if (nrm) launch_ttm_reg<true, true>(xf, v, mode, U, R, Z, norm_part, norm_out, res_part, res_out, fl, by, s);
    else if (rese) launch_ttm_reg<false, true>(xf, v, mode, U, R, Z, nullptr, nullptr, res_part, res_out, fl, by, s);
    else launch_ttm_reg<false, false>(xf, v, mode, U, R, Z, nullptr, nullptr, nullptr, nullptr, fl, by, s);
  } else if (v.m <= kSmallModeM && R <= kSmallModeM) {
#define HT_SM32(TT, NN, RR)                                                                                   \
  launch_ttm_small<TT, float, NN, RR>(x, v, U, R, Z, NN ? norm_part : nullptr, NN ? norm_out : nullptr,       \
                                      RR ? res_part : nullptr, RR ? res_out : nullptr, KKind::TtmContract32, fl, \
                                      by, s)
    if (t == Elem::F32) {
      if (nrm && rese) HT_SM32(float, true, true);
      else if (rese) HT_SM32(float, false, true);
      else if (nrm) HT_SM32(float, true, false);
      else HT_SM32(float, false, false);
    } else {
      if (nrm && rese) HT_SM32(double, true, true);
      else if (rese) HT_SM32(double, false, true);
      else if (nrm) HT_SM32(double, true, false);
      else HT_SM32(double, false, false);
    }
#undef HT_SM32
  } else if (t == Elem::F32) {
    if (nrm && rese) HT_TTM32(float, true, true);
    else if (rese) HT_TTM32(float, false, true);
    else if (nrm) HT_TTM32(float, true, false);
    else HT_TTM32(float, false, false);
  } else {
    if (nrm && rese) HT_TTM32(double, true, true);
    else if (rese) HT_TTM32(double, false, true);
    else if (nrm) HT_TTM32(double, true, false);
    else HT_TTM32(double, false, false);
  }
#undef HT_TTM32
}

void ttm_expand(const double* Z, int64_t P, int R, int64_t S, const double* U, int64_t m, const void* M, Elem mt,
                void* out, Elem out_t, hipStream_t s) {
  const int64_t K = P * S;
  ProfScope prof(KKind::TtmExpand, s, 2.0 * R * m * (double)K,
                 (double)R * K * 8 + (double)m * K * (out_t == Elem::F32 ? 4 : 8) +
                     (M ? (double)m * K * (mt == Elem::F32 ? 4 : 8) : 0.0));
  dim3 grid((unsigned)((K + 63) / 64), (unsigned)((m + 63) / 64));
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

void orth_expand_batch(const OrthJob* jobs, int count, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&orth_expand_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (64 * 64 + kOrthLdsDoubles) * 8);
    attr = true;
  }
  for (int b0 = 0; b0 < count; b0 += kMaxOrthJobs) {
    const int n = std::min(kMaxOrthJobs, count - b0);
    OrthBatch b;
    int64_t staged = 0;
    for (int i = 0; i < n; ++i) {
      b.j[i] = jobs[b0 + i];
      const int64_t need = b.j[i].alpha * (int64_t)(b.j[i].r_old + b.j[i].rR);
      if (need <= kOrthLdsDoubles) staged = std::max(staged, need);
    }
    const size_t lds = (size_t)(64 * 64 + staged) * sizeof(double);
    ProfScope prof(KKind::Orth, s, 0.0, 0.0);
    orth_expand_kernel<<<n, 256, lds, s>>>(b);
  }
}

void orth_expand(const double* U_old, int64_t alpha, int r_old, double* V, int rR, double* core, double* scratch,
                 hipStream_t s) {
  (void)scratch;
  if (rR <= 0) return;
  const OrthJob j{U_old, V, core, alpha, r_old, rR};
  orth_expand_batch(&j, 1, s);
}

void pad_core(const double* src, int ra, int rb, int rp, double* dst, int ra2, int rb2, hipStream_t s) {
  const int64_t n = (int64_t)ra2 * rb2 * rp;
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  pad_core_kernel<<<grid_for(n), 256, 0, s>>>(src, ra, rb, rp, dst, ra2, rb2);
}

void root_append(const void* C1, Elem t, int64_t N, int r11, int r12, double* root, int64_t n_acc, int rcap,
                 hipStream_t s) {
  const int64_t n = N * rcap * rcap;
  ProfScope prof(KKind::Layout, s, 0.0, 0.0);
  if (t == Elem::F32)
    root_append_kernel<float><<<grid_for(n), 256, 0, s>>>(static_cast<const float*>(C1), N, r11, r12, root, n_acc,
                                                          rcap);
  else
    root_append_kernel<double><<<grid_for(n), 256, 0, s>>>(static_cast<const double*>(C1), N, r11, r12, root, n_acc,
                                                           rcap);
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
