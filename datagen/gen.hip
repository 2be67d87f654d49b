// GPU side of datagen's exactly reproducible separable fields: the same elements,
// bit for bit, as datagen.exact_field_batch computes on the host.  Input synthesis
// only; nothing of the tensor method lives here.
//
// y[s][p1][p2] = float32(sum_t A[t][s][p1] * B[t][p2] + scale * g(key, e)) with e the
// element's index in the batch.  A and B are 24-bit fixed point, so every product
// and partial sum of the signal is exact and its order immaterial; g is the
// Irwin-Hall sum of the four 16-bit fields of SplitMix64 (Steele, Lea & Flood 2014)
// at counter (key << 40) + e, an exact multiple of 2^-16.  The one rounding multiply
// and the one rounding add use explicit round-to-nearest intrinsics so that the
// compiler cannot fuse them.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t counter) {
  uint64_t z = (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void field_kernel(const double* __restrict__ A, const double* __restrict__ B,
                                                    int T, int64_t N, int64_t P1, int64_t P2, uint64_t key,
                                                    double scale, float* __restrict__ out) {
  const int64_t per = P1 * P2;
  const int64_t E = N * per;
  const uint64_t base = key << 40;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / per;
    const int64_t rem = e - s * per;
    const int64_t p1 = rem / P2;
    const int64_t p2 = rem - p1 * P2;
    double sig = 0.0;
    for (int t = 0; t < T; ++t) sig = __fma_rn(A[((int64_t)t * N + s) * P1 + p1], B[(int64_t)t * P2 + p2], sig);
    double y = sig;
    if (scale != 0.0) {
      const uint64_t z = splitmix64(base + (uint64_t)e);
      const int64_t n = (int64_t)(z & 0xFFFFull) + (int64_t)((z >> 16) & 0xFFFFull) +
                        (int64_t)((z >> 32) & 0xFFFFull) + (int64_t)(z >> 48);
      const double g = (double)(n - 131070) * 0x1p-16;
      y = __dadd_rn(sig, __dmul_rn(scale, g));
    }
    out[e] = __double2float_rn(y);
  }
}

}  // namespace

extern "C" int htgen_field(const double* A, const double* B, int32_t T, int64_t N, int64_t P1, int64_t P2,
                           uint64_t key, double scale, float* out, void* stream) {
  if (A == nullptr || B == nullptr || out == nullptr || T < 1 || T > 32 || N < 1 || P1 < 1 || P2 < 1) return 1;
  const int64_t E = N * P1 * P2;
  int64_t blocks = (E + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  field_kernel<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(A, B, T, N, P1, P2, key, scale, out);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}
