// Feature-map draw from a seed, for problems given without W and b (the
// random draw of the section on randomized kernel maps, generated here from
// a seed as the paper does instead of storing it).  The definition is stated
// with bsadmm_problem.seed in include/bsadmm.h.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace bs {

namespace {

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC 2011): ten rounds of two 32 x 32 -> 64-bit
// multiplications by M0, M1, the high halves XORed with the other two
// counter words and the round key, the key advanced by the Weyl increments
// W0, W1 after every round.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = uint4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// two uniforms in (0, 1) from the four words: (w0 2^32 + w1 + 1/2) 2^-64
__device__ __forceinline__ double philox_u64(uint32_t hi, uint32_t lo) {
  const uint64_t v = ((uint64_t)hi << 32) | lo;
  return ((double)(v >> 11) + 0.5) * 0x1.0p-53;
}

// W (d x s row-major): element pair (2t, 2t + 1) from counter t, stream 0;
// b[j] from counter j, stream 1.
__global__ void draw_features_kernel(uint64_t seed, int64_t count, int64_t s, double inv_sigma,
                                     float* __restrict__ W, float* __restrict__ b) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int64_t pairs = (count + 1) / 2;
  const double two_pi = 6.283185307179586;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < pairs + s;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (t < pairs) {
      const uint4 w = philox4x32_10(uint4{(uint32_t)t, (uint32_t)(t >> 32), 0u, 0u}, k0, k1);
      const double u1 = philox_u64(w.x, w.y), u2 = philox_u64(w.z, w.w);
      const double r = sqrt(-2.0 * log(u1)) * inv_sigma;
      W[2 * t] = (float)(r * cos(two_pi * u2));
      if (2 * t + 1 < count) W[2 * t + 1] = (float)(r * sin(two_pi * u2));
    } else {
      const int64_t j = t - pairs;
      const uint4 w = philox4x32_10(uint4{(uint32_t)j, (uint32_t)(j >> 32), 1u, 0u}, k0, k1);
      float v = (float)(two_pi * philox_u64(w.x, w.y));
      if (v >= (float)two_pi) v = 0.0f;
      b[j] = v;
    }
  }
}

}  // namespace

hipError_t draw_features(uint64_t seed, int64_t d, int64_t s, double sigma, float* W, float* b,
                         hipStream_t st) {
  if (d <= 0 || s <= 0 || !(sigma > 0.0)) return hipErrorInvalidValue;
  const int64_t work = (d * s + 1) / 2 + s;
  draw_features_kernel<<<(unsigned)std::min<int64_t>((work + 255) / 256, 65536), 256, 0, st>>>(seed, d * s, s, 1.0 / sigma, W, b);
  return hipGetLastError();
}

}  // namespace bs
