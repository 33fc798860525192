// Shared device helpers: precision traits, MFMA fragment steps, BF16
// rounding and the range-reduced cosine of the feature map.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define BS_PREC_F64 0
#define BS_PREC_F32 1
#define BS_PREC_BF16 2
#define BS_PREC_BF16X3 3  // BF16 head + BF16 residual operands, three products

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
// 16-byte staging register.  A native vector type: arrays of it stay in
// registers, where arrays of HIP's struct-based uint4 end up in scratch.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef short v4s __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------------------
// Precision traits.  op_t is the MFMA operand element, acc_t the accumulator
// element; FRAG_BYTES is what one lane loads for one fragment step and KC the
// number of k values one fragment step covers across the wave (4 lane groups).
// --------------------------------------------------------------------------
template <int P> struct Prec;

template <> struct Prec<BS_PREC_F64> {
  using op_t = double;
  using acc_t = double;
  using accv = v4d;
  static constexpr int VEC = 4;   // op elements per lane per fragment step
  static constexpr int KC = 16;
};
template <> struct Prec<BS_PREC_F32> {
  using op_t = float;
  using acc_t = float;
  using accv = v4f;
  static constexpr int VEC = 4;
  static constexpr int KC = 16;
};
template <> struct Prec<BS_PREC_BF16> {
  using op_t = uint16_t;
  using acc_t = float;
  using accv = v4f;
  static constexpr int VEC = 8;
  static constexpr int KC = 32;
};
template <> struct Prec<BS_PREC_BF16X3> {
  using op_t = uint16_t;
  using acc_t = float;
  using accv = v4f;
  static constexpr int VEC = 8;
  static constexpr int KC = 32;
};

// A fragment: the VEC consecutive-k operand values one lane holds.
template <int P> struct Frag;
template <> struct Frag<BS_PREC_F64> { double v[4]; };
template <> struct Frag<BS_PREC_F32> { float v[4]; };
template <> struct Frag<BS_PREC_BF16> { uint16_t v[8]; };
template <> struct Frag<BS_PREC_BF16X3> { uint16_t v[8]; };

// One fragment step of a 16x16 output tile.  Lane l holds rows/cols
// (l % 16) of its operand and the k values kbase + VEC * (l / 16) + t.
// For FP32 and FP64 the 16x16x4 instruction takes one value per lane, so the
// step issues VEC instructions, instruction t pairing value t of A with value
// t of B: the k summation order is a permutation of the natural one, which is
// harmless because A and B use the same permutation.
__device__ __forceinline__ void mfma_step(v4d& acc, const Frag<BS_PREC_F64>& a,
                                          const Frag<BS_PREC_F64>& b) {
#pragma unroll
  for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[t], b.v[t], acc, 0, 0, 0);
}
__device__ __forceinline__ void mfma_step(v4f& acc, const Frag<BS_PREC_F32>& a,
                                          const Frag<BS_PREC_F32>& b) {
#pragma unroll
  for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[t], b.v[t], acc, 0, 0, 0);
}
__device__ __forceinline__ void mfma_step(v4f& acc, const Frag<BS_PREC_BF16>& a,
                                          const Frag<BS_PREC_BF16>& b) {
  v8bf av, bv;
  __builtin_memcpy(&av, a.v, 16);
  __builtin_memcpy(&bv, b.v, 16);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
}
__device__ __forceinline__ void mfma_step(v4f& acc, const Frag<BS_PREC_BF16X3>& a,
                                          const Frag<BS_PREC_BF16X3>& b) {
  v8bf av, bv;
  __builtin_memcpy(&av, a.v, 16);
  __builtin_memcpy(&bv, b.v, 16);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
}

// Four adjacent elements of a stored Z (double, float or bf16 bits) as MFMA
// operands of the product kernels (FP64 for double, FP32 otherwise).
template <typename ZT> struct ZAcc { using type = float; };
template <> struct ZAcc<double> { using type = double; };
template <typename ZT>
__device__ __forceinline__ void load_z4(const ZT* p, typename ZAcc<ZT>::type (&v)[4]) {
  if constexpr (sizeof(ZT) == 8) {
    const double2* q = reinterpret_cast<const double2*>(p);
    double2 x = q[0], y = q[1];
    v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
  } else if constexpr (sizeof(ZT) == 4) {
    float4 x = *reinterpret_cast<const float4*>(p);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
    uint2 x = *reinterpret_cast<const uint2*>(p);
    v[0] = __builtin_bit_cast(float, x.x << 16);
    v[1] = __builtin_bit_cast(float, x.x & 0xffff0000u);
    v[2] = __builtin_bit_cast(float, x.y << 16);
    v[3] = __builtin_bit_cast(float, x.y & 0xffff0000u);
  }
}
__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 products with 16-byte (8 values) and 8-byte (4 values) fragments per
// lane; same lane layout as the other 16 x 16 instructions.
__device__ __forceinline__ v4f mfma_bf16x8(u32x4 a, u32x4 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_bf16x4(u32x2 a, u32x2 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, a),
                                                   __builtin_bit_cast(v4s, b), c, 0, 0, 0);
}

// Row (within a 16 x 16 tile) of the accumulator element a lane of group
// g = lane / 16 holds in register r; its column is lane % 16.  The FP32
// accumulators of the 16x16x4 / 16x16x32 instructions hold rows 4 g + r,
// the FP64 16x16x4 instruction holds rows g + 4 r.
template <typename ACC> __device__ __forceinline__ constexpr int acc_row(int g, int r);
template <> __device__ __forceinline__ constexpr int acc_row<float>(int g, int r) { return 4 * g + r; }
template <> __device__ __forceinline__ constexpr int acc_row<double>(int g, int r) { return g + 4 * r; }

// Load a fragment (VEC consecutive elements, 16-byte aligned).
template <int P>
__device__ __forceinline__ Frag<P> load_frag(const typename Prec<P>::op_t* p) {
  Frag<P> f;
  if constexpr (P == BS_PREC_F64) {
    const double2* q = reinterpret_cast<const double2*>(p);
    double2 x = q[0], y = q[1];
    f.v[0] = x.x; f.v[1] = x.y; f.v[2] = y.x; f.v[3] = y.y;
  } else if constexpr (P == BS_PREC_F32) {
    float4 x = *reinterpret_cast<const float4*>(p);
    f.v[0] = x.x; f.v[1] = x.y; f.v[2] = x.z; f.v[3] = x.w;
  } else {  // BF16 / BF16X3: 8 bf16
    uint4 x = *reinterpret_cast<const uint4*>(p);
    __builtin_memcpy(f.v, &x, 16);
  }
  return f;
}

// --------------------------------------------------------------------------
// BF16 round-to-nearest-even from float (NaN kept quiet).
// --------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
// Two FP32 values to a packed pair of BF16 (low half = a), round to nearest
// even through the gfx950 conversion instruction; equal to f32_to_bf16 on
// every non-NaN input.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  const bf16x2_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  uint32_t u = ((uint32_t)h) << 16;
  float x;
  __builtin_memcpy(&x, &u, 4);
  return x;
}
// A value as a BF16 head h = bf16(v) and a BF16 residual l = bf16(v - h):
// h + l carries about 16 significant bits of v.
__device__ __forceinline__ void split_bf16(double v, uint16_t& h, uint16_t& l) {
  h = f32_to_bf16((float)v);
  l = f32_to_bf16((float)(v - (double)bf16_to_f32(h)));
}

template <typename T> __device__ __forceinline__ T cvt_from_double(double x);
template <> __device__ __forceinline__ double cvt_from_double<double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt_from_double<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ uint16_t cvt_from_double<uint16_t>(double x) {
  return f32_to_bf16((float)x);
}
template <typename T> __device__ __forceinline__ T cvt_from_float(float x);
template <> __device__ __forceinline__ double cvt_from_float<double>(float x) { return x; }
template <> __device__ __forceinline__ float cvt_from_float<float>(float x) { return x; }
template <> __device__ __forceinline__ uint16_t cvt_from_float<uint16_t>(float x) { return f32_to_bf16(x); }

__device__ __forceinline__ double to_double(double x) { return x; }
__device__ __forceinline__ double to_double(float x) { return x; }
__device__ __forceinline__ double to_double(uint16_t x) { return bf16_to_f32(x); }

// --------------------------------------------------------------------------
// cos in FP32 for the feature map.
// Cody-Waite reduction x = k (pi/2) + r with pi/2 split in three float32
// parts (12, 12 and 24 significant bits, so k * hi and k * mid are exact for
// |k| < 4096, i.e. |x| < 6400), then cos(r) or +-sin(r) on |r| <= pi/4 by
// quadrant.  The polynomials in u = r^2 (degree 4) were fitted here by
// reweighted least squares on Chebyshev nodes (fit_cos_poly.py); their FP64
// error is below 5e-11 on the interval.
// --------------------------------------------------------------------------
__device__ __forceinline__ float rff_cosf(float x) {
  const float two_over_pi = 0x1.45f306p-1f;
  const float pio2_hi = 0x1.92p+0f;
  const float pio2_mid = 0x1.fb4p-12f;
  const float pio2_lo = 0x1.4442d2p-24f;
  float k = __builtin_rintf(x * two_over_pi);
  float r = __builtin_fmaf(-k, pio2_hi, x);
  r = __builtin_fmaf(-k, pio2_mid, r);
  r = __builtin_fmaf(-k, pio2_lo, r);
  float u = r * r;
  float c = __builtin_fmaf(u, 0x1.99070p-16f, -0x1.6c0786p-10f);
  c = __builtin_fmaf(u, c, 0x1.55553ap-5f);
  c = __builtin_fmaf(u, c, -0.5f);
  c = __builtin_fmaf(u, c, 1.0f);
  float sp = __builtin_fmaf(u, 0x1.6cb78cp-19f, -0x1.a00eeap-13f);
  sp = __builtin_fmaf(u, sp, 0x1.111108p-7f);
  sp = __builtin_fmaf(u, sp, -0x1.555556p-3f);
  float sn = __builtin_fmaf(u * r, sp, r);
  int q = ((int)k) & 3;
  float v = (q & 1) ? sn : c;
  return (q == 1 || q == 2) ? -v : v;
}

// cos for values that are rounded to BF16 afterwards: the hardware cosine
// (v_cos_f32 takes revolutions) on the argument reduced to [-1/2, 1/2]
// revolutions.  Its error is orders of magnitude below one BF16 rounding.
__device__ __forceinline__ float rff_cos_bf16out(float x) {
  float r = x * 0x1.45f306p-3f;  // x / (2 pi)
  r = r - __builtin_rintf(r);
  return __builtin_amdgcn_cosf(r);
}

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  // Workgroups are dealt round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tile ids so neighbouring tiles share its L2.
  const int nx = 8;
  int per = (nblocks + nx - 1) / nx;
  int x = bid % nx, k = bid / nx;
  int full = nblocks - (per - 1) * nx;  // XCDs that receive `per` blocks
  int t = (x < full) ? x * per + k : full * per + (x - full) * (per - 1) + k;
  return t;
}
