// Feature regeneration: the transform T[X_i, j] of Algorithm 1 (step 15)
// for random Fourier features, Z = sqrt(2/s) cos(X W + b) (section
// "Randomized Kernel Maps"; the transform is one GEMM followed by an
// entrywise cosine).  One MFMA GEMM per launch with the phase offset and the
// range-reduced cosine fused into its epilogue.
#include "common.h"
#include "kernels.h"

namespace bs {

namespace {

constexpr int BM = 128;          // rows of Z per workgroup
constexpr int BN = 128;          // features of Z per workgroup
constexpr int NTHREADS = 256;
constexpr int GROUP_M = 8;


// ---------------------------------------------------------------------------
// Operand preparation
// ---------------------------------------------------------------------------
// Row operands; BF16X3 writes the head plane at dst and the residual plane at
// dst + plane (elements).
template <int P>
__global__ void prep_rows_kernel(const float* __restrict__ src, int64_t rows, int64_t d,
                                 int64_t Kp, typename Prec<P>::op_t* __restrict__ dst,
                                 int64_t plane, int* __restrict__ flag) {
  using op_t = typename Prec<P>::op_t;
  int64_t total = rows * Kp;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e / Kp, k = e - r * Kp;
    float v = (k < d) ? src[r * d + k] : 0.0f;
    if (!__builtin_isfinite(v)) bad = 1;
    const op_t h = cvt_from_float<op_t>(v);
    dst[e] = h;
    if constexpr (P == BS_PREC_BF16X3) dst[plane + e] = f32_to_bf16(v - bf16_to_f32(h));
  }
  if (bad && flag) atomicOr(flag, 1);
}

// W is d x s (ld = s); Wt is s x Kp.  32 x 32 tiles through LDS.
template <int P>
__global__ void prep_w_kernel(const float* __restrict__ W, int64_t d, int64_t s, int64_t Kp,
                              typename Prec<P>::op_t* __restrict__ Wt, int64_t plane,
                              int* __restrict__ flag) {
  using op_t = typename Prec<P>::op_t;
  __shared__ float tile[32][33];
  int64_t f0 = (int64_t)blockIdx.x * 32, k0 = (int64_t)blockIdx.y * 32;
  int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: ty 0..7
  int bad = 0;
  for (int yy = ty; yy < 32; yy += 8) {
    int64_t k = k0 + yy, f = f0 + tx;
    float v = (k < d && f < s) ? W[k * s + f] : 0.0f;
    if (!__builtin_isfinite(v)) bad = 1;
    tile[yy][tx] = v;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    int64_t f = f0 + yy, k = k0 + tx;
    if (f < s && k < Kp) {
      const float v = tile[tx][yy];
      const op_t h = cvt_from_float<op_t>(v);
      Wt[f * Kp + k] = h;
      if constexpr (P == BS_PREC_BF16X3) Wt[plane + f * Kp + k] = f32_to_bf16(v - bf16_to_f32(h));
    }
  }
  if (bad && flag) atomicOr(flag, 1);
}

template <typename B>
__global__ void prep_bias_kernel(const float* __restrict__ b, int64_t s, B* __restrict__ out,
                                 int* __restrict__ flag) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f < s) {
    float v = b[f];
    if (!__builtin_isfinite(v) && flag) atomicOr(flag, 1);
    out[f] = (B)v;
  }
}

__global__ void check_finite_kernel(const float* __restrict__ p, int64_t count, int* flag) {
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    if (!__builtin_isfinite(p[e])) bad = 1;
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Regeneration GEMM.  Xp (rows x Kp) and Wt (cols x Kp) are both k-contiguous.
// A 256-thread workgroup computes a 128 x 128 tile of Z; its 4 waves each own
// a 64 x 64 quadrant made of 4 x 4 MFMA 16 x 16 tiles.  k advances in chunks
// staged through double-buffered LDS; the next chunk's global loads are in
// flight while the current one feeds the MFMAs.
//
// BF16X3 operands come in two planes (plane stride xps / wps elements): the
// BF16 head h = bf16(v) and the BF16 residual l = bf16(v - h).  The phase
// accumulates h_x h_w + h_x l_w + l_x h_w in FP32 (the dropped l_x l_w term is
// ~2^-16 of the product), so the phase keeps ~16 significant bits instead of
// the ~8 of a single BF16 product.
// ---------------------------------------------------------------------------
template <int V> struct Tag { static constexpr int value = V; };
template <int P> constexpr int planes() { return P == BS_PREC_BF16X3 ? 2 : 1; }
// Bytes of one staged k-chunk per row (per plane).  FP32 stages 16 values so
// that four 40 KB workgroups fill the LDS of a CU (4 waves per SIMD to cover
// each other's barrier and load waits); FP64 needs 128 bytes for one step.
template <int P> constexpr int krow_bytes() {
  return (P == BS_PREC_BF16X3 || P == BS_PREC_F32) ? 64 : 128;
}
// Workgroups per CU the register budget is sized for.
template <int P> constexpr int regen_wgs() { return P == BS_PREC_F32 ? 4 : 2; }

// Defect bf16(z - t) of an FP32-faithful feature z against its BF16 value t.
// z must be the rounded float (as stored): no contraction of the product that
// formed z with this difference, so both epilogue paths give the same bits.
__device__ __forceinline__ uint16_t feature_defect_bf16(float z, uint16_t t) {
#pragma clang fp contract(off)
  return f32_to_bf16(z - bf16_to_f32(t));
}

template <int P, typename ZT, bool DEFECT = false>
__global__ void __launch_bounds__(NTHREADS, regen_wgs<P>())
regen_kernel(const typename Prec<P>::op_t* __restrict__ Xp, int64_t xps, int64_t rows,
             const typename Prec<P>::op_t* __restrict__ Wt, int64_t wps, int64_t cols,
             const typename Prec<P>::acc_t* __restrict__ bias, int64_t Kp,
             typename Prec<P>::acc_t scale, ZT* __restrict__ Z, int64_t ldz,
             const uint16_t* __restrict__ Zt, uint16_t* __restrict__ Zd) {
  using op_t = typename Prec<P>::op_t;
  using acc_t = typename Prec<P>::acc_t;
  using accv = typename Prec<P>::accv;
  constexpr int VEC = Prec<P>::VEC;
  constexpr int KC = Prec<P>::KC;
  constexpr int NPL = planes<P>();
  constexpr int KROW = krow_bytes<P>();
  constexpr int PITCH = KROW + 16;
  constexpr int BK = KROW / (int)sizeof(op_t);
  constexpr int STEPS = BK / KC;           // fragment steps per chunk
  constexpr int SEGS = KROW / 16;          // 16-byte segments per staged row
  constexpr int NS = BM * SEGS / NTHREADS; // staged segments per thread, per plane

  __shared__ __attribute__((aligned(16))) unsigned char lds[2][2][NPL][BM * PITCH];

  const int tiles_m = (int)((rows + BM - 1) / BM);
  const int tiles_n = (int)((cols + BN - 1) / BN);
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int per_group = GROUP_M * tiles_n;
  const int g = t / per_group;
  const int first_m = g * GROUP_M;
  const int gsize = min(GROUP_M, tiles_m - first_m);
  const int tm = first_m + (t % per_group) % gsize;
  const int tn = (t % per_group) / gsize;
  const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const unsigned char* gA[NS];
  const unsigned char* gB[NS];
  int ldsoff[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int idx = tid + NTHREADS * i;
    const int r = idx / SEGS, seg = idx % SEGS;
    const int64_t ra = min(row0 + r, rows - 1);
    const int64_t rb = min(col0 + r, cols - 1);
    gA[i] = reinterpret_cast<const unsigned char*>(Xp + ra * Kp) + seg * 16;
    gB[i] = reinterpret_cast<const unsigned char*>(Wt + rb * Kp) + seg * 16;
    ldsoff[i] = r * PITCH + seg * 16;
  }
  const int64_t xpb = xps * (int64_t)sizeof(op_t), wpb = wps * (int64_t)sizeof(op_t);
  const int64_t nchunks = Kp / BK;
  // Global loads run DEPTH chunks ahead of the MFMAs through DEPTH register
  // sets (FP64 has no registers to spare for a second set; FP32 spends its
  // registers on occupancy instead).
  constexpr int DEPTH = (P == BS_PREC_F64 || P == BS_PREC_F32) ? 1 : 2;
  u32x4 sa[DEPTH][NPL][NS], sb[DEPTH][NPL][NS];

  accv acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  const int fr = lane & 15, fg = lane >> 4;
  // register set SET <- chunk `chunk` of the X and W tiles
  auto gload = [&](auto set, int64_t chunk) {
    constexpr int S = decltype(set)::value;
    const int64_t off = chunk * KROW;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        sa[S][pl][i] = *reinterpret_cast<const u32x4*>(gA[i] + pl * xpb + off);
        sb[S][pl][i] = *reinterpret_cast<const u32x4*>(gB[i] + pl * wpb + off);
      }
  };
  // LDS buffer BUF <- register set SET
  auto lstore = [&](auto set, auto buf) {
    constexpr int S = decltype(set)::value, B = decltype(buf)::value;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        *reinterpret_cast<u32x4*>(&lds[B][0][pl][ldsoff[i]]) = sa[S][pl][i];
        *reinterpret_cast<u32x4*>(&lds[B][1][pl][ldsoff[i]]) = sb[S][pl][i];
      }
  };
  // the MFMAs of the chunk staged in LDS buffer `buf`
  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < STEPS; ++ks) {
      const int kbyte = (ks * KC + VEC * fg) * (int)sizeof(op_t);
      Frag<P> fa[NPL][4], fb[NPL][4];
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          fa[pl][i] = load_frag<P>(reinterpret_cast<const op_t*>(
              &lds[buf][0][pl][(wm * 64 + i * 16 + fr) * PITCH + kbyte]));
          fb[pl][i] = load_frag<P>(reinterpret_cast<const op_t*>(
              &lds[buf][1][pl][(wn * 64 + i * 16 + fr) * PITCH + kbyte]));
        }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          mfma_step(acc[i][j], fa[0][i], fb[0][j]);
          if constexpr (NPL == 2) {
            mfma_step(acc[i][j], fa[0][i], fb[1][j]);
            mfma_step(acc[i][j], fa[1][i], fb[0][j]);
          }
        }
    }
  };
  constexpr Tag<0> T0{};
  constexpr Tag<1> T1{};

  if constexpr (DEPTH == 2) {
    // Chunk k travels in register set k % 2 and LDS buffer k % 2.  Loads are
    // issued unconditionally, past the last chunk as repeats of it, so that
    // no branch separates a load from the wait for it.
    // The loop runs over whole pairs of chunks so that no exit test sits
    // between a load and the store that consumes it (the compiler would sink
    // the load past the test), and the scheduling barriers keep each step's
    // loads ahead of its MFMAs and its LDS stores after them.
    const int64_t last = nchunks - 1;
    gload(T0, 0);
    gload(T1, min((int64_t)1, last));
    lstore(T0, T0);
    __syncthreads();
    for (int64_t c = 0; c + 1 < nchunks; c += 2) {
      gload(T0, min(c + 2, last));
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      __builtin_amdgcn_sched_barrier(0);
      lstore(T1, T1);  // chunk c + 1
      __syncthreads();
      gload(T1, min(c + 3, last));
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      __builtin_amdgcn_sched_barrier(0);
      lstore(T0, T0);  // chunk c + 2
      __syncthreads();
    }
    if (nchunks & 1) compute(0);  // the last chunk, staged in buffer 0
  } else {
    gload(T0, 0);
    lstore(T0, T0);
    __syncthreads();
    for (int64_t c = 0; c < nchunks; ++c) {
      const int buf = (int)(c & 1);
      const bool more = c + 1 < nchunks;
      if (more) gload(T0, c + 1);
      compute(buf);
      if (more) {
        if (buf) lstore(T0, T0);
        else lstore(T0, T1);
      }
      __syncthreads();
    }
  }

  // Epilogue: lane holds D[acc_row(lane / 16, r)][lane % 16] of each 16 x 16 tile.
  // Float Z of a whole tile leaves through LDS, half a tile (64 rows, the
  // rows of waves wm = h) at a time, as 512-byte rows with 16-byte
  // non-temporal stores; straight from the MFMA layout a store instruction
  // writes 64 bytes into each of 4 rows.  The LDS is free once every wave
  // has passed the barrier below (the last chunk's products may follow the
  // loop's last barrier).  DEFECT (FP32-faithful features of refined BF16):
  // the float values are not stored; the defect bf16(z - Zt) against the
  // BF16 features Zt of the same elements goes to Zd instead.
  if constexpr (sizeof(ZT) == 4) {
    constexpr int ZP = BN + 4;                     // floats per staged row (528 B)
    static_assert(BM / 2 * ZP * 4 <= (int)sizeof(lds), "half a Z tile fits in the staging LDS");
    if (row0 + BM <= rows && col0 + BN <= cols && ldz % 4 == 0 &&
        reinterpret_cast<uintptr_t>(DEFECT ? (const void*)Zd : (const void*)Z) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(Zt) % 8 == 0) {
      float* zt = reinterpret_cast<float*>(&lds[0][0][0][0]);
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (wm == h) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int cl = wn * 64 + j * 16 + fr;
            const acc_t bcol = bias[col0 + cl];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const float z = scale * rff_cosf(acc[i][j][r] + bcol);
                zt[(i * 16 + acc_row<acc_t>(fg, r)) * ZP + cl] = z;
              }
          }
        }
        __syncthreads();
        constexpr int RPP = NTHREADS / 32;         // rows per pass: 32 lanes a row
#pragma unroll 2
        for (int ps = 0; ps < BM / 2 / RPP; ++ps) {
          const int r = ps * RPP + tid / 32, sg = tid % 32;
          const v4f w = *reinterpret_cast<const v4f*>(zt + r * ZP + sg * 4);
          const int64_t off = (row0 + h * (BM / 2) + r) * ldz + col0 + sg * 4;
          if constexpr (DEFECT) {
            const uint2 t = *reinterpret_cast<const uint2*>(Zt + off);
            uint2 o;
            o.x = (uint32_t)feature_defect_bf16(w[0], (uint16_t)(t.x & 0xffffu)) |
                  ((uint32_t)feature_defect_bf16(w[1], (uint16_t)(t.x >> 16)) << 16);
            o.y = (uint32_t)feature_defect_bf16(w[2], (uint16_t)(t.y & 0xffffu)) |
                  ((uint32_t)feature_defect_bf16(w[3], (uint16_t)(t.y >> 16)) << 16);
            *reinterpret_cast<uint2*>(Zd + off) = o;
          } else {
            __builtin_nontemporal_store(w, reinterpret_cast<v4f*>(Z + off));
          }
        }
        __syncthreads();
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = col0 + wn * 64 + j * 16 + fr;
    const bool cok = col < cols;
    const acc_t bcol = cok ? bias[col] : (acc_t)0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + wm * 64 + i * 16 + acc_row<acc_t>(fg, r);
        if (cok && row < rows) {
          acc_t th = acc[i][j][r] + bcol;
          acc_t z;
          if constexpr (P == BS_PREC_F64)
            z = scale * cos(th);
          else if constexpr (P == BS_PREC_BF16)
            z = scale * rff_cos_bf16out(th);
          else
            z = scale * rff_cosf(th);
          if constexpr (sizeof(ZT) == 2) {
            Z[row * ldz + col] = f32_to_bf16((float)z);
          } else if constexpr (DEFECT) {
            Zd[row * ldz + col] = feature_defect_bf16((float)z, Zt[row * ldz + col]);
          } else {
            Z[row * ldz + col] = (ZT)z;
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Wide-tile regeneration for single-plane BF16 operands.  A 512-thread
// workgroup computes a 256 x 256 tile of Z (8 waves of 128 rows x 64
// features, 32 MFMA 16x16x32 tiles each), so each staged k-chunk feeds twice
// the MFMA work of the 128 x 128 kernel per byte moved from L2.
// Double-buffered LDS (147 KB) keeps one workgroup per CU.  The staging loads
// are raw buffer loads whose descriptor ends at the tile's last valid row, so
// rows past the edge read as zero and one 32-bit offset per thread addresses
// all of its segments.  The feature tile is the MFMA's M operand and the row
// tile its N operand: a lane ends with 4 adjacent features of one row, packed
// to BF16; the tile is then staged in LDS and stored as whole rows.  The
// k-steps are those of regen_kernel.
// ---------------------------------------------------------------------------
constexpr int WBM = 256, WBN = 256, WNT = 512, WKROW = 128, WPITCH = WKROW + 16;
constexpr int WSEG = WKROW / 16;                 // 16-byte segments per staged row
constexpr int WNS = WBM * WSEG / WNT;            // segments per thread and operand (4)
constexpr int WRSTEP = WNT / WSEG;               // rows between a thread's segments (64)
constexpr int WTJ = 4;                           // feature tiles per wave
constexpr int WZPITCH = 2 * WBN + 32;            // bytes per row of a Z tile staged in LDS
static_assert(WBM * WZPITCH <= 2 * (WBM + WBN) * WPITCH, "a Z tile fits in the staging LDS");

// Raw buffer descriptor over [p, p + bytes): loads past the end return zero.
// p and bytes are wave-uniform; rebuilding them from readfirstlane halves
// keeps the descriptor in scalar registers even where their arithmetic was
// done in vector registers.  A descriptor in vector registers wraps each load
// in a readfirstlane loop.  The byte counts below take min() of two int64
// values: HIP's math headers evaluate min() of an int64 and an int in double
// precision, in vector registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wide_rsrc(const void* p, int64_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  const int nb = __builtin_amdgcn_readfirstlane((int)bytes);
  void* q = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, nb, 0x00020000);
}

__device__ __forceinline__ void wide_load(const void* pa, int64_t na, const void* pb, int64_t nbb,
                                          int voff, int rowb, int koff, u32x4 (&sa)[WNS],
                                          u32x4 (&sb)[WNS]) {
  const __amdgpu_buffer_rsrc_t ra = wide_rsrc(pa, na), rb = wide_rsrc(pb, nbb);
#pragma unroll
  for (int i = 0; i < WNS; ++i)
    sa[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                          ra, voff, i * WRSTEP * rowb + koff, 0));
#pragma unroll
  for (int i = 0; i < WNS; ++i)
    sb[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                          rb, voff, i * WRSTEP * rowb + koff, 0));
}

__device__ __forceinline__ void wide_store(unsigned char* buf, int lofs, const u32x4 (&sa)[WNS],
                                           const u32x4 (&sb)[WNS]) {
#pragma unroll
  for (int i = 0; i < WNS; ++i)
    *reinterpret_cast<u32x4*>(buf + lofs + i * WRSTEP * WPITCH) = sa[i];
#pragma unroll
  for (int i = 0; i < WNS; ++i)
    *reinterpret_cast<u32x4*>(buf + WBM * WPITCH + lofs + i * WRSTEP * WPITCH) = sb[i];
}

// The MFMA work of one staged chunk (64 k values, two 16x16x32 steps).
__device__ __forceinline__ void wide_mfma(const unsigned char* buf, int wm, int wn, int fr, int fg,
                                          v4f (&acc)[WTJ][8]) {
  // quarter q = (k-step ks, row half h) of the chunk's two k-steps; its
  // fragments are read while the previous quarter's 16 products run
  static_assert(WKROW == 128, "two 32-value k-steps per chunk");
  auto load_w = [&](int ks, Frag<BS_PREC_BF16> (&fw)[WTJ]) {
#pragma unroll
    for (int j = 0; j < WTJ; ++j)
      fw[j] = load_frag<BS_PREC_BF16>(reinterpret_cast<const uint16_t*>(
          buf + (WBM + wn * (16 * WTJ) + j * 16 + fr) * WPITCH + ks * 64 + 16 * fg));
  };
  auto load_x = [&](int ks, int h, Frag<BS_PREC_BF16> (&fx)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      fx[i] = load_frag<BS_PREC_BF16>(reinterpret_cast<const uint16_t*>(
          buf + (wm * 128 + (4 * h + i) * 16 + fr) * WPITCH + ks * 64 + 16 * fg));
  };
  // a wave issuing its products takes issue priority over the other wave of
  // its SIMD, which is then reading fragments or staging (0.7% per launch)
  auto prod = [&](int h, const Frag<BS_PREC_BF16> (&fw)[WTJ], const Frag<BS_PREC_BF16> (&fx)[4]) {
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < WTJ; ++j) mfma_step(acc[j][4 * h + i], fw[j], fx[i]);
    __builtin_amdgcn_s_setprio(0);
  };
  Frag<BS_PREC_BF16> fw0[WTJ], fw1[WTJ], xa[4], xb[4];
  load_w(0, fw0);
  load_x(0, 0, xa);
  load_x(0, 1, xb);
  __builtin_amdgcn_sched_barrier(0);
  prod(0, fw0, xa);
  __builtin_amdgcn_sched_barrier(0);
  load_w(1, fw1);
  load_x(1, 0, xa);
  __builtin_amdgcn_sched_barrier(0);
  prod(1, fw0, xb);
  __builtin_amdgcn_sched_barrier(0);
  load_x(1, 1, xb);
  __builtin_amdgcn_sched_barrier(0);
  prod(0, fw1, xa);
  __builtin_amdgcn_sched_barrier(0);
  prod(1, fw1, xb);
}

// Persistent: the grid holds one workgroup per CU and each walks a list of
// tiles.  Workgroups are dealt round-robin over the 8 XCDs; workgroup b takes
// every (grid / 8)-th tile of XCD b % 8's contiguous tile range, so the tiles
// an XCD runs at once are neighbours that share its L2.  The next tile's
// first chunk is loaded during the current tile's last chunk and epilogue.
__global__ void __launch_bounds__(WNT, 1)
regen_bf16_wide_kernel(const uint16_t* __restrict__ Xp, int64_t rows,
                       const uint16_t* __restrict__ Wt, int64_t cols,
                       const float* __restrict__ bias, int64_t Kp, float scale,
                       uint16_t* __restrict__ Z, int64_t ldz) {
  constexpr int TJ = WTJ;
  constexpr int BK = WKROW / 2;               // 64 bf16 per chunk
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][(WBM + WBN) * WPITCH];

  const int tiles_m = (int)((rows + WBM - 1) / WBM);
  const int tiles_n = (int)((cols + WBN - 1) / WBN);
  const int T = tiles_m * tiles_n;
  // this XCD's tile range [tbeg, tend), split as in xcd_remap
  const int x = (int)(blockIdx.x % 8), wpx = (int)(gridDim.x / 8);
  const int per = (T + 7) / 8, full = T - (per - 1) * 8;
  const int tbeg = x < full ? x * per : full * per + (x - full) * (per - 1);
  const int tend = tbeg + (x < full ? per : per - 1);
  int t = tbeg + (int)(blockIdx.x / 8);
  if (t >= tend) return;  // uniform over the workgroup

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;     // 2 x 4 waves
  const int fr = lane & 15, fg = lane >> 4;
  // staging: thread tid moves segment tid % 8 of rows tid / 8 + 64 i
  const int rowb = (int)(Kp * 2);
  const int voff = (tid / WSEG) * rowb + (tid % WSEG) * 16;
  const int lofs = (tid / WSEG) * WPITCH + (tid % WSEG) * 16;
  const int per_group = GROUP_M * tiles_n;
  auto origin = [&](int tt, int64_t& r0, int64_t& c0) {
    const int g = tt / per_group;
    const int first_m = g * GROUP_M;
    const int gsize = min(GROUP_M, tiles_m - first_m);
    r0 = (int64_t)(first_m + (tt % per_group) % gsize) * WBM;
    c0 = (int64_t)((tt % per_group) / gsize) * WBN;
  };
  int64_t row0, col0;
  origin(t, row0, col0);
  const int64_t nchunks = Kp / BK;
  u32x4 sa[WNS], sb[WNS];
  wide_load(Xp + row0 * Kp, min(rows - row0, (int64_t)WBM) * rowb, Wt + col0 * Kp,
            min(cols - col0, (int64_t)WBN) * rowb, voff, rowb, 0, sa, sb);
  wide_store(lds[0], lofs, sa, sb);
  __syncthreads();

  for (;;) {
    const void* pa = Xp + row0 * Kp;
    const int64_t na = min(rows - row0, (int64_t)WBM) * rowb;
    const void* pb = Wt + col0 * Kp;
    const int64_t nbb = min(cols - col0, (int64_t)WBN) * rowb;
    const int tnext = t + wpx;
    const bool has_next = tnext < tend;
    int64_t nrow0 = 0, ncol0 = 0;
    if (has_next) origin(tnext, nrow0, ncol0);

    v4f acc[TJ][8];   // [feature tile][row tile]
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[j][i] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int64_t c = 0; c < nchunks; ++c) {
      const int buf = (int)(c & 1);
      const bool more = c + 1 < nchunks;
      if (more)
        wide_load(pa, na, pb, nbb, voff, rowb, (int)(c + 1) * WKROW, sa, sb);
      else if (has_next)
        wide_load(Xp + nrow0 * Kp, min(rows - nrow0, (int64_t)WBM) * rowb, Wt + ncol0 * Kp,
                  min(cols - ncol0, (int64_t)WBN) * rowb, voff, rowb, 0, sa, sb);
      wide_mfma(lds[buf], wm, wn, fr, fg, acc);
      if (more) wide_store(lds[buf ^ 1], lofs, sa, sb);
      __syncthreads();
    }

    // Epilogue: lane holds features 4 fg .. 4 fg + 3 of tile j for row fr of
    // tile i; phase + bias -> cos -> two packed BF16 pairs.  A whole tile
    // goes to LDS (free after the last chunk's barrier) as rows of 256
    // values, then leaves as 512-byte rows, 16 bytes a lane, with
    // non-temporal stores: an 8-byte store from the MFMA layout touches 16
    // rows.  Tiles that cross the row or feature edge store element by
    // element.
    if (row0 + WBM <= rows && col0 + WBN <= cols) {
      unsigned char* zt = &lds[0][0];
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const int fl = wn * (16 * TJ) + j * 16 + 4 * fg;
        const int64_t f = col0 + fl;
        const float b0 = bias[f], b1 = bias[f + 1], b2 = bias[f + 2], b3 = bias[f + 3];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          uint2 v;
          v.x = pack_bf16x2(scale * rff_cos_bf16out(acc[j][i][0] + b0),
                            scale * rff_cos_bf16out(acc[j][i][1] + b1));
          v.y = pack_bf16x2(scale * rff_cos_bf16out(acc[j][i][2] + b2),
                            scale * rff_cos_bf16out(acc[j][i][3] + b3));
          *reinterpret_cast<uint2*>(zt + (wm * 128 + i * 16 + fr) * WZPITCH + fl * 2) = v;
        }
      }
      __syncthreads();
      constexpr int RPP = WNT / 32;                // rows per pass: 32 lanes a row
#pragma unroll 1
      for (int ps = 0; ps < WBM / RPP; ++ps) {
        const int r = ps * RPP + tid / 32, sg = tid % 32;
        const u32x4 w = *reinterpret_cast<const u32x4*>(zt + r * WZPITCH + sg * 16);
        __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(Z + (row0 + r) * ldz + col0 + sg * 8));
      }
      __syncthreads();   // the next tile's first chunk reuses this LDS
    } else {
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const int64_t f = col0 + wn * (16 * TJ) + j * 16 + 4 * fg;
        float bj[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bj[r] = bias[min(f + r, cols - 1)];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int64_t row = row0 + wm * 128 + i * 16 + fr;
          if (row >= rows) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (f + r < cols) {
              const float z = scale * rff_cos_bf16out(acc[j][i][r] + bj[r]);
              Z[row * ldz + f + r] = (uint16_t)(pack_bf16x2(z, 0.f) & 0xffffu);
            }
        }
      }
    }
    if (!has_next) break;
    // every wave passed the last chunk's barrier: no one reads LDS any more
    wide_store(lds[0], lofs, sa, sb);
    __syncthreads();
    t = tnext;
    row0 = nrow0;
    col0 = ncol0;
  }
}

// ---------------------------------------------------------------------------
// Wide-tile regeneration for split BF16 operands (head h and residual l
// planes of X and W; phase = h_x h_w + h_x l_w + l_x h_w per 32-value k-step,
// in that order, as regen_kernel).  A 512-thread workgroup computes a
// 256 x 256 tile (8 waves of 128 rows x 64 features); each staged chunk is
// one k-step of the four planes, 1024 rows of 64 bytes (pitch 80), double
// buffered in all of the 160 KB of LDS, and feeds three products, so a
// staged byte feeds three times the MFMA work of the one-plane wide kernel.
// X is the MFMA's M operand, as in regen_kernel, so the bits are regen_kernel's.
// The FP32 features leave through LDS in two halves of 128 rows as whole
// 1 KB rows.  Persistent, one workgroup per CU, tiles dealt as in the wide
// kernel.  (The refinement defect stays with regen_kernel: through this
// kernel it measured 4.8% slower.)
// ---------------------------------------------------------------------------
constexpr int XBM = 256, XBN = 256, XNT = 512, XKROW = 64, XPITCH = XKROW + 16;
constexpr int XSET = 256 * XPITCH;                // bytes of one staged plane (X or W rows)
constexpr int XBUF = 4 * XSET;                    // one chunk: X head, X residual, W head, W residual
constexpr int XNS = 4 * 256 * (XKROW / 16) / XNT; // staged segments per thread (8)
constexpr int XZP = XBN + 4;                      // floats per staged Z row (1040 B)
static_assert(2 * XBUF <= 163840, "two chunks fit the LDS");
static_assert((XBM / 2) * XZP * 4 <= 2 * XBUF, "half a Z tile fits the LDS");

__global__ void __launch_bounds__(XNT, 1)
regen_bf16x3_wide_kernel(const uint16_t* __restrict__ Xp, int64_t xps, int64_t rows,
                         const uint16_t* __restrict__ Wt, int64_t wps, int64_t cols,
                         const float* __restrict__ bias, int64_t Kp, float scale,
                         float* __restrict__ Z, int64_t ldz) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * XBUF];

  const int tiles_m = (int)((rows + XBM - 1) / XBM);
  const int tiles_n = (int)((cols + XBN - 1) / XBN);
  const int T = tiles_m * tiles_n;
  const int x = (int)(blockIdx.x % 8), wpx = (int)(gridDim.x / 8);
  const int per = (T + 7) / 8, full = T - (per - 1) * 8;
  const int tbeg = x < full ? x * per : full * per + (x - full) * (per - 1);
  const int tend = tbeg + (x < full ? per : per - 1);
  int t = tbeg + (int)(blockIdx.x / 8);
  if (t >= tend) return;  // uniform over the workgroup

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;     // 2 x 4 waves
  const int fr = lane & 15, fg = lane >> 4;
  // staging: thread tid moves segment tid % 4 of rows tid / 4 and tid / 4 + 128
  // of each of the four planes
  const int rowb = (int)(Kp * 2);
  const int voff = (tid / 4) * rowb + (tid % 4) * 16;
  const int lofs = (tid / 4) * XPITCH + (tid % 4) * 16;
  const int per_group = GROUP_M * tiles_n;
  auto origin = [&](int tt, int64_t& r0, int64_t& c0) {
    const int g = tt / per_group;
    const int first_m = g * GROUP_M;
    const int gsize = min(GROUP_M, tiles_m - first_m);
    r0 = (int64_t)(first_m + (tt % per_group) % gsize) * XBM;
    c0 = (int64_t)((tt % per_group) / gsize) * XBN;
  };
  auto load = [&](int64_t r0, int64_t c0, int koff, u32x4 (&sg)[XNS]) {
    const int64_t na = min(rows - r0, (int64_t)XBM) * rowb;
    const int64_t nb = min(cols - c0, (int64_t)XBN) * rowb;
    const __amdgpu_buffer_rsrc_t rs[4] = {wide_rsrc(Xp + r0 * Kp, na), wide_rsrc(Xp + xps + r0 * Kp, na),
                                          wide_rsrc(Wt + c0 * Kp, nb), wide_rsrc(Wt + wps + c0 * Kp, nb)};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        sg[2 * q + h] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                                      rs[q], voff, h * 128 * rowb + koff, 0));
  };
  auto store = [&](unsigned char* buf, const u32x4 (&sg)[XNS]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        *reinterpret_cast<u32x4*>(buf + q * XSET + lofs + h * 128 * XPITCH) = sg[2 * q + h];
  };
  using F = Frag<BS_PREC_BF16X3>;
  auto frag = [&](const unsigned char* buf, int q, int row) {
    return load_frag<BS_PREC_BF16X3>(
        reinterpret_cast<const uint16_t*>(buf + q * XSET + row * XPITCH + 16 * fg));
  };

  int64_t row0, col0;
  origin(t, row0, col0);
  const int64_t nchunks = Kp / (XKROW / 2);
  u32x4 sg[XNS];
  load(row0, col0, 0, sg);
  store(lds, sg);
  __syncthreads();

  for (;;) {
    const int tnext = t + wpx;
    const bool has_next = tnext < tend;
    int64_t nrow0 = 0, ncol0 = 0;
    if (has_next) origin(tnext, nrow0, ncol0);

    v4f acc[8][4];   // [row tile][feature tile]
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int64_t c = 0; c < nchunks; ++c) {
      const unsigned char* cur = lds + (c & 1) * XBUF;
      const bool more = c + 1 < nchunks;
      if (more) load(row0, col0, (int)(c + 1) * XKROW, sg);
      else if (has_next) load(nrow0, ncol0, 0, sg);
      F wh[4], wl[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        wh[j] = frag(cur, 2, wn * 64 + j * 16 + fr);
        wl[j] = frag(cur, 3, wn * 64 + j * 16 + fr);
      }
#pragma unroll
      for (int qr = 0; qr < 4; ++qr) {   // row tiles 2 qr, 2 qr + 1
        F xh[2], xl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          xh[i] = frag(cur, 0, wm * 128 + (2 * qr + i) * 16 + fr);
          xl[i] = frag(cur, 1, wm * 128 + (2 * qr + i) * 16 + fr);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            mfma_step(acc[2 * qr + i][j], xh[i], wh[j]);
            mfma_step(acc[2 * qr + i][j], xh[i], wl[j]);
            mfma_step(acc[2 * qr + i][j], xl[i], wh[j]);
          }
      }
      if (more) store(lds + ((c + 1) & 1) * XBUF, sg);
      __syncthreads();
    }

    // Epilogue: lane holds rows 4 fg .. 4 fg + 3 of row tile i for feature fr
    // of feature tile j.
    const bool fast = row0 + XBM <= rows && col0 + XBN <= cols;
    if (fast) {
      float* zt = reinterpret_cast<float*>(lds);
#pragma unroll 1
      for (int h = 0; h < 2; ++h) {
        if (wm == h) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int cl = wn * 64 + j * 16 + fr;
            const float bcol = bias[col0 + cl];
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                zt[(i * 16 + acc_row<float>(fg, r)) * XZP + cl] =
                    scale * rff_cosf(acc[i][j][r] + bcol);
          }
        }
        __syncthreads();
#pragma unroll 2
        for (int ps = 0; ps < (XBM / 2) / (XNT / 64); ++ps) {
          const int r = ps * (XNT / 64) + tid / 64, sgi = tid % 64;
          const v4f w = *reinterpret_cast<const v4f*>(zt + r * XZP + sgi * 4);
          const int64_t off = (row0 + h * (XBM / 2) + r) * ldz + col0 + sgi * 4;
          __builtin_nontemporal_store(w, reinterpret_cast<v4f*>(Z + off));
        }
        __syncthreads();   // the LDS: the next half, or the next tile's first chunk
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = col0 + wn * 64 + j * 16 + fr;
        const bool cok = col < cols;
        const float bcol = cok ? bias[col] : 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + wm * 128 + i * 16 + acc_row<float>(fg, r);
            if (cok && row < rows) Z[row * ldz + col] = scale * rff_cosf(acc[i][j][r] + bcol);
          }
      }
    }
    if (!has_next) break;
    // every wave passed the last barrier: no one reads LDS any more
    store(lds, sg);
    __syncthreads();
    t = tnext;
    row0 = nrow0;
    col0 = ncol0;
  }
}

// Compute units of the current device (queried once per device).
int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

inline unsigned grid_1d(int64_t count, int threads, int64_t cap = 65536) {
  int64_t g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

int64_t padded_k(int prec, int64_t d) {
  // a whole number of the regeneration's k-chunks (the wide BF16 kernel's
  // chunk is 128 bytes, as regen_kernel's BF16 one)
  int krow = 128;
  if (prec == BS_PREC_F32) krow = krow_bytes<BS_PREC_F32>();
  else if (prec == BS_PREC_BF16X3) krow = krow_bytes<BS_PREC_BF16X3>();
  const int64_t bk = krow / (int64_t)op_bytes(prec);
  return ((d + bk - 1) / bk) * bk;
}

size_t op_bytes(int prec) {
  return prec == BS_PREC_F64 ? 8 : (prec == BS_PREC_F32 ? 4 : 2);
}

int op_planes(int prec) { return prec == BS_PREC_BF16X3 ? 2 : 1; }

size_t z_bytes(int prec) {
  return prec == BS_PREC_F64 ? 8 : (prec == BS_PREC_BF16 ? 2 : 4);
}

size_t vec_bytes(int prec) { return prec == BS_PREC_F64 ? 8 : 4; }

hipError_t prep_rows(int prec, const float* src, int64_t rows, int64_t d, int64_t Kp, void* dst,
                     int64_t plane, int* flag, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  unsigned g = grid_1d(rows * Kp, 256);
  switch (prec) {
    case BS_PREC_F64:
      prep_rows_kernel<BS_PREC_F64><<<g, 256, 0, st>>>(src, rows, d, Kp, (double*)dst, plane, flag);
      break;
    case BS_PREC_F32:
      prep_rows_kernel<BS_PREC_F32><<<g, 256, 0, st>>>(src, rows, d, Kp, (float*)dst, plane, flag);
      break;
    case BS_PREC_BF16:
      prep_rows_kernel<BS_PREC_BF16><<<g, 256, 0, st>>>(src, rows, d, Kp, (uint16_t*)dst, plane,
                                                         flag);
      break;
    default:
      prep_rows_kernel<BS_PREC_BF16X3><<<g, 256, 0, st>>>(src, rows, d, Kp, (uint16_t*)dst, plane,
                                                           flag);
  }
  return hipGetLastError();
}

hipError_t prep_w(int prec, const float* W, const float* b, int64_t d, int64_t s, int64_t Kp,
                  void* Wt, int64_t plane, void* bias, int* flag, hipStream_t st) {
  dim3 g((unsigned)((s + 31) / 32), (unsigned)((Kp + 31) / 32));
  switch (prec) {
    case BS_PREC_F64:
      prep_w_kernel<BS_PREC_F64><<<g, 256, 0, st>>>(W, d, s, Kp, (double*)Wt, plane, flag);
      prep_bias_kernel<double><<<grid_1d(s, 256), 256, 0, st>>>(b, s, (double*)bias, flag);
      break;
    case BS_PREC_F32:
      prep_w_kernel<BS_PREC_F32><<<g, 256, 0, st>>>(W, d, s, Kp, (float*)Wt, plane, flag);
      prep_bias_kernel<float><<<grid_1d(s, 256), 256, 0, st>>>(b, s, (float*)bias, flag);
      break;
    case BS_PREC_BF16:
      prep_w_kernel<BS_PREC_BF16><<<g, 256, 0, st>>>(W, d, s, Kp, (uint16_t*)Wt, plane, flag);
      prep_bias_kernel<float><<<grid_1d(s, 256), 256, 0, st>>>(b, s, (float*)bias, flag);
      break;
    default:
      prep_w_kernel<BS_PREC_BF16X3><<<g, 256, 0, st>>>(W, d, s, Kp, (uint16_t*)Wt, plane, flag);
      prep_bias_kernel<float><<<grid_1d(s, 256), 256, 0, st>>>(b, s, (float*)bias, flag);
  }
  return hipGetLastError();
}

hipError_t check_finite(const float* p, int64_t count, int* flag, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  check_finite_kernel<<<grid_1d(count, 256, 16384), 256, 0, st>>>(p, count, flag);
  return hipGetLastError();
}

namespace {

// Split-operand regeneration on wide tiles where its 16-byte row stores and
// 32-bit staging offsets allow; false where regen_kernel must run instead
// (same bits either way).
bool regen_bf16x3_wide(const void* Xp, int64_t xps, int64_t rows, const void* Wt, int64_t wps,
                       int64_t cols, const void* bias, int64_t Kp, double scale, float* Z,
                       int64_t ldz, hipStream_t st) {
  const int64_t wt = ((rows + XBM - 1) / XBM) * ((cols + XBN - 1) / XBN);
  if (ldz % 4 != 0 || reinterpret_cast<uintptr_t>(Z) % 16 != 0 || wt > 0x7fffffff ||
      Kp % (XKROW / 2) != 0 || Kp > ((int64_t)1 << 21))
    return false;
  const int64_t nwg = std::min<int64_t>(std::max(8, cu_count() / 8 * 8), (wt + 7) / 8 * 8);
  regen_bf16x3_wide_kernel<<<dim3((unsigned)nwg), XNT, 0, st>>>(
      (const uint16_t*)Xp, xps, rows, (const uint16_t*)Wt, wps, cols, (const float*)bias, Kp,
      (float)scale, Z, ldz);
  return true;
}

}  // namespace

hipError_t regen_defect(const void* Xp, int64_t xps, int64_t rows, const void* Wt, int64_t wps,
                        int64_t cols, const void* bias, int64_t Kp, double scale,
                        const uint16_t* Zt, uint16_t* Zd, int64_t ldz, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (!Zt || !Zd) return hipErrorInvalidValue;
  int64_t tiles = ((rows + BM - 1) / BM) * ((cols + BN - 1) / BN);
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  regen_kernel<BS_PREC_BF16X3, float, true><<<dim3((unsigned)tiles), NTHREADS, 0, st>>>(
      (const uint16_t*)Xp, xps, rows, (const uint16_t*)Wt, wps, cols, (const float*)bias, Kp,
      (float)scale, nullptr, ldz, Zt, Zd);
  return hipGetLastError();
}

hipError_t regen(int prec, const void* Xp, int64_t xps, int64_t rows, const void* Wt, int64_t wps,
                 int64_t cols, const void* bias, int64_t Kp, double scale, void* Z, int64_t ldz,
                 hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  int64_t tiles = ((rows + BM - 1) / BM) * ((cols + BN - 1) / BN);
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  dim3 g((unsigned)tiles);
  switch (prec) {
    case BS_PREC_F64:
      regen_kernel<BS_PREC_F64, double><<<g, NTHREADS, 0, st>>>(
          (const double*)Xp, xps, rows, (const double*)Wt, wps, cols, (const double*)bias, Kp,
          scale, (double*)Z, ldz, nullptr, nullptr);
      break;
    case BS_PREC_F32:
      regen_kernel<BS_PREC_F32, float><<<g, NTHREADS, 0, st>>>(
          (const float*)Xp, xps, rows, (const float*)Wt, wps, cols, (const float*)bias, Kp,
          (float)scale, (float*)Z, ldz, nullptr, nullptr);
      break;
    case BS_PREC_BF16: {
      // wide tiles: the 16-byte row stores of Z need ldz and the base 16-byte
      // aligned (else regen_kernel, same bits), the 32-bit buffer offsets a
      // tile of 256 rows below 2 GiB
      const int64_t wt = ((rows + WBM - 1) / WBM) * ((cols + WBN - 1) / WBN);
      if (ldz % 8 == 0 && reinterpret_cast<uintptr_t>(Z) % 16 == 0 && wt <= 0x7fffffff &&
          Kp <= ((int64_t)1 << 21)) {
        // persistent: one workgroup per CU (a multiple of the 8 XCDs)
        const int64_t nwg = std::min<int64_t>(std::max(8, cu_count() / 8 * 8), (wt + 7) / 8 * 8);
        regen_bf16_wide_kernel<<<dim3((unsigned)nwg), WNT, 0, st>>>(
            (const uint16_t*)Xp, rows, (const uint16_t*)Wt, cols, (const float*)bias, Kp,
            (float)scale, (uint16_t*)Z, ldz);
      } else {
        regen_kernel<BS_PREC_BF16, uint16_t><<<g, NTHREADS, 0, st>>>(
            (const uint16_t*)Xp, xps, rows, (const uint16_t*)Wt, wps, cols, (const float*)bias,
            Kp, (float)scale, (uint16_t*)Z, ldz, nullptr, nullptr);
      }
      break;
    }
    default:
      if (regen_bf16x3_wide(Xp, xps, rows, Wt, wps, cols, bias, Kp, scale, (float*)Z, ldz, st))
        break;
      regen_kernel<BS_PREC_BF16X3, float><<<g, NTHREADS, 0, st>>>(
          (const uint16_t*)Xp, xps, rows, (const uint16_t*)Wt, wps, cols, (const float*)bias, Kp,
          (float)scale, (float*)Z, ldz, nullptr, nullptr);
  }
  return hipGetLastError();
}

}  // namespace bs
