// Products against blocks of Z (Algorithm 1, steps 17 and 19; the paper's
// step 21 is replaced by the identity Z^T Z W' = rhs - W') and the Gram
// matrices Z_ij^T Z_ij behind the cached factors of eq. cache.
//
// Z lives in the iteration workspace, row-major.  Feature block j occupies
// the 64-aligned column range starting at coff_j; the columns between s_j and
// the next multiple of 64 are zero.  Every feature-indexed array uses this
// padded feature index, so kernels can sweep all of it without masks.
// All reductions run in a fixed order (split partials are summed by a second
// kernel), so results are bitwise repeatable.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace bs {

namespace {

template <typename T> struct V4;
template <> struct V4<double> { using type = v4d; };
template <> struct V4<float> { using type = v4f; };

// ---------------------------------------------------------------------------
// Partial transpose products, one row block per launch:
// part[sp][f][c] = sum_{r in split sp} Z[r][f] Rop[r][c].
// MFMA view: M = features, N = outputs, K = rows.  A lane loads 4 adjacent
// features of one row; instruction q of a step uses feature 4 m + q as its
// row m, so one 16-byte load feeds 4 instructions.  Each wave owns 64
// features; the 4 waves of a workgroup own 256 adjacent features and read
// the same rows of Rop.  U groups of 4 rows are loaded before they are
// consumed so that enough bytes are in flight to cover HBM latency.
// ---------------------------------------------------------------------------
template <typename ZT, int NTC, int U>
__global__ void __launch_bounds__(256)
ztr_kernel(const ZT* __restrict__ Z, int64_t ldz, int64_t rows, int64_t s,
           const typename ZAcc<ZT>::type* __restrict__ Rop, int64_t mp, int64_t split_rows,
           typename ZAcc<ZT>::type* __restrict__ part) {
  using op_t = typename ZAcc<ZT>::type;
  using accv = typename V4<op_t>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int64_t f0 = (int64_t)blockIdx.x * 256 + wave * 64;
  const int64_t sp = blockIdx.y;
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);
  const int64_t rbeg = sp * split_rows;
  const int64_t rend = min(rows, rbeg + split_rows);
  const int64_t fl = f0 + 4 * fr;  // first of this lane's 4 features (< ldz)

  accv acc[4][NTC];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < NTC; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[q][t][r] = 0;

  if (f0 < s) {
    for (int64_t rb = rbeg; rb < rend; rb += 4 * U) {
      op_t a[U][4];
      op_t bv[U][NTC];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = rb + 4 * u + fg;
        ok[u] = r < rend;
        const int64_t rl = ok[u] ? r : rend - 1;   // in-bounds row; its weight is zeroed
        load_z4<ZT>(Z + rl * ldz + fl, a[u]);
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
          const int nt = min(nc0 + t, ntiles - 1);
          bv[u][t] = Rop[rl * mp + nt * 16 + fr];
        }
      }
      // keep all U loads issued before the first use (no re-interleaving)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
          const op_t b = ok[u] ? bv[u][t] : (op_t)0;
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q][t] = mfma4(a[u][q], b, acc[q][t]);
        }
    }
  }
  // lane holds D[m = acc_row(fg, r)][n = fr]; feature = f0 + 4 m + q
#pragma unroll
  for (int t = 0; t < NTC; ++t) {
    const int nt = nc0 + t;
    if (nt >= ntiles) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t f = f0 + 4 * acc_row<op_t>(fg, r) + q;
        if (f < s) part[(sp * s + f) * mp + nt * 16 + fr] = acc[q][t][r];
      }
  }
}

// ---------------------------------------------------------------------------
// Transpose products from an FP32 Z for many output columns.  R of a 16-row
// step (NC columns) is staged once per workgroup into LDS, transposed to
// [column][16 rows] (row pitch 80 B), double-buffered, and shared by the 4
// waves; rows past the split are staged as zeros.  Lane group g takes rows
// 4 g .. 4 g + 3 of the step: four 16-byte loads give its 4 x 4 block of Z,
// one 16-byte LDS read gives the matching 4 rows of an R column, and
// instruction j of the step pairs row 4 g + j of both.  Same grid and output
// as ztr_kernel.
// ---------------------------------------------------------------------------
template <int NTC>
__global__ void __launch_bounds__(256, 2)
ztr_f32_lds_kernel(const float* __restrict__ Z, int64_t ldz, int64_t rows, int64_t s,
                   const float* __restrict__ Rop, int64_t mp, int64_t split_rows,
                   float* __restrict__ part) {
  constexpr int NC = NTC * 16, PITCH = 80;
  constexpr int SEGS = 16 * NC / 4;                // 16-byte segments of R per step
  constexpr int NSEG = (SEGS + 255) / 256;         // per thread
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][NC * PITCH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int64_t f0 = (int64_t)blockIdx.x * 256 + wave * 64;
  const int64_t sp = blockIdx.y;
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);
  const int64_t rbeg = sp * split_rows;
  const int64_t rend = min(rows, rbeg + split_rows);
  const int64_t fl = min(f0 + 4 * fr, s - 4);      // waves past s load in bounds, store nothing

  // staged segment q = tid + 256 u: row q % 16 of the step, columns
  // 4 (q / 16) .. + 3 of the workgroup's NC (clamped into R past mp)
  int srow[NSEG], scol[NSEG];
  bool sval[NSEG];
#pragma unroll
  for (int u = 0; u < NSEG; ++u) {
    const int q = min(tid + 256 * u, SEGS - 1);
    srow[u] = q % 16;
    scol[u] = 4 * (q / 16);
    sval[u] = tid + 256 * u < SEGS;
  }
  auto stage_load = [&](int64_t rb, v4f (&stg)[NSEG]) {
#pragma unroll
    for (int u = 0; u < NSEG; ++u) {
      const int64_t r = rb + srow[u];
      const int64_t col = min(nc0 * 16 + scol[u], (int)mp - 4);
      stg[u] = r < rend ? *reinterpret_cast<const v4f*>(Rop + r * mp + col)
                        : v4f{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto stage_store = [&](unsigned char* buf, const v4f (&stg)[NSEG]) {
#pragma unroll
    for (int u = 0; u < NSEG; ++u)
      if (sval[u]) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          *reinterpret_cast<float*>(buf + (scol[u] + i) * PITCH + srow[u] * 4) = stg[u][i];
      }
  };
  auto z_load = [&](int64_t rb, v4f (&a)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      a[j] = *reinterpret_cast<const v4f*>(Z + min(rb + 4 * fg + j, rows - 1) * ldz + fl);
  };

  v4f acc[4][NTC];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[q][t] = v4f{0.f, 0.f, 0.f, 0.f};

  v4f stg[NSEG], a[4], an[4];
  stage_load(rbeg, stg);
  z_load(rbeg, a);
  stage_store(lds[0], stg);
  __syncthreads();
  for (int64_t rb = rbeg; rb < rend; rb += 16) {
    const int buf = (int)(((rb - rbeg) >> 4) & 1);
    const bool more = rb + 16 < rend;
    if (more) {
      stage_load(rb + 16, stg);
      z_load(rb + 16, an);
    }
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const v4f b = *reinterpret_cast<const v4f*>(&lds[buf][(t * 16 + fr) * PITCH + 16 * fg]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q][t] = mfma4(a[j][q], b[j], acc[q][t]);
    }
    if (more) {
      stage_store(lds[buf ^ 1], stg);
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = an[j];
    }
    __syncthreads();
  }
  // lane holds D[m = acc_row(fg, r)][n = fr]; feature = f0 + 4 m + q
#pragma unroll
  for (int t = 0; t < NTC; ++t) {
    const int nt = nc0 + t;
    if (nt >= ntiles) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t f = f0 + 4 * acc_row<float>(fg, r) + q;
        if (f < s) part[(sp * s + f) * mp + nt * 16 + fr] = acc[q][t][r];
      }
  }
}

// rhs = W-bar - mu' + U + sum over splits (fixed order) + corr, per row
// block; without W-bar (null) the base is 0 and without corr nothing is added.
template <typename A>
__global__ void reduce_rhs_kernel(const A* __restrict__ part, int64_t nsplit_max, int64_t n,
                                  int R, int i0, int i1, int64_t split_rows, int64_t s, int64_t mp,
                                  const double* __restrict__ Wbar, const double* __restrict__ mup,
                                  const double* __restrict__ U, const double* __restrict__ corr,
                                  double* __restrict__ rhs) {
  const int64_t per = s * mp;
  const int64_t total = (int64_t)(i1 - i0) * per;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = i0 + (int)(e / per);
    const int64_t fc = e - (int64_t)(i - i0) * per;
    const int64_t ni = (int64_t)(i + 1) * n / R - (int64_t)i * n / R;
    const int64_t ns = (ni + split_rows - 1) / split_rows;
    const A* pp = part + (int64_t)i * nsplit_max * per + fc;
    // the loads of 8 splits go out together; the sum keeps split order
    double a = 0.0;
    int64_t sp = 0;
    for (; sp + 8 <= ns; sp += 8) {
      A v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[(sp + u) * per];
#pragma unroll
      for (int u = 0; u < 8; ++u) a += (double)v[u];
    }
    for (; sp < ns; ++sp) a += (double)pp[sp * per];
    const int64_t off = (int64_t)i * per + fc;
    double v = Wbar ? Wbar[fc] - mup[off] + U[off] + a : a;
    if (corr) v += corr[off];
    rhs[off] = v;
  }
}

// ---------------------------------------------------------------------------
// Forward product for one row block: P[r][c] = sum_f Z[r][f] W'[f][c], with
// W' stored transposed, Wt[c][f] (row stride s16).  MFMA view: M = rows,
// N = outputs, K = features.  A lane loads 4 adjacent features of its row of
// Z and the same 4 features of its column of Wt; instruction t of a step
// pairs feature 4 g + t of both.  Each wave owns 32 rows (two M tiles sharing
// every W' value); U fragment steps of 16 features are loaded before they are
// consumed.  Pad columns of Z and pad features of W' are zero.
// KS = 1: a workgroup owns 128 rows, each wave all features of its 32.
// KS = 4: the 4 waves share 32 rows and take every fourth group of 16 U
// features, so each round reads 4 x 16 U adjacent features of every row (the
// DRAM locality of the transpose product) instead of 16 U features of 128
// rows; their partial sums are added in wave order through LDS.
// ---------------------------------------------------------------------------
template <typename ZT, int NTC, int U, int KS>
__global__ void __launch_bounds__(256)
zw_kernel(const ZT* __restrict__ Z, int64_t ldz, int64_t rows, int64_t s16,
          const typename ZAcc<ZT>::type* __restrict__ Wop, int64_t mp, double* __restrict__ Pout) {
  using op_t = typename ZAcc<ZT>::type;
  using accv = typename V4<op_t>::type;
  static_assert(KS == 1 || KS == 4, "K split over 1 or 4 waves");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int64_t r0 = KS == 1 ? (int64_t)blockIdx.x * 128 + wave * 32 : (int64_t)blockIdx.x * 32;
  const int64_t fbeg = KS == 1 ? 0 : (int64_t)wave * 16 * U;
  const int nc0 = blockIdx.y * NTC;
  const int ntiles = (int)(mp / 16);
  accv acc[2][NTC];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < NTC; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[h][t][r] = 0;
  if (r0 < rows) {
    const auto* z0 = Z + min(r0 + fr, rows - 1) * ldz + 4 * fg;
    const auto* z1 = Z + min(r0 + 16 + fr, rows - 1) * ldz + 4 * fg;
    for (int64_t f0 = fbeg; f0 < s16; f0 += KS * 16 * U) {
      op_t a0[U][4], a1[U][4], b[U][NTC][4];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        load_z4<ZT>(z0 + f0 + 16 * u, a0[u]);
        load_z4<ZT>(z1 + f0 + 16 * u, a1[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const auto* wb = Wop + (int64_t)fr * s16 + f0 + 16 * u + 4 * fg;
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
          const int nt = min(nc0 + t, ntiles - 1);
          load_z4<op_t>(wb + (int64_t)nt * 16 * s16, b[u][t]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < NTC; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc[0][t] = mfma4(a0[u][q], b[u][t][q], acc[0][t]);
            acc[1][t] = mfma4(a1[u][q], b[u][t][q], acc[1][t]);
          }
    }
  }
  if constexpr (KS > 1) {  // r0 is uniform over the workgroup: every wave gets here
    __shared__ op_t red[KS - 1][2 * NTC * 4][64];
    if (wave > 0) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < NTC; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[wave - 1][(h * NTC + t) * 4 + r][lane] = acc[h][t][r];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < KS - 1; ++w)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < NTC; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[h][t][r] += red[w][(h * NTC + t) * 4 + r][lane];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const int nt = nc0 + t;
      if (nt >= ntiles) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 16 * h + acc_row<op_t>(fg, r);
        if (row < rows) Pout[row * mp + nt * 16 + fr] = (double)acc[h][t][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Forward product from an FP32 Z for many output columns.  The transposed W'
// of a 16-feature step (NC columns x 64 B) is staged once per workgroup into
// LDS (row pitch 80 B: the 16 columns a fragment read touches fall in
// distinct banks), double-buffered, and shared by the 4 waves of 32 rows, so
// W' moves from L2 once per workgroup instead of once per wave; each wave's
// next Z fragments and the next stage are loaded while the current step's
// products run.  The k-permutation and output are those of zw_kernel (KS = 1).
// One launch covers the row blocks i0 .. i0 + gridDim.y - 1 of the partition
// of n rows into R (grid row = row block, as in zw_bf16_kernel), so that a
// speech-sized block of 25000 rows does not leave most of the GPU idle.
// ---------------------------------------------------------------------------
template <int NTC>
__global__ void __launch_bounds__(256, 2)
zw_f32_lds_kernel(const float* __restrict__ Zg, int64_t ldz, int64_t n, int R, int i0,
                  int64_t s16, const float* __restrict__ Wg, int64_t wt_stride, int64_t mp,
                  double* __restrict__ Pg) {
  constexpr int NC = NTC * 16, PITCH = 80;
  constexpr int SEGS = NC * 4;                     // 16-byte segments per stage
  constexpr int NSEG = (SEGS + 255) / 256;         // per thread
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][NC * PITCH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int i = i0 + (int)blockIdx.y;
  const int64_t gi = (int64_t)i * n / R, rows = (int64_t)(i + 1) * n / R - gi;
  const float* Z = Zg + (gi - (int64_t)i0 * n / R) * ldz;
  const float* Wt = Wg + (int64_t)i * wt_stride;
  double* Pout = Pg + gi * mp;
  const int64_t r0 = (int64_t)blockIdx.x * 128 + wave * 32;
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);

  // staged segment q = tid + 256 u: column q / 4 of the workgroup's NC,
  // features 4 (q % 4) .. 4 (q % 4) + 3 of the step
  const float* gsrc[NSEG];
  int ldst[NSEG];
#pragma unroll
  for (int u = 0; u < NSEG; ++u) {
    const int q = min(tid + 256 * u, SEGS - 1);
    const int c = q / 4, part = q % 4;
    const int64_t col = min(nc0 * 16 + c, (int)mp - 1);
    gsrc[u] = Wt + col * s16 + part * 4;
    ldst[u] = tid + 256 * u < SEGS ? c * PITCH + part * 16 : -1;
  }
  // rows past the block read its last row (in bounds) and store nothing
  const float* z0 = Z + min(r0 + fr, rows - 1) * ldz + 4 * fg;
  const float* z1 = Z + min(r0 + 16 + fr, rows - 1) * ldz + 4 * fg;

  v4f acc[2][NTC];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[h][t] = v4f{0.f, 0.f, 0.f, 0.f};

  v4f stg[NSEG], a0 = *reinterpret_cast<const v4f*>(z0), a1 = *reinterpret_cast<const v4f*>(z1);
#pragma unroll
  for (int u = 0; u < NSEG; ++u) stg[u] = *reinterpret_cast<const v4f*>(gsrc[u]);
#pragma unroll
  for (int u = 0; u < NSEG; ++u)
    if (ldst[u] >= 0) *reinterpret_cast<v4f*>(&lds[0][ldst[u]]) = stg[u];
  __syncthreads();
  for (int64_t f0 = 0; f0 < s16; f0 += 16) {
    const int buf = (int)((f0 >> 4) & 1);
    const bool more = f0 + 16 < s16;
    v4f n0 = a0, n1 = a1;
    if (more) {
#pragma unroll
      for (int u = 0; u < NSEG; ++u) stg[u] = *reinterpret_cast<const v4f*>(gsrc[u] + f0 + 16);
      n0 = *reinterpret_cast<const v4f*>(z0 + f0 + 16);
      n1 = *reinterpret_cast<const v4f*>(z1 + f0 + 16);
    }
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const v4f b = *reinterpret_cast<const v4f*>(&lds[buf][(t * 16 + fr) * PITCH + 16 * fg]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[0][t] = mfma4(a0[q], b[q], acc[0][t]);
        acc[1][t] = mfma4(a1[q], b[q], acc[1][t]);
      }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < NSEG; ++u)
        if (ldst[u] >= 0) *reinterpret_cast<v4f*>(&lds[buf ^ 1][ldst[u]]) = stg[u];
      a0 = n0;
      a1 = n1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const int nt = nc0 + t;
      if (nt >= ntiles) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 16 * h + acc_row<float>(fg, r);
        if (row < rows) Pout[row * mp + nt * 16 + fr] = (double)acc[h][t][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Gram tile of one block: slot[a][b] tile = I + Z_b^T Z_b restricted to the
// 64 x 64 tile (ta, tb), ta >= tb.  The 4 waves take interleaved groups of 4
// rows and their partial sums are added in wave order through LDS.  Tiles in
// the XCD-aware super-tile order of gram_bf16_kernel (below).
// ---------------------------------------------------------------------------
template <typename ZT>
__global__ void __launch_bounds__(256)
gram_kernel(const ZT* __restrict__ Z, int64_t ldz, int64_t rows, int64_t coff,
            int64_t sj, double* __restrict__ slot, int64_t S) {
  using acc_t = typename ZAcc<ZT>::type;
  using accv = typename V4<acc_t>::type;
  __shared__ acc_t red[64 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  // slot -> super-tile (sa, sb), sa >= sb, and tile (ta, tb) inside it
  const int64_t L = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int64_t q = L / 64, u = L % 64;
  int64_t sa = (int64_t)((__builtin_sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while ((sa + 1) * (sa + 2) / 2 <= q) ++sa;
  while (sa * (sa + 1) / 2 > q) --sa;
  const int64_t sb = q - sa * (sa + 1) / 2;
  const int64_t ta = 8 * sa + u / 8, tb = 8 * sb + u % 8;
  if (tb > ta || 64 * ta >= sj) return;  // whole workgroup, before any barrier
  const int64_t fa = 64 * ta + 4 * fr, fb = 64 * tb + 4 * fr;  // block-local features

  accv acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  // Row steps of 4 rows (lane group fg takes row rb + fg); the loads of the
  // next GS steps are in flight while the current GS steps' products run
  // (FP32 Gram setup of the speech workload: 2, 4, 8 steps 0.286, 0.269,
  // 0.264 s).
  // Rows past the end and features past sj load as zero (the clamped address
  // is read and discarded).
  constexpr int GS = sizeof(acc_t) == 8 ? 4 : 8;   // FP64: 4 (registers)
  const bool fa_ok[4] = {fa < sj, fa + 1 < sj, fa + 2 < sj, fa + 3 < sj};
  const bool fb_ok[4] = {fb < sj, fb + 1 < sj, fb + 2 < sj, fb + 3 < sj};
  auto load_step = [&](int64_t rb, acc_t (&a)[4], acc_t (&b)[4]) {
    const int64_t r = rb + fg;
    const int64_t rc = r < rows ? r : rows - 1;
    load_z4<ZT>(Z + rc * ldz + coff + fa, a);
    load_z4<ZT>(Z + rc * ldz + coff + fb, b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (r >= rows || !fa_ok[q]) a[q] = 0;
      if (r >= rows || !fb_ok[q]) b[q] = 0;
    }
  };
  acc_t a[GS][4], b[GS][4];
  int64_t rb = 4 * wave;
#pragma unroll
  for (int g = 0; g < GS; ++g) load_step(rb + 16 * g, a[g], b[g]);
  for (; rb < rows; rb += 16 * GS) {
    acc_t na[GS][4], nb[GS][4];
    const bool more = rb + 16 * GS < rows;
    if (more) {
#pragma unroll
      for (int g = 0; g < GS; ++g) load_step(rb + 16 * (GS + g), na[g], nb[g]);
    }
#pragma unroll
    for (int g = 0; g < GS; ++g)
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) acc[qa][qb] = mfma4(a[g][qa], b[g][qb], acc[qa][qb]);
    if (more) {
#pragma unroll
      for (int g = 0; g < GS; ++g)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[g][q] = na[g][q];
          b[g][q] = nb[g][q];
        }
    }
  }
  // element (m = acc_row(fg, r), n = fr) of instruction (qa, qb) is
  // G[64 ta + 4 m + qa][64 tb + 4 n + qb]; local index (4 m + qa, 4 n + qb)
  for (int w = 1; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            red[(4 * acc_row<acc_t>(fg, r) + qa) * 64 + 4 * fr + qb] = acc[qa][qb][r];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[qa][qb][r] += red[(4 * acc_row<acc_t>(fg, r) + qa) * 64 + 4 * fr + qb];
    }
    __syncthreads();
  }
  if (wave == 0) {
#pragma unroll
    for (int qa = 0; qa < 4; ++qa)
#pragma unroll
      for (int qb = 0; qb < 4; ++qb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = 64 * ta + 4 * acc_row<acc_t>(fg, r) + qa;
          const int64_t gj = 64 * tb + 4 * fr + qb;
          if (gi < sj && gj < sj)
            slot[gi * S + gj] = (double)acc[qa][qb][r] + (gi == gj ? 1.0 : 0.0);
        }
  }
}

// ---------------------------------------------------------------------------
// Forward products from a BF16 Z on the 16x16x32 BF16 instruction, all row
// blocks of a group in one launch (grid.y = block):
// P[r][c] = sum_f Z[r][f] W'_i[f][c] for the rows r of block i.
// W'_i comes as BF16 head and residual planes stored transposed,
// Wt[p][c][f] (plane stride mp * s), and both planes are multiplied.
// A lane loads 8 adjacent features of one row of Z and of one column of each
// plane; a wave owns MT 16-row tiles.  KS = 1: a workgroup owns 4 MT tiles,
// each wave all features of its own.  KS = 4: the 4 waves share MT tiles and
// take every fourth group of 32 U features (4 x 32 U adjacent features of
// each row per round, as in zw_kernel), partial sums added in wave order.
// ---------------------------------------------------------------------------
template <int NTC, int MT, int U, int KS>
__global__ void __launch_bounds__(256)
zw_bf16_kernel(const uint16_t* __restrict__ Z, int64_t ldz, int64_t n, int R, int i0, int64_t s,
               const uint16_t* __restrict__ Wt, int64_t wt_stride, int64_t mp,
               double* __restrict__ Pout) {
  static_assert(KS == 1 || KS == 4, "K split over 1 or 4 waves");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int i = i0 + (int)blockIdx.y;
  const int64_t gi = (int64_t)i * n / R, ni = (int64_t)(i + 1) * n / R - gi;
  const int64_t zi = gi - (int64_t)i0 * n / R;   // first row of block i in Z
  const int64_t row0 = KS == 1 ? (int64_t)blockIdx.x * (64 * MT) + wave * (16 * MT)
                               : (int64_t)blockIdx.x * (16 * MT);
  if (row0 >= ni) return;  // with KS = 4 uniform over the workgroup
  const int64_t kbeg = KS == 1 ? 0 : (int64_t)wave * 32 * U;
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);
  const uint16_t* Wb = Wt + (int64_t)i * wt_stride;
  const int64_t pstride = mp * s;

  const uint16_t* zp[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
    zp[t] = Z + (zi + min(row0 + 16 * t + fr, ni - 1)) * ldz + 8 * fg;
  const uint16_t* wp[NTC];
#pragma unroll
  for (int t = 0; t < NTC; ++t)
    wp[t] = Wb + (int64_t)(min(nc0 + t, ntiles - 1) * 16 + fr) * s + 8 * fg;

  v4f acc[MT][NTC];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[a][t] = v4f{0.f, 0.f, 0.f, 0.f};

  for (int64_t k0 = kbeg; k0 < s; k0 += KS * 32 * U) {
    u32x4 a[U][MT], b[U][NTC][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int t = 0; t < MT; ++t)
        a[u][t] = *reinterpret_cast<const u32x4*>(zp[t] + k0 + 32 * u);
#pragma unroll
      for (int t = 0; t < NTC; ++t) {
        b[u][t][0] = *reinterpret_cast<const u32x4*>(wp[t] + k0 + 32 * u);
        b[u][t][1] = *reinterpret_cast<const u32x4*>(wp[t] + pstride + k0 + 32 * u);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < NTC; ++t)
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          acc[m][t] = mfma_bf16x8(a[u][m], b[u][t][0], acc[m][t]);
          acc[m][t] = mfma_bf16x8(a[u][m], b[u][t][1], acc[m][t]);
        }
  }
  if constexpr (KS > 1) {
    __shared__ float red[KS - 1][MT * NTC * 4][64];
    if (wave > 0) {
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTC; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[wave - 1][(m * NTC + t) * 4 + r][lane] = acc[m][t][r];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < KS - 1; ++w)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTC; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[m][t][r] += red[w][(m * NTC + t) * 4 + r][lane];
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const int nt = nc0 + t;
      if (nt >= ntiles) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 16 * m + acc_row<float>(fg, r);
        if (row < ni) Pout[(gi + row) * mp + nt * 16 + fr] = (double)acc[m][t][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Wait until at most N (0..15) of this wave's vector memory
// operations are outstanding and all of its LDS accesses have completed
// (expcnt unconstrained).  The compiler-level memory clobbers keep LDS
// accesses from moving across.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt immediate");
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0070 | N);
  asm volatile("" ::: "memory");
}
// Workgroup barrier without the memory fence of __syncthreads (which would
// wait for every outstanding load, including the prefetched stages); callers
// precede it with wait_vm, which also drains the wave's LDS accesses.
__device__ __forceinline__ void bare_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

#define BS_LDS __attribute__((address_space(3)))

// ---------------------------------------------------------------------------
// Transpose products from a BF16 Z for many output columns, fed by direct
// global-to-LDS loads.  Each 16-row step of the workgroup (Z: 16 rows x 256
// features; R: 2 planes x NC columns x 16 rows) goes into one of 4 LDS
// stages, loaded three steps ahead without passing through registers, so
// that about 55 KB per workgroup are in flight against HBM latency.  Every
// wave waits for its own loads of the step, then one barrier makes the whole
// stage visible; the barrier also orders the reads of the stage refilled
// next (the previous step's) before its refill.  A lane reads its 8-row x
// 4-feature block of Z from the stage and transposes it in registers with
// byte permutes; one 16x16x32 MFMA per output tile and feature takes
// k = 32 as the step's 16 rows against R's head plane (k < 16) and against
// its residual plane (k >= 16): lane group fg holds k = 8 fg .. 8 fg + 7,
// i.e. rows 8 (fg & 1) .. + 7 of plane fg / 2.
// Stage layouts, chosen so that fragment reads touch distinct banks with 32
// banks (8 lanes per cycle) or 64 banks (16 lanes per cycle):
// * Z row r (512 B) holds its 16-byte segment g at (g + 8 (r / 8)) mod 32;
// * R: 16-byte segment (plane p, column c, half h: rows 8h .. 8h + 7) at
//   index (p NC + c) 2 + (h ^ (((c >> 2) ^ (c >> 3)) & 1)).
// Output: part[sp][f][c] = sum over the rows r of split sp of Z[r][f] R[r][c];
// R comes as BF16 head and residual planes stored transposed, Rt[p][c][r]
// (plane stride mp * ldr, zero for 32 rows past the block's rows).  Grid:
// 256 features x splits x passes of NTC output tiles.
// ---------------------------------------------------------------------------
template <int NTC>
__global__ void __launch_bounds__(256, 2)
ztr_bf16_dma_kernel(const uint16_t* __restrict__ Z, int64_t ldz, int64_t rows, int64_t s,
                    const uint16_t* __restrict__ Rt, int64_t ldr, int64_t mp, int64_t split_rows,
                    float* __restrict__ part) {
  constexpr int NC = NTC * 16;
  constexpr int ZB = 16 * 512;                     // Z bytes of a stage
  constexpr int RB = 2 * NC * 32;                  // R bytes of a stage (NTC loads of 1 KB)
  __shared__ __attribute__((aligned(16))) unsigned char z0[ZB], z1[ZB], z2[ZB], z3[ZB];
  __shared__ __attribute__((aligned(16))) unsigned char q0[RB], q1[RB], q2[RB], q3[RB];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar branches
  const int fr = lane & 15, fg = lane >> 4;
  const int64_t fwg = (int64_t)blockIdx.x * 256;
  const int64_t f0 = fwg + wave * 64;
  const int64_t sp = blockIdx.y;
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);
  const int64_t rbeg = sp * split_rows;
  const int64_t rend = min(rows, rbeg + split_rows);
  const int64_t pstride = mp * ldr;
  const int nsteps = (int)((rend - rbeg + 15) / 16);

  // Z: load k = 2 wave + u writes stage rows 2k, 2k + 1; lane -> (row, slot)
  int64_t zrow[2], zcol[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = 2 * wave + u;
    const int pr = 2 * k + (lane >> 5), ps = lane & 31;
    const int g = (ps - 8 * (pr >> 3)) & 31;
    zrow[u] = pr;
    zcol[u] = min(fwg + 8 * g, s - 8);
  }
  // R: load k = wave + 4 u writes stage segments 64 k + lane; every wave
  // issues NRU loads per stage, those with k >= NTC repeating load NTC - 1
  // (same bytes to the same place), so that all waves count the same loads
  constexpr int NRU = (NTC + 3) / 4;
  constexpr int NLOAD = 2 + NRU;                   // loads per stage and wave
  int64_t roff[NRU];
#pragma unroll
  for (int u = 0; u < NRU; ++u) {
    const int k = min(wave + 4 * u, NTC - 1);
    const int q = 64 * k + lane;
    const int p = q / (2 * NC), c = (q >> 1) % NC;
    const int h = (q & 1) ^ (((c >> 2) ^ (c >> 3)) & 1);
    const int64_t col = min(nc0 * 16 + c, (int)mp - 1);
    roff[u] = p * pstride + col * ldr + 8 * h;
  }
  auto issue = [&](int64_t rb, unsigned char* zs, unsigned char* qs) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
      __builtin_amdgcn_global_load_lds(
          (const void*)(Z + min(rb + zrow[u], rows - 1) * ldz + zcol[u]),
          (BS_LDS void*)(zs + (2 * wave + u) * 1024), 16, 0, 0);
#pragma unroll
    for (int u = 0; u < NRU; ++u)
      __builtin_amdgcn_global_load_lds((const void*)(Rt + roff[u] + rb),
                                       (BS_LDS void*)(qs + min(wave + 4 * u, NTC - 1) * 1024),
                                       16, 0, 0);
  };

  v4f acc[4][NTC];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[q][t] = v4f{0.f, 0.f, 0.f, 0.f};

  // fragment offsets: Z rows 8 (fg & 1) + t, features wave * 64 + 4 fr .. + 3;
  // R plane fg / 2, column t * 16 + fr, half fg & 1
  const int rsub = 8 * (fg & 1);
  const int zoff = rsub * 512 + ((wave * 8 + (fr >> 1) + rsub) & 31) * 16 + 8 * (fr & 1);
  const int boff = (((fg >> 1) * NC + fr) * 2 + ((fg & 1) ^ (((fr >> 2) ^ (fr >> 3)) & 1))) * 16;
  auto compute = [&](const unsigned char* zs, const unsigned char* qs) {
    u32x2 zc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) zc[t] = *reinterpret_cast<const u32x2*>(zs + zoff + t * 512);
    u32x4 a[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      a[0][h] = __builtin_amdgcn_perm(zc[2 * h + 1].x, zc[2 * h].x, 0x05040100u);
      a[1][h] = __builtin_amdgcn_perm(zc[2 * h + 1].x, zc[2 * h].x, 0x07060302u);
      a[2][h] = __builtin_amdgcn_perm(zc[2 * h + 1].y, zc[2 * h].y, 0x05040100u);
      a[3][h] = __builtin_amdgcn_perm(zc[2 * h + 1].y, zc[2 * h].y, 0x07060302u);
    }
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const u32x4 bv = *reinterpret_cast<const u32x4*>(qs + boff + t * 512);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q][t] = mfma_bf16x8(a[q], bv, acc[q][t]);
    }
  };
  // Step c reads stage c % 4 and refills the stage of step c - 1 with step
  // c + 3.  Every step issues its refill, past the last step with the last
  // step's rows again (never read), so the loads in flight are always those
  // of the next two steps and no refill sits under a branch (which would make
  // the compiler wait for all of them before any LDS read).
  auto step = [&](int c, const unsigned char* zs, const unsigned char* qs, unsigned char* zn,
                  unsigned char* qn) {
    wait_vm<2 * NLOAD>();
    bare_barrier();
    issue(rbeg + 16 * (int64_t)min(c + 3, nsteps - 1), zn, qn);
    compute(zs, qs);
  };

  issue(rbeg, z0, q0);
  issue(rbeg + 16 * (int64_t)min(1, nsteps - 1), z1, q1);
  issue(rbeg + 16 * (int64_t)min(2, nsteps - 1), z2, q2);
  int c = 0;
  for (; c + 4 <= nsteps; c += 4) {
    step(c, z0, q0, z3, q3);
    step(c + 1, z1, q1, z0, q0);
    step(c + 2, z2, q2, z1, q1);
    step(c + 3, z3, q3, z2, q2);
  }
  if (c < nsteps) step(c, z0, q0, z3, q3);
  if (c + 1 < nsteps) step(c + 1, z1, q1, z0, q0);
  if (c + 2 < nsteps) step(c + 2, z2, q2, z1, q1);
  wait_vm<0>();   // no load into LDS may still be in flight when the workgroup ends
#pragma unroll
  for (int t = 0; t < NTC; ++t) {
    const int nt = nc0 + t;
    if (nt >= ntiles) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t f = f0 + 4 * acc_row<float>(fg, r) + q;
        if (f < s) part[(sp * s + f) * mp + nt * 16 + fr] = acc[q][t][r];
      }
  }
}

// ---------------------------------------------------------------------------
// BF16X3 transpose products for many output columns: Z in FP32, R as BF16
// head and residual planes (the layout of ztr_bf16_dma_kernel).  A lane
// splits each of its Z values into a BF16 head h = RNE(z) and residual
// l = RNE(z - h) (z - h is exact in FP32) and accumulates h x (R head +
// R residual) + l x R head in FP32: per output tile and feature one
// 16x16x32 MFMA with the head pairs the step's 16 rows with both R planes,
// and one with the residual in the lanes of the head plane (zero in those
// of the residual plane) adds l x R head.  The dropped l x R residual is
// below 2^-16 of the product.  Stages of 16 rows (16 KB of Z, 2 x NC x 32 B
// of R) fill a ring of 3 by direct global-to-LDS loads two steps ahead,
// with the waits, barrier and unconditional refills of ztr_bf16_dma_kernel;
// two workgroups fit a CU.  Z stage row r holds the workgroup's 256
// features in order (a lane's 16-byte fragment reads cover 256 contiguous
// bytes per 16 lanes).  Same grid and output as ztr_bf16_dma_kernel.
// ---------------------------------------------------------------------------
template <int NTC>
__global__ void __launch_bounds__(256, 2)
ztr_bf16x3_dma_kernel(const float* __restrict__ Z, int64_t ldz, int64_t rows, int64_t s,
                      const uint16_t* __restrict__ Rt, int64_t ldr, int64_t mp,
                      int64_t split_rows, float* __restrict__ part) {
  constexpr int NC = NTC * 16;
  constexpr int ZB = 16 * 1024;                    // Z bytes of a stage (16 loads of 1 KB)
  constexpr int RB = 2 * NC * 32;                  // R bytes of a stage (NTC loads of 1 KB)
  __shared__ __attribute__((aligned(16))) unsigned char z0[ZB], z1[ZB], z2[ZB];
  __shared__ __attribute__((aligned(16))) unsigned char q0[RB], q1[RB], q2[RB];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar branches
  const int fr = lane & 15, fg = lane >> 4;
  const int64_t fwg = (int64_t)blockIdx.x * 256;
  const int64_t f0 = fwg + wave * 64;
  const int64_t sp = blockIdx.y;
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);
  const int64_t rbeg = sp * split_rows;
  const int64_t rend = min(rows, rbeg + split_rows);
  const int64_t pstride = mp * ldr;
  const int nsteps = (int)((rend - rbeg + 15) / 16);

  // Z: load k = 4 wave + u writes stage row k, lane -> features 4 lane .. + 3
  const int64_t zcol = min(fwg + 4 * lane, s - 4);
  constexpr int NRU = (NTC + 3) / 4;
  constexpr int NLOAD = 4 + NRU;                   // loads per stage and wave
  int64_t roff[NRU];
#pragma unroll
  for (int u = 0; u < NRU; ++u) {
    const int k = min(wave + 4 * u, NTC - 1);
    const int q = 64 * k + lane;
    const int p = q / (2 * NC), c = (q >> 1) % NC;
    const int h = (q & 1) ^ (((c >> 2) ^ (c >> 3)) & 1);
    const int64_t col = min(nc0 * 16 + c, (int)mp - 1);
    roff[u] = p * pstride + col * ldr + 8 * h;
  }
  auto issue = [&](int64_t rb, unsigned char* zs, unsigned char* qs) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * wave + u;
      __builtin_amdgcn_global_load_lds((const void*)(Z + min(rb + k, rows - 1) * ldz + zcol),
                                       (BS_LDS void*)(zs + k * 1024), 16, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < NRU; ++u)
      __builtin_amdgcn_global_load_lds((const void*)(Rt + roff[u] + rb),
                                       (BS_LDS void*)(qs + min(wave + 4 * u, NTC - 1) * 1024),
                                       16, 0, 0);
  };

  v4f acc[4][NTC];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[q][t] = v4f{0.f, 0.f, 0.f, 0.f};

  // Z rows 8 (fg & 1) + t, features wave * 64 + 4 fr .. + 3; R fragment as
  // in ztr_bf16_dma_kernel; the residual enters in lane groups 0 and 1 only
  const int rsub = 8 * (fg & 1);
  const int zoff = rsub * 1024 + (wave * 64 + 4 * fr) * 4;
  const int boff = (((fg >> 1) * NC + fr) * 2 + ((fg & 1) ^ (((fr >> 2) ^ (fr >> 3)) & 1))) * 16;
  const bool lo_lane = fg < 2;
  // Two passes per step keep one set of A fragments live: the heads against
  // both R planes, then the residuals (lane groups 0, 1) against R's head.
  auto split = [&](const unsigned char* zs, bool lo, u32x4 (&a)[4]) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const v4f za = *reinterpret_cast<const v4f*>(zs + zoff + (2 * h) * 1024);
      const v4f zb = *reinterpret_cast<const v4f*>(zs + zoff + (2 * h + 1) * 1024);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t hp = pack_bf16x2(za[q], zb[q]);
        if (!lo) {
          a[q][h] = hp;
        } else {
          const float ha = __builtin_bit_cast(float, hp << 16);
          const float hb = __builtin_bit_cast(float, hp & 0xffff0000u);
          a[q][h] = lo_lane ? pack_bf16x2(za[q] - ha, zb[q] - hb) : 0u;
        }
      }
      if (h % 2 == 1) __builtin_amdgcn_sched_barrier(0);
    }
  };
  // R fragments are read one output tile ahead of their products
  auto prods = [&](const unsigned char* qs, const u32x4 (&a)[4]) {
    u32x4 bv = *reinterpret_cast<const u32x4*>(qs + boff);
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const u32x4 bn = *reinterpret_cast<const u32x4*>(qs + boff + min(t + 1, NTC - 1) * 512);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q][t] = mfma_bf16x8(a[q], bv, acc[q][t]);
      __builtin_amdgcn_sched_barrier(0);
      bv = bn;
    }
  };
  // (scheduling barriers keep the passes, and the steps, from overlapping in
  // registers)
  auto compute = [&](const unsigned char* zs, const unsigned char* qs) {
    u32x4 a[4];
    __builtin_amdgcn_sched_barrier(0);
    split(zs, false, a);
    prods(qs, a);
    __builtin_amdgcn_sched_barrier(0);
    split(zs, true, a);
    prods(qs, a);
    __builtin_amdgcn_sched_barrier(0);
  };
  // step c reads stage c % 3 and refills the stage of step c - 1 with step c + 2
  auto step = [&](int c, const unsigned char* zs, const unsigned char* qs, unsigned char* zn,
                  unsigned char* qn) {
    wait_vm<NLOAD>();
    bare_barrier();
    issue(rbeg + 16 * (int64_t)min(c + 2, nsteps - 1), zn, qn);
    compute(zs, qs);
  };

  issue(rbeg, z0, q0);
  issue(rbeg + 16 * (int64_t)min(1, nsteps - 1), z1, q1);
  int c = 0;
  for (; c + 3 <= nsteps; c += 3) {
    step(c, z0, q0, z2, q2);
    step(c + 1, z1, q1, z0, q0);
    step(c + 2, z2, q2, z1, q1);
  }
  if (c < nsteps) step(c, z0, q0, z2, q2);
  if (c + 1 < nsteps) step(c + 1, z1, q1, z0, q0);
  wait_vm<0>();   // no load into LDS may still be in flight when the workgroup ends
#pragma unroll
  for (int t = 0; t < NTC; ++t) {
    const int nt = nc0 + t;
    if (nt >= ntiles) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t f = f0 + 4 * acc_row<float>(fg, r) + q;
        if (f < s) part[(sp * s + f) * mp + nt * 16 + fr] = acc[q][t][r];
      }
  }
}

// ---------------------------------------------------------------------------
// BF16 Gram for large blocks: 128 x 128 output tiles (features fa0, fb0 of
// the lower triangle), one 64 x 64 quadrant per wave, every wave over all
// rows.  Each step of 32 rows stages the rows' 128 + 128 features (16 KB)
// in LDS once for the 4 waves, double-buffered (next step loaded from
// global while this step's products run), so a row segment moves from L2 once
// per 128 x 128 tile instead of once per wave and 64 x 64 tile.  Staged rows
// have a pitch of 272 bytes: the two 16-lane halves of a fragment read (rows
// 8 apart) fall in disjoint banks, and a 16-lane staging store writes one
// row's 256 contiguous bytes.  Fragments are read and transposed exactly as in
// gram_bf16_kernel.  Tiles in super-tiles of 4 x 4 tiles, XCD-aware.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
gram_bf16_wide_kernel(const uint16_t* __restrict__ Z, int64_t ldz, int64_t rows, int64_t coff,
                      int64_t sj, double* __restrict__ slot, int64_t S) {
  constexpr int PITCH = 272, MAT = 32 * PITCH, BUF = 2 * MAT;
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * BUF];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int wa = wave >> 1, wb = wave & 1;
  const int64_t L = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int64_t q = L / 16, u = L % 16;
  int64_t sa = (int64_t)((__builtin_sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while ((sa + 1) * (sa + 2) / 2 <= q) ++sa;
  while (sa * (sa + 1) / 2 > q) --sa;
  const int64_t sb = q - sa * (sa + 1) / 2;
  const int64_t ta = 4 * sa + u / 4, tb = 4 * sb + u % 4;
  if (tb > ta || 128 * ta >= sj) return;  // whole workgroup, before any barrier
  const int64_t fa0 = 128 * ta, fb0 = 128 * tb;

  // staging: segment v = tid + 256 k (k < 4) is matrix v / 512 (A, B), row
  // (v % 512) / 16 of the step, 16-byte segment v % 16 (8 features)
  int64_t gofs[4];
  int lofs[4];
  uint4 keepm[4];
  bool live[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int v = tid + 256 * k, mat = v / 512, row = (v % 512) / 16, seg = v % 16;
    const int64_t f = (mat ? fb0 : fa0) + 8 * seg;
    live[k] = f < sj;
    gofs[k] = (int64_t)row * ldz + coff + (live[k] ? f : 0);
    lofs[k] = mat * MAT + row * PITCH + 16 * seg;
    unsigned m[4];
#pragma unroll
    for (int h = 0; h < 4; ++h)
      m[h] = (f + 2 * h < sj ? 0x0000ffffu : 0u) | (f + 2 * h + 1 < sj ? 0xffff0000u : 0u);
    keepm[k] = uint4{m[0], m[1], m[2], m[3]};
  }
  auto fetch = [&](int64_t r0, uint4* stg) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int row = ((tid + 256 * k) % 512) / 16;
      uint4 v = uint4{0u, 0u, 0u, 0u};
      if (live[k] && r0 + row < rows)
        v = *reinterpret_cast<const uint4*>(Z + r0 * ldz + gofs[k]);
      stg[k] = uint4{v.x & keepm[k].x, v.y & keepm[k].y, v.z & keepm[k].z, v.w & keepm[k].w};
    }
  };
  auto stage = [&](int buf, const uint4* stg) {
#pragma unroll
    for (int k = 0; k < 4; ++k) *reinterpret_cast<uint4*>(&lds[buf * BUF + lofs[k]]) = stg[k];
  };

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  uint4 stg[4];
  fetch(0, stg);
  stage(0, stg);
  __syncthreads();
  const int aofs = (8 * fg) * PITCH + 128 * wa + 8 * fr;
  const int bofs = MAT + (8 * fg) * PITCH + 128 * wb + 8 * fr;
  for (int64_t r0 = 0; r0 < rows; r0 += 32) {
    const int buf = (int)((r0 >> 5) & 1);
    const bool more = r0 + 32 < rows;
    if (more) fetch(r0 + 32, stg);
    uint2 za[8], zb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      za[i] = *reinterpret_cast<const uint2*>(&lds[buf * BUF + aofs + i * PITCH]);
      zb[i] = *reinterpret_cast<const uint2*>(&lds[buf * BUF + bofs + i * PITCH]);
    }
    u32x4 a[4], b[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      a[0][h] = __builtin_amdgcn_perm(za[2 * h + 1].x, za[2 * h].x, 0x05040100u);
      a[1][h] = __builtin_amdgcn_perm(za[2 * h + 1].x, za[2 * h].x, 0x07060302u);
      a[2][h] = __builtin_amdgcn_perm(za[2 * h + 1].y, za[2 * h].y, 0x05040100u);
      a[3][h] = __builtin_amdgcn_perm(za[2 * h + 1].y, za[2 * h].y, 0x07060302u);
      b[0][h] = __builtin_amdgcn_perm(zb[2 * h + 1].x, zb[2 * h].x, 0x05040100u);
      b[1][h] = __builtin_amdgcn_perm(zb[2 * h + 1].x, zb[2 * h].x, 0x07060302u);
      b[2][h] = __builtin_amdgcn_perm(zb[2 * h + 1].y, zb[2 * h].y, 0x05040100u);
      b[3][h] = __builtin_amdgcn_perm(zb[2 * h + 1].y, zb[2 * h].y, 0x07060302u);
    }
#pragma unroll
    for (int qa = 0; qa < 4; ++qa)
#pragma unroll
      for (int qb = 0; qb < 4; ++qb) acc[qa][qb] = mfma_bf16x8(a[qa], b[qb], acc[qa][qb]);
    if (more) stage(buf ^ 1, stg);
    __syncthreads();
  }
  // element (m = acc_row(fg, r), n = fr) of instruction (qa, qb) is
  // G[fa0 + 64 wa + 4 m + qa][fb0 + 64 wb + 4 n + qb]
#pragma unroll
  for (int qa = 0; qa < 4; ++qa)
#pragma unroll
    for (int qb = 0; qb < 4; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = fa0 + 64 * wa + 4 * acc_row<float>(fg, r) + qa;
        const int64_t gj = fb0 + 64 * wb + 4 * fr + qb;
        if (gi < sj && gj < sj)
          slot[gi * S + gj] = (double)acc[qa][qb][r] + (gi == gj ? 1.0 : 0.0);
      }
}

// ---------------------------------------------------------------------------
// Forward products from a BF16 Z for many output columns: the W' planes of a
// 32-feature stage (2 x NC columns x 64 B) are loaded once per workgroup into
// LDS (row pitch 80 B: the 16 columns a fragment read touches fall in
// distinct banks) and shared by its 4 waves of 64 rows, so W' moves from L2
// 1.25 times per byte of Z instead of 10 times.  The next stage's W' and
// each wave's next Z fragments are loaded while the current stage's products
// run.  Same grid and output as zw_bf16_kernel.
// ---------------------------------------------------------------------------
template <int NTC>
__global__ void __launch_bounds__(256, 2)
zw_bf16_lds_kernel(const uint16_t* __restrict__ Z, int64_t ldz, int64_t n, int R, int i0,
                   int nblk, int64_t s, const uint16_t* __restrict__ Wt, int64_t wt_stride, int64_t mp,
                   double* __restrict__ Pout) {
  constexpr int MT = 4, NC = NTC * 16, PITCH = 80;
  constexpr int SEGS = 2 * NC * 4;                 // 16-byte segments per stage
  constexpr int NSEG = (SEGS + 255) / 256;         // per thread
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][2 * NC * PITCH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  // x runs over (row block, row tile) pairs, row block major; each XCD takes
  // a contiguous range of them, so the workgroups sharing an XCD's L2 mostly
  // read the same row block's W'
  const int tiles = (int)(gridDim.x / nblk);
  const int t = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int i = i0 + t / tiles;
  const int64_t gi = (int64_t)i * n / R, ni = (int64_t)(i + 1) * n / R - gi;
  const int64_t zi = gi - (int64_t)i0 * n / R;
  const int64_t row0 = (int64_t)(t % tiles) * (64 * MT) + wave * (16 * MT);
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);
  const uint16_t* Wb = Wt + (int64_t)i * wt_stride;
  const int64_t pstride = mp * s;

  // staged segment q = tid + 256 u: plane q / (4 NC), column (q / 4) % NC, part q % 4
  const uint16_t* gsrc[NSEG];
  int ldst[NSEG];
#pragma unroll
  for (int u = 0; u < NSEG; ++u) {
    const int q = min(tid + 256 * u, SEGS - 1);
    const int p = q / (4 * NC), c = (q / 4) % NC, part = q % 4;
    const int64_t col = min(nc0 * 16 + c, (int)mp - 1);
    gsrc[u] = Wb + p * pstride + col * s + part * 8;
    ldst[u] = tid + 256 * u < SEGS ? (p * NC + c) * PITCH + part * 16 : -1;
  }
  const uint16_t* zp[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
    zp[t] = Z + (zi + min(row0 + 16 * t + fr, ni - 1)) * ldz + 8 * fg;

  v4f acc[MT][NTC];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[a][t] = v4f{0.f, 0.f, 0.f, 0.f};

  u32x4 stg[NSEG], a_cur[MT], a_nxt[MT];
#pragma unroll
  for (int u = 0; u < NSEG; ++u) stg[u] = *reinterpret_cast<const u32x4*>(gsrc[u]);
#pragma unroll
  for (int t = 0; t < MT; ++t) a_cur[t] = *reinterpret_cast<const u32x4*>(zp[t]);
#pragma unroll
  for (int u = 0; u < NSEG; ++u)
    if (ldst[u] >= 0) *reinterpret_cast<u32x4*>(&lds[0][ldst[u]]) = stg[u];
  __syncthreads();
  for (int64_t k0 = 0; k0 < s; k0 += 32) {
    const int buf = (int)((k0 >> 5) & 1);
    const bool more = k0 + 32 < s;
    if (more) {
#pragma unroll
      for (int u = 0; u < NSEG; ++u) stg[u] = *reinterpret_cast<const u32x4*>(gsrc[u] + k0 + 32);
#pragma unroll
      for (int t = 0; t < MT; ++t) a_nxt[t] = *reinterpret_cast<const u32x4*>(zp[t] + k0 + 32);
    }
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const u32x4 bh = *reinterpret_cast<const u32x4*>(&lds[buf][(t * 16 + fr) * PITCH + 16 * fg]);
      const u32x4 bl =
          *reinterpret_cast<const u32x4*>(&lds[buf][(NC + t * 16 + fr) * PITCH + 16 * fg]);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        acc[m][t] = mfma_bf16x8(a_cur[m], bh, acc[m][t]);
        acc[m][t] = mfma_bf16x8(a_cur[m], bl, acc[m][t]);
      }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < NSEG; ++u)
        if (ldst[u] >= 0) *reinterpret_cast<u32x4*>(&lds[buf ^ 1][ldst[u]]) = stg[u];
#pragma unroll
      for (int t = 0; t < MT; ++t) a_cur[t] = a_nxt[t];
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const int nt = nc0 + t;
      if (nt >= ntiles) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 16 * m + acc_row<float>(fg, r);
        if (row < ni) Pout[(gi + row) * mp + nt * 16 + fr] = (double)acc[m][t][r];
      }
    }
}

// ---------------------------------------------------------------------------
// BF16X3 forward products for many output columns: Z in FP32, W' as BF16
// head and residual planes (the layout of zw_bf16_lds_kernel, staged the same
// way).  A lane splits its 8 Z values of a 32-feature stage into heads
// h = RNE(z) and residuals l = RNE(z - h) and accumulates h x W' head +
// h x W' residual + l x W' head (three 16x16x32 MFMAs per row tile and output
// tile; the dropped l x W' residual is below 2^-16 of the product).  The
// next stage's Z (two 16-byte loads per row tile) and W' are loaded while
// the current stage's products run.  Same grid and output as zw_bf16_kernel.
// ---------------------------------------------------------------------------
template <int NTC>
__global__ void __launch_bounds__(256, 2)
zw_bf16x3_lds_kernel(const float* __restrict__ Z, int64_t ldz, int64_t n, int R, int i0,
                     int64_t s, const uint16_t* __restrict__ Wt, int64_t wt_stride, int64_t mp,
                     double* __restrict__ Pout) {
  constexpr int MT = 4, NC = NTC * 16, PITCH = 80;
  constexpr int SEGS = 2 * NC * 4;                 // 16-byte segments per stage
  constexpr int NSEG = (SEGS + 255) / 256;         // per thread
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][2 * NC * PITCH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int i = i0 + (int)blockIdx.y;
  const int64_t gi = (int64_t)i * n / R, ni = (int64_t)(i + 1) * n / R - gi;
  const int64_t zi = gi - (int64_t)i0 * n / R;
  const int64_t row0 = (int64_t)blockIdx.x * (64 * MT) + wave * (16 * MT);
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);
  const uint16_t* Wb = Wt + (int64_t)i * wt_stride;
  const int64_t pstride = mp * s;

  // staged segment q = tid + 256 u: plane q / (4 NC), column (q / 4) % NC, part q % 4
  const uint16_t* gsrc[NSEG];
  int ldst[NSEG];
#pragma unroll
  for (int u = 0; u < NSEG; ++u) {
    const int q = min(tid + 256 * u, SEGS - 1);
    const int p = q / (4 * NC), c = (q / 4) % NC, part = q % 4;
    const int64_t col = min(nc0 * 16 + c, (int)mp - 1);
    gsrc[u] = Wb + p * pstride + col * s + part * 8;
    ldst[u] = tid + 256 * u < SEGS ? (p * NC + c) * PITCH + part * 16 : -1;
  }
  const float* zp[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
    zp[t] = Z + (zi + min(row0 + 16 * t + fr, ni - 1)) * ldz + 8 * fg;

  v4f acc[MT][NTC];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[a][t] = v4f{0.f, 0.f, 0.f, 0.f};

  // heads and residuals of a lane's 8 consecutive features, packed in pairs
  // (low half = the even feature)
  auto split = [&](const v4f& z0, const v4f& z1, u32x4& h, u32x4& l) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float a = j < 2 ? z0[2 * j] : z1[2 * j - 4];
      const float b = j < 2 ? z0[2 * j + 1] : z1[2 * j - 3];
      const uint32_t hp = pack_bf16x2(a, b);
      h[j] = hp;
      l[j] = pack_bf16x2(a - __builtin_bit_cast(float, hp << 16),
                         b - __builtin_bit_cast(float, hp & 0xffff0000u));
    }
  };

  u32x4 stg[NSEG], ah[MT], al[MT];
  v4f zn[MT][2];
#pragma unroll
  for (int u = 0; u < NSEG; ++u) stg[u] = *reinterpret_cast<const u32x4*>(gsrc[u]);
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    zn[t][0] = *reinterpret_cast<const v4f*>(zp[t]);
    zn[t][1] = *reinterpret_cast<const v4f*>(zp[t] + 4);
  }
#pragma unroll
  for (int u = 0; u < NSEG; ++u)
    if (ldst[u] >= 0) *reinterpret_cast<u32x4*>(&lds[0][ldst[u]]) = stg[u];
#pragma unroll
  for (int t = 0; t < MT; ++t) split(zn[t][0], zn[t][1], ah[t], al[t]);
  __syncthreads();
  for (int64_t k0 = 0; k0 < s; k0 += 32) {
    const int buf = (int)((k0 >> 5) & 1);
    const bool more = k0 + 32 < s;
    if (more) {
#pragma unroll
      for (int u = 0; u < NSEG; ++u) stg[u] = *reinterpret_cast<const u32x4*>(gsrc[u] + k0 + 32);
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        zn[t][0] = *reinterpret_cast<const v4f*>(zp[t] + k0 + 32);
        zn[t][1] = *reinterpret_cast<const v4f*>(zp[t] + k0 + 36);
      }
    }
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const u32x4 bh = *reinterpret_cast<const u32x4*>(&lds[buf][(t * 16 + fr) * PITCH + 16 * fg]);
      const u32x4 bl =
          *reinterpret_cast<const u32x4*>(&lds[buf][(NC + t * 16 + fr) * PITCH + 16 * fg]);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        acc[m][t] = mfma_bf16x8(ah[m], bh, acc[m][t]);
        acc[m][t] = mfma_bf16x8(ah[m], bl, acc[m][t]);
        acc[m][t] = mfma_bf16x8(al[m], bh, acc[m][t]);
      }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < NSEG; ++u)
        if (ldst[u] >= 0) *reinterpret_cast<u32x4*>(&lds[buf ^ 1][ldst[u]]) = stg[u];
#pragma unroll
      for (int t = 0; t < MT; ++t) split(zn[t][0], zn[t][1], ah[t], al[t]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const int nt = nc0 + t;
      if (nt >= ntiles) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 16 * m + acc_row<float>(fg, r);
        if (row < ni) Pout[(gi + row) * mp + nt * 16 + fr] = (double)acc[m][t][r];
      }
    }
}

// Loads batched per wave before their MFMAs: more when each load feeds few
// instructions (few output tiles), fewer when the tile count is large.
template <int NTC> constexpr int ztr_unroll() { return NTC <= 2 ? 8 : 4; }
template <int NTC> constexpr int zw_unroll() { return NTC <= 2 ? 4 : (NTC <= 6 ? 2 : 1); }

template <typename ZT, int NTC>
static void launch_ztr(const void* Z, int64_t ldz, int64_t rows, int64_t s, const void* Rop,
                       int64_t mp, int64_t split_rows, void* part, hipStream_t st) {
  using op_t = typename ZAcc<ZT>::type;
  const int ntiles = (int)(mp / 16);
  const int64_t nsplit = (rows + split_rows - 1) / split_rows;
  dim3 g((unsigned)((s + 255) / 256), (unsigned)nsplit, (unsigned)((ntiles + NTC - 1) / NTC));
  ztr_kernel<ZT, NTC, ztr_unroll<NTC>()><<<g, 256, 0, st>>>(
      (const ZT*)Z, ldz, rows, s, (const op_t*)Rop, mp, split_rows, (op_t*)part);
}

template <int NTC>
static void launch_ztr_lds(const void* Z, int64_t ldz, int64_t rows, int64_t s, const void* Rop,
                           int64_t mp, int64_t split_rows, void* part, hipStream_t st) {
  const int ntiles = (int)(mp / 16);
  const int64_t nsplit = (rows + split_rows - 1) / split_rows;
  dim3 g((unsigned)((s + 255) / 256), (unsigned)nsplit, (unsigned)((ntiles + NTC - 1) / NTC));
  ztr_f32_lds_kernel<NTC><<<g, 256, 0, st>>>((const float*)Z, ldz, rows, s, (const float*)Rop,
                                             mp, split_rows, (float*)part);
}

// One pass over Z covers all output tiles when there are at most 10 (FP32
// operands; more than two share R through LDS) or 2 (FP64); beyond that,
// passes of 8 (FP32) or 2 (FP64) tiles.
// The FP64 branch is resolved at compile time so its wide variants are never
// instantiated.
template <typename ZT>
static void ztr_dispatch(const void* Z, int64_t ldz, int64_t rows, int64_t s, const void* Rop,
                         int64_t mp, int64_t split_rows, void* part, hipStream_t st) {
  const int nt = (int)(mp / 16);
  if constexpr (sizeof(ZT) == 8) {
    if (nt == 1) launch_ztr<ZT, 1>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
    else launch_ztr<ZT, 2>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
  } else {
    if (nt == 1) launch_ztr<ZT, 1>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
    else if (nt == 2) launch_ztr<ZT, 2>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
    else if (nt <= 4) launch_ztr_lds<4>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
    else if (nt <= 6) launch_ztr_lds<6>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
    else if (nt <= 8) launch_ztr_lds<8>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
    else if (nt <= 10) launch_ztr_lds<10>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
    else launch_ztr_lds<8>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
  }
}

template <int NTC>
static void launch_ztr_bf16_dma(const void* Z, int64_t ldz, int64_t rows, int64_t s,
                                const void* Rt, int64_t ldr, int64_t mp, int64_t split_rows,
                                void* part, hipStream_t st) {
  const int ntiles = (int)(mp / 16);
  const int64_t nsplit = (rows + split_rows - 1) / split_rows;
  dim3 g((unsigned)((s + 255) / 256), (unsigned)nsplit, (unsigned)((ntiles + NTC - 1) / NTC));
  ztr_bf16_dma_kernel<NTC><<<g, 256, 0, st>>>((const uint16_t*)Z, ldz, rows, s,
                                              (const uint16_t*)Rt, ldr, mp, split_rows,
                                              (float*)part);
}

template <int NTC>
static void launch_ztr_bf16x3_dma(const void* Z, int64_t ldz, int64_t rows, int64_t s,
                                  const void* Rt, int64_t ldr, int64_t mp, int64_t split_rows,
                                  void* part, hipStream_t st) {
  const int ntiles = (int)(mp / 16);
  const int64_t nsplit = (rows + split_rows - 1) / split_rows;
  dim3 g((unsigned)((s + 255) / 256), (unsigned)nsplit, (unsigned)((ntiles + NTC - 1) / NTC));
  ztr_bf16x3_dma_kernel<NTC><<<g, 256, 0, st>>>((const float*)Z, ldz, rows, s,
                                                (const uint16_t*)Rt, ldr, mp, split_rows,
                                                (float*)part);
}

// BF16X3 with more than two output tiles (bf16_planes): one pass over Z for up
// to 8 tiles (10 do not fit the registers), two passes of 5 for 9 or 10,
// passes of 8 beyond.
static void ztr_bf16x3_dispatch(const void* Z, int64_t ldz, int64_t rows, int64_t s,
                                const void* Rt, int64_t ldr, int64_t mp, int64_t split_rows,
                                void* part, hipStream_t st) {
  const int nt = (int)(mp / 16);
  if (nt <= 4) launch_ztr_bf16x3_dma<4>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else if (nt <= 6) launch_ztr_bf16x3_dma<6>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else if (nt <= 8) launch_ztr_bf16x3_dma<8>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else if (nt <= 10) launch_ztr_bf16x3_dma<5>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else launch_ztr_bf16x3_dma<8>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
}

// All tile counts go through the LDS stages (passes of 8 beyond 10 tiles).
static void ztr_bf16_dispatch(const void* Z, int64_t ldz, int64_t rows, int64_t s, const void* Rt,
                              int64_t ldr, int64_t mp, int64_t split_rows, void* part,
                              hipStream_t st) {
  const int nt = (int)(mp / 16);
  if (nt == 1) launch_ztr_bf16_dma<1>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else if (nt == 2) launch_ztr_bf16_dma<2>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else if (nt <= 4) launch_ztr_bf16_dma<4>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else if (nt <= 6) launch_ztr_bf16_dma<6>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else if (nt <= 8) launch_ztr_bf16_dma<8>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else if (nt <= 10) launch_ztr_bf16_dma<10>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
  else launch_ztr_bf16_dma<8>(Z, ldz, rows, s, Rt, ldr, mp, split_rows, part, st);
}


// ---------------------------------------------------------------------------
// Gram tile of one block of a BF16 Z on BF16 MFMA: the lower 64 x 64 tile
// (ta, tb) of I + Z_b^T Z_b.  Products of BF16 values are exact in FP32, so
// this is the same arithmetic as widening Z to FP32 (FP32 accumulation), at
// the rate of the 16x16x32 BF16 instruction.  A step is 32 rows: lane
// (f = lane % 16, g = lane / 16) loads rows 8 g .. 8 g + 7 of features
// 4 f .. 4 f + 3 of both feature tiles (8-byte loads, 128 contiguous bytes of
// a row per 16 lanes) and transposes them in registers with byte permutes
// into four 8-row fragments per tile, one for each feature 4 f + q.  The k of
// an instruction is then the 32 rows of the step and instruction (qa, qb)
// accumulates G[4 m + qa][4 n + qb], m, n < 16.  The 4 waves take interleaved
// steps; their partial sums are added in wave order through LDS.
// Tile order: the grid has 64 slots per super-tile of 8 x 8 tiles of the
// lower triangle (slots above the diagonal or past the edge exit at once),
// and each XCD takes a contiguous range of slots, so the workgroups resident
// on an XCD read the 16 feature strips of about one super-tile and its L2
// serves their re-reads (tiles in plain triangle order spread the strips
// over all XCDs and re-read Z from beyond L2 about 30 times).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
gram_bf16_kernel(const uint16_t* __restrict__ Z, int64_t ldz, int64_t rows, int64_t coff,
                 int64_t sj, double* __restrict__ slot, int64_t S) {
  __shared__ float red[64 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int64_t L = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int64_t q = L / 64, u = L % 64;
  int64_t sa = (int64_t)((__builtin_sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while ((sa + 1) * (sa + 2) / 2 <= q) ++sa;
  while (sa * (sa + 1) / 2 > q) --sa;
  const int64_t sb = q - sa * (sa + 1) / 2;
  const int64_t ta = 8 * sa + u / 8, tb = 8 * sb + u % 8;
  if (tb > ta || 64 * ta >= sj) return;  // whole workgroup, before any barrier
  const int64_t fa = 64 * ta + 4 * fr, fb = 64 * tb + 4 * fr;  // block-local features
  // features at or past s_j read as zero: mask of the 4 packed halves
  auto keep = [&](int64_t f0) -> uint2 {
    uint2 k;
    k.x = (f0 < sj ? 0x0000ffffu : 0u) | (f0 + 1 < sj ? 0xffff0000u : 0u);
    k.y = (f0 + 2 < sj ? 0x0000ffffu : 0u) | (f0 + 3 < sj ? 0xffff0000u : 0u);
    return k;
  };
  const uint2 ka = keep(fa), kb = keep(fb);
  const bool la = fa < sj, lb = fb < sj;
  const uint16_t* za_base = Z + coff + fa;
  const uint16_t* zb_base = Z + coff + fb;

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  // a step is 32 rows of this wave (rows r0 + 8 fg + 0..7 per lane); the
  // next step's rows are loaded while this step's products run
  auto load_step = [&](int64_t r0, uint2* za, uint2* zb) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t r = r0 + 8 * fg + i;
      uint2 a = {0u, 0u}, b = {0u, 0u};
      if (r < rows) {
        if (la) a = *reinterpret_cast<const uint2*>(za_base + r * ldz);
        if (lb) b = *reinterpret_cast<const uint2*>(zb_base + r * ldz);
      }
      za[i] = uint2{a.x & ka.x, a.y & ka.y};
      zb[i] = uint2{b.x & kb.x, b.y & kb.y};
    }
  };
  uint2 za[8], zb[8];
  load_step(32 * wave, za, zb);
  for (int64_t r0 = 32 * wave; r0 < rows; r0 += 128) {
    uint2 na[8], nb[8];
    load_step(r0 + 128, na, nb);   // rows past the end load as zero
    u32x4 a[4], b[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      a[0][h] = __builtin_amdgcn_perm(za[2 * h + 1].x, za[2 * h].x, 0x05040100u);
      a[1][h] = __builtin_amdgcn_perm(za[2 * h + 1].x, za[2 * h].x, 0x07060302u);
      a[2][h] = __builtin_amdgcn_perm(za[2 * h + 1].y, za[2 * h].y, 0x05040100u);
      a[3][h] = __builtin_amdgcn_perm(za[2 * h + 1].y, za[2 * h].y, 0x07060302u);
      b[0][h] = __builtin_amdgcn_perm(zb[2 * h + 1].x, zb[2 * h].x, 0x05040100u);
      b[1][h] = __builtin_amdgcn_perm(zb[2 * h + 1].x, zb[2 * h].x, 0x07060302u);
      b[2][h] = __builtin_amdgcn_perm(zb[2 * h + 1].y, zb[2 * h].y, 0x05040100u);
      b[3][h] = __builtin_amdgcn_perm(zb[2 * h + 1].y, zb[2 * h].y, 0x07060302u);
    }
#pragma unroll
    for (int qa = 0; qa < 4; ++qa)
#pragma unroll
      for (int qb = 0; qb < 4; ++qb) acc[qa][qb] = mfma_bf16x8(a[qa], b[qb], acc[qa][qb]);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      za[i] = na[i];
      zb[i] = nb[i];
    }
  }
  // element (m = acc_row(fg, r), n = fr) of instruction (qa, qb) is
  // G[64 ta + 4 m + qa][64 tb + 4 n + qb]; local index (4 m + qa, 4 n + qb)
  for (int w = 1; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            red[(4 * acc_row<float>(fg, r) + qa) * 64 + 4 * fr + qb] = acc[qa][qb][r];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[qa][qb][r] += red[(4 * acc_row<float>(fg, r) + qa) * 64 + 4 * fr + qb];
    }
    __syncthreads();
  }
  if (wave == 0) {
#pragma unroll
    for (int qa = 0; qa < 4; ++qa)
#pragma unroll
      for (int qb = 0; qb < 4; ++qb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = 64 * ta + 4 * acc_row<float>(fg, r) + qa;
          const int64_t gj = 64 * tb + 4 * fr + qb;
          if (gi < sj && gj < sj)
            slot[gi * S + gj] = (double)acc[qa][qb][r] + (gi == gj ? 1.0 : 0.0);
        }
  }
}

}  // namespace

hipError_t ztr_partial(int prec, const void* Z, int64_t ldz, int64_t rows, int64_t s,
                       const void* Rop, int64_t ldr, int64_t mp, int64_t split_rows, void* part,
                       hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  if (prec == BS_PREC_F64) ztr_dispatch<double>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
  else if (prec == BS_PREC_BF16) {
    if (split_rows % 32 != 0) return hipErrorInvalidValue;
    ztr_bf16_dispatch(Z, ldz, rows, s, Rop, ldr, mp, split_rows, part, st);
  } else if (bf16_planes(prec, mp)) {
    if (split_rows % 32 != 0) return hipErrorInvalidValue;
    ztr_bf16x3_dispatch(Z, ldz, rows, s, Rop, ldr, mp, split_rows, part, st);
  } else ztr_dispatch<float>(Z, ldz, rows, s, Rop, mp, split_rows, part, st);
  return hipGetLastError();
}

hipError_t reduce_rhs(int prec, const void* part, int64_t nsplit_max, int64_t n, int R, int i0,
                      int i1, int64_t split_rows, int64_t s, int64_t mp, const double* Wbar,
                      const double* mup, const double* U, const double* corr, double* rhs,
                      hipStream_t st) {
  int64_t total = (int64_t)(i1 - i0) * s * mp;
  if (total <= 0) return hipSuccess;
  unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  if (prec == BS_PREC_F64)
    reduce_rhs_kernel<double><<<g, 256, 0, st>>>((const double*)part, nsplit_max, n, R, i0, i1,
                                                 split_rows, s, mp, Wbar, mup, U, corr, rhs);
  else
    reduce_rhs_kernel<float><<<g, 256, 0, st>>>((const float*)part, nsplit_max, n, R, i0, i1,
                                                split_rows, s, mp, Wbar, mup, U, corr, rhs);
  return hipGetLastError();
}

namespace {

template <typename ZT, int NTC>
static void launch_zw(const void* Z, int64_t ldz, int64_t rows, int64_t s16, const void* Wop,
                      int64_t mp, double* Pout, hipStream_t st) {
  using op_t = typename ZAcc<ZT>::type;
  const int ntiles = (int)(mp / 16);
  // up to two output tiles: HBM-bound, K split over the waves for locality
  constexpr int KS = NTC <= 2 ? 4 : 1;
  const int64_t wrows = KS == 1 ? 128 : 32;
  dim3 g((unsigned)((rows + wrows - 1) / wrows), (unsigned)((ntiles + NTC - 1) / NTC));
  zw_kernel<ZT, NTC, zw_unroll<NTC>(), KS><<<g, 256, 0, st>>>((const ZT*)Z, ldz, rows, s16,
                                                             (const op_t*)Wop, mp, Pout);
}

template <int NTC>
static void launch_zw_lds(const void* Z, int64_t ldz, int64_t n, int R, int i0, int nblk,
                          int64_t nmax, int64_t s16, const void* Wop, int64_t wop_stride,
                          int64_t mp, double* Pout, hipStream_t st) {
  const int ntiles = (int)(mp / 16);
  dim3 g((unsigned)((nmax + 127) / 128), (unsigned)nblk, (unsigned)((ntiles + NTC - 1) / NTC));
  zw_f32_lds_kernel<NTC><<<g, 256, 0, st>>>((const float*)Z, ldz, n, R, i0, s16,
                                            (const float*)Wop, wop_stride, mp, Pout);
}

// FP32 operands with more than two output tiles: all row blocks in one
// launch, one pass over Z for up to 10 tiles, passes of 8 beyond.
static void zw_f32_lds_dispatch(const void* Z, int64_t ldz, int64_t n, int R, int i0, int nblk,
                                int64_t nmax, int64_t s16, const void* Wop, int64_t wop_stride,
                                int64_t mp, double* Pout, hipStream_t st) {
  const int nt = (int)(mp / 16);
#define BS_ZWF(NTC) \
  launch_zw_lds<NTC>(Z, ldz, n, R, i0, nblk, nmax, s16, Wop, wop_stride, mp, Pout, st)
  if (nt <= 4) BS_ZWF(4);
  else if (nt <= 6) BS_ZWF(6);
  else if (nt <= 8) BS_ZWF(8);
  else if (nt <= 10) BS_ZWF(10);
  else BS_ZWF(8);
#undef BS_ZWF
}

template <typename ZT>
static void zw_dispatch(const void* Z, int64_t ldz, int64_t rows, int64_t s16, const void* Wop,
                        int64_t mp, double* Pout, hipStream_t st) {
  const int nt = (int)(mp / 16);
  if constexpr (sizeof(ZT) == 8) {
    if (nt == 1) launch_zw<ZT, 1>(Z, ldz, rows, s16, Wop, mp, Pout, st);
    else launch_zw<ZT, 2>(Z, ldz, rows, s16, Wop, mp, Pout, st);
  } else {  // FP32 operands, one or two tiles (more: zw_f32_lds_dispatch)
    if (nt == 1) launch_zw<ZT, 1>(Z, ldz, rows, s16, Wop, mp, Pout, st);
    else launch_zw<ZT, 2>(Z, ldz, rows, s16, Wop, mp, Pout, st);
  }
}

template <int NTC, int MT, int U>
static void launch_zw_bf16(const void* Z, int64_t ldz, int64_t n, int R, int i0, int nblk,
                           int64_t nmax, int64_t s, const void* Wt, int64_t wt_stride, int64_t mp,
                           double* Pout, hipStream_t st) {
  const int ntiles = (int)(mp / 16);
  constexpr int KS = NTC <= 2 ? 4 : 1;  // K split over the waves for DRAM locality
  const int64_t wrows = (KS == 1 ? 64 : 16) * MT;
  dim3 g((unsigned)((nmax + wrows - 1) / wrows), (unsigned)nblk,
         (unsigned)((ntiles + NTC - 1) / NTC));
  zw_bf16_kernel<NTC, MT, U, KS><<<g, 256, 0, st>>>((const uint16_t*)Z, ldz, n, R, i0, s,
                                                    (const uint16_t*)Wt, wt_stride, mp, Pout);
}

template <int NTC>
static void launch_zw_bf16_lds(const void* Z, int64_t ldz, int64_t n, int R, int i0, int nblk,
                               int64_t nmax, int64_t s, const void* Wt, int64_t wt_stride,
                               int64_t mp, double* Pout, hipStream_t st) {
  const int ntiles = (int)(mp / 16);
  dim3 g((unsigned)((nmax + 255) / 256 * nblk), 1u, (unsigned)((ntiles + NTC - 1) / NTC));
  zw_bf16_lds_kernel<NTC><<<g, 256, 0, st>>>((const uint16_t*)Z, ldz, n, R, i0, nblk, s,
                                             (const uint16_t*)Wt, wt_stride, mp, Pout);
}

template <int NTC>
static void launch_zw_bf16x3_lds(const void* Z, int64_t ldz, int64_t n, int R, int i0, int nblk,
                                 int64_t nmax, int64_t s, const void* Wt, int64_t wt_stride,
                                 int64_t mp, double* Pout, hipStream_t st) {
  const int ntiles = (int)(mp / 16);
  dim3 g((unsigned)((nmax + 255) / 256), (unsigned)nblk, (unsigned)((ntiles + NTC - 1) / NTC));
  zw_bf16x3_lds_kernel<NTC><<<g, 256, 0, st>>>((const float*)Z, ldz, n, R, i0, s,
                                               (const uint16_t*)Wt, wt_stride, mp, Pout);
}

// One pass over Z for up to 10 output tiles (passes of 8 beyond): up to two
// tiles read W' directly, more share it through LDS.
static void zw_bf16_dispatch(const void* Z, int64_t ldz, int64_t n, int R, int i0, int nblk,
                             int64_t nmax, int64_t s, const void* Wt, int64_t wt_stride,
                             int64_t mp, double* Pout, hipStream_t st) {
  const int nt = (int)(mp / 16);
#define BS_ZWB(NTC, MT, U) \
  launch_zw_bf16<NTC, MT, U>(Z, ldz, n, R, i0, nblk, nmax, s, Wt, wt_stride, mp, Pout, st)
#define BS_ZWL(NTC) \
  launch_zw_bf16_lds<NTC>(Z, ldz, n, R, i0, nblk, nmax, s, Wt, wt_stride, mp, Pout, st)
  if (nt == 1) BS_ZWB(1, 4, 2);
  else if (nt == 2) BS_ZWB(2, 4, 2);
  else if (nt <= 4) BS_ZWL(4);
  else if (nt <= 6) BS_ZWL(6);
  else if (nt <= 8) BS_ZWL(8);
  else if (nt <= 10) BS_ZWL(10);
  else BS_ZWL(8);
#undef BS_ZWB
#undef BS_ZWL
}

}  // namespace

hipError_t zw(int prec, const void* Z, int64_t ldz, int64_t n, int R, int i0, int i1, int64_t s,
              const void* Wop, int64_t wop_stride, int64_t mp, double* Pout, hipStream_t st) {
  if (i1 <= i0 || n <= 0) return hipSuccess;
  if (s % 64 != 0) return hipErrorInvalidValue;
  if (bf16_planes(prec, mp)) {
    int64_t nmax = 0;
    for (int i = i0; i < i1; ++i)
      nmax = std::max<int64_t>(nmax, (int64_t)(i + 1) * n / R - (int64_t)i * n / R);
    if (prec == BS_PREC_BF16)
      zw_bf16_dispatch(Z, ldz, n, R, i0, i1 - i0, nmax, s, Wop, wop_stride, mp, Pout, st);
    else  // BF16X3: passes of up to 5 output tiles (the registers of 3 products)
      launch_zw_bf16x3_lds<5>(Z, ldz, n, R, i0, i1 - i0, nmax, s, Wop, wop_stride, mp, Pout, st);
    return hipGetLastError();
  }
  if (prec != BS_PREC_F64 && mp > 32) {
    int64_t nmax = 0;
    for (int i = i0; i < i1; ++i)
      nmax = std::max<int64_t>(nmax, (int64_t)(i + 1) * n / R - (int64_t)i * n / R);
    zw_f32_lds_dispatch(Z, ldz, n, R, i0, i1 - i0, nmax, s, Wop, wop_stride, mp, Pout, st);
    return hipGetLastError();
  }
  const int64_t r0 = (int64_t)i0 * n / R;
  const size_t eb = prec == BS_PREC_F64 ? 8 : 4;       // operand element bytes
  const size_t zb = prec == BS_PREC_F64 ? 8 : 4;       // stored Z element bytes
  for (int i = i0; i < i1; ++i) {
    const int64_t gi = (int64_t)i * n / R, rows = (int64_t)(i + 1) * n / R - gi;
    if (rows <= 0) continue;
    const void* Zi = (const char*)Z + (size_t)(gi - r0) * ldz * zb;
    const void* Wi = (const char*)Wop + (size_t)i * wop_stride * eb;
    if (prec == BS_PREC_F64) zw_dispatch<double>(Zi, ldz, rows, s, Wi, mp, Pout + gi * mp, st);
    else zw_dispatch<float>(Zi, ldz, rows, s, Wi, mp, Pout + gi * mp, st);
  }
  return hipGetLastError();
}

hipError_t gram(int prec, const void* Z, int64_t ldz, int64_t rows, int64_t coff, int64_t sj,
                double* slot, int64_t S, hipStream_t st) {
  // 64 workgroup slots per super-tile of 8 x 8 tiles of the lower triangle
  const int64_t T = (sj + 63) / 64, ST = (T + 7) / 8;
  const dim3 g((unsigned)(ST * (ST + 1) / 2 * 64));
  if (prec == BS_PREC_F64)
    gram_kernel<double><<<g, 256, 0, st>>>((const double*)Z, ldz, rows, coff, sj, slot, S);
  else if (prec == BS_PREC_BF16 && T >= 64 && ldz % 8 == 0 && coff % 8 == 0 &&
           reinterpret_cast<uintptr_t>(Z) % 16 == 0) {
    // large blocks (s_j > 4032): 128 x 128 tiles, 16 slots per super-tile
    // of 4 x 4 tiles; smaller ones keep 64 x 64 tiles with the rows split
    // over the waves, which fills the chip with more workgroups
    const int64_t T2 = (sj + 127) / 128, ST2 = (T2 + 3) / 4;
    gram_bf16_wide_kernel<<<dim3((unsigned)(ST2 * (ST2 + 1) / 2 * 16)), 256, 0, st>>>(
        (const uint16_t*)Z, ldz, rows, coff, sj, slot, S);
  } else if (prec == BS_PREC_BF16 && ldz % 4 == 0 && coff % 4 == 0 &&
             reinterpret_cast<uintptr_t>(Z) % 8 == 0)
    gram_bf16_kernel<<<g, 256, 0, st>>>((const uint16_t*)Z, ldz, rows, coff, sj, slot, S);
  else if (prec == BS_PREC_BF16)
    gram_kernel<uint16_t><<<g, 256, 0, st>>>((const uint16_t*)Z, ldz, rows, coff, sj, slot, S);
  else
    gram_kernel<float><<<g, 256, 0, st>>>((const float*)Z, ldz, rows, coff, sj, slot, S);
  return hipGetLastError();
}

}  // namespace bs
