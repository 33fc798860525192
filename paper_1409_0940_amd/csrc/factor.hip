// FP64 factor cache of eq. cache and the graph-projection solve of eq. gpWij.
//
// The paper caches either Q_ij = (Z_ij^T Z_ij + I)^{-1} or its Cholesky
// factors.  Here the explicit inverse is cached: the per-iteration solve
// W'_ij = Q_ij rhs_ij becomes one batched FP64 product with no sequential
// triangular sweeps, and its cost (2 s_j^2 m flops, s_j^2 doubles streamed)
// is the same as two triangular solves.  Setup, per matrix A = I + G:
//   1. blocked Cholesky A = L L^T (64 x 64 tiles; trailing updates applied
//      per panel of 4 tile columns),
//   2. X = L^{-1} by recursive doubling over tile blocks
//      (X_CA = -X_CC L_CA X_AA for sibling blocks A, C),
//   3. Q = X^T X, written as a full symmetric matrix.
// Every 64 x 64 x 64 tile product runs on the FP64 16x16x4 MFMA.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace bs {

namespace {

constexpr int NB = 64;
constexpr int LDP = NB + 1;  // LDS row pitch (doubles)

typedef double tile_t[NB][LDP];

// Load a 64 x 64 tile (row-major, leading dimension ld) into LDS, optionally
// transposed.  256 threads.
__device__ __forceinline__ void load_tile(tile_t& dst, const double* __restrict__ src, int64_t ld,
                                          bool transpose) {
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    int r = e >> 6, c = e & 63;
    double v = src[r * ld + c];
    if (transpose)
      dst[c][r] = v;
    else
      dst[r][c] = v;
  }
}

// The same load split in two, so that the global loads of the next tile
// product can be issued before the current one's MFMAs: thread t holds
// elements (t / 64 + 4 i, t % 64), i < 16, in registers.
__device__ __forceinline__ void fetch_tile(double (&r)[16], const double* __restrict__ src,
                                           int64_t ld) {
  const int row = threadIdx.x >> 6, c = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 16; ++i) r[i] = src[(int64_t)(row + 4 * i) * ld + c];
}
__device__ __forceinline__ void put_tile(tile_t& dst, const double (&r)[16], bool transpose) {
  const int row = threadIdx.x >> 6, c = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (transpose)
      dst[c][row + 4 * i] = r[i];
    else
      dst[row + 4 * i][c] = r[i];
  }
}

// acc += A B^T over k < 64, A and B in LDS as [row][k].  Wave w owns the
// 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 MFMA tiles.
__device__ __forceinline__ void tile_mma_nt(v4d (&acc)[2][2], const tile_t& A, const tile_t& B) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int fr = lane & 15, fg = lane >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < NB; k0 += 4) {
    double a0 = A[wm * 32 + fr][k0 + fg];
    double a1 = A[wm * 32 + 16 + fr][k0 + fg];
    double b0 = B[wn * 32 + fr][k0 + fg];
    double b1 = B[wn * 32 + 16 + fr][k0 + fg];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__device__ __forceinline__ void zero_acc(v4d (&acc)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
}

// Visit the elements of the accumulator: f(row, col, value) in tile coords.
template <typename F>
__device__ __forceinline__ void for_acc(const v4d (&acc)[2][2], F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int fr = lane & 15, fg = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        f(wm * 32 + i * 16 + acc_row<double>(fg, r), wn * 32 + j * 16 + fr, acc[i][j][r]);
}

// ---------------------------------------------------------------------------
// Diagonal tile kb: unblocked Cholesky in LDS, then the inverse of the
// triangular factor.  One workgroup per matrix.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
potrf_diag_kernel(double* __restrict__ slots, int64_t S, int kb, double* __restrict__ dinv,
                  int* __restrict__ flag) {
  __shared__ tile_t L;
  __shared__ tile_t Li;
  double* A = slots + (int64_t)blockIdx.x * S * S + (int64_t)kb * NB * S + (int64_t)kb * NB;
  const int tid = threadIdx.x;
  load_tile(L, A, S, false);
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    if (tid == 0) {
      double dj = L[j][j];
      if (!(dj > 0.0)) {
        atomicOr(flag, 2);
        dj = 1.0;
      }
      L[j][j] = __builtin_sqrt(dj);
    }
    __syncthreads();
    const double inv = 1.0 / L[j][j];
    for (int i = j + 1 + tid; i < NB; i += 256) L[i][j] *= inv;
    __syncthreads();
    // trailing update of the lower triangle: L[i][k] -= L[i][j] L[k][j], j < k <= i;
    // thread (tid / 64, tid % 64) takes column k = tid % 64 of every fourth row
    {
      const int k = tid & 63;
      if (k > j) {
        const double lkj = L[k][j];
        for (int i = k + (tid >> 6); i < NB; i += 4) L[i][k] -= L[i][j] * lkj;
      }
    }
    __syncthreads();
  }
  // Li = L^{-1}, one column per thread of wave 0 (forward substitution), the
  // column in registers: the loops are unrolled over all rows, so that no
  // product waits for a value the same lane has just written to LDS.  Terms
  // k < c multiply a zero entry and leave the +0 sum at +0, so the sums and
  // the bits are those of the substitution that starts at k = c.
  if (tid < NB) {
    const int c = tid;
    double li[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) acc += L[i][k] * li[k];
      const double diag = L[i][i];
      li[i] = i < c ? 0.0 : (i == c ? 1.0 / diag : -acc / diag);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) Li[i][c] = li[i];
  }
  __syncthreads();
  double* D = dinv + (int64_t)blockIdx.x * S * NB + (int64_t)kb * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    int r = e >> 6, c = e & 63;
    A[r * S + c] = (c <= r) ? L[r][c] : 0.0;
    D[e] = Li[r][c];
  }
}

// Panel: L[ib][kb] = A[ib][kb] Linv_kk^T for ib > kb.
__global__ void __launch_bounds__(256)
trsm_kernel(double* __restrict__ slots, int64_t S, int kb, const double* __restrict__ dinv) {
  __shared__ tile_t At;
  __shared__ tile_t Bt;
  const int ib = kb + 1 + blockIdx.x;
  double* base = slots + (int64_t)blockIdx.y * S * S;
  double* T = base + (int64_t)ib * NB * S + (int64_t)kb * NB;
  load_tile(At, T, S, false);
  load_tile(Bt, dinv + (int64_t)blockIdx.y * S * NB + (int64_t)kb * NB * NB, NB, false);
  __syncthreads();
  v4d acc[2][2];
  zero_acc(acc);
  tile_mma_nt(acc, At, Bt);
  for_acc(acc, [&](int r, int c, double v) { T[r * S + c] = v; });
}

// Trailing updates in panels of PW tile columns (left-looking inside the
// panel, right-looking across panels): after column kb of the panel
// [K, K + PW) is factored, only the panel's later columns take its update
// (syrk_panel_kernel); the columns past the panel take the updates of all
// PW columns at once (syrk_multi_kernel), so each of their tiles is read
// and written once per panel instead of once per column.
constexpr int PW = 4;

// A[ib][jb] -= L[ib][kb] L[jb][kb]^T for kb < jb < jend, jb <= ib < nblk;
// grid (rows below kb, panel columns after kb, matrices).
__global__ void __launch_bounds__(256)
syrk_panel_kernel(double* __restrict__ slots, int64_t S, int kb, int jend) {
  __shared__ tile_t At;
  __shared__ tile_t Bt;
  const int64_t ib = kb + 1 + blockIdx.x, jb = kb + 1 + blockIdx.y;
  if (ib < jb || jb >= jend) return;  // whole workgroup
  double* base = slots + (int64_t)blockIdx.z * S * S;
  load_tile(At, base + ib * NB * S + (int64_t)kb * NB, S, false);
  load_tile(Bt, base + jb * NB * S + (int64_t)kb * NB, S, false);
  __syncthreads();
  v4d acc[2][2];
  zero_acc(acc);
  tile_mma_nt(acc, At, Bt);
  double* T = base + ib * NB * S + jb * NB;
  for_acc(acc, [&](int r, int c, double v) { T[r * S + c] -= v; });
}

// A[ib][jb] -= sum_{k = K}^{K + nk - 1} L[ib][k] L[jb][k]^T for
// K + nk <= jb <= ib; grid (triangle of the trailing tiles, matrices).
__global__ void __launch_bounds__(256)
syrk_multi_kernel(double* __restrict__ slots, int64_t S, int K, int nk) {
  __shared__ tile_t At;
  __shared__ tile_t Bt;
  const int64_t t = blockIdx.x;
  int64_t a = (int64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  const int64_t b = t - a * (a + 1) / 2;
  const int64_t ib = K + nk + a, jb = K + nk + b;
  double* base = slots + (int64_t)blockIdx.y * S * S;
  v4d acc[2][2];
  zero_acc(acc);
  double ra[16], rb[16];
  fetch_tile(ra, base + ib * NB * S + (int64_t)K * NB, S);
  fetch_tile(rb, base + jb * NB * S + (int64_t)K * NB, S);
  for (int k = K; k < K + nk; ++k) {
    put_tile(At, ra, false);
    put_tile(Bt, rb, false);
    __syncthreads();
    if (k + 1 < K + nk) {
      fetch_tile(ra, base + ib * NB * S + (int64_t)(k + 1) * NB, S);
      fetch_tile(rb, base + jb * NB * S + (int64_t)(k + 1) * NB, S);
    }
    tile_mma_nt(acc, At, Bt);
    __syncthreads();
  }
  double* T = base + ib * NB * S + jb * NB;
  for_acc(acc, [&](int r, int c, double v) { T[r * S + c] -= v; });
}

// X = L^{-1} by recursive doubling over the T = S / 64 tile rows.  The
// diagonal tiles X_ii = Linv_ii come from the factorization.  At level b
// (b = 1, 2, 4, ...) the tile range [2 p b, 2 p b + 2 b) splits into A, its
// first b tiles, and C, the rest; with X_AA and X_CC complete,
//   X_CA = -X_CC L_CA X_AA,
// the off-diagonal block of the inverse of [[L_AA, 0], [L_CA, L_CC]].  Each
// level is two batched tile-product launches: Y = L_CA X_AA, written into the
// upper triangle of `work` (tile (A0 + a, C0 + c) holds Y's tile (c, a); the
// upper triangle of X is never read), then X_CA = -X_CC Y.  The chain of
// dependent tile products is about 2 T, against T^2 / 2 for block forward
// substitution row by row.
__global__ void __launch_bounds__(256)
trinv_diag_kernel(const double* __restrict__ dinv, int64_t S, double* __restrict__ work) {
  const int i = blockIdx.x;
  const double* D = dinv + (int64_t)blockIdx.y * S * NB + (int64_t)i * NB * NB;
  double* out = work + (int64_t)blockIdx.y * S * S + (int64_t)i * NB * S + (int64_t)i * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) out[(e >> 6) * S + (e & 63)] = D[e];
}

// Output tile (c, a) of pair p at level b; false if past the last tile row.
__device__ __forceinline__ bool trinv_tile(int b, int nblk, int64_t& A0, int64_t& C0, int& c,
                                           int& a) {
  const int t = blockIdx.x;
  const int p = t / (b * b), rem = t - p * b * b;
  c = rem / b;
  a = rem - c * b;
  A0 = (int64_t)2 * p * b;
  C0 = A0 + b;
  return C0 + c < nblk;
}

// Y(c, a) = sum_{j = a}^{b-1} L(C0 + c, A0 + j) X(A0 + j, A0 + a)  (X_AA lower).
__global__ void __launch_bounds__(256)
trinv_y_kernel(const double* __restrict__ slots, int64_t S, int b, double* __restrict__ work) {
  __shared__ tile_t At;
  __shared__ tile_t Bt;
  int64_t A0, C0;
  int c, a;
  if (!trinv_tile(b, (int)(S / NB), A0, C0, c, a)) return;
  const double* Lb = slots + (int64_t)blockIdx.y * S * S;
  double* Xb = work + (int64_t)blockIdx.y * S * S;
  v4d acc[2][2];
  zero_acc(acc);
  double ra[16], rb[16];
  fetch_tile(ra, Lb + (C0 + c) * NB * S + (A0 + a) * NB, S);
  fetch_tile(rb, Xb + (A0 + a) * NB * S + (A0 + a) * NB, S);
  for (int j = a; j < b; ++j) {
    put_tile(At, ra, false);
    put_tile(Bt, rb, true);
    __syncthreads();
    if (j + 1 < b) {
      fetch_tile(ra, Lb + (C0 + c) * NB * S + (A0 + j + 1) * NB, S);
      fetch_tile(rb, Xb + (A0 + j + 1) * NB * S + (A0 + a) * NB, S);
    }
    tile_mma_nt(acc, At, Bt);
    __syncthreads();
  }
  double* out = Xb + (A0 + a) * NB * S + (C0 + c) * NB;
  for_acc(acc, [&](int r, int cc, double v) { out[r * S + cc] = v; });
}

// X(C0 + c, A0 + a) = -sum_{j = 0}^{c} X(C0 + c, C0 + j) Y(j, a)  (X_CC lower).
__global__ void __launch_bounds__(256)
trinv_x_kernel(int64_t S, int b, double* __restrict__ work) {
  __shared__ tile_t At;
  __shared__ tile_t Bt;
  int64_t A0, C0;
  int c, a;
  if (!trinv_tile(b, (int)(S / NB), A0, C0, c, a)) return;
  double* Xb = work + (int64_t)blockIdx.y * S * S;
  v4d acc[2][2];
  zero_acc(acc);
  double ra[16], rb[16];
  fetch_tile(ra, Xb + (C0 + c) * NB * S + C0 * NB, S);
  fetch_tile(rb, Xb + (A0 + a) * NB * S + C0 * NB, S);
  for (int j = 0; j <= c; ++j) {
    put_tile(At, ra, false);
    put_tile(Bt, rb, true);
    __syncthreads();
    if (j + 1 <= c) {
      fetch_tile(ra, Xb + (C0 + c) * NB * S + (C0 + j + 1) * NB, S);
      fetch_tile(rb, Xb + (A0 + a) * NB * S + (C0 + j + 1) * NB, S);
    }
    tile_mma_nt(acc, At, Bt);
    __syncthreads();
  }
  double* out = Xb + (C0 + c) * NB * S + (A0 + a) * NB;
  for_acc(acc, [&](int r, int cc, double v) { out[r * S + cc] = -v; });
}

// Q_ab = sum_{c >= a} X_ca^T X_cb for a >= b; Q_ba = Q_ab^T.
__global__ void __launch_bounds__(256)
xtx_kernel(const double* __restrict__ work, int64_t S, double* __restrict__ slots) {
  __shared__ tile_t At;
  __shared__ tile_t Bt;
  const int64_t t = blockIdx.x;
  int64_t a = (int64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  const int64_t b = t - a * (a + 1) / 2;
  const int64_t nblk = S / NB;
  const double* Xb = work + (int64_t)blockIdx.y * S * S;
  double* Qb = slots + (int64_t)blockIdx.y * S * S;
  v4d acc[2][2];
  zero_acc(acc);
  double ra[16], rb[16];
  fetch_tile(ra, Xb + a * NB * S + a * NB, S);
  fetch_tile(rb, Xb + a * NB * S + b * NB, S);
  for (int64_t c = a; c < nblk; ++c) {
    put_tile(At, ra, true);
    put_tile(Bt, rb, true);
    __syncthreads();
    if (c + 1 < nblk) {
      fetch_tile(ra, Xb + (c + 1) * NB * S + a * NB, S);
      fetch_tile(rb, Xb + (c + 1) * NB * S + b * NB, S);
    }
    tile_mma_nt(acc, At, Bt);
    __syncthreads();
  }
  // On a diagonal tile only the lower half is written (and mirrored), so each
  // element has exactly one writer.
  for_acc(acc, [&](int r, int cc, double v) {
    if (a != b || r >= cc) {
      Qb[(a * NB + r) * S + b * NB + cc] = v;
      Qb[(b * NB + cc) * S + a * NB + r] = v;
    }
  });
}

// Identity in the pad rows / columns [sj, S) of each slot.
__global__ void identity_pad_kernel(double* __restrict__ slot, int64_t S, int64_t sj) {
  const int64_t total = S * S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e / S, c = e - r * S;
    if (r >= sj || c >= sj) slot[e] = (r == c) ? 1.0 : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Projection solve for one or two output tiles (mp <= 32), where the product
// streams Q (s_j^2 doubles a block) for very little arithmetic: a workgroup
// owns 16 rows of W'_b and its 4 waves split the k-steps (wave w takes steps
// w, w + 4, ...), so a block of s_j rows has s_j / 16 workgroups in flight
// instead of s_j / 64.  Each wave issues the Q and rhs loads of U steps before
// their MFMAs, and the 4 partial sums are added in wave order through LDS.
// Lane (fr, fg) loads 4 adjacent doubles of row row0 + fr of Q, and the 4
// matching rhs rows make the B fragment: one FP64 MFMA per step and tile.
// OUT is the type of the operand copy of W' for the forward products:
// double or float in W''s own layout, or uint16_t for BF16 head and residual
// planes stored transposed, [i][plane][mp][spad].
// ---------------------------------------------------------------------------
template <typename OUT, int NT>
__global__ void __launch_bounds__(256)
solve_ks_kernel(const double* __restrict__ Q, int64_t S, int C, int b0,
                const int64_t* __restrict__ coff, const int64_t* __restrict__ sjs, int64_t spad,
                int64_t mp, const double* __restrict__ rhs, double* __restrict__ Wp,
                double* __restrict__ U, OUT* __restrict__ Wop) {
  constexpr int KS = 4, UN = 4;
  __shared__ double red[KS - 1][NT][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int b = b0 + (int)blockIdx.y;
  const int i = b / C, j = b - i * C;
  const int64_t sj = sjs[j];
  const int64_t row0 = (int64_t)blockIdx.x * 16;
  if (row0 >= sj) return;  // whole workgroup: no barrier is skipped by part of it
  const int ntiles = (int)(mp / 16);
  const double* Qb = Q + (int64_t)b * S * S;
  const int64_t base = ((int64_t)i * spad + coff[j]) * mp;
  const double* rb = rhs + base;
  const int64_t nk = (sj + 15) / 16;  // 16-value k-steps; Q pad columns are zero off the diagonal
  const double* qrow = Qb + (row0 + fr) * S + 4 * fg;
  v4d acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[t][r] = 0.0;
  for (int64_t ks = wave; ks < nk; ks += KS * UN) {
    Frag<BS_PREC_F64> a[UN];
    Frag<BS_PREC_F64> bb[UN][NT];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int64_t k = ks + (int64_t)u * KS;
      if (k < nk) {
        const int64_t k0 = 16 * k;
        a[u] = load_frag<BS_PREC_F64>(qrow + k0);
        const double* rk = rb + (k0 + 4 * fg) * mp + fr;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) bb[u][t].v[q] = t < ntiles ? rk[q * mp + t * 16] : 0.0;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[u].v[q] = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) bb[u][t].v[q] = 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) mfma_step(acc[t], a[u], bb[u][t]);
  }
  if (wave > 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave - 1][t][r][lane] = acc[t][r];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < KS - 1; ++w)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[t][r] += red[w][t][r][lane];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t >= ntiles) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + acc_row<double>(fg, r);
      if (row < sj) {
        const int64_t o = base + row * mp + t * 16 + fr;
        const double w = acc[t][r];
        Wp[o] = w;
        U[o] = rhs[o] - w;
        if constexpr (sizeof(OUT) == 2) {
          uint16_t hi, lo;
          split_bf16(w, hi, lo);
          const int64_t tcol = ((int64_t)i * 2 * mp + t * 16 + fr) * spad + coff[j] + row;
          Wop[tcol] = hi;
          Wop[tcol + mp * spad] = lo;
        } else {  // [i][mp][spad], like the BF16 planes
          Wop[((int64_t)i * mp + t * 16 + fr) * spad + coff[j] + row] = (OUT)w;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Projection solve for many output columns (ntiles > 2): one pass over Q for
// all column tiles.  A workgroup owns 128 rows of W'_b (each wave two 16-row
// tiles) and every column; per 16-value k-step the rows k0 .. k0 + 15 of
// rhs_b (16 x mp doubles) are staged once in LDS, double-buffered, and read by
// all 4 waves, so rhs moves from L2 once per 128 rows instead of once per 16.
// A lane loads 4 adjacent doubles of a row of Q, which feed instructions
// q = 0..3 with the matching rhs rows (the k-permutation of solve_ks_kernel).
// ---------------------------------------------------------------------------
template <typename OUT, int NTC>
__global__ void __launch_bounds__(256, 2)
solve_wide_kernel(const double* __restrict__ Q, int64_t S, int C, int b0,
                  const int64_t* __restrict__ coff, const int64_t* __restrict__ sjs, int64_t spad,
                  int64_t mp, const double* __restrict__ rhs, double* __restrict__ Wp,
                  double* __restrict__ U, OUT* __restrict__ Wop) {
  constexpr int NC = NTC * 16;
  constexpr int PITCH = NC + 4;  // doubles per staged row: rows 4 apart 32 banks apart
  constexpr int NSEG = NTC / 2;                    // 16-byte segments per thread per stage
  static_assert(NTC % 2 == 0, "a stage is 8 NC segments, NTC / 2 per thread");
  __shared__ __attribute__((aligned(16))) double stage[2][16 * PITCH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int b = b0 + (int)blockIdx.y;
  const int i = b / C, j = b - i * C;
  const int64_t sj = sjs[j];
  if ((int64_t)blockIdx.x * 128 >= sj) return;  // uniform over the workgroup
  const int64_t row0 = (int64_t)blockIdx.x * 128 + wave * 32;
  const int nc0 = blockIdx.z * NTC;
  const int ntiles = (int)(mp / 16);
  const double* Qb = Q + (int64_t)b * S * S;
  const int64_t base = ((int64_t)i * spad + coff[j]) * mp;
  const double* rb = rhs + base;
  const int64_t k16 = (sj + 15) / 16 * 16;          // Q pad columns are zero off the diagonal
  // rows past sj read row sj - 1 of Q (in bounds) and store nothing
  const double* qrow0 = Qb + min(row0 + fr, sj - 1) * S + 4 * fg;
  const double* qrow1 = Qb + min(row0 + 16 + fr, sj - 1) * S + 4 * fg;

  // staged segment q = tid + 256 u: rhs row q / (NC / 2) of the step, columns
  // 2 (q % (NC / 2)) + 0..1 of the workgroup's NC (clamped into rhs past mp;
  // those staged values feed accumulators that are never stored)
  int soff[NSEG], goff[NSEG];
#pragma unroll
  for (int u = 0; u < NSEG; ++u) {
    const int q = tid + 256 * u;
    const int r = q / (NC / 2), c2 = 2 * (q % (NC / 2));
    goff[u] = r * (int)mp + min(nc0 * 16 + c2, (int)mp - 2);
    soff[u] = r * PITCH + c2;
  }

  v4d acc[2][NTC];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int t = 0; t < NTC; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][t][r] = 0.0;

  typedef double d2 __attribute__((ext_vector_type(2)));
  d2 stg[NSEG];
#pragma unroll
  for (int u = 0; u < NSEG; ++u) stg[u] = *reinterpret_cast<const d2*>(rb + goff[u]);
#pragma unroll
  for (int u = 0; u < NSEG; ++u) *reinterpret_cast<d2*>(&stage[0][soff[u]]) = stg[u];
  __syncthreads();
  for (int64_t k0 = 0; k0 < k16; k0 += 16) {
    const int buf = (int)((k0 >> 4) & 1);
    const bool more = k0 + 16 < k16;
    if (more) {
#pragma unroll
      for (int u = 0; u < NSEG; ++u)
        stg[u] = *reinterpret_cast<const d2*>(rb + (k0 + 16) * mp + goff[u]);
    }
    const Frag<BS_PREC_F64> a0 = load_frag<BS_PREC_F64>(qrow0 + k0);
    const Frag<BS_PREC_F64> a1 = load_frag<BS_PREC_F64>(qrow1 + k0);
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      Frag<BS_PREC_F64> bb;
#pragma unroll
      for (int q = 0; q < 4; ++q) bb.v[q] = stage[buf][(4 * fg + q) * PITCH + t * 16 + fr];
      mfma_step(acc[0][t], a0, bb);
      mfma_step(acc[1][t], a1, bb);
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < NSEG; ++u) *reinterpret_cast<d2*>(&stage[buf ^ 1][soff[u]]) = stg[u];
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const int nt = nc0 + t;
      if (nt >= ntiles) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 16 * m + acc_row<double>(fg, r);
        if (row < sj) {
          const int64_t o = base + row * mp + nt * 16 + fr;
          const double w = acc[m][t][r];
          Wp[o] = w;
          U[o] = rhs[o] - w;
          if constexpr (sizeof(OUT) == 2) {
            uint16_t hi, lo;
            split_bf16(w, hi, lo);
            const int64_t tcol = ((int64_t)i * 2 * mp + nt * 16 + fr) * spad + coff[j] + row;
            Wop[tcol] = hi;
            Wop[tcol + mp * spad] = lo;
          } else {  // [i][mp][spad], like the BF16 planes
            Wop[((int64_t)i * mp + nt * 16 + fr) * spad + coff[j] + row] = (OUT)w;
          }
        }
      }
    }
}

template <typename OUT>
void launch_solve(const double* Q, int64_t S, int C, int b0, int nb, const int64_t* coff,
                  const int64_t* sjs, int64_t spad, int64_t mp, const double* rhs, double* Wp,
                  double* U, OUT* Wop, hipStream_t st) {
  const int ntiles = (int)(mp / 16);
  if (ntiles <= 2) {  // few columns: Q streamed once, k split over the 4 waves
    dim3 g((unsigned)(S / 16), (unsigned)nb);
    if (ntiles == 1)
      solve_ks_kernel<OUT, 1><<<g, 256, 0, st>>>(Q, S, C, b0, coff, sjs, spad, mp, rhs, Wp, U,
                                                 Wop);
    else
      solve_ks_kernel<OUT, 2><<<g, 256, 0, st>>>(Q, S, C, b0, coff, sjs, spad, mp, rhs, Wp, U,
                                                 Wop);
    return;
  }
#define BS_SOLVE_WIDE(NTC)                                                                 \
  solve_wide_kernel<OUT, NTC><<<dim3((unsigned)((S + 127) / 128), (unsigned)nb,            \
                                     (unsigned)((ntiles + NTC - 1) / NTC)), 256, 0, st>>>( \
      Q, S, C, b0, coff, sjs, spad, mp, rhs, Wp, U, Wop)
  if (ntiles <= 4) BS_SOLVE_WIDE(4);
  else if (ntiles <= 6) BS_SOLVE_WIDE(6);
  else if (ntiles <= 8) BS_SOLVE_WIDE(8);
  else if (ntiles <= 10) BS_SOLVE_WIDE(10);
  else BS_SOLVE_WIDE(8);
#undef BS_SOLVE_WIDE
}

}  // namespace

hipError_t identity_pad(double* slots, int batch, int64_t S, const int64_t* sj_host,
                        hipStream_t st) {
  for (int b = 0; b < batch; ++b) {
    if (sj_host[b] >= S) continue;
    unsigned g = (unsigned)std::min<int64_t>((S * S + 255) / 256, 16384);
    identity_pad_kernel<<<g, 256, 0, st>>>(slots + (int64_t)b * S * S, S, sj_host[b]);
  }
  return hipGetLastError();
}

hipError_t spd_inverse(double* slots, int batch, int64_t S, double* work, double* dinv, int* flag,
                       hipStream_t st) {
  const int nblk = (int)(S / NB);
  for (int K = 0; K < nblk; K += PW) {
    const int jend = std::min(nblk, K + PW);
    for (int kb = K; kb < jend; ++kb) {
      potrf_diag_kernel<<<batch, 256, 0, st>>>(slots, S, kb, dinv, flag);
      const int T = nblk - kb - 1;
      if (T > 0) {
        trsm_kernel<<<dim3(T, batch), 256, 0, st>>>(slots, S, kb, dinv);
        if (jend - kb - 1 > 0)
          syrk_panel_kernel<<<dim3(T, jend - kb - 1, batch), 256, 0, st>>>(slots, S, kb, jend);
      }
    }
    const int T2 = nblk - jend;
    if (T2 > 0)
      syrk_multi_kernel<<<dim3(T2 * (T2 + 1) / 2, batch), 256, 0, st>>>(slots, S, K, jend - K);
  }
  trinv_diag_kernel<<<dim3(nblk, batch), 256, 0, st>>>(dinv, S, work);
  for (int b = 1; b < nblk; b *= 2) {
    const int pairs = (nblk - b + 2 * b - 1) / (2 * b);  // p with 2 p b + b < nblk
    const dim3 g((unsigned)(pairs * b * b), (unsigned)batch);
    trinv_y_kernel<<<g, 256, 0, st>>>(slots, S, b, work);
    trinv_x_kernel<<<g, 256, 0, st>>>(S, b, work);
  }
  xtx_kernel<<<dim3(nblk * (nblk + 1) / 2, batch), 256, 0, st>>>(work, S, slots);
  return hipGetLastError();
}

hipError_t solve(int prec, const double* Q, int64_t S, int C, int b0, int nb, const int64_t* coff,
                 const int64_t* sjs, int64_t spad, int64_t mp, const double* rhs, double* Wp,
                 double* U, void* Wop, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  if (prec == BS_PREC_F64)
    launch_solve<double>(Q, S, C, b0, nb, coff, sjs, spad, mp, rhs, Wp, U, (double*)Wop, st);
  else if (bf16_planes(prec, mp))  // BF16, and BF16X3 with more than two output tiles
    launch_solve<uint16_t>(Q, S, C, b0, nb, coff, sjs, spad, mp, rhs, Wp, U, (uint16_t*)Wop, st);
  else  // FP32, and BF16X3 with one or two output tiles, multiply FP32 operands
    launch_solve<float>(Q, S, C, b0, nb, coff, sjs, spad, mp, rhs, Wp, U, (float*)Wop, st);
  return hipGetLastError();
}

}  // namespace bs
