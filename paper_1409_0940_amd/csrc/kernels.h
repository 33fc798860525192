// Host-side launchers of the HIP kernels (internal to libbsadmm).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace bs {

// Whether the products take R and W' as BF16 head and residual planes (the
// transposed layouts below): always in BF16, and in BF16X3 when there are
// more than two output tiles, where three BF16 products (head x head,
// head x residual, residual x head) replace the MFMA-bound FP32 ones.
inline bool bf16_planes(int prec, int64_t mp) {
  return prec == BS_PREC_BF16 || (prec == BS_PREC_BF16X3 && mp > 32);
}

// Operand row width (k padded) for a precision: multiple of the K chunk.
int64_t padded_k(int prec, int64_t d);
// Bytes of one operand element (per plane), operand planes (2 for BF16X3:
// head and residual), bytes of one stored Z element, and bytes of one
// element of the product operands R and W' (FP64 or FP32).
size_t op_bytes(int prec);
int op_planes(int prec);
size_t z_bytes(int prec);
size_t vec_bytes(int prec);

// Rows [0, rows) of a float32 matrix (ld = d) -> operand layout (ld = Kp,
// zero padded; BF16X3 writes the residual plane at dst + plane elements).
// Sets *flag |= 1 if a value is not finite.
hipError_t prep_rows(int prec, const float* src, int64_t rows, int64_t d, int64_t Kp,
                     void* dst, int64_t plane, int* flag, hipStream_t st);
// W (d x s, ld = s) -> Wt (s x Kp), transposed and padded (residual plane at
// Wt + plane); bias copy.
hipError_t prep_w(int prec, const float* W, const float* b, int64_t d, int64_t s, int64_t Kp,
                  void* Wt, int64_t plane, void* bias, int* flag, hipStream_t st);
// Non-finite check of a float32 array.
hipError_t check_finite(const float* p, int64_t count, int* flag, hipStream_t st);

// Z[r][f] = scale * cos(sum_k Xp[r][k] Wt[f][k] + bias[f]) for r < rows,
// f < cols; Z has leading dimension ldz and the stored type of the precision
// (double / float / bf16 bits / float).  xps, wps: plane strides (BF16X3).
hipError_t regen(int prec, const void* Xp, int64_t xps, int64_t rows, const void* Wt, int64_t wps,
                 int64_t cols, const void* bias, int64_t Kp, double scale, void* Z, int64_t ldz,
                 hipStream_t st);
// Feature-map draw from a seed (Philox4x32-10 and Box-Muller, as documented
// with bsadmm_problem.seed): W (d x s, N(0, 1/sigma^2)) and b (s, U[0, 2 pi)).
hipError_t draw_features(uint64_t seed, int64_t d, int64_t s, double sigma, float* W, float* b,
                         hipStream_t st);
// Refined BF16: BF16X3 (FP32-faithful) features of the same block, not
// stored; their defect bf16(z - Zt) against the BF16 features Zt goes to Zd
// (both BF16, row stride ldz).
hipError_t regen_defect(const void* Xp, int64_t xps, int64_t rows, const void* Wt, int64_t wps,
                        int64_t cols, const void* bias, int64_t Kp, double scale,
                        const uint16_t* Zt, uint16_t* Zd, int64_t ldz, hipStream_t st);

// The padded feature index: feature block j occupies [coff_j, coff_j + s_j)
// with coff_j a multiple of 64; spad is the padded total; pad entries are 0.

// Product operands.  FP64, FP32 and BF16X3 multiply R as [n][mp] and W'
// transposed, [i][mp][spad], in the operand type (double, float, float).
// BF16 multiplies BF16 head and residual planes of both, stored transposed:
// R as [plane][mp][ldr] with ldr = R * nbpad and row block i in the segment
// starting at i * nbpad (zero for at least 32 rows past its rows), W' as
// [i][plane][mp][spad].  BF16X3 with more than two output tiles takes R and
// W' in those plane layouts too (bf16_planes) and splits its float Z into
// head and residual in the kernels.

// Partial transpose products for one row block:
// part[sp][f][c] = sum_{r in split sp} Z[r][f] * R[r][c], f < spad, c < mp.
// Rop points at the block's rows; ldr is used by the plane layout only
// (bf16_planes), whose split_rows must be a multiple of 32.
hipError_t ztr_partial(int prec, const void* Z, int64_t ldz, int64_t rows, int64_t spad,
                       const void* Rop, int64_t ldr, int64_t mp, int64_t split_rows, void* part,
                       hipStream_t st);
// For row blocks i in [i0, i1): rhs_i = W-bar - mu'_i + U_i + sum_sp part_i[sp]
// + corr_i (part laid out [i][sp < nsplit_max][spad][mp]; the split count of
// block i follows from the row partition of n into R blocks).  Wbar, mup, U
// null: the base is 0 (the plain sum of the partials); corr null: no term.
hipError_t reduce_rhs(int prec, const void* part, int64_t nsplit_max, int64_t n, int R, int i0,
                      int i1, int64_t split_rows, int64_t spad, int64_t mp, const double* Wbar,
                      const double* mup, const double* U, const double* corr, double* rhs,
                      hipStream_t st);
// For the row blocks i in [i0, i1) of the partition of n rows into R blocks:
// Pout[r][c] = sum_f Z[r][f] * W'_i[f][c], f < spad (a multiple of 64),
// c < mp, W'_i in the transposed operand layout with row stride spad.  Z
// points at row floor(i0 n / R), Pout at row 0; W'_i starts wop_stride
// operand elements after W'_{i-1} (0: one W' for every block).
hipError_t zw(int prec, const void* Z, int64_t ldz, int64_t n, int R, int i0, int i1,
              int64_t spad, const void* Wop, int64_t wop_stride, int64_t mp, double* Pout,
              hipStream_t st);
// Gram of one block (rows x [coff, coff + sj)) of Z into slot (ld = S):
// lower 64 x 64 tiles of I + Z^T Z.
hipError_t gram(int prec, const void* Z, int64_t ldz, int64_t rows, int64_t coff, int64_t sj,
                double* slot, int64_t S, hipStream_t st);

// Batched FP64 factor cache.  `slots` holds `batch` matrices of S x S
// (S multiple of 64) whose lower triangle is I + G; on exit it holds the
// full symmetric inverse.  `work` needs batch * S * S doubles, `dinv`
// batch * S * 64 doubles.  Pivot failures set *flag |= 2.
hipError_t identity_pad(double* slots, int batch, int64_t S, const int64_t* sj_host,
                        hipStream_t st);
hipError_t spd_inverse(double* slots, int batch, int64_t S, double* work, double* dinv,
                       int* flag, hipStream_t st);

// W'_b = Q_b rhs_b for blocks b in [b0, b0 + nb) (b = i * C + j); U = rhs - W';
// Wop = W' in the operand layout of the precision.  coff / sjs are device
// arrays of length C.
hipError_t solve(int prec, const double* Q, int64_t S, int C, int b0, int nb, const int64_t* coff,
                 const int64_t* sjs, int64_t spad, int64_t mp, const double* rhs, double* Wp,
                 double* U, void* Wop, hipStream_t st);

// Elementwise steps (FP64 state, n x mp / s x mp, only c < m touched).
hipError_t row_pre(int prec, int loss, const double* wts, double cfac, int64_t n, int R, int64_t m,
                   int64_t mp, int64_t nbpad, const float* Y, const double* Obar, const double* nu,
                   const double* Dbar, double* O, void* Rop, hipStream_t st);
// Pc (nullable): defect of the forward product, added to P (and P updated).
hipError_t row_post(int64_t n, int64_t m, int64_t mp, int C, const double* O, double* P,
                    const double* Pc, double* Obar, double* nu, double* Dbar, hipStream_t st);
hipError_t col_pre(const double* wts, int64_t s, int64_t m, int64_t mp, const double* Wbar,
                   const double* mu, double* Wc, hipStream_t st);
hipError_t col_post(int R, int64_t s, int64_t m, int64_t mp, const double* Wc, const double* Wp,
                    double* Wbar, double* mu, double* mup, hipStream_t st);
// Copy between padded (ld = mp) FP64 state and a dense (ld = m) buffer.
hipError_t unpad(const double* src, int64_t rows, int64_t m, int64_t mp, double* dst,
                 hipStream_t st);
hipError_t pad(const double* src, int64_t rows, int64_t m, int64_t mp, double* dst,
               hipStream_t st);
// Penalty adaptation: the eight fixed-order sums the residual-balancing step
// needs, from the state after an iteration and a copy of it from before:
// out[0] = ||Dbar||^2, out[1] = ||Wc - Wbar||^2, out[2] = sum_i ||Wp_i - Wbar||^2,
// out[3] = ||dObar||^2, out[4] = ||dWbar||^2, out[5] = <dWp, dU>,
// out[6] = <dO, dDbar>, out[7] = ||dDbar||^2 (d: change over the iteration;
// part holds 8 nb partials).
struct ResidualArgs {
  const double *Dbar, *Wc, *Wp, *Wbar, *Obar, *O, *U;
  const double *Obar_prev, *Wbar_prev, *Wp_prev, *O_prev, *Dbar_prev, *U_prev;
};
hipError_t residuals(const ResidualArgs& a, int R, int64_t n, int64_t spad, int64_t m,
                     int64_t mp, double* part, int nb, double* out, hipStream_t st);
// dst[e] = src[e] for e < count (a kernel, so it may sit in a captured graph).
hipError_t copy(double* dst, const double* src, int64_t count, hipStream_t st);
// y[e] += x[e] for e < count.
hipError_t axpy(double* y, const double* x, int64_t count, hipStream_t st);
// a[e] *= *f for e < count (nothing when *f == 1).
hipError_t scale(double* a, int64_t count, const double* f, hipStream_t st);
// Penalty block on the device (doubles): rho, the loss-prox weight 1/rho, the
// regulariser weight n lambda / rho, the factor for the scaled duals from the
// last change, and the number of changes made by adapt.
enum { BS_W_RHO = 0, BS_W_TAU = 1, BS_W_KAPPA = 2, BS_W_DUAL = 3, BS_W_CHANGES = 4, BS_W_COUNT = 8 };
// Residual balancing from the eight sums of residuals(): updates wts.
hipError_t adapt(const double* sums, double* wts, int R, int C, double n_lambda, double mu,
                 double tau_f, hipStream_t st);
// out[0..1] = primal and dual residual norms from the sums of residuals() at
// the penalty in wts (read when the kernel runs).
hipError_t residual_norms(const double* sums, const double* wts, int R, int C, double* out,
                          hipStream_t st);
// wts <- penalty rho (dual factor rho_old / rho when rescale, else 1).
hipError_t set_rho(double* wts, double rho, double n_lambda, int rescale, hipStream_t st);
// Operand copy of nblk blocks of W' ([spad][mp] doubles each) in the layout
// the forward products of the precision read.
hipError_t to_wop(int prec, const double* src, int64_t nblk, int64_t spad, int64_t mp, void* dst,
                  hipStream_t st);
// Deterministic partial sums (one per workgroup, nblocks <= 65536, summed by
// the caller in order): sum of V(y_rc, P_rc) over r < n, c < m (loss 0:
// squared, otherwise hinge), and sum of squares of a.
hipError_t loss_partial(int loss, const double* P, const float* Y, int64_t n, int64_t m,
                        int64_t mp, double* part, int nblocks, hipStream_t st);
hipError_t sumsq_partial(const double* a, int64_t count, double* part, int nblocks,
                         hipStream_t st);
// Convergence monitor (no synchronisation): out[0] = sum V(y, P),
// out[1] = sum_i ||Wp_i||^2 / R, out[2] = sum_i ||Wp_i - Wbar||^2,
// out[3] = ||Dbar||^2, via nb partial sums per quantity in `part` (4 nb).
// Fenchel dual bound (not in the paper): alpha = rho (Delta-bar/(C+1) + nu)
// moved into the conjugate's domain (loss 0 squared, 1 hinge), written into
// the R operand layout, with the conjugate terms' partial sums in part[0, nb).
hipError_t dual_rows(int prec, int loss, const double* wts, double cfac, int64_t n, int R,
                     int64_t m, int64_t mp, int64_t nbpad, const float* Y, const double* nu,
                     const double* Dbar, void* Rop, double* part, int nb, hipStream_t st);
// out = {D, conj / n, ||Z^T alpha||^2 / (4 lambda n^2)} from part[0, nb) and
// A = Z_ij^T alpha_i (R blocks of `per` values, summed over i).
hipError_t dual_final(const double* A, int R, int64_t per, int64_t n, double lambda, double* part,
                      int nb, double* out, hipStream_t st);
hipError_t monitor(int loss, const double* P, const float* Y, const double* Wp,
                   const double* Wbar, const double* Dbar, int R, int64_t n, int64_t spad,
                   int64_t m, int64_t mp, double* part, int nb, double* out, hipStream_t st);
// Scores out[r][c] = (float) P[r][c], c < m.
hipError_t scores_out(const double* P, int64_t rows, int64_t m, int64_t mp, float* out,
                      hipStream_t st);

}  // namespace bs
