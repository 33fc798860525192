// Elementwise steps of Algorithm 1 on the FP64 ADMM state.
//
// Row side (n x m, padded to mp columns; pad columns stay zero):
//   row_pre  : O = prox_{tau V}(O-bar - nu)                        (step 4)
//              R = Delta-bar / (C+1) + nu as product operand        (step 17)
//   row_post : Delta-bar = O - sum_j O'_ij                         (steps 11, 20, 25)
//              O-bar = C/(C+1) O + sum_j O'_ij / (C+1)             (steps 12, 22)
//              nu += O - O-bar                                       (step 33)
// Column side (padded feature index x mp):
//   col_pre  : W = prox_{kappa r}(W-bar - mu)                        (step 6)
//   col_post : W-bar = (W + sum_i W'_i) / (R+1), summed in order i   (steps 28-29)
//              mu += W - W-bar, mu'_i += W'_i - W-bar (new W-bar, as in the
//              block-splitting update equations)
#include "common.h"
#include "kernels.h"

namespace bs {

namespace {

inline unsigned grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

#define GRID_STRIDE(e, total)                                                   \
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (total); \
       e += (int64_t)gridDim.x * blockDim.x)

// Kernel loss codes: 0 squared ||y - o||^2, 1 hinge max(0, 1 - y o) (also
// one-vs-all), 2 l1 |y - o|: elementwise proxes; 3 Crammer-Singer hinge and
// 4 multinomial logistic: row-wise proxes (row_prox_kernel).
__device__ __forceinline__ double prox_loss(int loss, double v, double y, double tau) {
  if (loss == 0) return (v + 2.0 * tau * y) / (1.0 + 2.0 * tau);  // ||y - o||^2
  if (loss == 2) {  // |y - o|: soft-threshold v - y at tau
    const double d = v - y, a = fabs(d) - tau;
    return a > 0.0 ? y + (d > 0.0 ? a : -a) : y;
  }
  // max(0, 1 - y o): move by y * clamp(1 - y v, 0, tau)
  double g = 1.0 - y * v;
  g = g < 0.0 ? 0.0 : (g > tau ? tau : g);
  return v + y * g;
}

// Row-wise proxes, one thread per row r of the padded n x mp state; the
// argument of the prox is v_k = O-bar[r][k] - nu[r][k] and the result goes to
// O[r][k], which also holds the iterate while it is being computed.
//
// Crammer-Singer, f(o) = max_k (o_k + delta_k) - o_y with delta_k = [k != y]:
// prox_{tau f}(v) = w - tau P(w / tau) - delta with w = v + tau e_y + delta and
// P the projection onto the probability simplex, P(u)_k = max(u_k - theta, 0).
// theta is found by support shrinking: starting from all k, theta = (sum of
// u over the support - 1) / (support size), and entries not above theta leave
// the support until it is stable (at most m passes; exact).
//
// Multinomial logistic, f(o) = log sum_k exp(o_k) - y^T o: Newton's method on
// h(o) = tau f(o) + 1/2 ||o - v||^2.  Its Hessian is D - tau p p^T with
// D = diag(1 + tau p), p = softmax(o), so by Sherman-Morrison the step is
// H^{-1} g = g / d + tau (p / d) (sum p g / d) / (1 - tau sum p^2 / d).  A step
// is halved until the gradient norm drops; the iteration stops when it no
// longer does (rounding level) or after 100 steps.
__device__ __forceinline__ double row_v(const double* Obar, const double* nu, int64_t o) {
  return Obar[o] - nu[o];
}

__global__ void row_prox_kernel(int loss, const double* __restrict__ wts, int64_t n, int64_t m,
                                int64_t mp, const float* __restrict__ Y,
                                const double* __restrict__ Obar, const double* __restrict__ nu,
                                double* __restrict__ O) {
  const double tau = wts[BS_W_TAU];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = r * mp;
    const float* y = Y + r * m;
    if (loss == 3) {
      // w into O; the support test runs on u = w / tau
      for (int64_t k = 0; k < m; ++k) {
        const double e = y[k] > 0.5f ? 1.0 : 0.0;
        O[b + k] = row_v(Obar, nu, b + k) + tau * e + (1.0 - e);
      }
      double theta = -__builtin_inf();
      int64_t cnt = -1;
      for (int pass = 0; pass <= m; ++pass) {
        double sum = 0.0;
        int64_t c = 0;
        for (int64_t k = 0; k < m; ++k) {
          const double u = O[b + k] / tau;
          if (u > theta) {
            sum += u;
            ++c;
          }
        }
        const double th = (sum - 1.0) / (double)c;
        if (c == cnt) break;  // support unchanged: theta is final
        cnt = c;
        theta = th;
      }
      for (int64_t k = 0; k < m; ++k) {
        const double w = O[b + k], u = w / tau;
        const double q = u > theta ? u - theta : 0.0;
        O[b + k] = w - tau * q - (y[k] > 0.5f ? 0.0 : 1.0);
      }
    } else {  // loss == 4
      for (int64_t k = 0; k < m; ++k) O[b + k] = row_v(Obar, nu, b + k);
      // softmax normaliser and gradient norm of the current iterate
      auto stats = [&](double t, double mx0, double se0, double a, double c, double& mx,
                       double& se, double& gmax) {
        // iterate o - t * step (t = 0: o itself), step from (mx0, se0, a, c)
        mx = -__builtin_inf();
        for (int64_t k = 0; k < m; ++k) {
          double x = O[b + k];
          if (t != 0.0) {
            const double p = exp(x - mx0) / se0, d = 1.0 + tau * p;
            const double g = tau * (p - (double)y[k]) + x - row_v(Obar, nu, b + k);
            x -= t * (g / d + tau * (p / d) * a / (1.0 - tau * c));
          }
          mx = x > mx ? x : mx;
        }
        se = 0.0;
        for (int64_t k = 0; k < m; ++k) {
          double x = O[b + k];
          if (t != 0.0) {
            const double p = exp(x - mx0) / se0, d = 1.0 + tau * p;
            const double g = tau * (p - (double)y[k]) + x - row_v(Obar, nu, b + k);
            x -= t * (g / d + tau * (p / d) * a / (1.0 - tau * c));
          }
          se += exp(x - mx);
        }
        gmax = 0.0;
        for (int64_t k = 0; k < m; ++k) {
          double x = O[b + k];
          if (t != 0.0) {
            const double p = exp(x - mx0) / se0, d = 1.0 + tau * p;
            const double g = tau * (p - (double)y[k]) + x - row_v(Obar, nu, b + k);
            x -= t * (g / d + tau * (p / d) * a / (1.0 - tau * c));
          }
          const double g = tau * (exp(x - mx) / se - (double)y[k]) + x - row_v(Obar, nu, b + k);
          gmax = fabs(g) > gmax ? fabs(g) : gmax;
        }
      };
      double mx, se, gn;
      stats(0.0, 0.0, 1.0, 0.0, 0.0, mx, se, gn);
      for (int it = 0; it < 100; ++it) {
        // Sherman-Morrison sums at the current iterate
        double a = 0.0, c = 0.0;
        for (int64_t k = 0; k < m; ++k) {
          const double x = O[b + k];
          const double p = exp(x - mx) / se, d = 1.0 + tau * p;
          const double g = tau * (p - (double)y[k]) + x - row_v(Obar, nu, b + k);
          a += p * g / d;
          c += p * p / d;
        }
        double t = 1.0, mxc = 0.0, sec = 0.0, gc = 0.0;
        bool ok = false;
        for (int h = 0; h < 45; ++h, t *= 0.5) {
          stats(t, mx, se, a, c, mxc, sec, gc);
          if (gc < gn) {
            ok = true;
            break;
          }
        }
        if (!ok) break;  // no further decrease: at rounding level
        for (int64_t k = 0; k < m; ++k) {
          const double x = O[b + k];
          const double p = exp(x - mx) / se, d = 1.0 + tau * p;
          const double g = tau * (p - (double)y[k]) + x - row_v(Obar, nu, b + k);
          O[b + k] = x - t * (g / d + tau * (p / d) * a / (1.0 - tau * c));
        }
        mx = mxc;
        se = sec;
        gn = gc;
      }
    }
  }
}

template <typename OP>
__global__ void row_pre_kernel(int loss, const double* __restrict__ wts, double cfac, int64_t n,
                               int64_t m, int64_t mp,
                               const float* __restrict__ Y, const double* __restrict__ Obar,
                               const double* __restrict__ nu, const double* __restrict__ Dbar,
                               double* __restrict__ O, OP* __restrict__ Rop) {
  const double tau = wts[BS_W_TAU];
  GRID_STRIDE(e, n * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    const double nv = nu[o];
    if (loss < 3) O[o] = prox_loss(loss, Obar[o] - nv, (double)Y[e], tau);
    Rop[o] = cvt_from_double<OP>(Dbar[o] * cfac + nv);
  }
}

// BF16 products: R as BF16 head and residual planes stored transposed,
// Rt[plane][c][i * nbpad + (r - first row of block i)].
__global__ void row_pre_bf16_kernel(int loss, const double* __restrict__ wts, double cfac,
                                    int64_t n, int R,
                                    int64_t m, int64_t mp, int64_t nbpad,
                                    const float* __restrict__ Y, const double* __restrict__ Obar,
                                    const double* __restrict__ nu, const double* __restrict__ Dbar,
                                    double* __restrict__ O, uint16_t* __restrict__ Rt) {
  const double tau = wts[BS_W_TAU];
  const int64_t ldr = (int64_t)R * nbpad;
  GRID_STRIDE(e, n * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    const double nv = nu[o];
    if (loss < 3) O[o] = prox_loss(loss, Obar[o] - nv, (double)Y[e], tau);
    // row block of r: the largest i with floor(i n / R) <= r
    int64_t i = r * R / n;
    while (i + 1 < R && (i + 1) * n / R <= r) ++i;
    while (i > 0 && i * n / R > r) --i;
    uint16_t hi, lo;
    split_bf16(Dbar[o] * cfac + nv, hi, lo);
    const int64_t t = c * ldr + i * nbpad + (r - i * n / R);
    Rt[t] = hi;
    Rt[t + mp * ldr] = lo;
  }
}

// With Pc (the stored defect of the forward product, refined BF16) the
// product is P + Pc, written back to P so later readers see the sum.
__global__ void row_post_kernel(int64_t n, int64_t m, int64_t mp, double a, double bfac,
                                const double* __restrict__ O, double* __restrict__ P,
                                const double* __restrict__ Pc, double* __restrict__ Obar,
                                double* __restrict__ nu, double* __restrict__ Dbar) {
  GRID_STRIDE(e, n * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    double pv = P[o];
    if (Pc) {
      pv += Pc[o];
      P[o] = pv;
    }
    const double ov = O[o];
    const double ob = a * ov + bfac * pv;
    Dbar[o] = ov - pv;
    Obar[o] = ob;
    nu[o] = nu[o] + ov - ob;
  }
}

__global__ void col_pre_kernel(const double* __restrict__ wts, int64_t rows, int64_t m, int64_t mp,
                               const double* __restrict__ Wbar, const double* __restrict__ mu,
                               double* __restrict__ Wc) {
  const double den = 1.0 / (1.0 + 2.0 * wts[BS_W_KAPPA]);
  GRID_STRIDE(e, rows * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    Wc[o] = (Wbar[o] - mu[o]) * den;
  }
}

__global__ void col_post_kernel(int R, int64_t rows, int64_t m, int64_t mp,
                                const double* __restrict__ Wc, const double* __restrict__ Wp,
                                double* __restrict__ Wbar, double* __restrict__ mu,
                                double* __restrict__ mup) {
  const int64_t per = rows * mp;
  const double inv = 1.0 / (double)(R + 1);
  GRID_STRIDE(e, rows * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    const double wc = Wc[o];
    double sum = wc;
    for (int i = 0; i < R; ++i) sum += Wp[(int64_t)i * per + o];
    const double wb = sum * inv;
    Wbar[o] = wb;
    mu[o] = mu[o] + wc - wb;
    for (int i = 0; i < R; ++i) {
      const int64_t oi = (int64_t)i * per + o;
      mup[oi] = mup[oi] + Wp[oi] - wb;
    }
  }
}

__global__ void unpad_kernel(const double* __restrict__ src, int64_t rows, int64_t m, int64_t mp,
                             double* __restrict__ dst) {
  GRID_STRIDE(e, rows * m) {
    const int64_t r = e / m, c = e - r * m;
    dst[e] = src[r * mp + c];
  }
}

__global__ void pad_kernel(const double* __restrict__ src, int64_t rows, int64_t m, int64_t mp,
                           double* __restrict__ dst) {
  GRID_STRIDE(e, rows * m) {
    const int64_t r = e / m, c = e - r * m;
    dst[r * mp + c] = src[e];
  }
}

__global__ void scores_kernel(const double* __restrict__ P, int64_t rows, int64_t m, int64_t mp,
                              float* __restrict__ out) {
  GRID_STRIDE(e, rows * m) {
    const int64_t r = e / m, c = e - r * m;
    out[e] = (float)P[r * mp + c];
  }
}

// Fixed-order block reduction helper: 256 threads, result in red[0].
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// part[block] = sum over this block's grid-stride elements of V(y, o)
// (squared: (y - o)^2; hinge: max(0, 1 - y o)).
__global__ void loss_partial_kernel(int loss, const double* __restrict__ P,
                                    const float* __restrict__ Y, int64_t n, int64_t m, int64_t mp,
                                    double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  if (loss < 3) {
    GRID_STRIDE(e, n * m) {
      const int64_t r = e / m, c = e - r * m;
      const double o = P[r * mp + c], y = (double)Y[e];
      if (loss == 0) {
        const double d = y - o;
        acc += d * d;
      } else if (loss == 2) {
        acc += fabs(y - o);
      } else {
        const double h = 1.0 - y * o;
        acc += h > 0.0 ? h : 0.0;
      }
    }
  } else {  // row-wise: Crammer-Singer max_k (o_k + delta_k) - o_y, or log sum exp(o) - o_y
    GRID_STRIDE(r, n) {
      const double* o = P + r * mp;
      const float* y = Y + r * m;
      double mx = -__builtin_inf(), oy = 0.0;
      for (int64_t k = 0; k < m; ++k) {
        const bool cls = y[k] > 0.5f;
        const double v = o[k] + (loss == 3 && !cls ? 1.0 : 0.0);
        mx = v > mx ? v : mx;
        if (cls) oy = o[k];
      }
      if (loss == 3) {
        acc += mx - oy;
      } else {
        double se = 0.0;
        for (int64_t k = 0; k < m; ++k) se += exp(o[k] - mx);
        acc += mx + log(se) - oy;
      }
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void sumsq_partial_kernel(const double* __restrict__ a, int64_t count,
                                     double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  GRID_STRIDE(e, count) acc += a[e] * a[e];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// part[block] = sum over this block's share of sum_i (Wp_i - Wbar)^2 on the
// first `rows * m` entries of each padded (rows x mp) array.
__global__ void diffsq_partial_kernel(const double* __restrict__ Wp, const double* __restrict__ Wbar,
                                      int R, int64_t rows, int64_t m, int64_t mp,
                                      double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t per = rows * mp;
  double acc = 0.0;
  GRID_STRIDE(e, rows * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    const double wb = Wbar[o];
    for (int i = 0; i < R; ++i) {
      const double d = Wp[(int64_t)i * per + o] - wb;
      acc += d * d;
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// part[block] = this block's share of sum (a - ap) * (b - bp) over the first
// `m` columns of `rows` padded (ld = mp) rows.
__global__ void diffdot_partial_kernel(const double* __restrict__ a, const double* __restrict__ ap,
                                       const double* __restrict__ b, const double* __restrict__ bp,
                                       int64_t rows, int64_t m, int64_t mp,
                                       double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  GRID_STRIDE(e, rows * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    acc += (a[o] - ap[o]) * (b[o] - bp[o]);
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void copy_kernel(double* __restrict__ dst, const double* __restrict__ src,
                            int64_t count) {
  GRID_STRIDE(e, count) dst[e] = src[e];
}

__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ x, int64_t count) {
  GRID_STRIDE(e, count) y[e] += x[e];
}

__global__ void scale_kernel(double* __restrict__ a, int64_t count, const double* __restrict__ f) {
  const double v = *f;
  if (v == 1.0) return;
  GRID_STRIDE(e, count) a[e] *= v;
}

// Residual balancing step on the device (one thread).  The sums q are those
// of residuals(): with the exchange gap Delta-bar = O - P (P = sum_j O'_ij),
// ADMM on the block problem written as x = z has
//   primal^2 = ||Delta-bar||^2 / (C+1) + ||W - W-bar||^2 + sum_i ||W'_i - W-bar||^2
// (O_i - O-bar_i = Delta-bar_i / (C+1) and O'_ij - O-bar_ij = -Delta-bar_i / (C+1)
// for each of the C blocks), and
//   dual^2 / rho^2 = ||dO-bar||^2 + sum_ij ||dO-bar_ij||^2 + (R+1) ||dW-bar||^2
// with O-bar_ij = O'_ij + Delta-bar_i / (C+1).  Expanding the middle sum,
//   sum_ij ||dO'_ij||^2 = sum_ij <dW'_ij, dU_ij>  (O'_ij = Z_ij W'_ij, U_ij = G_ij W'_ij)
//   + 2 <dP, dDelta-bar> / (C+1) + C ||dDelta-bar||^2 / (C+1)^2,
// and <dP, dDelta-bar> = <dO, dDelta-bar> - ||dDelta-bar||^2.  The penalty
// block is updated; wts[BS_W_DUAL] gets the factor for the scaled duals
// (1 when rho stays).
__device__ inline void residual_pair(const double* __restrict__ q, double rho, int R, int C,
                                     double& r, double& sd) {
  const double c1 = (double)(C + 1);
  r = sqrt(q[0] / c1 + q[1] + q[2]);
  const double blocks = q[5] + 2.0 * (q[6] - q[7]) / c1 + (double)C * q[7] / (c1 * c1);
  const double s2 = q[3] + (double)(R + 1) * q[4] + blocks;
  sd = rho * sqrt(s2 > 0.0 ? s2 : 0.0);
}

__global__ void adapt_kernel(const double* __restrict__ q, double* __restrict__ wts, int R, int C,
                             double n_lambda, double mu, double tau_f) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double rho = wts[BS_W_RHO];
  double r, sd;
  residual_pair(q, rho, R, C, r, sd);
  const double f = r > mu * sd ? tau_f : (sd > mu * r ? 1.0 / tau_f : 1.0);
  wts[BS_W_DUAL] = 1.0 / f;
  if (f != 1.0) {
    const double nr = rho * f;
    wts[BS_W_RHO] = nr;
    wts[BS_W_TAU] = 1.0 / nr;
    wts[BS_W_KAPPA] = n_lambda / nr;
    wts[BS_W_CHANGES] += 1.0;
  }
}

// out[0], out[1] = primal and dual residual norms from the sums q at the
// current penalty (the same formulas as the balancing step).
__global__ void residual_norms_kernel(const double* __restrict__ q,
                                      const double* __restrict__ wts, int R, int C,
                                      double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double r, sd;
  residual_pair(q, wts[BS_W_RHO], R, C, r, sd);
  out[0] = r;
  out[1] = sd;
}

// Penalty set from the host: rho, the two prox weights and the dual factor
// rho_old / rho (or 1 without rescaling).
__global__ void set_rho_kernel(double* __restrict__ wts, double rho, double n_lambda, int rescale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  wts[BS_W_DUAL] = rescale ? wts[BS_W_RHO] / rho : 1.0;
  wts[BS_W_RHO] = rho;
  wts[BS_W_TAU] = 1.0 / rho;
  wts[BS_W_KAPPA] = n_lambda / rho;
}

// out[q] = scale[q] * sum_k part[q * nb + k], one workgroup per quantity
// (quantities past the fourth take the fourth scale).
__global__ void final_reduce_kernel(const double* __restrict__ part, int nb, double s0, double s1,
                                    double s2, double s3, double* __restrict__ out) {
  __shared__ double red[256];
  const int q = blockIdx.x;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) acc += part[q * nb + k];
  const double t = block_sum(acc, red);
  const double sc = q == 0 ? s0 : (q == 1 ? s1 : (q == 2 ? s2 : s3));
  if (threadIdx.x == 0) out[q] = sc * t;
}

// ---------------------------------------------------------------------------
// Lower bound on the optimum of F through its Fenchel dual (not in the
// paper): for any alpha (n x m) in the domain of the conjugate losses,
//   D(alpha) = (1/n) sum_r -V*(-alpha_r) - ||Z^T alpha||^2 / (4 lambda n^2)
// is at most min F.  -V*(-a) is a y - a^2 / 4 for the squared loss and a y
// for the hinge losses, whose domain is a y in [0, 1].  The dual point is
// the penalty times the row operand, rho (Delta-bar / (C+1) + nu), moved
// into that domain (hinge: y clip(y a, 0, 1)); at the ADMM fixed point it is
// the dual solution.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dual_value(int loss, double a, double y) {
  if (loss == 0) return a;
  double t = y * a;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  return y * t;
}

// alpha into the FP64 / FP32 operand layout of R (n x mp); part[block] =
// sum of the conjugate terms of the rounded alpha (the operand the product
// sees, still in the domain: rounding keeps 0 <= y a <= 1).
template <typename OP>
__global__ void dual_rows_kernel(int loss, const double* __restrict__ wts, double cfac, int64_t n,
                                 int64_t m, int64_t mp, const float* __restrict__ Y,
                                 const double* __restrict__ nu, const double* __restrict__ Dbar,
                                 OP* __restrict__ Rop, double* __restrict__ part) {
  __shared__ double red[256];
  const double rho = wts[BS_W_RHO];
  double conj = 0.0;
  GRID_STRIDE(e, n * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    const double y = (double)Y[e];
    const OP q = cvt_from_double<OP>(dual_value(loss, rho * (Dbar[o] * cfac + nu[o]), y));
    Rop[o] = q;
    const double a = to_double(q);
    conj += loss == 0 ? a * y - 0.25 * a * a : a * y;
  }
  const double t = block_sum(conj, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// The same into the BF16 head and residual planes (layout of row_pre_bf16).
__global__ void dual_rows_bf16_kernel(int loss, const double* __restrict__ wts, double cfac,
                                      int64_t n, int R, int64_t m, int64_t mp, int64_t nbpad,
                                      const float* __restrict__ Y, const double* __restrict__ nu,
                                      const double* __restrict__ Dbar, uint16_t* __restrict__ Rt,
                                      double* __restrict__ part) {
  __shared__ double red[256];
  const double rho = wts[BS_W_RHO];
  const int64_t ldr = (int64_t)R * nbpad;
  double conj = 0.0;
  GRID_STRIDE(e, n * m) {
    const int64_t r = e / m, c = e - r * m;
    const int64_t o = r * mp + c;
    const double y = (double)Y[e];
    const double v = dual_value(loss, rho * (Dbar[o] * cfac + nu[o]), y);
    int64_t i = r * R / n;
    while (i + 1 < R && (i + 1) * n / R <= r) ++i;
    while (i > 0 && i * n / R > r) --i;
    uint16_t hi, lo;
    split_bf16(v, hi, lo);
    const int64_t t = c * ldr + i * nbpad + (r - i * n / R);
    Rt[t] = hi;
    Rt[t + mp * ldr] = lo;
    const double a = (double)bf16_to_f32(hi) + (double)bf16_to_f32(lo);
    conj += loss == 0 ? a * y - 0.25 * a * a : a * y;
  }
  const double t = block_sum(conj, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// part[block] = sum over this block's share of the feature x column entries
// e of (sum_i A[i][e])^2: Z^T alpha = sum over row blocks of Z_ij^T alpha_i.
__global__ void colsum_sumsq_partial_kernel(const double* __restrict__ A, int R, int64_t per,
                                            double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  GRID_STRIDE(e, per) {
    double v = 0.0;
    for (int i = 0; i < R; ++i) v += A[(int64_t)i * per + e];
    acc += v * v;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out = {D, conjugate part / n, quadratic part}, partials as in dual_bound
__global__ void dual_final_kernel(const double* __restrict__ part, int nb, double n,
                                  double lambda, double* __restrict__ out) {
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) {
    a += part[k];
    b += part[nb + k];
  }
  const double conj = block_sum(a, red[0]);
  const double sq = block_sum(b, red[1]);
  if (threadIdx.x == 0) {
    const double c = conj / n, q = sq / (4.0 * lambda * n * n);
    out[0] = c - q;
    out[1] = c;
    out[2] = q;
  }
}

}  // namespace

hipError_t monitor(int loss, const double* P, const float* Y, const double* Wp,
                   const double* Wbar, const double* Dbar, int R, int64_t n, int64_t spad,
                   int64_t m, int64_t mp, double* part, int nb, double* out, hipStream_t st) {
  loss_partial_kernel<<<nb, 256, 0, st>>>(loss, P, Y, n, m, mp, part);
  sumsq_partial_kernel<<<nb, 256, 0, st>>>(Wp, (int64_t)R * spad * mp, part + nb);
  diffsq_partial_kernel<<<nb, 256, 0, st>>>(Wp, Wbar, R, spad, m, mp, part + 2 * nb);
  sumsq_partial_kernel<<<nb, 256, 0, st>>>(Dbar, n * mp, part + 3 * nb);
  final_reduce_kernel<<<4, 256, 0, st>>>(part, nb, 1.0, 1.0 / (double)R, 1.0, 1.0, out);
  return hipGetLastError();
}

hipError_t residuals(const ResidualArgs& a, int R, int64_t n, int64_t spad, int64_t m,
                     int64_t mp, double* part, int nb, double* out, hipStream_t st) {
  const int64_t cols = (int64_t)R * spad;
  sumsq_partial_kernel<<<nb, 256, 0, st>>>(a.Dbar, n * mp, part);
  diffsq_partial_kernel<<<nb, 256, 0, st>>>(a.Wc, a.Wbar, 1, spad, m, mp, part + nb);
  diffsq_partial_kernel<<<nb, 256, 0, st>>>(a.Wp, a.Wbar, R, spad, m, mp, part + 2 * nb);
  diffsq_partial_kernel<<<nb, 256, 0, st>>>(a.Obar, a.Obar_prev, 1, n, m, mp, part + 3 * nb);
  diffsq_partial_kernel<<<nb, 256, 0, st>>>(a.Wbar, a.Wbar_prev, 1, spad, m, mp, part + 4 * nb);
  diffdot_partial_kernel<<<nb, 256, 0, st>>>(a.Wp, a.Wp_prev, a.U, a.U_prev, cols, m, mp,
                                             part + 5 * nb);
  diffdot_partial_kernel<<<nb, 256, 0, st>>>(a.O, a.O_prev, a.Dbar, a.Dbar_prev, n, m, mp,
                                             part + 6 * nb);
  diffsq_partial_kernel<<<nb, 256, 0, st>>>(a.Dbar, a.Dbar_prev, 1, n, m, mp, part + 7 * nb);
  final_reduce_kernel<<<8, 256, 0, st>>>(part, nb, 1.0, 1.0, 1.0, 1.0, out);
  return hipGetLastError();
}

hipError_t dual_rows(int prec, int loss, const double* wts, double cfac, int64_t n, int R,
                     int64_t m, int64_t mp, int64_t nbpad, const float* Y, const double* nu,
                     const double* Dbar, void* Rop, double* part, int nb, hipStream_t st) {
  if (bf16_planes(prec, mp))
    dual_rows_bf16_kernel<<<nb, 256, 0, st>>>(loss, wts, cfac, n, R, m, mp, nbpad, Y, nu, Dbar,
                                              (uint16_t*)Rop, part);
  else if (prec == BS_PREC_F64)
    dual_rows_kernel<double><<<nb, 256, 0, st>>>(loss, wts, cfac, n, m, mp, Y, nu, Dbar,
                                                 (double*)Rop, part);
  else
    dual_rows_kernel<float><<<nb, 256, 0, st>>>(loss, wts, cfac, n, m, mp, Y, nu, Dbar,
                                                (float*)Rop, part);
  return hipGetLastError();
}

hipError_t dual_final(const double* A, int R, int64_t per, int64_t n, double lambda, double* part,
                      int nb, double* out, hipStream_t st) {
  colsum_sumsq_partial_kernel<<<nb, 256, 0, st>>>(A, R, per, part + nb);
  dual_final_kernel<<<1, 256, 0, st>>>(part, nb, (double)n, lambda, out);
  return hipGetLastError();
}

hipError_t copy(double* dst, const double* src, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  copy_kernel<<<grid_for(count), 256, 0, st>>>(dst, src, count);
  return hipGetLastError();
}

hipError_t axpy(double* y, const double* x, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  axpy_kernel<<<grid_for(count), 256, 0, st>>>(y, x, count);
  return hipGetLastError();
}

hipError_t scale(double* a, int64_t count, const double* f, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  scale_kernel<<<grid_for(count), 256, 0, st>>>(a, count, f);
  return hipGetLastError();
}

hipError_t adapt(const double* sums, double* wts, int R, int C, double n_lambda, double mu,
                 double tau_f, hipStream_t st) {
  adapt_kernel<<<1, 64, 0, st>>>(sums, wts, R, C, n_lambda, mu, tau_f);
  return hipGetLastError();
}

hipError_t residual_norms(const double* sums, const double* wts, int R, int C, double* out,
                          hipStream_t st) {
  residual_norms_kernel<<<1, 64, 0, st>>>(sums, wts, R, C, out);
  return hipGetLastError();
}

hipError_t set_rho(double* wts, double rho, double n_lambda, int rescale, hipStream_t st) {
  set_rho_kernel<<<1, 64, 0, st>>>(wts, rho, n_lambda, rescale);
  return hipGetLastError();
}

hipError_t loss_partial(int loss, const double* P, const float* Y, int64_t n, int64_t m,
                        int64_t mp, double* part, int nblocks, hipStream_t st) {
  loss_partial_kernel<<<nblocks, 256, 0, st>>>(loss, P, Y, n, m, mp, part);
  return hipGetLastError();
}

hipError_t sumsq_partial(const double* a, int64_t count, double* part, int nblocks,
                         hipStream_t st) {
  sumsq_partial_kernel<<<nblocks, 256, 0, st>>>(a, count, part);
  return hipGetLastError();
}

hipError_t row_pre(int prec, int loss, const double* wts, double cfac, int64_t n, int R, int64_t m,
                   int64_t mp, int64_t nbpad, const float* Y, const double* Obar, const double* nu,
                   const double* Dbar, double* O, void* Rop, hipStream_t st) {
  unsigned g = grid_for(n * m);
  if (loss >= 3)
    row_prox_kernel<<<grid_for(n), 256, 0, st>>>(loss, wts, n, m, mp, Y, Obar, nu, O);
  if (bf16_planes(prec, mp))
    row_pre_bf16_kernel<<<g, 256, 0, st>>>(loss, wts, cfac, n, R, m, mp, nbpad, Y, Obar, nu, Dbar,
                                           O, (uint16_t*)Rop);
  else if (prec == BS_PREC_F64)
    row_pre_kernel<double><<<g, 256, 0, st>>>(loss, wts, cfac, n, m, mp, Y, Obar, nu, Dbar, O,
                                               (double*)Rop);
  else
    row_pre_kernel<float><<<g, 256, 0, st>>>(loss, wts, cfac, n, m, mp, Y, Obar, nu, Dbar, O,
                                              (float*)Rop);
  return hipGetLastError();
}

hipError_t row_post(int64_t n, int64_t m, int64_t mp, int C, const double* O, double* P,
                    const double* Pc, double* Obar, double* nu, double* Dbar, hipStream_t st) {
  const double a = (double)C / (double)(C + 1), bfac = 1.0 / (double)(C + 1);
  row_post_kernel<<<grid_for(n * m), 256, 0, st>>>(n, m, mp, a, bfac, O, P, Pc, Obar, nu, Dbar);
  return hipGetLastError();
}

hipError_t col_pre(const double* wts, int64_t s, int64_t m, int64_t mp, const double* Wbar,
                   const double* mu, double* Wc, hipStream_t st) {
  col_pre_kernel<<<grid_for(s * m), 256, 0, st>>>(wts, s, m, mp, Wbar, mu, Wc);
  return hipGetLastError();
}

hipError_t col_post(int R, int64_t s, int64_t m, int64_t mp, const double* Wc, const double* Wp,
                    double* Wbar, double* mu, double* mup, hipStream_t st) {
  col_post_kernel<<<grid_for(s * m), 256, 0, st>>>(R, s, m, mp, Wc, Wp, Wbar, mu, mup);
  return hipGetLastError();
}

hipError_t unpad(const double* src, int64_t rows, int64_t m, int64_t mp, double* dst,
                 hipStream_t st) {
  if (rows * m == 0) return hipSuccess;
  unpad_kernel<<<grid_for(rows * m), 256, 0, st>>>(src, rows, m, mp, dst);
  return hipGetLastError();
}

hipError_t pad(const double* src, int64_t rows, int64_t m, int64_t mp, double* dst,
               hipStream_t st) {
  if (rows * m == 0) return hipSuccess;
  pad_kernel<<<grid_for(rows * m), 256, 0, st>>>(src, rows, m, mp, dst);
  return hipGetLastError();
}

namespace {
// W' (blocks of [spad][mp] doubles) as BF16 head and residual planes stored
// transposed, [b][plane][mp][spad].
__global__ void to_wop_bf16_kernel(const double* __restrict__ src, int64_t nblk, int64_t spad,
                                   int64_t mp, uint16_t* __restrict__ dst) {
  const int64_t per = spad * mp;
  GRID_STRIDE(e, nblk * per) {
    const int64_t b = e / per, rem = e - b * per;
    const int64_t f = rem / mp, c = rem - f * mp;
    uint16_t hi, lo;
    split_bf16(src[e], hi, lo);
    const int64_t t = (b * 2 * mp + c) * spad + f;
    dst[t] = hi;
    dst[t + mp * spad] = lo;
  }
}
template <typename T>
__global__ void to_wop_kernel(const double* __restrict__ src, int64_t nblk, int64_t spad,
                              int64_t mp, T* __restrict__ dst) {
  const int64_t per = spad * mp;
  GRID_STRIDE(e, nblk * per) {
    const int64_t b = e / per, rem = e - b * per;
    const int64_t f = rem / mp, c = rem - f * mp;
    dst[(b * mp + c) * spad + f] = (T)src[e];
  }
}
}  // namespace

hipError_t to_wop(int prec, const double* src, int64_t nblk, int64_t spad, int64_t mp, void* dst,
                  hipStream_t st) {
  const int64_t count = nblk * spad * mp;
  if (count == 0) return hipSuccess;
  const unsigned g = grid_for(count);
  if (bf16_planes(prec, mp))
    to_wop_bf16_kernel<<<g, 256, 0, st>>>(src, nblk, spad, mp, (uint16_t*)dst);
  else if (prec == BS_PREC_F64)
    to_wop_kernel<double><<<g, 256, 0, st>>>(src, nblk, spad, mp, (double*)dst);
  else
    to_wop_kernel<float><<<g, 256, 0, st>>>(src, nblk, spad, mp, (float*)dst);
  return hipGetLastError();
}

hipError_t scores_out(const double* P, int64_t rows, int64_t m, int64_t mp, float* out,
                      hipStream_t st) {
  if (rows * m == 0) return hipSuccess;
  scores_kernel<<<grid_for(rows * m), 256, 0, st>>>(P, rows, m, mp, out);
  return hipGetLastError();
}

}  // namespace bs
