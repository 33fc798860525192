// libbsadmm host library: the C ABI of include/bsadmm.h.
//
// A handle owns, in HBM: operand copies of X and W (k padded, in the
// arithmetic precision), the cached inverses Q_ij (FP64), the FP64 ADMM
// state of Algorithm 1 and a workspace for the blocks Z_ij of one group of
// row blocks.  One iteration enqueues, on the handle's stream:
//   row_pre, col_pre                      steps 4, 6 (+ operand of step 17)
//   per row-block group:
//     regen (one launch per column block) step 15
//     ztr partial + reduce_rhs            step 17 and the rhs of step 18
//     solve                               step 18 (+ U, step 21)
//     zw                                  step 19 (sums of steps 20, 22)
//   row_post, col_post                    steps 25, 27-29, 33
#include "bsadmm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(BSADMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

inline int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Loss code of the elementwise kernels: 0 squared, 1 hinge (one-vs-all
// included), 2 l1, 3 Crammer-Singer, 4 multinomial logistic.
inline int kernel_loss(int loss) {
  switch (loss) {
    case BSADMM_SQUARED: return 0;
    case BSADMM_L1: return 2;
    case BSADMM_CS_HINGE: return 3;
    case BSADMM_SOFTMAX: return 4;
    default: return 1;
  }
}

constexpr int kMonBlocks = 256;  // partial sums per monitored quantity

// Sizes and layout derived from a problem; computed on the host only.
struct Plan {
  int prec = 0;
  // Refined BF16 (BSADMM_BF16R): the iteration runs the BF16 kernels (prec is
  // BF16) and every refine_every-th iteration also regenerates FP32-faithful
  // features (BF16X3) to refresh the stored defects of the two products.
  bool refine = false;
  int refine_every = 0;
  int fprec = 0;  // feature precision of the objective and of predictions
  int64_t n = 0, d = 0, m = 0, s = 0, mp = 0, Kp = 0, spad = 0, S = 0;
  int R = 1, C = 1;
  std::vector<int64_t> rstart, cstart, coff, sj;
  std::vector<std::pair<int, int>> groups;  // row-block ranges [i0, i1)
  int64_t ws_rows = 0;
  int64_t split_rows = 2048, nsplit_max = 1;
  int64_t nbpad = 0;             // per-block row segment of the transposed BF16 R
  int fac_batch = 1;
  bool keep = false;             // Z generated once and kept (BSADMM_Z_KEEP)
  size_t op = 4, zb = 4, vb = 4;  // operand, stored Z, product-operand bytes
  int planes = 1;
  // byte counts
  size_t b_xp = 0, b_wt = 0, b_bias = 0, b_q = 0, b_ws = 0, b_row = 0, b_rop = 0, b_col = 0,
         b_colR = 0, b_wop = 0, b_part = 0, b_small = 0, b_fac_tmp = 0, b_prev = 0;
  // refined BF16: feature defects (BF16) and FP32-faithful features of a
  // row-block group, and the stored defects of the two products
  size_t b_wsd = 0, b_ca = 0, b_cp = 0, b_feat = 0;
  // operand elements between the W' copies of consecutive row blocks
  int64_t wop_stride() const { return bs::bf16_planes(prec, mp) ? 2 * mp * spad : spad * mp; }
  size_t total() const {
    return b_xp + b_wt + b_bias + b_q + b_ws + 5 * b_row + b_rop + 3 * b_col + 4 * b_colR + b_wop +
           b_part + b_small + b_fac_tmp + b_prev + b_wsd + b_ca + b_cp + b_feat;
  }
};

int validate(const bsadmm_problem* p) {
  if (!p) return fail(BSADMM_EINVAL, "problem is NULL");
  if (p->R < 1 || p->C < 1) return fail(BSADMM_EINVAL, "R and C must be >= 1");
  if (p->n < p->R) return fail(BSADMM_EINVAL, "need n >= R");
  if (p->s < p->C) return fail(BSADMM_EINVAL, "need s >= C");
  if (p->d < 1) return fail(BSADMM_EINVAL, "need d >= 1");
  if (p->m < 1 || p->m > 1024) return fail(BSADMM_EINVAL, "need 1 <= m <= 1024");
  if (p->loss < BSADMM_SQUARED || p->loss > BSADMM_SOFTMAX) return fail(BSADMM_EINVAL, "unknown loss");
  if (p->loss == BSADMM_HINGE && p->m != 1) return fail(BSADMM_EINVAL, "HINGE needs m == 1");
  if ((p->loss == BSADMM_CS_HINGE || p->loss == BSADMM_SOFTMAX) && p->m < 2)
    return fail(BSADMM_EINVAL, "CS_HINGE and SOFTMAX need m >= 2");
  if (p->reg != BSADMM_L2) return fail(BSADMM_EINVAL, "unknown regulariser");
  if (p->precision < BSADMM_FP64 || p->precision > BSADMM_BF16R)
    return fail(BSADMM_EINVAL, "unknown precision");
  if (p->refine_every < 0) return fail(BSADMM_EINVAL, "need refine_every >= 0");
  if (p->refine_every > 0 && p->precision != BSADMM_BF16R)
    return fail(BSADMM_EINVAL, "refine_every applies to BSADMM_BF16R only");
  if (p->z_mode != BSADMM_Z_AUTO && p->z_mode != BSADMM_Z_STORE && p->z_mode != BSADMM_Z_KEEP)
    return fail(BSADMM_EINVAL, "unknown z_mode");
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return fail(BSADMM_EINVAL, "need lambda >= 0");
  if (!(p->rho > 0.0) || !std::isfinite(p->rho)) return fail(BSADMM_EINVAL, "need rho > 0");
  if (!(p->sigma > 0.0) || !std::isfinite(p->sigma)) return fail(BSADMM_EINVAL, "need sigma > 0");
  if (p->rho_adapt_every < 0) return fail(BSADMM_EINVAL, "need rho_adapt_every >= 0");
  if (p->flags & ~BSADMM_F_GRAPH) return fail(BSADMM_EINVAL, "unknown flag bits");
  if (p->rho_adapt_mu != 0.0 && !(p->rho_adapt_mu > 1.0 && std::isfinite(p->rho_adapt_mu)))
    return fail(BSADMM_EINVAL, "rho_adapt_mu must be 0 or finite and > 1");
  if (p->rho_adapt_tau != 0.0 && !(p->rho_adapt_tau > 1.0 && std::isfinite(p->rho_adapt_tau)))
    return fail(BSADMM_EINVAL, "rho_adapt_tau must be 0 or finite and > 1");
  if (!p->X || !p->Y) return fail(BSADMM_EINVAL, "X and Y must be non-NULL");
  if (!p->W != !p->b)
    return fail(BSADMM_EINVAL, "W and b must both be given, or both NULL (drawn from seed)");
  const void* ptrs[4] = {p->X, p->Y, p->W, p->b};
  for (const void* q : ptrs)
    if (reinterpret_cast<uintptr_t>(q) % 16 != 0)
      return fail(BSADMM_EINVAL, "X, Y, W, b must be 16-byte aligned");
  return BSADMM_OK;
}

int make_plan(const bsadmm_problem* p, Plan& L) {
  int rc = validate(p);
  if (rc) return rc;
  L.refine = p->precision == BSADMM_BF16R;
  L.prec = L.refine ? BS_PREC_BF16 : p->precision;
  L.refine_every = L.refine ? (p->refine_every > 0 ? p->refine_every : 5) : 0;
  L.fprec = L.refine ? BS_PREC_BF16X3 : L.prec;
  L.n = p->n; L.d = p->d; L.m = p->m; L.s = p->s; L.R = p->R; L.C = p->C;
  L.mp = rup(L.m, 16);
  L.op = bs::op_bytes(L.prec);
  // refined BF16 keeps X and W as BF16 head and residual planes: the head is
  // the BF16 operand, both planes make the BF16X3 features
  L.planes = L.refine ? 2 : bs::op_planes(L.prec);
  L.zb = bs::z_bytes(L.prec);
  L.vb = bs::vec_bytes(L.prec);
  L.Kp = bs::padded_k(L.prec, L.d);
  L.rstart.resize(L.R + 1);
  for (int i = 0; i <= L.R; ++i) L.rstart[i] = (int64_t)i * L.n / L.R;
  L.cstart.resize(L.C + 1);
  for (int j = 0; j <= L.C; ++j) L.cstart[j] = (int64_t)j * L.s / L.C;
  L.coff.resize(L.C);
  L.sj.resize(L.C);
  int64_t off = 0, smax = 0;
  for (int j = 0; j < L.C; ++j) {
    L.sj[j] = L.cstart[j + 1] - L.cstart[j];
    L.coff[j] = off;
    off += rup(L.sj[j], 64);
    smax = std::max(smax, L.sj[j]);
  }
  L.spad = off;
  L.S = rup(smax, 64);
  // Row-block groups for the Z workspace (one group of all rows when Z is kept).
  L.keep = p->z_mode == BSADMM_Z_KEEP;
  // refined BF16 keeps the BF16 features and their defect (2 + 2 bytes)
  const size_t row_bytes = (size_t)L.spad * (L.refine ? 4 : L.zb);
  if (L.keep && p->workspace_bytes && p->workspace_bytes < (size_t)L.n * row_bytes)
    return fail(BSADMM_ENOMEM, "BSADMM_Z_KEEP needs " + std::to_string((size_t)L.n * row_bytes) +
                                   " B of workspace, workspace_bytes is smaller");
  size_t cap = L.keep ? SIZE_MAX : (p->workspace_bytes ? p->workspace_bytes : (size_t)32 << 30);
  L.groups.clear();
  int i = 0;
  L.ws_rows = 0;
  while (i < L.R) {
    int i1 = i + 1;
    while (i1 < L.R && (size_t)(L.rstart[i1 + 1] - L.rstart[i]) * row_bytes <= cap) ++i1;
    L.groups.push_back({i, i1});
    L.ws_rows = std::max(L.ws_rows, L.rstart[i1] - L.rstart[i]);
    i = i1;
  }
  int64_t nmax = 0;
  for (int r = 0; r < L.R; ++r) nmax = std::max(nmax, L.rstart[r + 1] - L.rstart[r]);
  // Rows per split of the transpose product: at most 2048 (the partial sums
  // of a split, spad x mp, stay small against the Z rows it reads), and fewer
  // for small problems, so that the (spad / 256) x splits workgroups of a
  // launch reach about 1024; at least 256, a multiple of 32.
  {
    const int64_t colg = std::max<int64_t>(1, L.spad / 256);
    const int64_t want = std::max<int64_t>(1, (1024 + colg - 1) / colg);
    L.split_rows = std::min<int64_t>(2048, std::max<int64_t>(256, rup((nmax + want - 1) / want, 32)));
  }
  L.nbpad = rup(nmax, 32) + 32;
  L.nsplit_max = (nmax + L.split_rows - 1) / L.split_rows;
  const size_t slot = (size_t)L.S * L.S * 8;
  const size_t fac_cap = (size_t)4 << 30;
  L.fac_batch = (int)std::max<size_t>(1, std::min<size_t>((size_t)L.R * L.C, fac_cap / slot));
  // a feature map drawn from the seed is kept for bsadmm_get_features
  L.b_feat = p->W ? 0 : ((size_t)L.d * L.s + (size_t)L.s) * 4 + 256;
  L.b_xp = (size_t)L.n * L.Kp * L.op * L.planes;
  L.b_wt = (size_t)L.s * L.Kp * L.op * L.planes;
  L.b_bias = (size_t)L.s * (L.prec == BSADMM_FP64 ? 8 : 4);
  L.b_q = (size_t)L.R * L.C * slot;
  L.b_ws = (size_t)L.ws_rows * L.spad * L.zb;
  if (L.refine) {
    // the defect of the workspace's (or the kept) BF16 features; the
    // FP32-faithful features it comes from are never stored
    L.b_wsd = (size_t)L.ws_rows * L.spad * 2;
    L.b_ca = (size_t)L.R * L.spad * L.mp * 8;
    L.b_cp = (size_t)L.n * L.mp * 8;
  }
  L.b_row = (size_t)L.n * L.mp * 8;
  L.b_rop = bs::bf16_planes(L.prec, L.mp) ? (size_t)2 * L.mp * L.R * L.nbpad * 2
                                  : (size_t)L.n * L.mp * L.vb;
  L.b_col = (size_t)L.spad * L.mp * 8;
  L.b_colR = (size_t)L.R * L.spad * L.mp * 8;
  L.b_wop = (size_t)L.R * L.spad * L.mp * L.vb;
  L.b_part = (size_t)L.R * L.nsplit_max * L.spad * L.mp * L.vb;
  L.b_small = 256 + 2 * (size_t)L.C * 8 + 9 * kMonBlocks * 8 + bs::BS_W_COUNT * 8;
  // copies of O-bar, O, Delta-bar, W-bar, W', U from before a checked
  // iteration, for the dual residual of penalty adaptation
  L.b_prev = p->rho_adapt_every > 0 ? 3 * L.b_row + L.b_col + 2 * L.b_colR : 0;
  L.b_fac_tmp = (size_t)L.fac_batch * (slot + (size_t)L.S * 64 * 8);
  return BSADMM_OK;
}

}  // namespace

struct bsadmm_handle {
  Plan L;
  bsadmm_problem p{};
  hipStream_t st = nullptr;
  double scale = 0;
  double* wts = nullptr;  // device penalty block (bs::BS_W_*)
  double *Obar_prev = nullptr, *Wbar_prev = nullptr, *O_prev = nullptr, *Dbar_prev = nullptr,
         *Wp_prev = nullptr, *U_prev = nullptr;
  std::vector<void*> allocs;
  void *Xp = nullptr, *Wt = nullptr, *bias = nullptr, *Z = nullptr, *Rop = nullptr,
       *Wop = nullptr, *part = nullptr;
  void* Zd = nullptr;  // refined BF16: feature defect bf16(Zf - Z) of the workspace rows
  double *cA = nullptr, *cP = nullptr;  // refined BF16: stored product defects
  double* dualA = nullptr;  // refined BF16 dual bound: defect part of Z^T alpha (lazy)
  float *W_own = nullptr, *b_own = nullptr;  // feature map drawn from the seed (W = b = NULL)
  double *Q = nullptr, *O = nullptr, *Obar = nullptr, *nu = nullptr, *Dbar = nullptr,
         *P = nullptr, *Wbar = nullptr, *mu = nullptr, *Wc = nullptr, *Wp = nullptr,
         *mup = nullptr, *U = nullptr, *rhs = nullptr;
  int64_t *d_coff = nullptr, *d_sj = nullptr;
  double* mon_part = nullptr;
  int* dflag = nullptr;
  int64_t iters = 0;
  bool poisoned = false;
  std::vector<hipEvent_t> evpool;
  // HIP graphs of the iteration (BSADMM_F_GRAPH): one plain and one checked
  // iteration, and a chunk of iterations; captured on `cap`, launched on st.
  hipStream_t cap = nullptr;
  hipGraphExec_t gx_one[4] = {nullptr, nullptr, nullptr, nullptr};  // [checked + 2 refined]
  hipGraphExec_t gx_chunk = nullptr;

  // Stream-ordered allocations on the handle's stream: freeing a handle does
  // not synchronise the device, so other solves keep running.
  hipError_t alloc(void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMallocAsync(ptr, bytes, st);
    if (e == hipSuccess) allocs.push_back(*ptr);
    return e;
  }
  ~bsadmm_handle() {
    for (hipGraphExec_t g : {gx_one[0], gx_one[1], gx_one[2], gx_one[3], gx_chunk})
      if (g) (void)hipGraphExecDestroy(g);
    if (cap) (void)hipStreamDestroy(cap);
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    for (void* a : allocs) (void)hipFreeAsync(a, st);
  }
};

namespace {

#define HCHK(expr)                                        \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);     \
  } while (0)

// Feature regeneration of the rows of row blocks [i0, i1) into a workspace:
// precision `prec` (the handle's, or BF16X3 for the FP32-faithful features
// of refined BF16), `zb` bytes per stored element.
hipError_t regen_group(bsadmm_handle* h, int i0, int i1, hipStream_t s, int prec, void* out,
                       size_t zb) {
  const Plan& L = h->L;
  const int64_t r0 = L.rstart[i0], rows = L.rstart[i1] - r0;
  const size_t bb = L.prec == BSADMM_FP64 ? 8 : 4;
  const int64_t xps = L.n * L.Kp;
  for (int j = 0; j < L.C; ++j) {
    hipError_t e = bs::regen(prec, (const char*)h->Xp + (size_t)r0 * L.Kp * L.op, xps, rows,
                             (const char*)h->Wt + (size_t)L.cstart[j] * L.Kp * L.op, L.s * L.Kp,
                             L.sj[j], (const char*)h->bias + (size_t)L.cstart[j] * bb, L.Kp,
                             h->scale, (char*)out + (size_t)L.coff[j] * zb, L.spad, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t regen_group(bsadmm_handle* h, int i0, int i1, hipStream_t s) {
  return regen_group(h, i0, i1, s, h->L.prec, h->Z, h->L.zb);
}

// Refined BF16: the FP32-faithful (BF16X3) features of the group, formed in
// the regeneration kernel and not stored, and their defect bf16(Zf - Z)
// against the group's BF16 features into Zd.
hipError_t defect_group(bsadmm_handle* h, int i0, int i1, hipStream_t s) {
  const Plan& L = h->L;
  const int64_t r0 = L.rstart[i0], rows = L.rstart[i1] - r0;
  const int64_t xps = L.n * L.Kp;
  for (int j = 0; j < L.C; ++j) {
    hipError_t e = bs::regen_defect(
        (const char*)h->Xp + (size_t)r0 * L.Kp * L.op, xps, rows,
        (const char*)h->Wt + (size_t)L.cstart[j] * L.Kp * L.op, L.s * L.Kp, L.sj[j],
        (const char*)h->bias + (size_t)L.cstart[j] * 4, L.Kp, h->scale,
        (const uint16_t*)h->Z + L.coff[j], (uint16_t*)h->Zd + L.coff[j], L.spad, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct PhaseTimer {
  bsadmm_handle* h;
  bool on;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks{};
  size_t used = 0;
  hipEvent_t get() {
    if (used == h->evpool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      h->evpool.push_back(e);
    }
    return h->evpool[used++];
  }
  hipEvent_t start_ev = nullptr;
  void begin() {
    if (!on) return;
    start_ev = get();
    if (start_ev) (void)hipEventRecord(start_ev, h->st);
  }
  void end(int phase) {
    if (!on || !start_ev) return;
    hipEvent_t e = get();
    if (!e) return;
    (void)hipEventRecord(e, h->st);
    marks.push_back({phase, {start_ev, e}});
    start_ev = nullptr;
  }
};

// Multiply the scaled duals nu, mu, mu' by the device factor wts[BS_W_DUAL].
hipError_t rescale_duals(bsadmm_handle* h, hipStream_t s) {
  const Plan& L = h->L;
  const double* f = h->wts + bs::BS_W_DUAL;
  hipError_t e = bs::scale(h->nu, L.n * L.mp, f, s);
  if (e == hipSuccess) e = bs::scale(h->mu, L.spad * L.mp, f, s);
  if (e == hipSuccess) e = bs::scale(h->mup, (int64_t)L.R * L.spad * L.mp, f, s);
  return e;
}

// New penalty (stream-ordered); with rescale the scaled duals are multiplied
// by rho_old / rho.
hipError_t apply_rho(bsadmm_handle* h, double rho, bool rescale) {
  hipError_t e = bs::set_rho(h->wts, rho, (double)h->L.n * h->p.lambda, rescale ? 1 : 0, h->st);
  if (e == hipSuccess && rescale) e = rescale_duals(h, h->st);
  return e;
}

// F(W) of eq. problem_linear for Wmodel (device s x m FP64) or W-bar: one
// regeneration pass over all rows and one forward product, fixed-order sums.
int objective_of(bsadmm_handle* h, const double* Wmodel, double* F) {
  const Plan& L = h->L;
  hipStream_t st = h->st;
  constexpr int NB = 1024;
  double *wpad = nullptr, *part = nullptr, *pd = nullptr;
  void* wop = nullptr;
  auto cleanup = [&]() {
    if (wpad) (void)hipFreeAsync(wpad, st);
    if (part) (void)hipFreeAsync(part, st);
    if (wop) (void)hipFreeAsync(wop, st);
    if (pd) (void)hipFreeAsync(pd, st);
  };
  if (hipMallocAsync((void**)&wpad, (size_t)L.spad * L.mp * 8, st) != hipSuccess ||
      hipMallocAsync((void**)&part, 2 * NB * 8, st) != hipSuccess ||
      hipMallocAsync(&wop, (size_t)L.spad * L.mp * L.vb, st) != hipSuccess ||
      (L.refine && hipMallocAsync((void**)&pd, (size_t)L.n * L.mp * 8, st) != hipSuccess)) {
    cleanup();
    return fail(BSADMM_ENOMEM, "device allocation failed in objective");
  }
  hipError_t e = hipSuccess;
  if (Wmodel) {
    e = hipMemsetAsync(wpad, 0, (size_t)L.spad * L.mp * 8, st);
    for (int j = 0; j < L.C && e == hipSuccess; ++j)
      e = bs::pad(Wmodel + (size_t)L.cstart[j] * L.m, L.sj[j], L.m, L.mp,
                  wpad + (size_t)L.coff[j] * L.mp, st);
  } else {
    e = hipMemcpyAsync(wpad, h->Wbar, (size_t)L.spad * L.mp * 8, hipMemcpyDeviceToDevice, st);
  }
  if (e == hipSuccess) e = bs::to_wop(L.prec, wpad, 1, L.spad, L.mp, wop, st);
  // forward pass Z W over all rows into the P buffer (free between
  // iterations); refined BF16 adds the product with the feature defect, as
  // its iteration does (BF16 features + defect = FP32-faithful features)
  for (size_t g = 0; g < L.groups.size() && e == hipSuccess; ++g) {
    const int i0 = L.groups[g].first, i1 = L.groups[g].second;
    if (!L.keep) e = regen_group(h, i0, i1, st);
    if (e == hipSuccess && L.refine && !L.keep) e = defect_group(h, i0, i1, st);
    if (e == hipSuccess)
      e = bs::zw(L.prec, h->Z, L.spad, L.n, L.R, i0, i1, L.spad, wop, 0, L.mp, h->P, st);
    if (e == hipSuccess && L.refine)
      e = bs::zw(L.prec, h->Zd, L.spad, L.n, L.R, i0, i1, L.spad, wop, 0, L.mp, pd, st);
  }
  if (e == hipSuccess && L.refine) e = bs::axpy(h->P, pd, L.n * L.mp, st);
  if (e == hipSuccess)
    e = bs::loss_partial(kernel_loss(h->p.loss), h->P, h->p.Y, L.n, L.m, L.mp, part,
                         NB, st);
  if (e == hipSuccess) e = bs::sumsq_partial(wpad, L.spad * L.mp, part + NB, NB, st);
  std::vector<double> hp(2 * NB);
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, 2 * NB * 8, hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "objective");
  }
  if (e2 != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e2, "objective synchronize");
  }
  double loss = 0.0, reg = 0.0;
  for (int k = 0; k < NB; ++k) loss += hp[k];
  for (int k = 0; k < NB; ++k) reg += hp[NB + k];
  *F = loss / (double)L.n + h->p.lambda * reg;
  return BSADMM_OK;
}

// Transpose products Z_ij^T R_i of the row blocks [i0, i1) of a group into
// the split partials; z is the group's feature workspace (the features of
// the handle's precision, or the defect of refined BF16) and R the operand
// buffer as the row step (or the dual bound) wrote it.
hipError_t ztr_rows(bsadmm_handle* h, int i0, int i1, const void* z, hipStream_t s) {
  const Plan& L = h->L;
  const int64_t r0 = L.rstart[i0];
  for (int i = i0; i < i1; ++i) {
    const int64_t ri = L.rstart[i], ni = L.rstart[i + 1] - ri;
    const char* Ri = bs::bf16_planes(L.prec, L.mp)
                         ? (const char*)h->Rop + (size_t)i * L.nbpad * 2
                         : (const char*)h->Rop + (size_t)ri * L.mp * L.vb;
    hipError_t e = bs::ztr_partial(
        L.prec, (const char*)z + (size_t)(ri - r0) * L.spad * L.zb, L.spad, ni, L.spad, Ri,
        (int64_t)L.R * L.nbpad, L.mp, L.split_rows,
        (char*)h->part + (size_t)i * L.nsplit_max * L.spad * L.mp * L.vb, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Enqueue the dual bound on the handle's stream: alpha from the current
// state into the R operand buffer (free between iterations), Z^T alpha over
// every group into rhs (also free between iterations; refined BF16 adds the
// defect product, so the bound is that of the FP32-faithful features), and
// the final sums into out[0..2].
int enqueue_dual_bound(bsadmm_handle* h, int loss, double* out) {
  const Plan& L = h->L;
  const hipStream_t st = h->st;
  const double cfac = 1.0 / (double)(L.C + 1);
  HCHK(bs::dual_rows(L.prec, loss, h->wts, cfac, L.n, L.R, L.m, L.mp, L.nbpad, h->p.Y, h->nu,
                     h->Dbar, h->Rop, h->mon_part, kMonBlocks, st));
  for (const auto& g : L.groups) {
    const int i0 = g.first, i1 = g.second;
    if (!L.keep) HCHK(regen_group(h, i0, i1, st));
    if (L.refine) {
      if (!L.keep) HCHK(defect_group(h, i0, i1, st));
      HCHK(ztr_rows(h, i0, i1, h->Zd, st));
      HCHK(bs::reduce_rhs(L.prec, h->part, L.nsplit_max, L.n, L.R, i0, i1, L.split_rows, L.spad,
                          L.mp, nullptr, nullptr, nullptr, nullptr, h->dualA, st));
    }
    HCHK(ztr_rows(h, i0, i1, h->Z, st));
    HCHK(bs::reduce_rhs(L.prec, h->part, L.nsplit_max, L.n, L.R, i0, i1, L.split_rows, L.spad,
                        L.mp, nullptr, nullptr, nullptr, L.refine ? h->dualA : nullptr, h->rhs,
                        st));
  }
  HCHK(bs::dual_final(h->rhs, L.R, L.spad * L.mp, L.n, h->p.lambda, h->mon_part, kMonBlocks, out,
                      st));
  return BSADMM_OK;
}

// Whether iteration number `k` (1-based over the handle's life) ends with a
// residual-balancing check.
inline bool checked_iteration(const bsadmm_handle* h, int64_t k) {
  const int every = h->p.rho_adapt_every;
  return every > 0 && k % every == 0;
}

// Whether iteration `k` refreshes the product defects of refined BF16: the
// first one and every refine_every-th after it.
inline bool refined_iteration(const bsadmm_handle* h, int64_t k) {
  return h->L.refine && (k - 1) % h->L.refine_every == 0;
}

// Enqueue one iteration on stream `s` (the handle's stream, or the capture
// stream of a HIP graph; then tm is null: no events are recorded).
int enqueue_iteration(bsadmm_handle* h, hipStream_t s, bool check, bool refine, bool want_res,
                      PhaseTimer* tm, int& launches) {
  const Plan& L = h->L;
  const double cfac = 1.0 / (double)(L.C + 1);
  const double amu = h->p.rho_adapt_mu > 0.0 ? h->p.rho_adapt_mu : 10.0;
  const double atau = h->p.rho_adapt_tau > 0.0 ? h->p.rho_adapt_tau : 2.0;
  const hipStream_t st = s;
  auto begin = [&]() { if (tm) tm->begin(); };
  auto end = [&](int ph) { if (tm) tm->end(ph); };
  if (check || want_res) {  // the state before this iteration, for the dual residual
    const int64_t rowc = L.n * L.mp, colc = L.spad * L.mp, colRc = (int64_t)L.R * colc;
    HCHK(bs::copy(h->Obar_prev, h->Obar, rowc, s));
    HCHK(bs::copy(h->O_prev, h->O, rowc, s));
    HCHK(bs::copy(h->Dbar_prev, h->Dbar, rowc, s));
    HCHK(bs::copy(h->Wbar_prev, h->Wbar, colc, s));
    HCHK(bs::copy(h->Wp_prev, h->Wp, colRc, s));
    HCHK(bs::copy(h->U_prev, h->U, colRc, s));
  }
  begin();
  HCHK(bs::row_pre(L.prec, kernel_loss(h->p.loss), h->wts, cfac, L.n, L.R, L.m, L.mp, L.nbpad,
                   h->p.Y, h->Obar, h->nu, h->Dbar, h->O, h->Rop, s));
  end(BSADMM_PH_ROW);
  begin();
  HCHK(bs::col_pre(h->wts, L.spad, L.m, L.mp, h->Wbar, h->mu, h->Wc, s));
  end(BSADMM_PH_COL);
  for (const auto& g : L.groups) {
    const int i0 = g.first, i1 = g.second;
    if (!L.keep) {  // a kept Z was generated at setup
      begin();
      HCHK(regen_group(h, i0, i1, st));
      launches += L.C;
      end(BSADMM_PH_REGEN);
    }
    auto ztr_group = [&](const void* z) { return ztr_rows(h, i0, i1, z, s); };
    if (refine) {
      // Refinement of the projection's products: FP32-faithful features of
      // the group, their defect against the BF16 features, and the defects
      // of both products, kept for the BF16 iterations until the next
      // refinement: cA_i = dZ_ij^T R_i, cP_i = sum_j dZ_ij W'_ij.
      begin();
      if (!L.keep) HCHK(defect_group(h, i0, i1, st));
      HCHK(ztr_group(h->Zd));
      HCHK(bs::reduce_rhs(L.prec, h->part, L.nsplit_max, L.n, L.R, i0, i1, L.split_rows, L.spad,
                          L.mp, nullptr, nullptr, nullptr, nullptr, h->cA, s));
      end(BSADMM_PH_REFINE);
    }
    begin();
    HCHK(ztr_group(h->Z));
    HCHK(bs::reduce_rhs(L.prec, h->part, L.nsplit_max, L.n, L.R, i0, i1, L.split_rows, L.spad,
                        L.mp, h->Wbar, h->mup, h->U, L.refine ? h->cA : nullptr, h->rhs, s));
    end(BSADMM_PH_ZTR);
    begin();
    HCHK(bs::solve(L.prec, h->Q, L.S, L.C, i0 * L.C, (i1 - i0) * L.C, h->d_coff, h->d_sj, L.spad,
                   L.mp, h->rhs, h->Wp, h->U, h->Wop, s));
    end(BSADMM_PH_SOLVE);
    if (refine) {
      begin();
      HCHK(bs::zw(L.prec, h->Zd, L.spad, L.n, L.R, i0, i1, L.spad, h->Wop, L.wop_stride(), L.mp,
                  h->cP, s));
      end(BSADMM_PH_REFINE);
    }
    begin();
    HCHK(bs::zw(L.prec, h->Z, L.spad, L.n, L.R, i0, i1, L.spad, h->Wop, L.wop_stride(), L.mp, h->P,
                s));
    end(BSADMM_PH_ZW);
  }
  begin();
  HCHK(bs::row_post(L.n, L.m, L.mp, L.C, h->O, h->P, L.refine ? h->cP : nullptr, h->Obar, h->nu,
                    h->Dbar, s));
  end(BSADMM_PH_ROW);
  begin();
  HCHK(bs::col_post(L.R, L.spad, L.m, L.mp, h->Wc, h->Wp, h->Wbar, h->mu, h->mup, s));
  end(BSADMM_PH_COL);
  if (check || want_res) {
    double* sums = h->mon_part + 8 * kMonBlocks;
    const bs::ResidualArgs ra{h->Dbar,    h->Wc,      h->Wp,        h->Wbar,      h->Obar,
                              h->O,       h->U,       h->Obar_prev, h->Wbar_prev, h->Wp_prev,
                              h->O_prev,  h->Dbar_prev, h->U_prev};
    HCHK(bs::residuals(ra, L.R, L.n, L.spad, L.m, L.mp, h->mon_part, kMonBlocks, sums, s));
    // norms at the penalty of this iteration, before a balancing step changes it
    if (want_res) HCHK(bs::residual_norms(sums, h->wts, L.R, L.C, sums + 8, s));
    if (check) {  // residual balancing, decided on the device (no read-back)
      HCHK(bs::adapt(sums, h->wts, L.R, L.C, (double)L.n * h->p.lambda, amu, atau, s));
      HCHK(rescale_duals(h, s));
    }
  }
  return BSADMM_OK;
}

// Capture `count` iterations, the first of which is iteration k0 + 1 of the
// handle's life, into an executable HIP graph (kernel nodes only).
int capture_iterations(bsadmm_handle* h, int count, int64_t k0, hipGraphExec_t* out) {
  *out = nullptr;
  if (!h->cap) HCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  HCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  int launches = 0, rc = BSADMM_OK;
  for (int t = 0; t < count && rc == BSADMM_OK; ++t)
    rc = enqueue_iteration(h, h->cap, checked_iteration(h, k0 + t + 1),
                           refined_iteration(h, k0 + t + 1), false, nullptr, launches);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap, &g);
  if (rc != BSADMM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return BSADMM_OK;
}

// Iterations by graph replay: chunks of `chunk` iterations (one adaptation
// period, or 16 without adaptation) where the count and alignment allow,
// single iterations (plain or checked) otherwise.
int replay_iterations(bsadmm_handle* h, int iters, int& launches) {
  const Plan& L = h->L;
  const int every = h->p.rho_adapt_every;
  // no chunks under refinement: its period and the adaptation period would
  // have to be aligned
  const int chunk = L.refine ? 0 : (every > 0 ? (every <= 64 ? every : 0) : 16);
  const int per_iter = L.keep ? 0 : L.C * (int)L.groups.size();
  int it = 0;
  while (it < iters) {
    const int64_t k0 = h->iters + it;
    const bool aligned = every > 0 ? k0 % every == 0 : true;
    hipGraphExec_t* gx;
    int count;
    if (chunk > 1 && aligned && iters - it >= chunk) {
      gx = &h->gx_chunk;
      count = chunk;
    } else {
      gx = &h->gx_one[(checked_iteration(h, k0 + 1) ? 1 : 0) +
                      (refined_iteration(h, k0 + 1) ? 2 : 0)];
      count = 1;
    }
    if (!*gx) {
      int rc = capture_iterations(h, count, k0, gx);
      if (rc) return rc;
    }
    HCHK(hipGraphLaunch(*gx, h->st));
    it += count;
    launches += count * per_iter;
  }
  return BSADMM_OK;
}

int run_iterations(bsadmm_handle* h, int iters, bsadmm_stats* st) {
  PhaseTimer tm{h, st && st->timed != 0};
  hipEvent_t all0 = nullptr, all1 = nullptr;
  if (st) {
    all0 = tm.get();
    all1 = tm.get();
    if (all0) HCHK(hipEventRecord(all0, h->st));
  }
  int launches = 0;
  const bool want_res = st && (st->want & BSADMM_WANT_RESIDUALS) && iters > 0;
  if (want_res && !h->Obar_prev) {  // state copies, allocated on first request
    const Plan& L = h->L;
    for (auto pr : {std::make_pair(&h->Obar_prev, L.b_row), std::make_pair(&h->O_prev, L.b_row),
                    std::make_pair(&h->Dbar_prev, L.b_row), std::make_pair(&h->Wbar_prev, L.b_col),
                    std::make_pair(&h->Wp_prev, L.b_colR), std::make_pair(&h->U_prev, L.b_colR)})
      if (h->alloc((void**)pr.first, pr.second) != hipSuccess)
        return fail(BSADMM_ENOMEM, "device allocation failed for the residual copies");
  }
  // with residuals asked for, the last iteration runs eagerly and reports them
  const int bulk = want_res ? iters - 1 : iters;
  if ((h->p.flags & BSADMM_F_GRAPH) && !tm.on) {
    int rc = replay_iterations(h, bulk, launches);
    if (rc) return rc;
    h->iters += bulk;
  } else {
    for (int it = 0; it < bulk; ++it) {
      int rc = enqueue_iteration(h, h->st, checked_iteration(h, h->iters + 1),
                                 refined_iteration(h, h->iters + 1), false, &tm, launches);
      if (rc) return rc;
      h->iters += 1;
    }
  }
  if (want_res) {
    int rc = enqueue_iteration(h, h->st, checked_iteration(h, h->iters + 1),
                               refined_iteration(h, h->iters + 1), true, &tm, launches);
    if (rc) return rc;
    h->iters += 1;
  }
  if (st) {
    if (all1) HCHK(hipEventRecord(all1, h->st));
    HCHK(hipStreamSynchronize(h->st));
    for (int k = 0; k < BSADMM_PH_COUNT; ++k) st->phase_ms[k] = 0.0;
    for (auto& mk : tm.marks) {
      float ms = 0.f;
      HCHK(hipEventElapsedTime(&ms, mk.second.first, mk.second.second));
      st->phase_ms[mk.first] += ms;
    }
    float all = 0.f;
    if (all0 && all1) HCHK(hipEventElapsedTime(&all, all0, all1));
    st->iterate_ms = all;
    st->launches = launches;
    double w[bs::BS_W_COUNT];
    HCHK(hipMemcpy(w, h->wts, sizeof w, hipMemcpyDeviceToHost));
    st->rho = w[bs::BS_W_RHO];
    st->rho_changes = (int32_t)w[bs::BS_W_CHANGES];
    st->iters_done = h->iters;
    st->objective = 0.0;
    if (st->want & BSADMM_WANT_OBJECTIVE) {
      int rc = objective_of(h, nullptr, &st->objective);
      if (rc) return rc;
    }
    st->r_primal = st->r_dual = 0.0;
    if (want_res) {
      double rs[2];
      HCHK(hipMemcpy(rs, h->mon_part + 8 * kMonBlocks + 8, sizeof rs, hipMemcpyDeviceToHost));
      st->r_primal = rs[0];
      st->r_dual = rs[1];
    }
  }
  return BSADMM_OK;
}

int do_setup(bsadmm_handle* h) {
  Plan& L = h->L;
  const bsadmm_problem& p = h->p;
  h->st = (hipStream_t)p.stream;
  h->scale = std::sqrt(2.0 / (double)L.s);

  void* tmp = nullptr;
#define ALLOC(ptr, bytes)                                                         \
  do {                                                                            \
    hipError_t e_ = h->alloc((void**)&(ptr), (bytes));                            \
    if (e_ != hipSuccess) return fail(BSADMM_ENOMEM, "device allocation failed for " #ptr); \
  } while (0)
  ALLOC(h->Xp, L.b_xp);
  ALLOC(h->Wt, L.b_wt);
  ALLOC(h->bias, L.b_bias);
  ALLOC(h->Q, L.b_q);
  ALLOC(h->Z, L.b_ws);
  ALLOC(h->O, L.b_row);
  ALLOC(h->Obar, L.b_row);
  ALLOC(h->nu, L.b_row);
  ALLOC(h->Dbar, L.b_row);
  ALLOC(h->P, L.b_row);
  ALLOC(h->Rop, L.b_rop);
  ALLOC(h->Wbar, L.b_col);
  ALLOC(h->mu, L.b_col);
  ALLOC(h->Wc, L.b_col);
  ALLOC(h->Wp, L.b_colR);
  ALLOC(h->mup, L.b_colR);
  ALLOC(h->U, L.b_colR);
  ALLOC(h->rhs, L.b_colR);
  ALLOC(h->Wop, L.b_wop);
  ALLOC(h->part, L.b_part);
  if (L.refine) {
    ALLOC(h->Zd, L.b_wsd);
    ALLOC(h->cA, L.b_ca);
    ALLOC(h->cP, L.b_cp);
  }
  if (L.b_prev) {
    ALLOC(h->Obar_prev, L.b_row);
    ALLOC(h->O_prev, L.b_row);
    ALLOC(h->Dbar_prev, L.b_row);
    ALLOC(h->Wbar_prev, L.b_col);
    ALLOC(h->Wp_prev, L.b_colR);
    ALLOC(h->U_prev, L.b_colR);
  }
  ALLOC(tmp, L.b_small);
  h->dflag = (int*)tmp;
  h->d_coff = (int64_t*)((char*)tmp + 256);
  h->d_sj = h->d_coff + L.C;
  h->mon_part = (double*)(h->d_sj + L.C);
  h->wts = h->mon_part + 9 * kMonBlocks;
  hipStream_t st = h->st;
  HCHK(hipMemcpyAsync(h->d_coff, L.coff.data(), L.C * 8, hipMemcpyHostToDevice, st));
  HCHK(hipMemcpyAsync(h->d_sj, L.sj.data(), L.C * 8, hipMemcpyHostToDevice, st));
  HCHK(hipMemsetAsync(h->dflag, 0, 256, st));
  HCHK(hipMemsetAsync(h->wts, 0, bs::BS_W_COUNT * 8, st));
  // n F(W) scaling of the penalty: loss prox weight 1/rho, regulariser n lambda / rho
  HCHK(apply_rho(h, p.rho, false));
  for (void* z : {(void*)h->O, (void*)h->Obar, (void*)h->nu, (void*)h->Dbar, (void*)h->P})
    HCHK(hipMemsetAsync(z, 0, L.b_row, st));
  HCHK(hipMemsetAsync(h->Rop, 0, L.b_rop, st));
  for (void* z : {(void*)h->Wbar, (void*)h->mu, (void*)h->Wc})
    HCHK(hipMemsetAsync(z, 0, L.b_col, st));
  for (void* z : {(void*)h->Wp, (void*)h->mup, (void*)h->U, (void*)h->rhs})
    HCHK(hipMemsetAsync(z, 0, L.b_colR, st));
  HCHK(hipMemsetAsync(h->Wop, 0, L.b_wop, st));
  HCHK(hipMemsetAsync(h->Z, 0, L.b_ws, st));
  if (L.refine) {  // pad columns of the workspaces stay zero
    HCHK(hipMemsetAsync(h->Zd, 0, L.b_wsd, st));
    HCHK(hipMemsetAsync(h->cA, 0, L.b_ca, st));
    HCHK(hipMemsetAsync(h->cP, 0, L.b_cp, st));
  }
  // the feature map from the seed when W = b = NULL (the random draw of the
  // section on randomized kernel maps), kept for bsadmm_get_features
  if (!p.W) {
    void* feat = nullptr;
    ALLOC(feat, L.b_feat);
    h->W_own = (float*)feat;
    h->b_own = h->W_own + ((L.d * L.s + 63) / 64) * 64;
    HCHK(bs::draw_features(p.seed, L.d, L.s, p.sigma, h->W_own, h->b_own, st));
    h->p.W = h->W_own;
    h->p.b = h->b_own;
  }
  // operands and input checks (refined BF16: BF16 head and residual planes,
  // the head being the BF16 operand)
  const int pprec = L.refine ? BS_PREC_BF16X3 : L.prec;
  HCHK(bs::prep_rows(pprec, p.X, L.n, L.d, L.Kp, h->Xp, L.n * L.Kp, h->dflag, st));
  HCHK(bs::prep_w(pprec, p.W, p.b, L.d, L.s, L.Kp, h->Wt, L.s * L.Kp, h->bias, h->dflag, st));
  HCHK(bs::check_finite(p.Y, L.n * L.m, h->dflag, st));
  int flag = 0;
  HCHK(hipMemcpyAsync(&flag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  HCHK(hipStreamSynchronize(st));
  if (flag & 1) return fail(BSADMM_ENONFINITE, "X, Y, W or b holds NaN or Inf");
  if (p.loss != BSADMM_SQUARED && p.loss != BSADMM_L1) {
    // target encodings, checked on a host copy of Y: +-1 for the hinge
    // losses, one-hot rows for the two multiclass losses with a class index
    std::vector<float> y((size_t)L.n * L.m);
    HCHK(hipMemcpyAsync(y.data(), p.Y, y.size() * 4, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    if (p.loss == BSADMM_HINGE || p.loss == BSADMM_MC_HINGE) {
      for (float v : y)
        if (v != 1.0f && v != -1.0f) return fail(BSADMM_EINVAL, "hinge targets must be +1 or -1");
    } else {
      for (int64_t r = 0; r < L.n; ++r) {
        int ones = 0;
        for (int64_t k = 0; k < L.m; ++k) {
          const float v = y[(size_t)r * L.m + k];
          if (v == 1.0f) ++ones;
          else if (v != 0.0f) ones = 2;
        }
        if (ones != 1)
          return fail(BSADMM_EINVAL, "CS_HINGE / SOFTMAX targets must be one-hot rows");
      }
    }
  }
  // Gram blocks and the FP64 inverse cache (eq. cache)
  const size_t slot = (size_t)L.S * L.S;
  // Refined BF16 builds the cache from its BF16 features, as plain BF16 does
  // (the refinement corrects the products through that same factor); a kept
  // Z also keeps its defect, formed here.
  int grc = BSADMM_OK;
  for (const auto& g : L.groups) {
    const int i0 = g.first, i1 = g.second;
    const int64_t r0 = L.rstart[i0];
    hipError_t e = regen_group(h, i0, i1, st);
    if (e == hipSuccess && L.refine && L.keep) e = defect_group(h, i0, i1, st);
    for (int i = i0; i < i1 && e == hipSuccess; ++i)
      for (int j = 0; j < L.C && e == hipSuccess; ++j)
        e = bs::gram(L.prec, (const char*)h->Z + (size_t)(L.rstart[i] - r0) * L.spad * L.zb,
                     L.spad, L.rstart[i + 1] - L.rstart[i], L.coff[j], L.sj[j],
                     h->Q + (size_t)(i * L.C + j) * slot, L.S, st);
    if (e != hipSuccess) {
      grc = hip_fail(e, "setup Gram");
      break;
    }
  }
  if (grc) return grc;
  std::vector<int64_t> sjb((size_t)L.R * L.C);
  for (int i = 0; i < L.R; ++i)
    for (int j = 0; j < L.C; ++j) sjb[(size_t)i * L.C + j] = L.sj[j];
  HCHK(bs::identity_pad(h->Q, L.R * L.C, L.S, sjb.data(), st));
  double* work = nullptr;
  {
    hipError_t e = hipMallocAsync((void**)&work, L.b_fac_tmp, st);
    if (e != hipSuccess) return fail(BSADMM_ENOMEM, "device allocation failed for the factor workspace");
  }
  double* dinv = work + (size_t)L.fac_batch * slot;
  int rc = BSADMM_OK;
  for (int b0 = 0; b0 < L.R * L.C && rc == BSADMM_OK; b0 += L.fac_batch) {
    const int nb = std::min(L.fac_batch, L.R * L.C - b0);
    hipError_t e = bs::spd_inverse(h->Q + (size_t)b0 * slot, nb, L.S, work, dinv, h->dflag, st);
    if (e != hipSuccess) rc = hip_fail(e, "spd_inverse");
  }
  hipError_t e1 = hipMemcpyAsync(&flag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFreeAsync(work, st);
  if (rc) return rc;
  if (e1 != hipSuccess) return hip_fail(e1, "flag copy");
  if (e2 != hipSuccess) return hip_fail(e2, "setup synchronize");
  if (flag & 2) return fail(BSADMM_ENOTPD, "Cholesky pivot of I + Z^T Z not positive");
  return BSADMM_OK;
}

// Which array, its rows and whether it is row-side (n), column-side (s) or
// per-row-block column-side (R x s).
struct StateRef {
  double* ptr;
  int kind;  // 0: n x m, 1: s x m, 2: R x s x m, 3: {rho, iterations} on the host
};

StateRef state_ref(const bsadmm_handle* h, int which) {
  switch (which) {
    case BSADMM_ST_O: return {h->O, 0};
    case BSADMM_ST_OBAR: return {h->Obar, 0};
    case BSADMM_ST_NU: return {h->nu, 0};
    case BSADMM_ST_DBAR: return {h->Dbar, 0};
    case BSADMM_ST_WC: return {h->Wc, 1};
    case BSADMM_ST_WBAR: return {h->Wbar, 1};
    case BSADMM_ST_MU: return {h->mu, 1};
    case BSADMM_ST_WP: return {h->Wp, 2};
    case BSADMM_ST_MUP: return {h->mup, 2};
    case BSADMM_ST_U: return {h->U, 2};
    case BSADMM_ST_META: return {h->wts, 3};
    // refined BF16 only (null otherwise): the stored product defects
    case BSADMM_ST_DEFECT_A: return {h->cA, 2};
    case BSADMM_ST_DEFECT_P: return {h->cP, 0};
    default: return {nullptr, -1};
  }
}

int copy_state(const bsadmm_handle* h, int which, double* dense, bool to_dense) {
  const Plan& L = h->L;
  StateRef s = state_ref(h, which);
  if (!s.ptr)
    return fail(BSADMM_EINVAL, (which == BSADMM_ST_DEFECT_A || which == BSADMM_ST_DEFECT_P)
                                   ? "product defects exist for BSADMM_BF16R handles only"
                                   : "unknown state array");
  hipStream_t st = h->st;
  if (s.kind == 3) {  // {rho, iterations}: small synchronous copies
    double meta[2];
    HCHK(hipStreamSynchronize(st));
    if (to_dense) {
      HCHK(hipMemcpy(meta, h->wts + bs::BS_W_RHO, 8, hipMemcpyDeviceToHost));
      meta[1] = (double)h->iters;
      HCHK(hipMemcpy(dense, meta, sizeof meta, hipMemcpyHostToDevice));
      return BSADMM_OK;
    }
    HCHK(hipMemcpy(meta, dense, sizeof meta, hipMemcpyDeviceToHost));
    if (!(meta[0] > 0.0) || !std::isfinite(meta[0]) || !(meta[1] >= 0.0) ||
        meta[1] != std::floor(meta[1]))
      return fail(BSADMM_EINVAL, "META needs rho > 0 and a whole iteration count >= 0");
    bsadmm_handle* hm = const_cast<bsadmm_handle*>(h);
    HCHK(apply_rho(hm, meta[0], false));
    HCHK(hipStreamSynchronize(st));
    hm->iters = (int64_t)meta[1];
    return BSADMM_OK;
  }
  auto mv = [&](double* padded, int64_t rows, double* dn) -> hipError_t {
    return to_dense ? bs::unpad(padded, rows, L.m, L.mp, dn, st)
                    : bs::pad(dn, rows, L.m, L.mp, padded, st);
  };
  if (s.kind == 0) {
    HCHK(mv(s.ptr, L.n, dense));
  } else {
    const int reps = s.kind == 1 ? 1 : L.R;
    for (int i = 0; i < reps; ++i)
      for (int j = 0; j < L.C; ++j)
        HCHK(mv(s.ptr + ((size_t)i * L.spad + L.coff[j]) * L.mp, L.sj[j],
                dense + ((size_t)i * L.s + L.cstart[j]) * L.m));
  }
  if (!to_dense && which == BSADMM_ST_WP) {
    // keep the operand copy of W' in step with the imported state
    HCHK(bs::to_wop(L.prec, h->Wp, L.R, L.spad, L.mp, h->Wop, st));
  }
  HCHK(hipStreamSynchronize(st));
  return BSADMM_OK;
}

// ---------------------------------------------------------------------------
// Scratch of rff_map_noalloc: the operand staging that rff_map allocates per
// call (W and b in the operand layout, a chunk of X rows) lives here instead.
// Each GPU the library runs on holds its own copy until the process ends.  In
// host code `scratch` only names the symbol: its device address on the
// current device comes from hipGetSymbolAddress, looked up once per device on
// the first call there and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(void** out) {
  int dev = -1;
  HCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(BSADMM_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(BSADMM_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BSADMM_OK;
}

}  // namespace

extern "C" {

const char* bsadmm_last_error(void) { return g_err.c_str(); }

int bsadmm_validate(const bsadmm_problem* p) {
  g_err.clear();
  return validate(p);
}

int bsadmm_footprint(const bsadmm_problem* p, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(BSADMM_EINVAL, "bytes is NULL");
  Plan L;
  int rc = make_plan(p, L);
  if (rc) return rc;
  *bytes = L.total();
  return BSADMM_OK;
}

int bsadmm_setup(const bsadmm_problem* p, bsadmm_handle** out) {
  g_err.clear();
  if (!out) return fail(BSADMM_EINVAL, "out is NULL");
  *out = nullptr;
  Plan L;
  int rc = make_plan(p, L);
  if (rc) return rc;
  if (p->hbm_budget_bytes && L.total() > p->hbm_budget_bytes)
    return fail(BSADMM_ENOMEM, "footprint " + std::to_string(L.total()) + " B exceeds budget " +
                                   std::to_string(p->hbm_budget_bytes) + " B");
  bsadmm_handle* h = new (std::nothrow) bsadmm_handle();
  if (!h) return fail(BSADMM_ENOMEM, "host allocation failed");
  h->L = L;
  h->p = *p;
  rc = do_setup(h);
  if (rc) {
    std::string msg = g_err;
    (void)hipStreamSynchronize(h->st);
    delete h;
    g_err = msg;
    return rc;
  }
  *out = h;
  return BSADMM_OK;
}

int bsadmm_iterate(bsadmm_handle* h, int32_t iters, bsadmm_stats* st) {
  g_err.clear();
  if (!h) return fail(BSADMM_EINVAL, "handle is NULL");
  if (iters < 0) return fail(BSADMM_EINVAL, "iters must be >= 0");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  int rc = run_iterations(h, iters, st);
  if (rc == BSADMM_EDEVICE) h->poisoned = true;
  return rc;
}

int bsadmm_set_rho(bsadmm_handle* h, double rho, int32_t rescale_duals) {
  g_err.clear();
  if (!h) return fail(BSADMM_EINVAL, "handle is NULL");
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(BSADMM_EINVAL, "need rho > 0 and finite");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  hipError_t e = apply_rho(h, rho, rescale_duals != 0);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "set_rho");
  }
  return BSADMM_OK;
}

int bsadmm_get_coef(const bsadmm_handle* h, double* Wbar) {
  g_err.clear();
  if (!h || !Wbar) return fail(BSADMM_EINVAL, "NULL argument");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  return copy_state(h, BSADMM_ST_WBAR, Wbar, true);
}

int bsadmm_state_size(const bsadmm_handle* h, int32_t which, int64_t* count) {
  g_err.clear();
  if (!h || !count) return fail(BSADMM_EINVAL, "NULL argument");
  StateRef s = state_ref(h, which);
  if (!s.ptr)
    return fail(BSADMM_EINVAL, (which == BSADMM_ST_DEFECT_A || which == BSADMM_ST_DEFECT_P)
                                   ? "product defects exist for BSADMM_BF16R handles only"
                                   : "unknown state array");
  const Plan& L = h->L;
  *count = s.kind == 0 ? L.n * L.m
                       : (s.kind == 1 ? L.s * L.m : (s.kind == 2 ? (int64_t)L.R * L.s * L.m : 2));
  return BSADMM_OK;
}

int bsadmm_export_state(const bsadmm_handle* h, int32_t which, double* dst) {
  g_err.clear();
  if (!h || !dst) return fail(BSADMM_EINVAL, "NULL argument");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  return copy_state(h, which, dst, true);
}

int bsadmm_import_state(bsadmm_handle* h, int32_t which, const double* src) {
  g_err.clear();
  if (!h || !src) return fail(BSADMM_EINVAL, "NULL argument");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  return copy_state(h, which, const_cast<double*>(src), false);
}

int bsadmm_predict(bsadmm_handle* h, const float* Xt, int64_t nt, float* out, void* stream) {
  g_err.clear();
  if (!h) return fail(BSADMM_EINVAL, "handle is NULL");
  if (nt < 0) return fail(BSADMM_EINVAL, "nt must be >= 0");
  if (nt > 0 && (!Xt || !out)) return fail(BSADMM_EINVAL, "Xt and out must be non-NULL");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  if (nt == 0) return BSADMM_OK;
  const Plan& L = h->L;
  hipStream_t st = stream ? (hipStream_t)stream : h->st;
  if (st != h->st) {
    // order after the handle's pending work
    hipEvent_t e;
    HCHK(hipEventCreate(&e));
    HCHK(hipEventRecord(e, h->st));
    HCHK(hipStreamWaitEvent(st, e, 0));
    (void)hipEventDestroy(e);
  }
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nt, std::min<int64_t>(L.ws_rows, 65536)));
  void *xop = nullptr, *wop = nullptr, *zt = nullptr;
  double* pbuf = nullptr;
  auto cleanup = [&]() {
    if (xop) (void)hipFreeAsync(xop, st);
    if (wop) (void)hipFreeAsync(wop, st);
    if (zt) (void)hipFreeAsync(zt, st);
    if (pbuf) (void)hipFreeAsync(pbuf, st);
  };
  // own feature buffer: the handle's workspace may hold a kept Z
  // refined BF16 predicts with its FP32-faithful (BF16X3) features
  const int fp = L.fprec;
  const size_t fzb = bs::z_bytes(fp), fvb = bs::vec_bytes(fp);
  if (hipMallocAsync(&xop, (size_t)chunk * L.Kp * bs::op_bytes(fp) * bs::op_planes(fp), st) !=
          hipSuccess ||
      hipMallocAsync(&wop, (size_t)L.spad * L.mp * fvb, st) != hipSuccess ||
      hipMallocAsync(&zt, (size_t)chunk * L.spad * fzb, st) != hipSuccess ||
      hipMallocAsync((void**)&pbuf, (size_t)chunk * L.mp * 8, st) != hipSuccess) {
    cleanup();
    return fail(BSADMM_ENOMEM, "device allocation failed in predict");
  }
  const size_t bb = L.prec == BSADMM_FP64 ? 8 : 4;
  hipError_t e = hipMemsetAsync(zt, 0, (size_t)chunk * L.spad * fzb, st);  // pad columns
  if (e == hipSuccess) e = bs::to_wop(fp, h->Wbar, 1, L.spad, L.mp, wop, st);
  for (int64_t r0 = 0; r0 < nt && e == hipSuccess; r0 += chunk) {
    const int64_t rows = std::min(chunk, nt - r0);
    e = bs::prep_rows(fp, Xt + r0 * L.d, rows, L.d, L.Kp, xop, chunk * L.Kp, nullptr, st);
    for (int j = 0; j < L.C && e == hipSuccess; ++j)
      e = bs::regen(fp, xop, chunk * L.Kp, rows,
                    (const char*)h->Wt + (size_t)L.cstart[j] * L.Kp * L.op, L.s * L.Kp, L.sj[j],
                    (const char*)h->bias + (size_t)L.cstart[j] * bb, L.Kp, h->scale,
                    (char*)zt + (size_t)L.coff[j] * fzb, L.spad, st);
    if (e == hipSuccess) e = bs::zw(fp, zt, L.spad, rows, 1, 0, 1, L.spad, wop, 0, L.mp, pbuf, st);
    if (e == hipSuccess) e = bs::scores_out(pbuf, rows, L.m, L.mp, out + r0 * L.m, st);
  }
  hipError_t e2 = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "predict");
  if (e2 != hipSuccess) return hip_fail(e2, "predict synchronize");
  if (st != h->st) HCHK(hipStreamSynchronize(h->st));
  return BSADMM_OK;
}

int bsadmm_monitor(bsadmm_handle* h, double* out) {
  g_err.clear();
  if (!h || !out) return fail(BSADMM_EINVAL, "NULL argument");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  const Plan& L = h->L;
  hipError_t e = bs::monitor(kernel_loss(h->p.loss), h->P, h->p.Y, h->Wp, h->Wbar,
                             h->Dbar, L.R, L.n, L.spad, L.m, L.mp, h->mon_part, kMonBlocks, out,
                             h->st);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "monitor");
  }
  return BSADMM_OK;
}

int bsadmm_dual_bound(bsadmm_handle* h, double* out) {
  g_err.clear();
  if (!h || !out) return fail(BSADMM_EINVAL, "NULL argument");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  const int loss = kernel_loss(h->p.loss);
  if (h->p.loss != BSADMM_SQUARED && h->p.loss != BSADMM_HINGE && h->p.loss != BSADMM_MC_HINGE)
    return fail(BSADMM_EINVAL, "dual bound: squared, hinge and one-vs-all hinge losses only");
  const Plan& L = h->L;
  if (L.refine && !h->dualA) {
    if (h->alloc((void**)&h->dualA, (size_t)L.R * L.spad * L.mp * 8) != hipSuccess)
      return fail(BSADMM_ENOMEM, "device allocation failed in dual bound");
  }
  const int rc = enqueue_dual_bound(h, loss, out);
  if (rc != BSADMM_OK) h->poisoned = true;
  return rc;
}

int bsadmm_get_features(const bsadmm_handle* h, float* W, float* b) {
  g_err.clear();
  if (!h || !W || !b) return fail(BSADMM_EINVAL, "NULL argument");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  if (!h->W_own) return fail(BSADMM_EINVAL, "W and b were given at setup, not drawn from the seed");
  const Plan& L = h->L;
  hipError_t e = hipMemcpyAsync(W, h->W_own, (size_t)L.d * L.s * 4, hipMemcpyDeviceToDevice, h->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b, h->b_own, (size_t)L.s * 4, hipMemcpyDeviceToDevice, h->st);
  if (e != hipSuccess) return hip_fail(e, "get_features");
  return BSADMM_OK;
}

int bsadmm_objective(bsadmm_handle* h, const double* Wmodel, double* F) {
  g_err.clear();
  if (!h || !F) return fail(BSADMM_EINVAL, "NULL argument");
  if (h->poisoned) return fail(BSADMM_ESTATE, "handle poisoned by an earlier device error");
  return objective_of(h, Wmodel, F);
}

int bsadmm_destroy(bsadmm_handle* h) {
  g_err.clear();
  if (!h) return BSADMM_OK;
  (void)hipStreamSynchronize(h->st);
  delete h;
  return BSADMM_OK;
}

int rff_map(const float* X, int64_t n, int64_t d, const float* W, const float* b, int64_t s,
            int32_t precision, void* Z_out, void* stream) {
  g_err.clear();
  if (precision < BSADMM_FP64 || precision > BSADMM_BF16X3)
    return fail(BSADMM_EINVAL, precision == BSADMM_BF16R
                                   ? "BF16R is an iteration mode: map features with BF16 or BF16X3"
                                   : "unknown precision");
  if (n < 0 || d < 1 || s < 1) return fail(BSADMM_EINVAL, "need n >= 0, d >= 1, s >= 1");
  if (n == 0) return BSADMM_OK;
  if (!X || !W || !b || !Z_out) return fail(BSADMM_EINVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  const int64_t Kp = bs::padded_k(precision, d);
  const size_t op = bs::op_bytes(precision) * bs::op_planes(precision);
  void *xop = nullptr, *wt = nullptr, *bias = nullptr;
  auto cleanup = [&]() {
    if (xop) (void)hipFreeAsync(xop, st);
    if (wt) (void)hipFreeAsync(wt, st);
    if (bias) (void)hipFreeAsync(bias, st);
  };
  if (hipMallocAsync(&xop, (size_t)n * Kp * op, st) != hipSuccess ||
      hipMallocAsync(&wt, (size_t)s * Kp * op, st) != hipSuccess ||
      hipMallocAsync(&bias, (size_t)s * 8, st) != hipSuccess) {
    cleanup();
    return fail(BSADMM_ENOMEM, "device allocation failed in rff_map");
  }
  hipError_t e = bs::prep_rows(precision, X, n, d, Kp, xop, n * Kp, nullptr, st);
  if (e == hipSuccess) e = bs::prep_w(precision, W, b, d, s, Kp, wt, s * Kp, bias, nullptr, st);
  if (e == hipSuccess)
    e = bs::regen(precision, xop, n * Kp, n, wt, s * Kp, s, bias, Kp, std::sqrt(2.0 / (double)s),
                  Z_out, s, st);
  hipError_t e2 = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "rff_map");
  if (e2 != hipSuccess) return hip_fail(e2, "rff_map synchronize");
  return BSADMM_OK;
}

int rff_map_noalloc(const float* X, int64_t n, int64_t d, const float* W, const float* b,
                    int64_t s, int32_t precision, void* Z_out, void* stream) {
  g_err.clear();
  if (precision < BSADMM_FP64 || precision > BSADMM_BF16X3)
    return fail(BSADMM_EINVAL, precision == BSADMM_BF16R
                                   ? "BF16R is an iteration mode: map features with BF16 or BF16X3"
                                   : "unknown precision");
  if (n < 0 || d < 1 || s < 1) return fail(BSADMM_EINVAL, "need n >= 0, d >= 1, s >= 1");
  if (n == 0) return BSADMM_OK;
  if (!X || !W || !b || !Z_out) return fail(BSADMM_EINVAL, "NULL pointer");
  // scratch layout: Wt (s x Kp operand planes), bias, then X rows in chunks
  const int64_t Kp = bs::padded_k(precision, d);
  const size_t opb = bs::op_bytes(precision) * bs::op_planes(precision);
  const size_t wbytes = (size_t)rup((int64_t)s * Kp * (int64_t)opb, 256);
  const size_t bbytes = (size_t)rup(s * (precision == BSADMM_FP64 ? 8 : 4), 256);
  const size_t row_bytes = (size_t)Kp * opb;
  constexpr int64_t kMinChunk = 256;
  if (wbytes + bbytes + (size_t)kMinChunk * row_bytes > kScratchBytes)
    return fail(BSADMM_EINVAL, "rff_map_noalloc: W (" + std::to_string(wbytes) + " B staged) and " +
                                   "256 rows of X need more than the " +
                                   std::to_string(kScratchBytes >> 20) + " MiB scratch");
  int64_t chunk = (int64_t)((kScratchBytes - wbytes - bbytes) / row_bytes) / kMinChunk * kMinChunk;
  chunk = std::min<int64_t>(chunk, n);
  void* base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  char* wt = (char*)base;
  char* bias = wt + wbytes;
  char* xop = bias + bbytes;
  hipStream_t st = (hipStream_t)stream;
  const size_t zb = bs::z_bytes(precision);
  hipError_t e = bs::prep_w(precision, W, b, d, s, Kp, wt, s * Kp, bias, nullptr, st);
  for (int64_t r0 = 0; r0 < n && e == hipSuccess; r0 += chunk) {
    const int64_t rows = std::min(chunk, n - r0);
    e = bs::prep_rows(precision, X + r0 * d, rows, d, Kp, xop, chunk * Kp, nullptr, st);
    if (e == hipSuccess)
      e = bs::regen(precision, xop, chunk * Kp, rows, wt, s * Kp, s, bias, Kp,
                    std::sqrt(2.0 / (double)s), (char*)Z_out + (size_t)r0 * s * zb, s, st);
  }
  if (e != hipSuccess) return hip_fail(e, "rff_map_noalloc");
  return BSADMM_OK;
}

}  // extern "C"
