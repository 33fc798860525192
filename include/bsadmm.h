/*
 * bsadmm.h -- C ABI of the MI355X block-splitting ADMM solver over random
 * Fourier features.
 *
 * The method is the one of Sindhwani & Avron, "High-performance Kernel
 * Machines with Implicit Distributed Optimization and Randomization"
 * (arXiv 1409.0940): the regularised risk problem (eq. basicproblem) is
 * linearised with random Fourier features (eq. problem_linear, section
 * "Randomized Kernel Maps") and solved with the block-splitting ADMM of
 * Algorithm 1 (BlockADMM) over an R x C grid of blocks of the feature matrix
 * Z, which is regenerated from X instead of being kept between iterations.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status (bsadmm_status).  Nothing throws
 *   across the ABI.  On a non-OK status a message is available from
 *   bsadmm_last_error() (thread-local, valid until the next call on the
 *   same thread).  BSADMM_EINVAL leaves every output and handle untouched.
 * - Pointers named "device" are HIP device pointers on the current device;
 *   pointers named "host" are ordinary host memory.  All matrices are dense
 *   row-major with the leading dimension equal to the column count.
 * - "stream" is a hipStream_t passed as void*; NULL means the default stream.
 *   Work is enqueued on it asynchronously unless a function says it
 *   synchronises.
 * - The caller owns every buffer it passes.  The library owns every buffer
 *   it allocates and releases all of them in bsadmm_destroy.
 * - Block split rule (the paper leaves uneven splits open): row block i of
 *   n rows is [floor(i n / R), floor((i+1) n / R)), feature block j of s
 *   features is [floor(j s / C), floor((j+1) s / C)).
 */
#ifndef BSADMM_H
#define BSADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define BSADMM_API __attribute__((visibility("default")))
#else
#define BSADMM_API
#endif

/* ---------------------------------------------------------------- status */
typedef enum {
  BSADMM_OK = 0,
  BSADMM_EINVAL = 1,     /* invalid argument (sizes, enums, pointers, values)   */
  BSADMM_ENOMEM = 2,     /* footprint above hbm_budget_bytes, or hipMalloc failed */
  BSADMM_EDEVICE = 3,    /* a HIP runtime call or kernel launch failed           */
  BSADMM_ENOTPD = 4,     /* a Cholesky pivot of I + Z_ij^T Z_ij was not positive */
  BSADMM_ENONFINITE = 5, /* NaN or Inf in X, Y, W or b                           */
  BSADMM_ESTATE = 6,     /* handle poisoned by an earlier EDEVICE / ENOTPD       */
  BSADMM_ENOTIMPL = 7    /* combination not implemented                          */
} bsadmm_status;

/* ------------------------------------------------------------- precision */
/* Arithmetic of the feature regeneration and of the Z products.  The ADMM
 * state, the Cholesky factorisation and the cached inverse are always FP64.
 * R = Delta-bar/(C+1) + nu is the operand of the transpose product Z^T R and
 * W' that of the forward product Z W'.
 *   FP64  : phase X W + b, cos and products in FP64 (FP64 MFMA).
 *   FP32  : FP32 MFMA with FP32 accumulation, phase and cos in FP32; Z FP32;
 *           R and W' rounded to FP32 for the products.
 *   BF16  : X and W rounded to BF16 (round to nearest even), BF16 MFMA with
 *           FP32 accumulation, b added to the FP32 phase, cos in FP32, Z
 *           stored in BF16.  The products are BF16 MFMA with FP32
 *           accumulation over the exact BF16 Z and two BF16 planes of R and
 *           W' each, a head h = bf16(v) and a residual bf16(v - h), so the
 *           operand keeps about 16 significant bits.  The phase error is about
 *           2^-8 |X||W| per element; objective error <= 1e-2 (measured far
 *           below it on the benchmark workloads).
 *   BF16X3: split-operand BF16 features.  X and W are each split into a BF16
 *           head and a BF16 residual (the rounding error of the head), and the
 *           phase sums the three products head*head + head*residual +
 *           residual*head on BF16 MFMA with FP32 accumulation (phase error
 *           <= 3 * 2^-16 sum |x||w|); Z is stored in FP32.  With at most two
 *           16-column output tiles (m <= 32) the products are FP32 MFMA; with
 *           more they are three BF16 MFMA products per element (Z's head and
 *           residual against the head and residual planes of R and W', the
 *           residual-by-residual term dropped, below 2^-16 of the product).
 *           rff_map returns float for BF16X3.
 *   BF16R : BF16 iterations with iterative refinement of the products of the
 *           graph projection (eq. gpWij) through the same FP64 factor: the
 *           cache of eq. cache is that of BF16.  Every iteration
 *           regenerates BF16 features Zt and runs the BF16 products; on the
 *           first iteration and every refine_every-th after it (a refinement
 *           iteration) it also regenerates BF16X3 features Zf, forms the
 *           defect dZ = bf16(Zf - Zt) and the defects of both products,
 *           dZ_ij^T R_i and sum_j dZ_ij W'_ij, which every iteration until
 *           the next refinement adds to its BF16 products.  The added defect
 *           is that of the last refinement's operands, so at a fixed point
 *           the corrected products equal the FP32-faithful ones; the
 *           remaining difference to the FP32-faithful fixed point is that of
 *           the factor (BF16 against FP32-faithful Gram).  The first
 *           iteration starts from R = W' = 0 and leaves the defects at 0, so
 *           the first refinement that corrects anything is iteration
 *           1 + refine_every.  The objective uses Zt + dZ and predictions the
 *           BF16X3 features.  rff_map rejects BF16R.                        */
enum { BSADMM_FP64 = 0, BSADMM_FP32 = 1, BSADMM_BF16 = 2, BSADMM_BF16X3 = 3, BSADMM_BF16R = 4 };

/* ------------------------------------------------------------------ loss */
/* V(y, o) of eq. basicproblem, entering only through its prox (paragraph
 * "Modularity").
 *   SQUARED : ||y - o||^2 (no 1/2), any m.
 *   HINGE   : max(0, 1 - y o), m = 1, y in {-1, +1}.
 *   MC_HINGE: one-vs-all sum_k max(0, 1 - y_k o_k), y in {-1, +1}^m.
 * Further losses with cheap proxes (not in the paper's experiments):
 *   L1      : sum_k |y_k - o_k|, any m (soft-thresholding prox).
 *   CS_HINGE: Crammer-Singer multiclass hinge max_k (o_k + [k != c]) - o_c,
 *             m >= 2, y one-hot (1 at class c, 0 elsewhere); row-wise prox
 *             through a projection onto the probability simplex.
 *   SOFTMAX : multinomial logistic log sum_k exp(o_k) - o_c, m >= 2, y
 *             one-hot; row-wise prox by Newton's method.                   */
enum {
  BSADMM_SQUARED = 0,
  BSADMM_HINGE = 1,
  BSADMM_MC_HINGE = 2,
  BSADMM_L1 = 3,
  BSADMM_CS_HINGE = 4,
  BSADMM_SOFTMAX = 5
};

/* ----------------------------------------------------------- regulariser */
/* r(W) = ||W||_F^2, separable over feature blocks (l2 case of the block
 * reformulation, eq. prob2).                                               */
enum { BSADMM_L2 = 0 };

/* ------------------------------------------------------------ Z handling */
/* STORE: each iteration regenerates the blocks Z_ij of a group of row
 *        blocks once into a library workspace and both products of the
 *        iteration read them (the paper keeps Z_ij for the products of one
 *        block visit, steps 15-21); nothing of Z survives the iteration.
 * AUTO : STORE with the largest row-block groups that fit the workspace cap.
 * KEEP : Z is generated once, at setup, for all rows and kept in HBM for
 *        every iteration (no regeneration).  Needs n x spad elements of
 *        workspace (spad = sum_j s_j rounded up to 64 per block); setup fails
 *        with ENOMEM if workspace_bytes is set and smaller.  Results equal
 *        STORE bit for bit.
 * A workspace element is the stored feature: 8 bytes (FP64), 4 (FP32,
 * BF16X3), 2 (BF16), 4 for BF16R (the BF16 feature and its defect; the
 * FP32-faithful features it comes from are never stored).                 */
enum { BSADMM_Z_AUTO = 0, BSADMM_Z_STORE = 1, BSADMM_Z_KEEP = 2 };

/* -------------------------------------------------------------- problem */
/* Problem flags.
 * BSADMM_F_GRAPH: bsadmm_iterate calls that do not ask for per-phase timing
 *   replay HIP graphs of the iteration instead of launching its kernels one
 *   by one: the launch sequence of one iteration (and of a chunk of 16, or of
 *   one adaptation period of at most 64 iterations) is captured on first use
 *   on a private stream and launched on the handle's stream.  The kernels and
 *   their order are the same, so the iterates are bit for bit those of the
 *   eager path; the gain is host launch time, which bounds small problems. */
enum { BSADMM_F_GRAPH = 1 };

/* Problem of eq. problem_linear with Z = sqrt(2/s) cos(X W + b):
 *   minimise (1/n) sum_r V(y_r, W_model^T z(x_r)) + lambda ||W_model||_F^2.
 * The ADMM penalty rho applies to n times that objective (the loss prox has
 * weight 1/rho and the regulariser prox weight n lambda / rho); this is the
 * paper's update with its rho replaced by rho / n, and has the same
 * minimiser.                                                              */
typedef struct bsadmm_problem {
  int64_t n;        /* examples (rows of X, Y), >= R                        */
  int64_t d;        /* input dimension, >= 1                                */
  int64_t m;        /* outputs / classes (columns of Y), 1 <= m <= 1024     */
  int64_t s;        /* random features, >= C                                */
  int32_t R;        /* row blocks, >= 1                                     */
  int32_t C;        /* feature (column) blocks, >= 1                        */
  int32_t loss;     /* BSADMM_SQUARED | BSADMM_HINGE | BSADMM_MC_HINGE      */
  int32_t reg;      /* BSADMM_L2                                            */
  int32_t precision;/* BSADMM_FP64 | FP32 | BF16 | BF16X3                    */
  int32_t z_mode;   /* BSADMM_Z_AUTO | BSADMM_Z_STORE | BSADMM_Z_KEEP       */
  double lambda;    /* >= 0                                                 */
  double rho;       /* > 0                                                  */
  double sigma;     /* kernel bandwidth the caller drew W with; > 0; used
                       only for validation and reporting                    */
  const float* X;   /* device, n x d, caller-owned, must outlive the handle */
  const float* Y;   /* device, n x m, caller-owned, must outlive the handle */
  const float* W;   /* device, d x s feature directions (N(0, 1/sigma^2)),
                       caller-owned; copied at setup.  NULL together with b:
                       drawn by the library from `seed` (below)             */
  const float* b;   /* device, s feature offsets (U[0, 2 pi)); copied       */
  void* stream;     /* hipStream_t for every call on the handle             */
  size_t hbm_budget_bytes;  /* 0 = no limit; else setup fails with ENOMEM
                               when the footprint exceeds it                */
  size_t workspace_bytes;   /* cap on the Z workspace; 0 = automatic        */
  /* Penalty adaptation (not in the paper): residual balancing of Boyd,
   * Parikh, Chu, Peleato and Eckstein (2011), section 3.4.1.  After every
   * rho_adapt_every-th iteration (counted over the handle's life; 0 = fixed
   * rho) the primal residual r and the dual residual s of that iteration are
   * compared: rho is multiplied by tau when r > mu s and divided by tau when
   * s > mu r, and the scaled duals nu, mu, mu' are divided by the same
   * factor.  r and s are those of ADMM on the block problem (eq. prob2)
   * written as x = z (Boyd et al., section 3.3): x stacks O_i, W_j and the
   * graph-projection outputs O_ij = Z_ij W'_ij, W'_ij; z their projections
   * O-bar_i, W-bar_j, O-bar_ij (eq. obar_ij), W-bar; r = ||x - z|| and
   * s = rho ||z - z_prev|| over every stacked copy.  In terms of the kept
   * state, r^2 = ||Delta-bar||^2/(C+1) + ||W - W-bar||^2 + sum_i ||W'_i - W-bar||^2,
   * and the O-bar_ij part of s uses ||Z_ij dW'_ij||^2 = <dW'_ij, dU_ij>.
   * The cached factors do not depend on rho.  The check and the decision run
   * on the device, stream-ordered: no host synchronisation.                */
  int32_t rho_adapt_every;  /* >= 0                                         */
  int32_t flags;            /* 0 or BSADMM_F_GRAPH                          */
  double rho_adapt_mu;      /* > 1; 0 selects 10                            */
  double rho_adapt_tau;     /* > 1; 0 selects 2                             */
  int32_t refine_every;     /* BF16R: iterations between refinements, >= 0;
                               0 selects 5.  Must be 0 for other precisions */
  int32_t reserved2;        /* 0                                            */
  /* Feature-map draw when W and b are both NULL (the random draw of the
   * section on randomized kernel maps, which the paper generates from a
   * seed rather than storing): with Philox4x32-10 (Salmon, Moraes, Dror and
   * Shaw, SC 2011) under key (seed mod 2^32, seed / 2^32), the counter
   * (t mod 2^32, t / 2^32, 0, 0) gives the pair W[2t], W[2t + 1] of the
   * row-major d x s array: its words (w0, w1, w2, w3) as two uniforms
   * u = (floor((w_hi 2^32 + w_lo) / 2^11) + 1/2) 2^-53 in (0, 1), u1 from
   * (w0, w1) and u2 from (w2, w3), then Box-Muller,
   * sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) / sigma; the counter
   * (j mod 2^32, j / 2^32, 1, 0) gives b[j] = 2 pi u1 (0 if that rounds to
   * 2 pi in FP32).  Evaluated in FP64, stored in FP32; bsadmm_get_features
   * copies the draw out.                                                  */
  uint64_t seed;
} bsadmm_problem;

/* Phases timed with HIP events on the handle's stream (bsadmm_stats). */
enum {
  BSADMM_PH_REGEN = 0,   /* feature regeneration Z = sqrt(2/s) cos(XW + b)  */
  BSADMM_PH_ZTR = 1,     /* A_ij = Z_ij^T (Delta-bar_i/(C+1) + nu_i)        */
  BSADMM_PH_SOLVE = 2,   /* W'_ij = (I + Z_ij^T Z_ij)^{-1} rhs_ij, U update */
  BSADMM_PH_ZW = 3,      /* sum_j Z_ij W'_ij                                */
  BSADMM_PH_ROW = 4,     /* loss prox, exchange and nu updates              */
  BSADMM_PH_COL = 5,     /* regulariser prox, consensus and mu updates      */
  BSADMM_PH_REFINE = 6,  /* BF16R refinement: BF16X3 features, their defect
                            and the two defect products                    */
  BSADMM_PH_COUNT = 8
};

/* Requests of bsadmm_stats.want. */
enum { BSADMM_WANT_RESIDUALS = 1, BSADMM_WANT_OBJECTIVE = 2 };

typedef struct bsadmm_stats {
  int64_t iters_done;       /* out: total iterations run on the handle      */
  int32_t timed;            /* in: nonzero asks for per-phase timing        */
  int32_t launches;         /* out: launches of the regeneration kernel in
                               the call (one per row-block group per
                               iteration)                                  */
  double phase_ms[BSADMM_PH_COUNT];  /* out: summed over the call          */
  double iterate_ms;        /* out: whole call, HIP events                 */
  double rho;               /* out: penalty after the call                 */
  int32_t rho_changes;      /* out: penalty changes by adaptation over the
                               handle's life                               */
  int32_t want;             /* in: BSADMM_WANT_* bits                       */
  double r_primal;          /* out (WANT_RESIDUALS, iters > 0): primal and   */
  double r_dual;            /* dual residual of the call's last iteration, as
                               defined for penalty adaptation (0 otherwise) */
  double objective;         /* out (WANT_OBJECTIVE): F(W-bar) after the call
                               (as bsadmm_objective; one extra regeneration
                               pass), 0 otherwise                          */
} bsadmm_stats;

typedef struct bsadmm_handle bsadmm_handle;

/* ----------------------------------------------------------------------
 * rff_map -- the transform T of Algorithm 1, step 15, for the random
 * Fourier feature map of section "Randomized Kernel Maps":
 *   Z[r][f] = sqrt(2/s) * cos(sum_k X[r][k] W[k][f] + b[f]).
 * X: device n x d float32.  W: device d x s float32.  b: device s float32.
 * Z_out: device n x s of double (FP64), float (FP32, BF16X3) or bf16 bits
 * stored as uint16 (BF16).  n may be 0 (no work).  Allocates and frees a small
 * operand staging buffer; synchronises the stream before returning.
 * Errors: EINVAL (null pointers with n > 0, d < 1, s < 1, bad precision),
 * ENOMEM, EDEVICE.
 * -------------------------------------------------------------------- */
BSADMM_API int rff_map(const float* X, int64_t n, int64_t d, const float* W, const float* b,
            int64_t s, int32_t precision, void* Z_out, void* stream);

/* ----------------------------------------------------------------------
 * rff_map_noalloc -- rff_map for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, layouts and results as rff_map (the same
 * kernels, so the same bits), but it allocates nothing and does not
 * synchronise: the operand staging lives in a 64 MiB array the library keeps
 * on each GPU for the life of the process, and the work is only enqueued on
 * `stream`.  The caller still passes X, W, b and Z_out.
 * Limit: W staged in the operand layout (s x Kp elements of 8, 4 or 2 bytes,
 * two planes for BF16X3; Kp = d rounded up to the kernel's K chunk) plus the
 * s offsets plus 256 rows of X must fit in the 64 MiB; X is staged in row
 * chunks, so n is not limited.  Larger problems fail with EINVAL and a
 * message naming the limit.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on a
 * GPU (different streams, or host threads, without ordering between them)
 * race and may return wrong features.  Order them on one stream or
 * synchronise between them.  Nothing in the scratch needs to start at zero
 * (each call writes all staging it reads).
 * Errors: as rff_map (EINVAL also for the size limit); device errors of the
 * enqueued kernels surface at the caller's next synchronisation.
 * -------------------------------------------------------------------- */
BSADMM_API int rff_map_noalloc(const float* X, int64_t n, int64_t d, const float* W,
                               const float* b, int64_t s, int32_t precision, void* Z_out,
                               void* stream);

/* ----------------------------------------------------------------------
 * bsadmm_validate -- host-only argument checks of a problem (no HIP call,
 * no device access): n >= R >= 1, s >= C >= 1, d >= 1, 1 <= m <= 1024,
 * m == 1 for HINGE, m >= 2 for CS_HINGE and SOFTMAX, lambda >= 0, rho > 0,
 * sigma > 0, known enums, non-null
 * X, Y, W, b, 16-byte alignment of X, Y, W, b, rho_adapt_every >= 0 and
 * rho_adapt_mu, rho_adapt_tau either 0 or finite and > 1.  Returns OK or
 * EINVAL.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_validate(const bsadmm_problem* p);

/* ----------------------------------------------------------------------
 * bsadmm_footprint -- device bytes bsadmm_setup will allocate for p
 * (operand copies, factor cache R*C*S^2 doubles with S = s_j rounded up to
 * 64, ADMM state, Z workspace, partial sums).  Host-only; validates p
 * first.  The paper's own per-node model is eq. mem of paragraph "Memory
 * Requirements"; this is its device counterpart.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_footprint(const bsadmm_problem* p, size_t* bytes);

/* ----------------------------------------------------------------------
 * bsadmm_setup -- validate, allocate, copy W and b into the operand
 * layout, set the ADMM state of Algorithm 1, step 2 to zero and build the
 * cache of eq. cache: for every block, Q_ij = (I + Z_ij^T Z_ij)^{-1} in
 * FP64 through a Cholesky factorisation (the paper builds it in the first
 * iteration, step 16).  Synchronises the stream.
 * Errors: EINVAL (also targets that are not +-1 for HINGE / MC_HINGE or
 * not one-hot rows for CS_HINGE / SOFTMAX), ENONFINITE (NaN/Inf in X, Y, W
 * or b), ENOMEM, EDEVICE, ENOTPD.  On error *out is NULL and nothing stays allocated.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_setup(const bsadmm_problem* p, bsadmm_handle** out);

/* ----------------------------------------------------------------------
 * bsadmm_iterate -- run `iters` (>= 0) iterations of Algorithm 1 with the
 * graph-projection right-hand side of eq. gpWij (it includes Z_ij^T nu_i)
 * and the dual updates of mu, mu' made with the new consensus W-bar, as in
 * the block-splitting update equations.  Enqueued on the handle's stream;
 * if st != NULL the call synchronises and fills st.  With
 * rho_adapt_every > 0 the penalty is balanced after every K-th iteration
 * (see bsadmm_problem), on the device.
 * Errors: EINVAL (iters < 0, null handle), ESTATE, EDEVICE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_iterate(bsadmm_handle* h, int32_t iters, bsadmm_stats* st);

/* ----------------------------------------------------------------------
 * bsadmm_predict -- scores of the consensus model: out = Z(Xt) W-bar
 * (prediction f(x) = W^T z(x) of the linearised hypothesis space).
 * Xt: device nt x d float32.  out: device nt x m float32.  Uses the
 * handle's precision for the feature map.  nt may be 0.  Synchronises.
 * Errors: EINVAL, ESTATE, ENOMEM, EDEVICE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_predict(bsadmm_handle* h, const float* Xt, int64_t nt, float* out, void* stream);

/* ----------------------------------------------------------------------
 * bsadmm_get_coef -- copy the consensus model W-bar (s x m, FP64) into a
 * caller-owned device buffer.  The paper does not name the model a run
 * returns; read here as W-bar, the consensus model that the root averages
 * from the local models and distributes to every node (Algorithm 1, the
 * reduce and broadcast of W-bar, and the schematic figure that follows it).
 * At convergence W-bar = W = W'_i.  Synchronises.  Errors: EINVAL, ESTATE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_get_coef(const bsadmm_handle* h, double* Wbar);

/* State arrays of the iteration (names of Algorithm 1; sizes in doubles). */
enum {
  BSADMM_ST_O = 0,     /* n x m   loss-prox output O                        */
  BSADMM_ST_OBAR = 1,  /* n x m   O-bar                                     */
  BSADMM_ST_NU = 2,    /* n x m   nu                                        */
  BSADMM_ST_DBAR = 3,  /* n x m   Delta-bar                                 */
  BSADMM_ST_WC = 4,    /* s x m   regulariser-prox output W                 */
  BSADMM_ST_WBAR = 5,  /* s x m   consensus W-bar                           */
  BSADMM_ST_MU = 6,    /* s x m   mu                                        */
  BSADMM_ST_WP = 7,    /* R x s x m local models W'                         */
  BSADMM_ST_MUP = 8,   /* R x s x m mu'                                     */
  BSADMM_ST_U = 9,     /* R x s x m U = Z_ij^T Z_ij W'_ij                   */
  BSADMM_ST_META = 10, /* 2       penalty rho and iterations done (importing
                                  them sets both; duals are not rescaled)   */
  BSADMM_ST_COUNT = 11,
  /* BSADMM_BF16R handles only (EINVAL otherwise): the product defects kept
   * between refinements, part of the state of a refined run.              */
  BSADMM_ST_DEFECT_A = 11, /* R x s x m  dZ_ij^T R_i of the last refinement  */
  BSADMM_ST_DEFECT_P = 12  /* n x m      sum_j dZ_ij W'_ij of the last one   */
};

/* ----------------------------------------------------------------------
 * bsadmm_state_size -- number of doubles of state array `which`.
 * bsadmm_export_state / bsadmm_import_state -- copy one state array to /
 * from a caller-owned device buffer, dense row-major with the sizes listed
 * above.  The arrays are the variables Algorithm 1 initialises to zero and
 * carries from one iteration to the next (its initialisation step), with
 * W'_i stacked over the row blocks, so they are the whole state of the
 * iteration: exporting all BSADMM_ST_COUNT arrays, META included (and, for
 * BSADMM_BF16R, the two product defects), and importing them into a handle
 * set up from the same inputs continues the run exactly, also under penalty
 * adaptation (checkpoint and resume).  The
 * factor cache (eq. cache) is not state: setup rebuilds it from X, W, b.
 * Both synchronise.  Errors: EINVAL (bad `which`, null pointer, an imported
 * META with rho <= 0 or a negative count), ESTATE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_state_size(const bsadmm_handle* h, int32_t which, int64_t* count);
BSADMM_API int bsadmm_export_state(const bsadmm_handle* h, int32_t which, double* dst);
BSADMM_API int bsadmm_import_state(bsadmm_handle* h, int32_t which, const double* src);

/* ----------------------------------------------------------------------
 * bsadmm_get_features -- copy the feature-map draw of a handle set up with
 * W = b = NULL (the problem's seed) into the caller's device arrays
 * W (d x s, row-major FP32) and b (s FP32), enqueued on the handle's stream
 * (no synchronisation).  Passing them back as W and b to another setup
 * gives the same run.
 * Errors: EINVAL (null argument; the handle was given W and b), ESTATE,
 * EDEVICE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_get_features(const bsadmm_handle* h, float* W, float* b);

/* ----------------------------------------------------------------------
 * bsadmm_objective -- F(W) = (1/n) sum_r V(y_r, W^T z(x_r)) + lambda ||W||_F^2
 * (eq. problem_linear) on the handle's training data, with the handle's
 * feature map and precision: one regeneration pass over all rows and one
 * forward product, summed in a fixed order.  Wmodel: device s x m FP64
 * model, or NULL for the handle's consensus W-bar.  *F: host.  Overwrites
 * the Z workspace (no effect on the iteration).  Synchronises.
 * Errors: EINVAL (null handle or F), ESTATE, ENOMEM, EDEVICE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_objective(bsadmm_handle* h, const double* Wmodel, double* F);

/* ----------------------------------------------------------------------
 * bsadmm_monitor -- enqueue on the handle's stream, without synchronising,
 * fixed-order reductions of the state left by the last iteration into the
 * caller-owned device array out[0..3] (doubles):
 *   out[0] = sum_r V(y_r, o'_r), o' = sum_j Z_ij W'_ij (outputs of the local
 *            models of step 19),
 *   out[1] = (1/R) sum_i ||W'_i||_F^2,
 *   out[2] = sum_i ||W'_i - W-bar||_F^2  (consensus residual, steps 28-29),
 *   out[3] = ||Delta-bar||_F^2           (exchange residual, step 25).
 * With R = 1, out[0] / n + lambda out[1] is the objective F of the local
 * model W' (eq. problem_linear) at no extra feature regeneration; a serving
 * loop reads it asynchronously as its stopping statistic.
 * Errors: EINVAL (null argument), ESTATE, EDEVICE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_monitor(bsadmm_handle* h, double* out);

/* ----------------------------------------------------------------------
 * bsadmm_dual_bound -- a lower bound on min F (eq. problem_linear), for
 * certifying the objective error of a run; not in the paper.  With V_r* the
 * convex conjugate of o -> V(y_r, o), weak Fenchel duality gives for every
 * alpha (n x m)
 *   F(W) >= D(alpha) = (1/n) sum_r -V_r*(-alpha_r) - ||Z^T alpha||^2 / (4 lambda n^2),
 * with -V*(-a) = a y - a^2/4 (squared loss) and a y on the domain
 * 0 <= a y <= 1 (hinge, one-vs-all hinge).  alpha is the penalty times the
 * row operand of the state left by the last iteration,
 * rho (Delta-bar/(C+1) + nu), moved into that domain (y clip(y a, 0, 1));
 * at the ADMM fixed point it is the dual solution and D = min F.
 * Enqueued on the handle's stream without synchronising: one transpose
 * product over Z (two for BF16R, whose bound uses the BF16 features plus
 * their defect; feature regeneration first unless Z is kept), into the
 * caller-owned device array out[0..2] (doubles):
 *   out[0] = D(alpha),  out[1] = the conjugate part,  out[2] = the
 *   ||Z^T alpha||^2 / (4 lambda n^2) part.
 * alpha enters the product as the precision's operand of R (FP64, FP32, or
 * BF16 head and residual planes) and the conjugate part is summed over that
 * rounded alpha, so out[0] is the dual objective of a point of the domain.
 * It overwrites the R operand and right-hand-side buffers and the Z
 * workspace, all rewritten by the next iteration, so the iteration is not
 * changed.  With R = 1, F(W') from bsadmm_monitor minus out[0] bounds the
 * objective error of the local model W' (state BSADMM_ST_WP).  BF16R
 * allocates an R x s x m FP64 buffer at the first call (stream-ordered).
 * Errors: EINVAL (null argument; a loss other than squared, hinge or
 * one-vs-all hinge), ESTATE, ENOMEM, EDEVICE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_dual_bound(bsadmm_handle* h, double* out);

/* ----------------------------------------------------------------------
 * bsadmm_set_rho -- change the ADMM penalty to rho (> 0, finite) for the
 * following iterations.  The loss-prox weight becomes 1/rho and the
 * regulariser weight n lambda / rho; with rescale_duals != 0 the scaled
 * duals nu, mu, mu' are multiplied by rho_old / rho, which keeps the
 * unscaled duals and hence the fixed point (the usual penalty update);
 * with 0 they are left as they are.  The factor cache is unchanged: it has
 * no rho.  Enqueued on the handle's stream.
 * Errors: EINVAL (null handle, rho <= 0 or not finite), ESTATE, EDEVICE.
 * -------------------------------------------------------------------- */
BSADMM_API int bsadmm_set_rho(bsadmm_handle* h, double rho, int32_t rescale_duals);

/* bsadmm_destroy -- wait for the handle's stream, then free everything the
 * handle owns: operand copies, the factor cache of eq. cache, the state and
 * the workspaces (the memory of the paper's per-process model, eq. mem).
 * The caller's X, Y, W, b are untouched.  NULL is allowed.  Returns OK.   */
BSADMM_API int bsadmm_destroy(bsadmm_handle* h);

/* Message of the last non-OK status on this thread ("" if none); a library
 * convention, not part of the method.  The string stays valid until the
 * next call into the library on the same thread.                         */
BSADMM_API const char* bsadmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BSADMM_H */
