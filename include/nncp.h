/*
 * nncp.h -- C ABI of the MI355X (gfx950) library for dense nonnegative CP
 * decomposition (NNCP) by alternating updates, after PLANC
 * (Eswar, Hayashi, Ballard, Kannan, Matheson, Park; arXiv 1909.01149).
 *
 * Problem (Section 1, Eq. eqn:nncp): given a nonnegative N-way tensor X of
 * size I_0 x ... x I_{N-1}, find nonnegative factors H^(n) (I_n x R) that
 * minimise || X - sum_r H^(0)(:,r) o ... o H^(N-1)(:,r) ||^2.  The library
 * computes the alternating-update iteration of Algorithm 1: for each mode n,
 * the MTTKRP M^(n), the Hadamard product S^(n) of the other Gram matrices,
 * an MU (Eq. eqn:muupd) or HALS (Eq. eqn:halsupd) update, column
 * normalisation, and the relative error through the identity of the
 * appendix (Algorithm 4).  MTTKRP runs through the dimension tree of
 * Section 4.2 (Algorithm 3): two partial MTTKRPs (one GEMM each) at the root
 * and multi-TTVs below.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Modes are 0-based (the paper numbers them from 1).
 *
 * Tensor layout: X is dense, mode 0 varies fastest: entry (i_0, ..., i_{N-1})
 * is at linear index i_0 + I_0 (i_1 + I_1 (i_2 + ...)), the local storage
 * order of Section 4.1.2 (column-major carried to N modes).  In
 * PyTorch this is a contiguous tensor of shape (I_{N-1}, ..., I_0).
 *
 * Factor layout: H^(n) is I_n x R, row-major (entry (i, r) at i*R + r).  The
 * paper's factors are column-major; the transposition keeps each row's R
 * values together for the row-parallel updates.  MTTKRP outputs M and
 * gradients use the same layout and the factor dtype.
 *
 * Dtypes (x_dtype, h_dtype): (NNCP_F64, NNCP_F64) "FP64 mode", (NNCP_F32,
 * NNCP_F32), (NNCP_BF16, NNCP_F32), (NNCP_F16, NNCP_F32).  Anything else
 * returns NNCP_E_DTYPE.  Partial-MTTKRP accumulation, dimension-tree
 * temporaries and M use the factor dtype; Gram matrices, S, lambda, the loss
 * and all scalar reductions are FP64.
 *
 * Memory: every pointer argument is device memory unless its comment says
 * "host".  X, H, lambda, outputs and the workspace belong to the caller and
 * are borrowed until nncp_destroy; the library never allocates or frees
 * device memory.  X is only read.  H and lambda are updated in place by
 * nncp_update_*, nncp_sweep and nncp_pgd.  Device pointers must be 16-byte
 * aligned.
 *
 * Streams: every kernel is launched on the stream given to nncp_init (a
 * hipStream_t passed as void*; NULL is the default stream).  Calls are
 * asynchronous and outputs are valid once the stream has been synchronised.
 * No call waits for the device except nncp_pgd, which synchronises to take
 * its step-size decisions, and the timer calls nncp_timers_enable and
 * nncp_timers_read.
 *
 * Errors: every call returns an int status.  Arguments are validated before
 * anything is launched, so a failing call launches nothing.  A HIP launch
 * failure returns NNCP_E_HIP.  nncp_last_error() gives a message for the
 * calling thread's last failure.  No C++ exception crosses the ABI.  A
 * context belongs to one stream and is not thread-safe.
 */
#ifndef NNCP_H
#define NNCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NNCP_MAX_MODES 16

enum nncp_status {
  NNCP_OK = 0,
  NNCP_E_INVAL = -1,       /* N, dims, R, mode, algo or a pointer is invalid     */
  NNCP_E_DTYPE = -2,       /* unsupported (x_dtype, h_dtype) pair                */
  NNCP_E_WORKSPACE = -3,   /* workspace smaller than nncp_workspace_size()       */
  NNCP_E_HIP = -4,         /* a HIP call or kernel launch failed                 */
  NNCP_E_STATE = -5,       /* context is NULL or already destroyed               */
  NNCP_E_UNSUPPORTED = -6  /* valid request outside the library's limits (R > 256, or
                              R > 64 for BPP, ADMM, NES and PGD)     */
};

enum nncp_dtype { NNCP_F64 = 0, NNCP_F32 = 1, NNCP_BF16 = 2, NNCP_F16 = 3 };

/* NNCP_NES_OUTER (nncp_sweep only): the Nesterov-type updates plus the outer
 * extrapolation of Section 4.3.5 (Eq. eqn:nesouterupd) after every sweep. */
enum nncp_algo {
  NNCP_MU = 0,
  NNCP_HALS = 1,
  NNCP_BPP = 2,
  NNCP_ADMM = 3,
  NNCP_NES = 4,
  NNCP_NES_OUTER = 5
};

/* Options (pass NULL for the defaults, shown in brackets). */
typedef struct nncp_options {
  int split;        /* root split: modes 0..split-1 form the left subtree.  0 =
                       automatic [0]: the smallest S with
                       prod(I_0..I_{S-1}) >= prod(I_S..I_{N-1}), clamped to
                       [1, N-1] (Section 4.2.2; ">=" is the reading of the
                       strict comparison there that gives a balanced split
                       for equal halves).  */
  int krp_split;    /* BF16/FP16 tensors: 1 = feed the Khatri-Rao operand to the
                       matrix cores as a hi+lo pair of the tensor's type (error
                       about 2^-16 instead of 2^-8), 0 = single rounding [1]. */
  int generic;      /* 1 = force the portable vector-ALU partial-MTTKRP kernels
                       instead of the matrix-core ones [0].                    */
  double eps_mu;    /* MU denominator guard, added to the denominator of
                       Eq. eqn:muupd [1e-16].                                  */
  int graphs;       /* 1 = nncp_sweep replays its launches as a HIP graph
                       (captured once per (algo, nsweeps, relerr_hist) and
                       factor binding), 0 = plain launches [1].                */
  int fused_grad;   /* 1 = nncp_grad computes both root partial MTTKRPs in one
                       pass over X where that path applies (BF16 tensor,
                       R <= 32, at least two modes on the left of the root
                       split) and the grid is large enough to fill the GPU
                       (at least 192 workgroups of 1024 columns), 2 = wherever
                       it applies, whatever the grid, 0 = one pass per root
                       product [1].                                            */
  int krp_kernel;   /* 1 = build every matrix-core product's Khatri-Rao operand
                       with its own kernel; 0 = where the operand is a single
                       fast mode times at most one slow mode (R a multiple of
                       16, not FP16), the product kernel reads the factors and
                       forms the operand itself, one launch fewer [0].        */
} nncp_options;

typedef struct nncp_ctx nncp_ctx;

/*
 * Bytes of device workspace that nncp_init needs for this problem.  Returns 0
 * if the arguments are invalid (see nncp_last_error).
 *   N      number of modes, 2..NNCP_MAX_MODES
 *   dims   host array of N mode sizes, each >= 1
 *   R      rank, 1..256
 */
size_t nncp_workspace_size(int N, const int64_t *dims, int R, int x_dtype, int h_dtype,
                           const nncp_options *opt);

/*
 * Create a context and run the initialisation of Algorithm 1 / Algorithm 4:
 * the Gram matrix G^(n) = H^(n)^T H^(n) of every factor and alpha = ||X||^2.
 *   ctx        host out: the new context
 *   X          tensor (layout above), x_dtype, prod(dims) entries
 *   H          host array of N device pointers to the factors (start iterate,
 *              all N modes; Algorithm 1 initialises only modes 2..N but MU and
 *              HALS need a start value for every mode)
 *   lambda     R FP64 column weights of the model [[lambda; H]] (pass ones
 *              for an unnormalised start)
 *   workspace  device buffer of at least nncp_workspace_size() bytes
 *   stream     hipStream_t, may be NULL
 */
int nncp_init(nncp_ctx **ctx, int N, const int64_t *dims, int R, int x_dtype, const void *X,
              int h_dtype, void *const *H, double *lambda, void *workspace, size_t ws_bytes,
              void *stream, const nncp_options *opt);

/* Point the context at other factor / lambda buffers of the same shapes and
 * recompute the Gram matrices (lambda may be NULL to keep the current one). */
int nncp_set_factors(nncp_ctx *ctx, void *const *H, double *lambda);

/*
 * MTTKRP of one mode at the current factors (Algorithm 1, MTTKRP line):
 *   M^(n) = X_(n) (H^(N-1) kr ... kr H^(n+1) kr H^(n-1) kr ... kr H^(0)),
 * computed through the dimension tree (Algorithm 3 with the transposes and
 * Khatri-Rao ranges corrected): the partial MTTKRP at the root of n's
 * subtree, then multi-TTVs down to n.
 * Nodes of the tree that an earlier nncp_mttkrp left in the workspace are
 * reused when every factor they were contracted with is unchanged since
 * (the reuse of Algorithm 3): the context keeps a version per factor, bumped
 * by every call that writes factors (nncp_update_*, nncp_sweep, nncp_pgd,
 * nncp_set_factors) and by nncp_factors_changed, which a caller must use
 * after writing a factor buffer itself.  Calls for modes 0..N-1 in order at
 * fixed factors therefore read X twice, not N times; a call whose nodes are
 * stale reads X once.  Any other entry point that uses the workspace drops
 * the cached nodes.  The result does not depend on the call order.
 *   M  I_n x R, row-major, h_dtype.
 */
int nncp_mttkrp(nncp_ctx *ctx, int mode, void *M);

/* The caller has written factor `mode` (every factor when mode = -1) in its
 * own buffer: bump its version (so no cached node built from the old values
 * is reused) and recompute its Gram matrix. */
int nncp_factors_changed(nncp_ctx *ctx, int mode);

/*
 * nncp_mttkrp without a context or workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Computes the same M^(n) with the same
 * kernels, grids and summation order as nncp_mttkrp on a context of the same
 * problem and options (so the two agree bitwise), from the root of n's
 * subtree.  The dimension-tree temporaries (Khatri-Rao operands, nodes,
 * split partials) live in a library-owned device array of
 * NNCP_NOALLOC_SCRATCH_BYTES, one per GPU, held from the first call on that
 * GPU until the process ends; nothing in it needs to start at zero, and it
 * keeps the last call's contents.  The call allocates nothing.
 *   N, dims, R, x_dtype, h_dtype, opt   as for nncp_init (opt may be NULL)
 *   X      tensor (layout above), read only
 *   H      host array of N device pointers to the factors, read only
 *   mode   0 .. N-1
 *   M      output, I_mode x R row-major, h_dtype
 *   stream hipStream_t of the current device (NULL: the default stream)
 * Returns NNCP_E_WORKSPACE when the temporaries of this problem exceed
 * NNCP_NOALLOC_SCRATCH_BYTES (nothing is launched), NNCP_E_INVAL when the
 * stream belongs to another device.  Calls on one GPU share its array, so
 * calls whose launches overlap on that GPU (on different streams, or from
 * different threads) race; calls that follow one another on one stream do
 * not.
 */
#define NNCP_NOALLOC_SCRATCH_BYTES (64u << 20)
int nncp_mttkrp_noalloc(int N, const int64_t *dims, int R, int x_dtype, const void *X,
                        int h_dtype, void *const *H, int mode, void *M, void *stream,
                        const nncp_options *opt);

/* G^(n) = H^(n)^T H^(n) (R x R, FP64, row-major) of the current factor; also
 * refreshes the context's copy used for S^(n). */
int nncp_gram(nncp_ctx *ctx, int mode, double *G);

/* S^(n) = Hadamard product of G^(k) for k != n (Algorithm 1), R x R FP64. */
int nncp_hadamard(nncp_ctx *ctx, int mode, double *S);

/*
 * One factor update of mode n from M = M^(n) (I_n x R, h_dtype) and
 * S = S^(n) (R x R FP64):  Hhat = H^(n) diag(lambda) (lambda folded into the
 * factor being solved for, Appendix B), then
 *   MU   (Eq. eqn:muupd):  Hhat <- Hhat * M / (Hhat S + eps)   [eps < 0: the
 *                          context's eps_mu]
 *   HALS (Eq. eqn:halsupd): for r = 0..R-1 in order, if S(r,r) > 0,
 *                          Hhat(:,r) <- max(0, Hhat(:,r) + (M(:,r) - Hhat S(:,r)) / S(r,r))
 * then lambda_r = ||Hhat(:,r)||_2, H^(n)(:,r) = Hhat(:,r) / lambda_r (a zero
 * column stays zero with lambda_r = 0), and G^(n) is recomputed.
 */
int nncp_update_mu(nncp_ctx *ctx, int mode, const void *M, const double *S, double eps);
int nncp_update_hals(nncp_ctx *ctx, int mode, const void *M, const double *S);

/*
 * BPP update of mode n (Section 4.3.3, Eq. eqn:snls): every row of Hhat
 * becomes the exact solution of the nonnegative least-squares subproblem
 *   min_{x >= 0} 0.5 x^T S x - m^T x   (m = that row of M),
 * found by block principal pivoting on the KKT conditions x >= 0,
 * y = S x - m >= 0, x_i y_i = 0, with S_FF solved by Cholesky in FP64 (the
 * pivoting rule is that of the method the paper cites: full switches while
 * the number of violating indices falls, three more, then the largest index
 * alone; at most 5 R + 10 solves per row, and a row whose S_FF is not
 * positive definite keeps its last solution clipped at 0).  Each row's
 * search starts from the support (the positive entries) of its current value
 * H^(n) diag(lambda), solved once; an empty support starts from x = 0.  The
 * NNLS solution does not depend on the start when S is positive definite;
 * the start only changes the number of solves.  Then normalisation and
 * G^(n) as above.  R <= 64
 * (NNCP_E_UNSUPPORTED otherwise); nncp_sweep accepts NNCP_BPP as its algo.
 */
int nncp_update_bpp(nncp_ctx *ctx, int mode, const void *M, const double *S);

/*
 * ADMM update of mode n (Section 4.3.4, Eqs. eqn:admmnls and eqn:admmupd),
 * written for the factor with the scaled dual U^(n) (I_n x R FP64, held in
 * the workspace, zero after nncp_init and nncp_set_factors, and kept from
 * one ADMM update of mode n to the next):
 *   rho = trace(S) / R;  Ht = (M + rho (Hhat + U)) (S + rho I)^-1;
 *   Hhat = max(0, Ht - U);  U = U + Hhat - Ht,
 * starting from Hhat = H^(n) diag(lambda), at most 5 passes, stopped after a
 * pass once ||Hhat - Ht||^2 / ||Hhat||^2 < 0.01 and
 * ||Hhat - Hhat_prev||^2 / ||U||^2 < 0.01 over the whole factor (the test of
 * the method the paper cites).  (S + rho I)^-1 is formed once per update by
 * Gauss-Jordan elimination (S + rho I is symmetric positive definite).  Then
 * normalisation and G^(n) as above.  R <= 64 (NNCP_E_UNSUPPORTED otherwise);
 * nncp_sweep accepts NNCP_ADMM as its algo.
 */
int nncp_update_admm(nncp_ctx *ctx, int mode, const void *M, const double *S);

/*
 * Nesterov-type update of mode n (Section 4.3.5, Eqs. eqn:nesnls and
 * eqn:nesinnerupd): every row x of Hhat takes 20 accelerated projected
 * gradient steps on the proximal subproblem
 *   min_{x >= 0} 0.5 x^T S x - m^T x + lam/2 ||x - x*||^2,
 * x* = the row of H^(n) diag(lambda) on entry (also the start value):
 *   x_{k+1} = max(0, y_k - alpha (y_k S - m + lam (y_k - x*))),
 *   y_{k+1} = x_{k+1} + beta (x_{k+1} - x_k),  y_0 = x_0 = x*.
 * The paper leaves lam, alpha and beta to the method it cites; here
 * L = the largest eigenvalue of S and L - mu the largest of L I - S, each by
 * 20 power steps from the all-ones vector; lam = max(0, (L - 100 mu) / 99)
 * (condition number of S + lam I at most 100); alpha = 1 / (L + lam);
 * beta = (1 - sqrt(q)) / (1 + sqrt(q)), q = (mu + lam) / (L + lam).  With
 * L <= 0 the rows keep their values.  Then normalisation and G^(n) as above.
 * The outer extrapolation of Eq. eqn:nesouterupd is not part of this call.
 * R <= 64 (NNCP_E_UNSUPPORTED otherwise); nncp_sweep accepts NNCP_NES as its
 * algo, and NNCP_NES_OUTER for these updates plus, after every sweep, the
 * outer step of outer iteration i (i counts the NNCP_NES_OUTER sweeps since
 * nncp_init or the last nncp_set_factors, from 1, on the device, so it
 * continues across calls and graph replays): with F^(n) = H^(n) for n < N-1 and
 * F^(N-1) = H^(N-1) diag(lambda), and F_prev the iterate before the sweep,
 * the candidate max(0, F + i^(1/N) (F - F_prev)) is normalised (lambda = the
 * product of its column norms) and replaces the iterate when its squared
 * relative error, from one extra MTTKRP of mode N-1, is lower; relerr_hist
 * then holds the candidate's error.  The outer step uses the workspace of
 * nncp_pgd for its copies.
 */
int nncp_update_nes(nncp_ctx *ctx, int mode, const void *M, const double *S);

/*
 * Loss of the current model through the identity of the appendix:
 *   ||X - [[lambda; H]]||^2 = alpha - 2 <M^(N-1), H^(N-1) diag(lambda)>
 *                             + lambda^T (Hadamard of all G) lambda.
 *   loss    1 FP64: 0.5 * ||X - [[lambda; H]]||^2 (may be NULL)
 *   relerr  1 FP64: sqrt(max(0, ||X - model||^2) / alpha) (may be NULL)
 * Costs one pass over X.
 */
int nncp_cp_loss(nncp_ctx *ctx, double *loss, double *relerr);

/*
 * nsweeps outer iterations of Algorithm 1 (modes 0..N-1 in order), each mode
 * as nncp_mttkrp + nncp_update_*, with the dimension-tree temporaries reused
 * across modes as in Algorithm 3 (two passes over X per sweep, three with
 * NNCP_NES_OUTER).  algo is one of enum nncp_algo.  After mode
 * N-1 the relative error is formed from that mode's M and Hhat (Algorithm 4):
 *   relerr_hist  nsweeps FP64: relative error after each sweep (may be NULL)
 * With options.graphs (the default) and timers off, the launches are captured
 * once on a private stream into a HIP graph and replayed on the context's
 * stream; the first call with a new (algo, nsweeps, relerr_hist) pays the
 * capture.  The graph holds kernel launches only.
 */
int nncp_sweep(nncp_ctx *ctx, int algo, int nsweeps, double *relerr_hist);

/* Capture (without running) the graph that nncp_sweep(ctx, algo, nsweeps,
 * relerr_hist) replays, so that the first such call does not pay for the
 * capture.  NNCP_E_INVAL if graphs are off or nsweeps < 1. */
int nncp_sweep_capture(nncp_ctx *ctx, int algo, int nsweeps, double *relerr_hist);

/*
 * Gradient of L = 0.5 ||X - [[H]]||^2 (lambda treated as all ones, no
 * normalisation) with respect to every factor at the current point:
 *   dL/dH^(n) = H^(n) S^(n) - M^(n),
 * with all N MTTKRPs at the same point, through the dimension tree from its
 * two root partial MTTKRPs.  Both roots come from one pass over X when
 * options.fused_grad is set and the fused path applies (BF16 tensor,
 * R <= 32, at least two modes left of the root split, its buffers within the
 * LDS; see options.fused_grad for the grid size); otherwise one pass per root
 * (two passes).  nncp_uses_fused_grad tells which.  For R <= 64 every
 * M^(n) is kept (M^(n), n < N-1, in grads[n] itself) until one launch forms
 * all gradients and the loss.
 *   grads  host array of N device pointers, each I_n x R h_dtype; they must
 *          not overlap each other, the factors or the workspace
 *   loss   1 FP64: L via the identity (may be NULL)
 */
int nncp_grad(nncp_ctx *ctx, void *const *grads, double *loss);

/* 1 if nncp_grad on this context reads X once (both root partial MTTKRPs in
 * one kernel), 0 if it reads X once per root product. */
int nncp_uses_fused_grad(const nncp_ctx *ctx);

/*
 * nsteps projected-gradient steps on L = 0.5 ||X - [[H]]||^2 (lambda = 1):
 * gradients at the current point, eta0 = 1 / max_n lmax(S^(n)) (lmax from
 * power_iters power-iteration steps from the all-ones vector), trial
 * H' = max(0, H - eta grad) for all modes at once, accepted when
 * L(H') <= L(H) - armijo_c * sum_n ||H' - H||^2 / eta, else eta is halved,
 * at most max_halvings times; without an accepted trial H is unchanged.
 *   loss_hist, eta_hist  host arrays of nsteps FP64 (may be NULL): L after
 *                        each step and the accepted eta (0 when rejected)
 * Synchronises the stream once per trial.  Needs R <= 64 (else
 * NNCP_E_UNSUPPORTED).
 */
int nncp_pgd(nncp_ctx *ctx, int nsteps, double armijo_c, int max_halvings, int power_iters,
             double *loss_hist, double *eta_hist);

/*
 * Per-category GPU time, from HIP events recorded on the context's stream
 * around each launch while timing is enabled (the time-breakdown categories
 * of the paper's experiments, restricted to one GPU):
 *   0  left partial MTTKRP kernel (GEMM over modes S..N-1); in nncp_grad
 *      with the fused path, the kernel computing both root products
 *   1  right partial MTTKRP kernel (GEMM over modes 0..S-1)
 *   2  Khatri-Rao operands of the partial MTTKRPs
 *   3  multi-TTVs and split-reduction finalize
 *   4  factor update (MU, HALS, BPP, ADMM, NES, normalisation, Gram,
 *      relative error, the NES outer step except its MTTKRP)
 * Inside nncp_sweep the Gram step of an update (slice sum, G^(n), gamma and
 * the next mode's S) runs as an extra workgroup of the next Khatri-Rao or
 * multi-TTV launch, so its time counts in category 2 or 3 there.
 * nncp_timers_enable(ctx, 1) starts recording (and clears the totals);
 * nncp_timers_read synchronises the stream and returns the totals in
 * milliseconds and the number of timed launches per category (host arrays of
 * NNCP_TIMER_CATEGORIES entries).  Recording adds two event records per
 * launch; it allocates no device memory.
 */
#define NNCP_TIMER_CATEGORIES 5
int nncp_timers_enable(nncp_ctx *ctx, int on);
int nncp_timers_read(nncp_ctx *ctx, double *ms, int64_t *launches);

/* Release the context (host memory only; borrowed buffers are untouched). */
int nncp_destroy(nncp_ctx *ctx);

/* Message for the calling thread's most recent failure ("" if none). */
const char *nncp_last_error(void);

/* Root split S chosen for this context (modes 0..S-1 on the left). */
int nncp_split(const nncp_ctx *ctx);

/*
 * Kernel path chosen for the two partial MTTKRPs (side 0 = left, reduces over
 * modes S..N-1; side 1 = right, reduces over modes 0..S-1): 1 = matrix cores
 * (MFMA), 0 = vector ALU.  Returns NNCP_E_INVAL for a bad side.
 */
int nncp_gemm_path(const nncp_ctx *ctx, int side);

/*
 * Launch plan of one partial MTTKRP (side as for nncp_gemm_path), for
 * inspection and for bounding its rounding error.  info is a host array of 8
 * entries:
 *   [0] 1 = matrix cores, 0 = vector ALU
 *   [1] Pf      length of the fast part of the reduced index (the Khatri-Rao
 *               rows held on chip; one accumulator block)
 *   [2] Ps      number of fast blocks (Pf * Ps = the reduced length)
 *   [3] nsplit  workgroups the reduction is split over (partials added in
 *               split order)
 *   [4] tiles   output tiles (the other grid dimension)
 *   [5] W       left side: fast indices staged in LDS at a time
 *   [6] hl      1 = the Khatri-Rao operand is a hi + lo pair of the tensor's
 *               16-bit type
 *   [7] direct  1 = the product kernel forms the operand from the factors
 *               (options.krp_kernel), 0 = a kernel of its own forms it first
 */
int nncp_gemm_plan(const nncp_ctx *ctx, int side, int64_t *info);

/*
 * Measurement helper: one streaming read of a device buffer (16-byte
 * non-temporal loads, grid-stride over `workgroups` workgroups of 256 threads), the attainable
 * read bandwidth that the partial MTTKRP's HBM rate is compared with.
 *   buf    device buffer of `bytes` bytes (a positive multiple of 16), read only
 *   out4   4 device bytes, written only if the XOR of everything read equals
 *          a fixed value (so the loads cannot be dropped)
 * Asynchronous on `stream`; time it with events on that stream.
 */
int nncp_read_probe(const void *buf, size_t bytes, int workgroups, void *out4, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NNCP_H */
