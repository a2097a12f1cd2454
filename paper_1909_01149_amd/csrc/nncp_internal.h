// Internal declarations shared by the HIP translation units of the NNCP
// library: element types, matrix-core wrappers, and the host-side launchers
// that the context code (nncp_ctx.hip) calls.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nncp.h"

namespace nncp {

typedef __bf16 bf16_t;
typedef _Float16 f16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Per-tensor-dtype traits for the matrix-core partial MTTKRP.
//   AT    accumulator / factor / temporary type
//   VEC   elements in one 16-byte load
//   KL    reduction elements each lane feeds to one MFMA (8 for the 16x16x32
//         BF16/FP16 instructions, 1 for the 16x16x4 FP32/FP64 ones)
// ---------------------------------------------------------------------------
template <typename XT> struct XTraits;
template <> struct XTraits<bf16_t> {
  typedef float AT;
  static constexpr int VEC = 8, KL = 8;
};
template <> struct XTraits<f16_t> {
  typedef float AT;
  static constexpr int VEC = 8, KL = 8;
};
template <> struct XTraits<float> {
  typedef float AT;
  static constexpr int VEC = 4, KL = 1;
};
template <> struct XTraits<double> {
  typedef double AT;
  static constexpr int VEC = 2, KL = 1;
};

// ---------------------------------------------------------------------------
// Plans for one partial MTTKRP (one side of the dimension-tree root).
//
// The tensor is viewed as a k x m row-major matrix Xr (m = prod of modes
// 0..S-1, contiguous; k = prod of modes S..N-1).
//   left  (GEMM-L):  T[i, r] = sum_j Xr[j, i] * K(j, r)   (reduce over rows)
//   right (GEMM-R):  T[j, r] = sum_i Xr[j, i] * K(i, r)   (reduce over columns)
// The Khatri-Rao operand of the reduced modes is factored as
//   K(rho, r) = Kfast(rho mod Pf, r) * Kslow(rho / Pf, r)
// where "fast" is a prefix of the reduced modes (Pf rows) and "slow" the rest.
// Kfast is staged in LDS in the tensor's element type (hi, and optionally a
// lo correction); Kslow is applied to each fast block's partial result.
// ---------------------------------------------------------------------------
struct GemmPlan {
  int side;          // 0 = left, 1 = right
  int mfma;          // 1 = matrix-core kernel, 0 = vector-ALU kernel
  int64_t m, k;      // Xr is k x m
  int64_t Pf, Ps;    // fast / slow sizes of the reduced index (Pf * Ps = reduced length)
  int64_t W;         // left kernel: fast indices staged in LDS at a time (W divides Pf)
  int NT;            // 16-column tiles (Rpad = 16 * NT)
  int Rpad;
  int hl;            // hi+lo Khatri-Rao operand
  int nt_loads;      // left kernel: non-temporal loads of X (large tensors)
  int nsplit;        // split of the reduction across workgroups
  int64_t tiles;     // output tiles (grid.x)
  size_t lds_bytes;  // dynamic LDS of the MFMA kernel
  int fast_lo, fast_hi, slow_lo, slow_hi;  // mode ranges [lo, hi) of the reduced modes
};

// Factor-set view passed to kernels (device pointers, row-major I_n x R).
struct FactorSet {
  const void *H[NNCP_MAX_MODES];
};

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files; all asynchronous on `st`)
// ---------------------------------------------------------------------------

// Khatri-Rao operand of a partial MTTKRP: Kfast [Rpad][Pf] (tensor type, hi
// then lo) and Kslow [Ps][Rpad] (factor type).  One launch.
hipError_t launch_krp_operands(int xdt, const GemmPlan &p, int R, const int64_t *dims, int N,
                               const FactorSet &F, void *kfast, void *kslow, hipStream_t st);

// Partial MTTKRP.  `out` receives [nsplit][...] partials (see the kernels) or,
// when nsplit == 1 and direct != 0, the node itself ([r][row] layout).
hipError_t launch_partial_mttkrp(int xdt, const GemmPlan &p, int R, const void *X,
                                 const int64_t *dims, int N, int S, const FactorSet &F,
                                 const void *kfast, const void *kslow, void *out,
                                 hipStream_t st);

// Sum split partials of a partial MTTKRP into a node ([r][row]) or, when
// leaf != 0, an M matrix ([row][r]).
hipError_t launch_finalize(int hdt, const GemmPlan &p, int R, const void *part, void *out,
                           int leaf, hipStream_t st);

// Multi-TTV, contiguous reduction over the node's first mode:
//   out(q, r) = sum_{i<Ia} T[r][i + Ia q] * H(i, r)
// out is a node [r][q] or, when leaf != 0, M [q][r].
hipError_t launch_mttv_contig(int hdt, const void *T, int64_t Ia, int64_t Q, int R,
                              const void *H, void *out, int leaf, hipStream_t st);

// Multi-TTV, strided reduction keeping the node's first mode:
//   M(i, r) = sum_q T[r][i + Ia q] * prod_{k in modes} H^(k)(digit_k(q), r)
// When M is NULL the split partials are left in `part` ([nsplit][Ia][R]) for
// the consumer to add; *nsplit_out receives their count.
hipError_t launch_mttv_strided(int hdt, const void *T, int64_t Ia, const int64_t *qdims, int nq,
                               const void *const *Hq, int R, void *M, void *part,
                               int64_t part_elems, hipStream_t st, int *nsplit_out);
int64_t mttv_strided_part_elems(int hdt, int64_t Ia, const int64_t *qdims, int nq, int R);

// Gram G = H^T H (FP64) for one factor; single workgroup.
hipError_t launch_gram(int hdt, const void *H, int64_t I, int R, double *G, hipStream_t st);

// S = Hadamard of G[k], k != mode (R x R), single workgroup.
hipError_t launch_hadamard(const double *G, int N, int R, int mode, double *S, hipStream_t st);

// ||X||^2 in FP64 (two-stage deterministic reduction; part >= 1024 doubles).
hipError_t launch_sumsq(int xdt, const void *X, int64_t n, double *part, double *out,
                        hipStream_t st);

struct UpdateArgs {
  int algo;             // NNCP_MU / NNCP_HALS
  int64_t I;            // rows
  int R;
  int N, mode;
  const void *M;        // I x R (hdt), or msplit partial copies of it
  int msplit;           // M = sum_{s < msplit} M[s * mstride ...], added in order
  int64_t mstride;
  const double *S;      // R x R (the Hadamard product of the Grams other than mode)
  double *S_next;       // if not NULL: receives the Hadamard product of the
  int next_mode;        //   Grams other than next_mode, after G^(mode) is new
  double *G;            // N x R x R Grams (G[mode] rewritten)
  void *H;              // factor (hdt), in/out
  double *lambda;       // R, in/out
  double *hhat;         // I x R FP64 scratch
  double *part;         // per-workgroup partials, update_part_elems(I, R) doubles
  double *gpart;        // R <= 64: per-slice Gram tiles, norm_gpart_elems(R) doubles
  unsigned *ticket;     // R <= 64: zero before the first launch; left at zero
  double eps;
  // error after a sweep (mode N-1 only): alpha, out pointers (may be NULL)
  const double *alpha;
  double *relerr_out;
  double *scal;         // [0]=beta [1]=gamma [2]=raw relerr^2
  // ADMM (R <= 64): the mode's dual U (I x R, in/out), the summed M of the
  // first pass (I x R), the inverse of S + rho I with rho and a failure flag
  // after it (R x R + 2), per-pass per-workgroup norms and per-pass status
  double *admmU, *admmMc, *admmP, *admmNorm;
  int *admmStatus;
};
constexpr int kAdmmMaxit = 5;         // passes per ADMM update (Section 4.3.4)
constexpr double kAdmmTol = 0.01;     // stopping tolerance of the cited method
hipError_t launch_update(int hdt, const UpdateArgs &a, hipStream_t st);
// workgroups of the finish kernel (R <= 64) and the rows each one normalises
constexpr int kNormWG = 16;
int norm_workgroups(int64_t I, int64_t *rows_per_wg);
// doubles of per-slice Gram tiles the finish kernel needs (R <= 64)
int norm_gpart_elems(int R);
int64_t update_part_elems(int64_t I, int R);

// loss of [[lambda; H]] from M^(N-1): loss = 0.5 (alpha - 2 beta + gamma)
hipError_t launch_loss(int hdt, int N, int R, int64_t In, const void *M, const void *H,
                       const double *lambda, const double *G, const double *alpha, double *loss,
                       double *relerr, double *scal, hipStream_t st);

// grad = H S - M (lambda = 1), S from the Grams (R <= 64) or the given S
hipError_t launch_grad(int hdt, int64_t I, int R, int N, int mode, const void *M, const void *H,
                       const double *G, const double *S, void *grad, hipStream_t st);

// eta0 = 1 / max_n lmax(S^(n)) by power iteration; writes eta[0] (R <= 64)
hipError_t launch_pgd_eta(const double *G, int N, int R, int iters, double *eta, hipStream_t st);

// H' = max(0, H - eta g); accumulates sum (H'-H)^2 into part[blockIdx] then d[0]
hipError_t launch_pgd_trial(int hdt, int64_t n, const void *H, const void *g, double eta,
                            void *Hn, double *part, double *d_out, hipStream_t st);

}  // namespace nncp
