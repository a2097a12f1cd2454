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
// Waves per workgroup of the right matrix-core partial MTTKRP (they take
// contiguous pieces of the workgroup's share of the reduction); eight
// measured 4-6% faster than four on the 16-bit tensors, equal on FP32.
constexpr int kRightWaves = 8;

// Waves per workgroup of the left matrix-core partial MTTKRP (es = element
// size of the tensor, QV columns per lane, NT 16-column tiles, slow = the
// Khatri-Rao operand has a slow part): eight, except where the slow part's
// extra accumulators would not fit the registers of two waves per SIMD.
__host__ __device__ constexpr int left_waves(int es, int QV, int NT, bool slow) {
  return slow && ((es == 2 && QV == 8) || (es == 8 && NT == 4)) ? 4 : 8;
}

struct GemmPlan {
  int side;          // 0 = left, 1 = right
  int mfma;          // 1 = matrix-core kernel, 0 = vector-ALU kernel
  int64_t m, k;      // Xr is k x m
  int64_t Pf, Ps;    // fast / slow sizes of the reduced index (Pf * Ps = reduced length)
  int64_t W;         // left kernel: fast indices staged in LDS at a time (W divides Pf)
  int NT;            // 16-column tiles (Rpad = 16 * NT)
  int Rpad;
  int hl;            // hi+lo Khatri-Rao operand
  int nt_loads;      // left kernel: non-temporal loads of X (tensors over 1 GiB)
  int nsplit;        // split of the reduction across workgroups
  int64_t tiles;     // output tiles (grid.x)
  size_t lds_bytes;  // dynamic LDS of the MFMA kernel
  int fast_lo, fast_hi, slow_lo, slow_hi;  // mode ranges [lo, hi) of the reduced modes
  int direct;        // MFMA kernel reads the factors as its operand (one fast
                     // mode, at most one slow mode, not FP16): no operand kernel
};

// Factor-set view passed to kernels (device pointers, row-major I_n x R).
struct FactorSet {
  const void *H[NNCP_MAX_MODES];
};

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files; all asynchronous on `st`)
// ---------------------------------------------------------------------------

struct GramJob;  // the Gram step of an update (below)

// Khatri-Rao operand of a partial MTTKRP: Kfast [Rpad][Pf] (tensor type, hi
// then lo) and Kslow [Ps][Rpad] (factor type).  One launch.
// A non-empty *carry is run by an extra workgroup of the launch and emptied.
hipError_t launch_krp_operands(int xdt, const GemmPlan &p, int R, const int64_t *dims, int N,
                               const FactorSet &F, void *kfast, void *kslow, hipStream_t st,
                               GramJob *carry = nullptr);
// The operands of two plans in one launch (not FP16, no Gram step carried):
// the same values as two launch_krp_operands calls.
hipError_t launch_krp_operands2(int xdt, const GemmPlan &p0, void *kf0, void *ks0,
                                const GemmPlan &p1, void *kf1, void *ks1, int R,
                                const int64_t *dims, int N, const FactorSet &F, hipStream_t st);

// Partial MTTKRP.  `out` receives [nsplit][...] partials (see the kernels) or,
// when nsplit == 1, the node itself ([r][row] layout) for the left product.
// The matrix-core kernels take their operand from kfast / kslow
// (launch_krp_operands) or, when p.direct, from the factors F.  A non-empty
// *carry, which must be a split Gram step (parts > 0), is run by extra
// workgroups of a matrix-core launch and emptied; the vector-ALU path cannot
// carry one (hipErrorInvalidValue).
hipError_t launch_partial_mttkrp(int xdt, const GemmPlan &p, int R, const void *X,
                                 const int64_t *dims, int N, int S, const FactorSet &F,
                                 const void *kfast, const void *kslow, void *out,
                                 hipStream_t st, GramJob *carry = nullptr);

// Both root partial MTTKRPs in one pass over X (BF16 tensor, NT <= 2, the
// left product written straight into its node out_l, [r][m]); the right
// product leaves dual_tiles(m) partials in out_r, [tile][R][k] when
// r_major != 0 (the node layout: added by launch_finalize with part_rmajor
// 1) else [tile][k][R] (the layout of M), to be added in tile order
// (launch_finalize with nsplit = dual_tiles(m)).  kfl / ksl are
// the right plan's Khatri-Rao operands (launch_krp_operands with pr); kfr is
// the left product's whole operand K_R, [hl][Rpad][k] (launch_krp_operands
// with dual_full_plan(pl)).
hipError_t launch_dual_mttkrp(int xdt, const GemmPlan &pl, const GemmPlan &pr, int R,
                              const void *X, const void *kfr, const void *kfl, const void *ksl,
                              void *out_l, void *out_r, int r_major, hipStream_t st);
// the left plan with every reduced mode in the fast part (Pf = k, Ps = 1)
inline GemmPlan dual_full_plan(const GemmPlan &pl, int S, int N) {
  GemmPlan p = pl;
  p.fast_lo = S;
  p.fast_hi = N;
  p.slow_lo = N;
  p.slow_hi = N;
  p.Pf = pl.k;
  p.Ps = 1;
  return p;
}
size_t dual_lds_bytes(int NT, int hl, int64_t PfL);
int64_t dual_tiles(int64_t m);

// Sum split partials of a partial MTTKRP into a node ([r][row]) or, when
// leaf != 0, an M matrix ([row][r]).  The partials are [split][R][rows] for
// the left product and [split][rows][R] for the right one, unless
// part_rmajor (0 or 1) says otherwise.
hipError_t launch_finalize(int hdt, const GemmPlan &p, int R, const void *part, void *out,
                           int leaf, hipStream_t st, int part_rmajor = -1);

// Multi-TTV, contiguous reduction over the node's first mode:
//   out(q, r) = sum_{i<Ia} T[r][i + Ia q] * H(i, r)
// out is a node [r][q] or, when leaf != 0, M [q][r].  A non-empty *carry is
// run (in an extra workgroup, or as a kernel of its own first) and emptied.
hipError_t launch_mttv_contig(int hdt, const void *T, int64_t Ia, int64_t Q, int R,
                              const void *H, void *out, int leaf, hipStream_t st,
                              GramJob *carry = nullptr);

// Multi-TTV, strided reduction keeping the node's first mode:
//   M(i, r) = sum_q T[r][i + Ia q] * prod_{k in modes} H^(k)(digit_k(q), r)
// When M is NULL the split partials are left in `part` ([nsplit][Ia][R]) for
// the consumer to add; *nsplit_out receives their count.  A non-empty *carry
// is run by an extra workgroup and emptied.
hipError_t launch_mttv_strided(int hdt, const void *T, int64_t Ia, const int64_t *qdims, int nq,
                               const void *const *Hq, int R, void *M, void *part,
                               int64_t part_elems, hipStream_t st, int *nsplit_out,
                               GramJob *carry = nullptr);
int64_t mttv_strided_part_elems(int hdt, int64_t Ia, const int64_t *qdims, int nq, int R);

// Launch parameters of a strided multi-TTV (the kernel's argument).
struct StridedArgs {
  const void *H[NNCP_MAX_MODES];
  int64_t qd[NNCP_MAX_MODES];
  int nq;
  int64_t Ia, Q;
  int R, IT, QS, nsplit;
};

// A multi-TTV planned instead of launched, for launch_mttv_jobs.
struct MttvJob {
  int kind;  // 0 strided (split partials left in out), 1 contiguous (packed form)
  const void *T;
  void *out;  // strided: the split partials; contiguous: the node or M
  StridedArgs sa;
  int64_t gx;  // strided: workgroups along i
  int64_t Ia, Q;
  int R, leaf;
  const void *H;
  int64_t blocks;
  int vec;                   // the job's kernel variant (strided V, contiguous GL)
  const char *rd0, *rd1;     // bytes read (T; the factors are only read)
  const char *wr0, *wr1;     // bytes written
};

// The launch launch_mttv_contig / launch_mttv_strided (partials left for the
// consumer, no Gram step to carry) would make, as a job, when it is one of
// the kinds launch_mttv_jobs can group (strided, or contiguous with
// Ia / (16 / sizeof element) a power of two below 64); false otherwise.
bool plan_mttv_contig(int hdt, const void *T, int64_t Ia, int64_t Q, int R, const void *H,
                      void *out, int leaf, MttvJob *j);
bool plan_mttv_strided(int hdt, const void *T, int64_t Ia, const int64_t *qdims, int nq,
                       const void *const *Hq, int R, void *part, int64_t part_elems, MttvJob *j,
                       int *nsplit_out);
// Run planned jobs in as few launches as their data dependencies allow: a job
// goes after every earlier job that writes bytes it reads or writes, or reads
// bytes it writes; independent jobs of one level share a launch (up to four,
// of matching kernel variants).  Results equal those of the separate launches
// in job order.
hipError_t launch_mttv_jobs(int hdt, const MttvJob *jobs, int n, hipStream_t st);

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
  double *gpart;        // R <= 64: norm_gpart_elems(R) doubles of scratch (GramJob)
  double *beta_out;     // R <= 64: receives beta for the Gram step (GramJob)
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
  // Nesterov-type update (R <= 64): [L, mu, lam, alpha, beta, ok] written by
  // its parameter kernel; always a valid address of 6 doubles
  double *nesParam;
  // the sweep's deferred MU/HALS path (R <= 64): rows written straight into
  // H without normalisation; lambda folded only when fold_lambda is set;
  // dead[r] != 0 (R doubles) marks a column whose model column has been zero
  // since an update zeroed it (where the normalised iteration's lambda_r is
  // 0, so every later start value of column r is zero)
  int defer, fold_lambda;
  const double *dead;
};
constexpr int kAdmmMaxit = 5;         // passes per ADMM update (Section 4.3.4)
constexpr double kAdmmTol = 0.01;     // stopping tolerance of the cited method
constexpr int kNesIters = 20;         // steps per Nesterov-type update (Section 4.3.5)
constexpr int kNesPower = 20;         // power steps for each extreme eigenvalue of S
constexpr double kNesKappa = 100.0;   // condition number the proximal weight allows
// workgroups of the finish kernel (R <= 64) and the rows each one normalises
constexpr int kNormWG = 8;
int norm_workgroups(int64_t I, int64_t *rows_per_wg);
// most Gram slices the Gram step adds (the finish kernel writes kNormWG, the
// row kernel of the sweep's deferred path up to this many)
constexpr int kGramSlices = 256;
// scratch of the Gram step (R <= 64): kGramSlices slices of Gram tiles, then
// the R x R Hadamard product of the Grams other than mode and next_mode
__host__ __device__ inline int64_t norm_pn_offset(int R) {
  const int T = (R + 15) / 16;
  return (int64_t)kGramSlices * (T * (T + 1) / 2) * 256;
}
int norm_gpart_elems(int R);
int64_t update_part_elems(int64_t I, int R);

// Cross-lane exchange through LDS inside one wave: the wave's LDS accesses
// are performed in order, so a wavefront-scope fence with a scheduling
// barrier is all that orders one lane's write before another lane's read.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// The Gram step of an update with R <= 64.  The update's last kernel leaves
// the Gram of the new factor as nw slices of upper 16 x 16 tiles (one slice
// per workgroup, tiles of the R x R grid in row-major order) together with
// lambda, beta and the product pn of the Grams other than mode and
// next_mode.  This step adds the slices in slice order into G^(mode) (both
// halves), forms gamma = lambda^T (S .* G^(mode)) lambda and the relative
// error when asked, and the next mode's S = pn .* G^(mode).  It runs as one
// workgroup (its first 256 threads), either a kernel of its own or an extra workgroup of
// the next kernel on the stream ("carrier"), which must not touch G, S or the
// error outputs.  R == 0 marks an empty job.
// ---------------------------------------------------------------------------
struct GramJob {
  const double *gpart;   // nw x ntile x 256 slices
  const double *pn;      // R x R, read when S_next is set and pn_inline is 0
  const double *beta_part;  // if not NULL: beta = sum of nbeta partials (in order)
  double *G;             // N x R x R Grams; G[mode] written
  const double *S;       // S of this mode (read for gamma)
  double *S_next;        // may be NULL; may alias S
  const double *lambda;  // R
  const double *beta;    // 1, written by the update (always a valid address)
  const double *alpha;   // ||X||^2 (always a valid address)
  double *relerr_out;    // may be NULL
  double *scal;          // may be NULL: [0]=beta [1]=gamma [2]=raw relerr^2
  int R, N, mode, next_mode, nw;
  int nbeta;
  int pn_inline;         // 1: the product of the Grams other than mode and
                         // next_mode is formed here from G (no pn buffer)
  double *dead;          // if not NULL: dead[x] = 1 where G^(mode)(x, x) == 0
  // parts > 0: the step is split over `parts` workgroups (gram_part), each
  // adding the slices of 32 upper-tile entries; gamma then comes from the
  // update's per-workgroup partials (gamma_part, nbeta of them) instead of
  // G and S
  int parts;
  const double *gamma_part;
};

// One workgroup (its first 256 threads).  Thread t takes the upper-tile entries u = t +
// 256 k (consecutive threads read consecutive slice entries) and writes both
// (x, y) and (y, x): G, S and pn are exactly symmetric (each pair is written
// from one value), so gamma adds the diagonal once and each off-diagonal pair
// twice.  Each thread reads S(x, y) before it writes S_next(x, y) and
// S_next(y, x), and no other thread touches either.  All loads of a round are
// unconditional (clamped indices) so that they are in flight together; the
// slices are added in slice order, eight at a time.
template <int FE>
__device__ inline void gram_finish(const GramJob &j) {
  __shared__ double gred[4];
  const int R = j.R, RR = R * R, T = (R + 15) >> 4, slice = (T * (T + 1) / 2) * 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool want_err = j.relerr_out || j.scal;
  // threads past the first 256 (a carrier of 512) only meet the barrier
  if (tid >= 256) {
    if (want_err) __syncthreads();
    return;
  }
  const int nw = j.nw;
  double *Gm = j.G + (int64_t)j.mode * RR;
  const double *pnp = (j.S_next && !j.pn_inline) ? j.pn : j.lambda;  // any valid address when unused
  const double *sp = want_err ? j.S : j.lambda;
  const double alpha = j.alpha[0];
  double beta = j.beta[0];  // both always valid addresses
  double gsum = 0.0;
  for (int u0 = tid; u0 < slice; u0 += 256 * FE) {
    double sv[FE], la[FE], lb[FE], pn[FE], sum[FE];
    int xs[FE], ys[FE];
    bool ok[FE];
#pragma unroll
    for (int kk = 0; kk < FE; ++kk) {
      const int u = u0 + 256 * kk < slice ? u0 + 256 * kk : slice - 1;
      // tile (tx, tx + q) of the upper tiles in row-major order (T <= 4)
      int tx = 0, q = u >> 8;
#pragma unroll
      for (int r = 0; r < 3; ++r)
        if (tx == r && q >= T - r) { q -= T - r; tx = r + 1; }
      const int xl = (u >> 4) & 15, yl = u & 15;
      const int x = 16 * tx + xl, y = 16 * (tx + q) + yl;
      ok[kk] = u0 + 256 * kk < slice && x < R && y < R && (q > 0 || xl <= yl);
      xs[kk] = x < R ? x : R - 1;
      ys[kk] = y < R ? y : R - 1;
      const int e = xs[kk] * R + ys[kk];
      la[kk] = j.lambda[xs[kk]];
      lb[kk] = j.lambda[ys[kk]];
      sv[kk] = sp[want_err ? e : 0];
      if (j.S_next && j.pn_inline) {
        double p = 1.0;
        for (int g = 0; g < j.N; ++g)
          if (g != j.mode && g != j.next_mode) p *= j.G[(int64_t)g * RR + e];
        pn[kk] = p;
      } else {
        pn[kk] = pnp[j.S_next ? e : 0];
      }
    }
    // the slices in order, eight loads per entry in flight
    for (int w0 = 0; w0 < nw; w0 += kNormWG) {
      double v[FE][kNormWG];
#pragma unroll
      for (int kk = 0; kk < FE; ++kk) {
        const int u = u0 + 256 * kk < slice ? u0 + 256 * kk : slice - 1;
#pragma unroll
        for (int w = 0; w < kNormWG; ++w)
          v[kk][w] = j.gpart[(int64_t)(w0 + w < nw ? w0 + w : nw - 1) * slice + u];
      }
#pragma unroll
      for (int kk = 0; kk < FE; ++kk) {
        double s0 = w0 == 0 ? v[kk][0] : sum[kk] + v[kk][0];
#pragma unroll
        for (int w = 1; w < kNormWG; ++w)
          if (w0 + w < nw) s0 += v[kk][w];
        sum[kk] = s0;
      }
    }
#pragma unroll
    for (int kk = 0; kk < FE; ++kk) {
      if (!ok[kk]) continue;
      const int x = xs[kk], y = ys[kk];
      Gm[x * R + y] = sum[kk];
      Gm[y * R + x] = sum[kk];
      if (j.dead && x == y && sum[kk] == 0.0) j.dead[x] = 1.0;
      if (want_err) gsum += (x == y ? 1.0 : 2.0) * (la[kk] * sv[kk] * sum[kk] * lb[kk]);
      if (j.S_next) {
        const double sn = j.next_mode == j.mode ? pn[kk] : pn[kk] * sum[kk];
        j.S_next[x * R + y] = sn;
        j.S_next[y * R + x] = sn;
      }
    }
  }
  if (!want_err) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) gsum += __shfl_xor(gsum, o);
  if (lane == 0) gred[wave] = gsum;
  __syncthreads();
  if (tid == 0) {
    if (j.beta_part) {
      beta = j.beta_part[0];
      for (int w = 1; w < j.nbeta; ++w) beta += j.beta_part[w];
    }
    const double gamma = gred[0] + gred[1] + gred[2] + gred[3];
    const double e2 = (alpha - 2.0 * beta + gamma) / alpha;
    if (j.scal) {
      j.scal[0] = beta;
      j.scal[1] = gamma;
      j.scal[2] = e2;
    }
    if (j.relerr_out) j.relerr_out[0] = sqrt(e2 > 0.0 ? e2 : 0.0);
  }
}

// Part p (0 <= p < j.parts) of a Gram step split over workgroups, one
// workgroup of at least 256 threads (the first 256 work): the upper-tile entries u = 32 p .. 32 p + 31.  Thread
// t adds the slices w = t / 32, t / 32 + 8, ... of entry 32 p + t % 32 in
// that order, and the eight groups are added in group order through LDS, so
// the sum is the same on every run.  Part 0 also forms beta, gamma and the
// relative error from the update's partials.  Only the thread of entry
// (x, y) writes G(x, y), G(y, x), S_next(x, y), S_next(y, x) and dead[x].
__device__ inline void gram_part(const GramJob &j, int p) {
  __shared__ double red[8][32];
  const int R = j.R, RR = R * R, T = (R + 15) >> 4, slice = (T * (T + 1) / 2) * 256;
  const int tid = threadIdx.x, e32 = tid & 31, grp = tid >> 5;
  // threads past the first 256 (a carrier of 512) only meet the barriers
  if (tid >= 256) {
    __syncthreads();
    if (p == 0 && (j.relerr_out || j.scal)) __syncthreads();
    return;
  }
  const int u = 32 * p + e32;
  const int uc = u < slice ? u : slice - 1;
  const int nw = j.nw;
  // this thread's slices eight at a time (few registers: the step rides
  // along with kernels whose own register use is small)
  double acc = 0.0;
  for (int w0 = grp; w0 < nw; w0 += 64) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int w = w0 + 8 * k;
      v[k] = w < nw ? j.gpart[(int64_t)w * slice + uc] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (w0 + 8 * k < nw) acc += v[k];
  }
  red[grp][e32] = acc;
  __syncthreads();
  if (tid < 32 && u < slice) {
    double sum = red[0][tid];
#pragma unroll
    for (int g = 1; g < 8; ++g) sum += red[g][tid];
    int tx = 0, q = u >> 8;
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (tx == r && q >= T - r) { q -= T - r; tx = r + 1; }
    const int xl = (u >> 4) & 15, yl = u & 15;
    const int x = 16 * tx + xl, y = 16 * (tx + q) + yl;
    if (x < R && y < R && (q > 0 || xl <= yl)) {
      double *Gm = j.G + (int64_t)j.mode * RR;
      Gm[x * R + y] = sum;
      Gm[y * R + x] = sum;
      if (j.dead && x == y && sum == 0.0) j.dead[x] = 1.0;
      if (j.S_next) {
        double pn = 1.0;
        if (j.pn_inline) {
          for (int g = 0; g < j.N; ++g)
            if (g != j.mode && g != j.next_mode) pn *= j.G[(int64_t)g * RR + x * R + y];
        } else {
          pn = j.pn[x * R + y];
        }
        const double sn = j.next_mode == j.mode ? pn : pn * sum;
        j.S_next[x * R + y] = sn;
        j.S_next[y * R + x] = sn;
      }
    }
  }
  if (p == 0 && (j.relerr_out || j.scal)) {
    // the update's beta and gamma partials: thread t adds partials t, t +
    // 256, ..., then a fixed butterfly per wave and the four waves in order
    __shared__ double bg[2][4];
    double b = 0.0, g = 0.0;
    for (int w = tid; w < j.nbeta; w += 256) {
      b += j.beta_part[w];
      g += j.gamma_part[w];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      b += __shfl_xor(b, o);
      g += __shfl_xor(g, o);
    }
    if ((tid & 63) == 0) {
      bg[0][tid >> 6] = b;
      bg[1][tid >> 6] = g;
    }
    __syncthreads();
    if (tid != 0) return;
    const double beta = bg[0][0] + bg[0][1] + bg[0][2] + bg[0][3];
    const double gamma = bg[1][0] + bg[1][1] + bg[1][2] + bg[1][3];
    const double alpha = j.alpha[0];
    const double e2 = (alpha - 2.0 * beta + gamma) / alpha;
    if (j.scal) {
      j.scal[0] = beta;
      j.scal[1] = gamma;
      j.scal[2] = e2;
    }
    if (j.relerr_out) j.relerr_out[0] = sqrt(e2 > 0.0 ? e2 : 0.0);
  }
}

// workgroups a Gram step needs (0 for an empty job)
__host__ __device__ inline int gram_blocks(const GramJob &j) {
  return j.R == 0 ? 0 : (j.parts > 0 ? j.parts : 1);
}
// run block p of a Gram step: FE = 3 entries per thread and round for the
// kernel of its own (one round up to R = 32), FE = 1 in a carrier, whose own
// kernel's register budget (and so its occupancy) it would otherwise set
template <int FE = 1>
__device__ inline void gram_run(const GramJob &j, int p) {
  if (j.parts > 0) {
    if (p < j.parts) gram_part(j, p);
  } else if (p == 0) {
    gram_finish<FE>(j);
  }
}

// Launches the update.  For R <= 64 the Gram step is left out and *job
// describes it (job->R == 0 otherwise); the caller runs it before anything
// reads G, S_next or the error outputs.  With a.defer (MU/HALS, R <= 64) the
// rows go straight into H unnormalised, in one kernel that also leaves the
// Gram slices and the <M, Hhat> partials for the Gram step.
hipError_t launch_update(int hdt, const UpdateArgs &a, hipStream_t st, GramJob *job);
// waves (rows per pass) of a workgroup of the deferred row kernel
constexpr int kDeferWaves = 4;
// workgroups of the deferred row kernel (at most kGramSlices)
int defer_workgroups(int64_t I);
// End of the sweep's deferred path: s_k(r) = sqrt(G^(k)(r, r)) for every
// mode, lambda_r = prod_k s_k(r); then H^(k)(:, r) /= s_k(r) and G^(k)(a, b)
// /= s_k(a) s_k(b), a column with lambda_r = 0 set to zero in every mode.
// scale: N x R + R doubles of scratch.
hipError_t launch_sweep_normalize(int hdt, const FactorSet &F, const int64_t *dims, int N, int R,
                                  double *G, double *lambda, double *scale, hipStream_t st);
// the Gram step as a kernel of its own (no-op for an empty job)
hipError_t launch_gram_finish(const GramJob &j, hipStream_t st);
// the norm kernel alone on rows left in a.hhat with nblocks per-workgroup
// partials in a.part (R <= 64); *job as for launch_update
hipError_t launch_norm_only(int hdt, const UpdateArgs &a, int nblocks, hipStream_t st,
                            GramJob *job);

// Outer extrapolation of the Nesterov-type sweeps (Eq. eqn:nesouterupd)
hipError_t launch_copy(size_t elem_bytes, const void *src, void *dst, int64_t n, hipStream_t st);
// raw = max(0, F + s (F - F_prev)), F = H (times lambda if last), FP64, with
// s = (count[0] + 1)^(1/N) and per-4-row column sums of squares in part;
// *nblocks receives their count
hipError_t launch_nes_extrap(int hdt, const void *H, const void *Hp, const double *lam,
                             const double *lamp, int last, const double *count, int N, int64_t I,
                             int R, double *raw, double *part, int *nblocks, hipStream_t st);
// lamc = product of the per-mode column norms; count[0] += 1
hipError_t launch_nes_lamc(const double *lamk, int N, int R, double *lamc, double *count,
                           hipStream_t st);
// p[0 .. n) = v (a kernel, so that it can sit in a captured graph)
hipError_t launch_fill(double *p, double v, int64_t n, hipStream_t st);
// dst = src when cand_e2 < cur_e2 (device scalars)
hipError_t launch_nes_accept(size_t elem_bytes, const void *src, void *dst, int64_t n,
                             const double *cand_e2, const double *cur_e2, hipStream_t st);
hipError_t launch_nes_accept_hist(const double *cand_e2, const double *cur_e2,
                                  const double *cand_rel, double *hist, hipStream_t st);

// loss of [[lambda; H]] from M^(N-1): loss = 0.5 (alpha - 2 beta + gamma)
hipError_t launch_loss(int hdt, int N, int R, int64_t In, const void *M, const void *H,
                       const double *lambda, const double *G, const double *alpha, double *loss,
                       double *relerr, double *scal, hipStream_t st);

// grad = H S - M (lambda = 1), S from the Grams (R <= 64) or the given S;
// M is msplit partial copies mstride apart, added in order (1: M itself)
hipError_t launch_grad(int hdt, int64_t I, int R, int N, int mode, const void *M, int msplit,
                       int64_t mstride, const void *H, const double *G, const double *S,
                       void *grad, hipStream_t st);

// Every mode's gradient grad[n] = H^(n) S^(n) - M^(n) (lambda = 1, R <= 64)
// and the loss from M^(N-1), in one launch.  M[n] holds msplit[n] partial
// copies mstride[n] apart (1: M itself) and may be grad[n] itself; M[N-1]
// must be M itself and not a gradient buffer.  wg0 is filled in by the
// launcher.
struct GradAllArgs {
  const void *M[NNCP_MAX_MODES];
  int64_t mstride[NNCP_MAX_MODES];
  const void *H[NNCP_MAX_MODES];
  void *grad[NNCP_MAX_MODES];
  int64_t I[NNCP_MAX_MODES];
  int msplit[NNCP_MAX_MODES];
  int wg0[NNCP_MAX_MODES + 1];
  int N, R;
  const double *G;
  const double *ones;   // R ones (lambda = 1)
  const double *alpha;
  double *loss;         // may be NULL
  double *scal;         // may be NULL: [0]=beta [1]=gamma [2]=raw relerr^2
};
hipError_t launch_grad_all(int hdt, GradAllArgs a, hipStream_t st);

// eta0 = 1 / max_n lmax(S^(n)) by power iteration; writes eta[0] (R <= 64)
hipError_t launch_pgd_eta(const double *G, int N, int R, int iters, double *eta, hipStream_t st);

// H' = max(0, H - eta g); accumulates sum (H'-H)^2 into part[blockIdx] then d[0]
hipError_t launch_pgd_trial(int hdt, int64_t n, const void *H, const void *g, double eta,
                            void *Hn, double *part, double *d_out, hipStream_t st);

// streaming read of `bytes` (a multiple of 16) with `workgroups` workgroups of
// 256 threads; writes out4 only in the (practically never taken) case that
// the XOR of everything read equals a fixed value
hipError_t launch_read_probe(const void *buf, size_t bytes, int workgroups, void *out4,
                             hipStream_t st);

}  // namespace nncp
