// Host side of the NNCP library: the C ABI declared in include/nncp.h, the
// planner (root split, Khatri-Rao factoring, grids), the workspace carve-up,
// the dimension-tree walk of Algorithm 3, the sweep of Algorithm 1 and the
// projected-gradient loop.  All device work is launched on the context's
// stream; nothing here allocates device memory.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nncp_internal.h"

using namespace nncp;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const int kMagic = 0x4E4E4350;  // "NNCP"
// index into the context's scalar block of the count of outer extrapolation
// steps (NNCP_NES_OUTER sweeps) since init / set_factors
const int kOuterCount = 62;
const size_t kAlign = 256;
const size_t kLdsMax = 64 * 1024;

size_t xsize(int dt) { return dt == NNCP_F64 ? 8 : dt == NNCP_F32 ? 4 : 2; }

int64_t prod(const int64_t *d, int lo, int hi) {
  int64_t p = 1;
  for (int k = lo; k < hi; ++k) p *= d[k];
  return p;
}

struct Layout {
  int N, R, S, xdt, hdt;
  int64_t dims[NNCP_MAX_MODES];
  nncp_options opt;
  GemmPlan gp[2];
  int64_t maxI, nodeA, nodeB, part_elems, kfast_elems, kslow_elems, sumI;
  // nncp_grad's single pass over X: both root products in one kernel
  int dual;
  int64_t dual_tiles, nodeR;
  // byte offsets into the workspace
  size_t off_G, off_Gt, off_S, off_scal, off_ones, off_hhat, off_upart, off_gpart,
      off_red, off_M, off_A, off_B, off_R, off_kfR, off_part, off_kf, off_ks, off_pgdH, off_pgdG, off_outer, off_admmU,
      off_admmMc, off_admmP, off_admmNorm, off_admmStatus, off_gradpart, total;
  // the gradient's strided multi-TTV partials, one region per mode (element
  // offsets into the region at off_gradpart and their sizes; 0 for a mode
  // whose M is not formed by a strided multi-TTV)
  int64_t gradpart_off[NNCP_MAX_MODES], gradpart_elems[NNCP_MAX_MODES];
};

nncp_options default_options() {
  nncp_options o;
  o.split = 0;
  o.krp_split = 1;
  o.generic = 0;
  o.eps_mu = 1e-16;
  o.graphs = 1;
  o.fused_grad = 1;
  o.krp_kernel = 0;
  return o;
}

int check_dtypes(int xdt, int hdt) {
  if (xdt == NNCP_F64 && hdt == NNCP_F64) return NNCP_OK;
  if ((xdt == NNCP_F32 || xdt == NNCP_BF16 || xdt == NNCP_F16) && hdt == NNCP_F32) return NNCP_OK;
  return fail(NNCP_E_DTYPE, "unsupported (x_dtype, h_dtype) = (%d, %d)", xdt, hdt);
}

// LDS bytes of the staged Khatri-Rao operand: rows of Pf elements, XOR-swizzled
// when a row has a multiple of 16 16-byte chunks, else padded by one chunk.
size_t stage_bytes(int Rpad, int64_t Pf, int es, int hl) {
  const int64_t sv = 16 / es;
  const int64_t ldk = ((Pf / sv) % 16 == 0) ? Pf : Pf + sv;
  return (size_t)Rpad * (size_t)ldk * es * (hl ? 2 : 1);
}

// Plan one partial MTTKRP.
void plan_side(Layout &L, int side) {
  GemmPlan &p = L.gp[side];
  memset(&p, 0, sizeof p);
  const int N = L.N, S = L.S, R = L.R;
  p.side = side;
  p.m = prod(L.dims, 0, S);
  p.k = prod(L.dims, S, N);
  const int lo = side == 0 ? S : 0, hi = side == 0 ? N : S;
  const int64_t red = prod(L.dims, lo, hi);
  p.Rpad = (R + 15) / 16 * 16;
  p.NT = p.Rpad / 16;
  const bool is16 = L.xdt == NNCP_BF16 || L.xdt == NNCP_F16;
  p.hl = is16 && L.opt.krp_split ? 1 : 0;
  const int es = (int)xsize(L.xdt);
  // tensors up to 1 GiB are read with normal loads (much of them is still in
  // the last-level cache for the next product); larger ones are streamed
  // with non-temporal loads by the left product (and the gradient's fused
  // pass); the right product measured slower with them on the 256^4 tensor
  // (4.99 against 5.47 TB/s)
  p.nt_loads = (double)p.m * (double)p.k * es > (double)(1ull << 30) ? 1 : 0;
  const int hs = (int)xsize(L.hdt);
  const int VEC = 16 / es;
  const int KL = is16 ? 8 : 1;
  const int KSTEP = side == 0 ? 4 * KL : 4 * VEC;
  const int MT = L.xdt == NNCP_F64 ? 1 : 2;
  const int QV = is16 ? (p.NT <= 2 ? 8 : 4) : VEC;

  bool mfma = !L.opt.generic && R <= 64;
  if (side == 0 && p.m % QV != 0) mfma = false;
  int64_t Pf = -1;
  int fhi = -1;
  int64_t W = -1;
  if (mfma) {
    // fast prefix: the shortest prefix of the reduced modes whose size is a
    // multiple of the step and at least 64.  The right kernel stages all of
    // it in LDS; the left kernel stages a window W that divides it.
    int64_t best = -1;
    int besthi = -1;
    for (int c = lo + 1; c <= hi; ++c) {
      const int64_t pf = prod(L.dims, lo, c);
      if (pf % KSTEP != 0) continue;
      if (side == 1 && stage_bytes(p.Rpad, pf, es, p.hl) > kLdsMax) break;
      best = pf;
      besthi = c;
      if (pf >= 64) break;
    }
    if (best >= 0) {
      W = best;
      if (side == 0)
        while (stage_bytes(p.Rpad, W, es, p.hl) > kLdsMax && W % 2 == 0 && (W / 2) % KSTEP == 0)
          W /= 2;
      if (stage_bytes(p.Rpad, W, es, p.hl) > kLdsMax) best = -1;
    }
    if (best < 0) mfma = false;
    Pf = best;
    fhi = besthi;
  }
  p.mfma = mfma ? 1 : 0;
  if (mfma) {
    p.Pf = Pf;
    p.W = W;
    p.Ps = red / Pf;
    p.fast_lo = lo; p.fast_hi = fhi; p.slow_lo = fhi; p.slow_hi = hi;
    // the operand straight from the factors: one fast mode, at most one slow
    // mode, R a multiple of 16, no FP16 column scaling, and (left product)
    // one LDS window
    p.direct = L.xdt != NNCP_F16 && fhi - lo == 1 && hi - fhi <= 1 && R == p.Rpad &&
                       (side == 1 || W == Pf) && !L.opt.krp_kernel ? 1 : 0;
    const size_t stage = stage_bytes(p.Rpad, W, es, p.hl);
    if (side == 1) {
      const size_t redb = (size_t)(kRightWaves - 1) * MT * p.NT * 4 * 64 * hs;
      p.lds_bytes = std::max(stage, redb);
      p.tiles = (p.k + 16 * MT - 1) / (16 * MT);
      const int64_t steps = p.m / KSTEP;
      // about one workgroup per CU in total: each one stages the Khatri-Rao
      // operand once, so fewer, longer workgroups re-stage less per byte of X
      int64_t ns = (256 + p.tiles - 1) / p.tiles;
      ns = std::min<int64_t>(ns, std::max<int64_t>(1, steps / 8));
      ns = std::min<int64_t>(ns, 4096);
      p.nsplit = (int)std::max<int64_t>(ns, 1);
    } else {
      // the epilogue stages 16 result columns of each wave's 16 QV columns
      // of T (rows padded by 16 bytes) in the same LDS
      const int WV = left_waves(es, QV, p.NT, p.Ps > 1);
      const size_t epi = (size_t)WV * 16 * (16 * QV * hs + 16);
      p.lds_bytes = std::max(stage, epi);
      p.tiles = (p.m + 16 * WV * QV - 1) / (16 * WV * QV);
      const int64_t steps = p.k / KSTEP;
      // no split (T written straight into the node) when the columns alone
      // give enough workgroups (about 1.5 waves per SIMD); otherwise split
      // the rows to reach about three
      const int64_t enough = 1536 / WV;
      int64_t ns = p.tiles >= enough ? 1 : (2 * enough + p.tiles - 1) / p.tiles;
      ns = std::min<int64_t>(ns, std::max<int64_t>(1, steps / 4));
      ns = std::min<int64_t>(ns, 4096);
      p.nsplit = (int)std::max<int64_t>(ns, 1);
    }
  } else {
    p.Pf = red; p.Ps = 1; p.W = red;
    p.fast_lo = lo; p.fast_hi = hi; p.slow_lo = hi; p.slow_hi = hi;
    p.direct = 0;
    p.lds_bytes = 0;
    if (side == 1) {
      p.tiles = p.k;
      int64_t ns = (1024 + p.k - 1) / p.k;
      ns = std::min<int64_t>(ns, std::max<int64_t>(1, p.m / 256));
      p.nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ns, 4096));
    } else {
      p.tiles = (p.m + 255) / 256;
      int64_t ns = (1024 + p.tiles - 1) / p.tiles;
      ns = std::min<int64_t>(ns, p.k);
      p.nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ns, 4096));
    }
  }
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int make_layout(Layout &L, int N, const int64_t *dims, int R, int xdt, int hdt,
                const nncp_options *opt) {
  if (N < 2 || N > NNCP_MAX_MODES) return fail(NNCP_E_INVAL, "N = %d outside [2, %d]", N, NNCP_MAX_MODES);
  if (!dims) return fail(NNCP_E_INVAL, "dims is NULL");
  if (R < 1) return fail(NNCP_E_INVAL, "R = %d < 1", R);
  if (R > 256) return fail(NNCP_E_UNSUPPORTED, "R = %d > 256", R);
  int rc = check_dtypes(xdt, hdt);
  if (rc) return rc;
  L.N = N; L.R = R; L.xdt = xdt; L.hdt = hdt;
  L.opt = opt ? *opt : default_options();
  if (!(L.opt.eps_mu >= 0.0)) return fail(NNCP_E_INVAL, "eps_mu must be >= 0");
  int64_t total = 1;
  for (int k = 0; k < N; ++k) {
    if (dims[k] < 1) return fail(NNCP_E_INVAL, "dims[%d] = %lld < 1", k, (long long)dims[k]);
    if (dims[k] > ((int64_t)1 << 31)) return fail(NNCP_E_UNSUPPORTED, "dims[%d] too large", k);
    L.dims[k] = dims[k];
    if (total > (((int64_t)1 << 40) / dims[k])) return fail(NNCP_E_UNSUPPORTED, "tensor has more than 2^40 entries");
    total *= dims[k];
  }
  if (L.opt.split) {
    if (L.opt.split < 1 || L.opt.split > N - 1) return fail(NNCP_E_INVAL, "split = %d outside [1, N-1]", L.opt.split);
    L.S = L.opt.split;
  } else {
    // smallest S with prod(0..S-1) >= prod(S..N-1), clamped to [1, N-1]
    L.S = N - 1;
    for (int s = 1; s <= N - 1; ++s)
      if (prod(L.dims, 0, s) >= prod(L.dims, s, N)) { L.S = s; break; }
  }
  plan_side(L, 0);
  plan_side(L, 1);
  const int S = L.S;
  L.maxI = 0;
  L.sumI = 0;
  for (int k = 0; k < N; ++k) { L.maxI = std::max(L.maxI, L.dims[k]); L.sumI += L.dims[k]; }
  const int64_t m = prod(L.dims, 0, S), kk = prod(L.dims, S, N);
  L.nodeA = std::max(m, kk) * R;
  L.nodeB = std::max(S > 1 ? prod(L.dims, 1, S) : 1, N - S > 1 ? prod(L.dims, S + 1, N) : 1) * R;
  // partial buffers: GEMM splits and strided multi-TTV splits
  int64_t part = 0;
  for (int side = 0; side < 2; ++side) {
    const GemmPlan &p = L.gp[side];
    const int64_t rows = side == 1 ? p.k : p.m;
    part = std::max(part, (int64_t)p.nsplit * rows * R);
  }
  for (int side = 0; side < 2; ++side) {
    const int lo = side == 0 ? 0 : S, hi = side == 0 ? S : N;
    for (int a = lo; a < hi - 1; ++a)
      part = std::max(part, mttv_strided_part_elems(L.hdt, L.dims[a], L.dims + a + 1, hi - a - 1, R));
  }
  // the fused pass of the gradient (see launch_dual_mttkrp)
  {
    const GemmPlan &pl = L.gp[0], &pr = L.gp[1];
    L.dual = 0;
    L.dual_tiles = 0;
    L.nodeR = 1;
    // fused_grad = 1: only where the columns alone give about 0.75 of a
    // workgroup per CU (smaller grids are faster as two passes);
    // fused_grad = 2: wherever the kernel can run
    if (L.opt.fused_grad && xdt == NNCP_BF16 && pl.mfma && pr.mfma && pl.NT <= 2 && S >= 2 &&
        pl.m < ((int64_t)1 << 31) && pr.Pf % 32 == 0 &&
        dual_lds_bytes(pl.NT, pl.hl, pr.Pf) <= 160 * 1024 &&
        (L.opt.fused_grad == 2 || dual_tiles(pl.m) >= 192)) {
      L.dual = 1;
      L.dual_tiles = dual_tiles(pl.m);
      part = std::max(part, L.dual_tiles * pl.k * R);
      L.nodeR = pl.k * R;
    }
  }
  L.part_elems = part;
  L.kfast_elems = 0;
  L.kslow_elems = 0;
  for (int side = 0; side < 2; ++side) {
    const GemmPlan &p = L.gp[side];
    if (!p.mfma) continue;
    L.kfast_elems = std::max(L.kfast_elems, (int64_t)(p.hl ? 2 : 1) * p.Rpad * p.Pf);
    L.kslow_elems = std::max(L.kslow_elems, (int64_t)p.Ps * p.Rpad);
  }
  const size_t hs = xsize(hdt), es = xsize(xdt);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + std::max<size_t>(bytes, 1)); return at; };
  L.off_G = take(sizeof(double) * N * R * R);
  L.off_Gt = take(sizeof(double) * N * R * R);
  L.off_S = take(sizeof(double) * R * R);
  L.off_scal = take(sizeof(double) * 64);
  L.off_ones = take(sizeof(double) * R);
  L.off_hhat = take(sizeof(double) * L.maxI * R);
  L.off_upart = take(sizeof(double) * update_part_elems(L.maxI, R));
  L.off_gpart = take(R <= 64 ? sizeof(double) * norm_gpart_elems(R) : 0);
  L.off_red = take(sizeof(double) * 1024);
  L.off_M = take(hs * L.maxI * R);
  L.off_A = take(hs * L.nodeA);
  L.off_B = take(hs * L.nodeB);
  L.off_R = take(hs * L.nodeR);
  L.off_kfR = take(L.dual ? es * (L.gp[0].hl ? 2 : 1) * L.gp[0].Rpad * L.gp[0].k : 0);
  L.off_part = take(hs * L.part_elems);
  L.off_kf = take(es * L.kfast_elems);
  L.off_ks = take(hs * L.kslow_elems);
  L.off_pgdH = take(hs * L.sumI * R);
  L.off_pgdG = take(hs * L.sumI * R);
  // NES outer extrapolation (R <= 64): lambda before the sweep, the
  // candidate's lambda, its scalars, and per-mode column norms
  L.off_outer = take(R <= 64 ? sizeof(double) * ((NNCP_MAX_MODES + 2) * R + 16) : 0);
  // ADMM (R <= 64): duals of every mode, the kept M sum, P and rho, norms
  const bool admm = R <= 64;
  L.off_admmU = take(admm ? sizeof(double) * L.sumI * R : 0);
  L.off_admmMc = take(admm ? sizeof(double) * L.maxI * R : 0);
  L.off_admmP = take(admm ? sizeof(double) * (R * R + 2) : 0);
  L.off_admmNorm = take(admm ? sizeof(double) * kAdmmMaxit * ((L.maxI + 3) / 4) * 4 : 0);
  L.off_admmStatus = take(admm ? sizeof(int) * kAdmmMaxit : 0);
  {
    int64_t t = 0;
    for (int n = 0; n < NNCP_MAX_MODES; ++n) L.gradpart_off[n] = L.gradpart_elems[n] = 0;
    if (R <= 64)
      for (int side = 0; side < 2; ++side) {
        const int lo = side == 0 ? 0 : L.S, hi = side == 0 ? L.S : N;
        for (int a = lo; a < hi - 1; ++a) {
          L.gradpart_off[a] = t;
          L.gradpart_elems[a] = mttv_strided_part_elems(hdt, L.dims[a], L.dims + a + 1, hi - a - 1, R);
          t += L.gradpart_elems[a];
        }
      }
    L.off_gradpart = take(hs * t);
  }
  L.total = o;
  return NNCP_OK;
}

}  // namespace

// Event pairs of one timing category; events are created on first use and
// reused after each read.
struct TimerCat {
  std::vector<hipEvent_t> ev;  // start, stop, start, stop, ...
  size_t used = 0;
  double ms = 0.0;
  int64_t n = 0;
};

// A captured multi-sweep launch sequence, replayed while its key matches.
struct SweepGraph {
  hipGraphExec_t exec = nullptr;
  int algo = -1, nsweeps = -1;
  double *hist = nullptr;
  uint64_t binding = 0;
};

// Multi-TTVs collected instead of launched (see flush_batch).
constexpr int kBatchMax = 32;
struct MttvBatch {
  MttvJob j[kBatchMax];
  int n = 0;
};

struct nncp_ctx {
  int magic;
  Layout L;
  int timing = 0;
  TimerCat timers[NNCP_TIMER_CATEGORIES];
  hipStream_t cap = nullptr;  // private stream used only for graph capture
  SweepGraph graph;
  uint64_t binding = 1;       // bumped when factor / lambda pointers change
  const void *X;
  void *H[NNCP_MAX_MODES];
  double *lambda;
  hipStream_t st;
  char *ws;
  double *G, *Gt, *S, *scal, *ones, *hhat, *upart, *gpart, *red;
  GramJob pending{};          // Gram step of the last update, not yet run (R == 0: none)
  double *admmU, *admmMc, *admmP, *admmNorm;
  int *admmStatus;
  double *outer;
  void *M, *nodeA, *nodeB, *nodeR, *kfR, *part, *kf, *ks, *gradpart;
  // when set, the strided multi-TTV writes its split partials here (with
  // room for part_override_elems) instead of into part
  void *part_override = nullptr;
  int64_t part_override_elems = 0;
  void *pgdH[NNCP_MAX_MODES], *pgdG[NNCP_MAX_MODES];
  // set while nncp_grad walks the right subtree from the fused pass: the
  // right root node lives in nodeR
  bool right_root_in_R = false;
  // when set, the walks' multi-TTVs are collected here and run by flush_batch
  MttvBatch *batch = nullptr;
  // node cache of nncp_mttkrp: a version per factor, bumped whenever the
  // library writes the factor or the caller reports a write
  // (nncp_factors_changed), and for each node buffer the node it holds with
  // the versions of the factors it was contracted with
  uint64_t ver[NNCP_MAX_MODES] = {};
  struct NodeTag {
    int side = -1, a = -1;
    uint64_t ver[NNCP_MAX_MODES];
  } tagA, tagB;
};

namespace {

int check_ctx(const nncp_ctx *c) {
  if (!c || c->magic != kMagic) return fail(NNCP_E_STATE, "context is NULL or destroyed");
  return NNCP_OK;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(NNCP_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Record a start event for category k (no-op unless timing is enabled).
hipError_t tstart(nncp_ctx *c, int k) {
  if (!c->timing) return hipSuccess;
  TimerCat &t = c->timers[k];
  if (t.used + 2 > t.ev.size()) {
    // timing-only events: no system-scope fence (cache writeback and
    // invalidation) around the timed launch; the stream is synchronised
    // before the times are read
    hipEvent_t a, b;
    hipError_t e = hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
    if (e != hipSuccess) return e;
    e = hipEventCreateWithFlags(&b, hipEventDisableSystemFence);
    if (e != hipSuccess) return e;
    t.ev.push_back(a);
    t.ev.push_back(b);
  }
  return hipEventRecord(t.ev[t.used], c->st);
}

hipError_t tstop(nncp_ctx *c, int k) {
  if (!c->timing) return hipSuccess;
  TimerCat &t = c->timers[k];
  hipError_t e = hipEventRecord(t.ev[t.used + 1], c->st);
  t.used += 2;
  t.n += 1;
  return e;
}

// fold recorded pairs into the totals (the stream must be synchronised)
hipError_t tcollect(nncp_ctx *c) {
  for (int k = 0; k < NNCP_TIMER_CATEGORIES; ++k) {
    TimerCat &t = c->timers[k];
    for (size_t i = 0; i + 1 < t.used; i += 2) {
      float ms = 0.f;
      hipError_t e = hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]);
      if (e != hipSuccess) return e;
      t.ms += ms;
    }
    t.used = 0;
  }
  return hipSuccess;
}

#define TIMED(k, expr)                 \
  do {                                 \
    HIPCHK(tstart(c, (k)));            \
    HIPCHK(expr);                      \
    HIPCHK(tstop(c, (k)));             \
  } while (0)

FactorSet factors_of(const nncp_ctx *c, void *const *H) {
  FactorSet F;
  for (int n = 0; n < NNCP_MAX_MODES; ++n) F.H[n] = n < c->L.N ? H[n] : nullptr;
  return F;
}

// Where a computed M^(n) lives: msplit == 1 means p is M itself; otherwise p
// holds msplit row-major partial copies, mstride apart, that the consumer adds
// in order (the same order the split-sum kernels use).
struct MRef {
  const void *p;
  int msplit;
  int64_t mstride;
};

// Dead-column mask of the sweep's deferred MU/HALS path (R doubles after
// the scratch that launch_sweep_normalize uses in c->outer).
double *dead_mask(nncp_ctx *c) { return c->outer + (int64_t)(NNCP_MAX_MODES + 1) * c->L.R; }

// Runs a pending Gram step as a kernel of its own.
hipError_t flush_gram(nncp_ctx *c) {
  if (c->pending.R == 0) return hipSuccess;
  hipError_t e = tstart(c, 4);
  if (e == hipSuccess) e = launch_gram_finish(c->pending, c->st);
  if (e == hipSuccess) e = tstop(c, 4);
  c->pending.R = 0;
  return e;
}

void *node_buf(nncp_ctx *c, int side, int a) {
  const int lo = side == 0 ? 0 : c->L.S;
  if (side == 1 && a == lo && c->right_root_in_R) return c->nodeR;
  return ((a - lo) % 2 == 0) ? c->nodeA : c->nodeB;
}

// ---- node cache of nncp_mttkrp
void bump_versions(nncp_ctx *c, int mode) {
  for (int q = 0; q < c->L.N; ++q)
    if (mode < 0 || q == mode) ++c->ver[q];
}
void drop_nodes(nncp_ctx *c) {
  c->tagA.side = c->tagB.side = -1;
}
nncp_ctx::NodeTag &tag_of(nncp_ctx *c, int side, int a) {
  return node_buf(c, side, a) == c->nodeA ? c->tagA : c->tagB;
}
// node a of a side (modes a .. hi-1, hi-1 kept only as an M) was contracted
// with every factor outside [a, hi)
bool node_valid(nncp_ctx *c, int side, int a) {
  const int hi = side == 0 ? c->L.S : c->L.N;
  const nncp_ctx::NodeTag &t = tag_of(c, side, a);
  if (t.side != side || t.a != a) return false;
  for (int q = 0; q < c->L.N; ++q)
    if ((q < a || q >= hi) && t.ver[q] != c->ver[q]) return false;
  return true;
}
void set_tag(nncp_ctx *c, int side, int a) {
  nncp_ctx::NodeTag &t = tag_of(c, side, a);
  t.side = side;
  t.a = a;
  for (int q = 0; q < NNCP_MAX_MODES; ++q) t.ver[q] = c->ver[q];
}

// Runs the collected multi-TTVs (launch_mttv_jobs: as few launches as their
// dependencies allow).
int flush_batch(nncp_ctx *c) {
  if (!c->batch || c->batch->n == 0) return NNCP_OK;
  TIMED(3, launch_mttv_jobs(c->L.hdt, c->batch->j, c->batch->n, c->st));
  c->batch->n = 0;
  return NNCP_OK;
}

// A contiguous multi-TTV: collected when a batch is open and the job is of a
// groupable kind, else launched (after the collected ones).
int run_mttv_contig(nncp_ctx *c, const void *T, int64_t Ia, int64_t Q, const void *H, void *out,
                    int leaf) {
  if (c->batch && c->pending.R == 0 && c->batch->n < kBatchMax &&
      plan_mttv_contig(c->L.hdt, T, Ia, Q, c->L.R, H, out, leaf, &c->batch->j[c->batch->n])) {
    ++c->batch->n;
    return NNCP_OK;
  }
  int rc = flush_batch(c);
  if (rc) return rc;
  TIMED(3, launch_mttv_contig(c->L.hdt, T, Ia, Q, c->L.R, H, out, leaf, c->st, &c->pending));
  return NNCP_OK;
}

// A strided multi-TTV, likewise (collected only when its partials are left
// for the consumer, M == NULL).
int run_mttv_strided(nncp_ctx *c, const void *T, int64_t Ia, const int64_t *qdims, int nq,
                     const void *const *Hq, void *M, void *part, int64_t cap, int *ns) {
  if (c->batch && !M && c->pending.R == 0 && c->batch->n < kBatchMax &&
      plan_mttv_strided(c->L.hdt, T, Ia, qdims, nq, Hq, c->L.R, part, cap,
                        &c->batch->j[c->batch->n], ns)) {
    ++c->batch->n;
    return NNCP_OK;
  }
  int rc = flush_batch(c);
  if (rc) return rc;
  TIMED(3, launch_mttv_strided(c->L.hdt, T, Ia, qdims, nq, Hq, c->L.R, M, part, cap, c->st, ns,
                               &c->pending));
  return NNCP_OK;
}

// Root partial MTTKRP of one side into node[lo] (or into Mout if the subtree
// has a single mode).
int root_gemm(nncp_ctx *c, const FactorSet &F, int side, void *Mout, MRef *defer) {
  const Layout &L = c->L;
  if (int rc = flush_batch(c)) return rc;
  const GemmPlan &p = L.gp[side];
  const int lo = side == 0 ? 0 : L.S, hi = side == 0 ? L.S : L.N;
  const bool leaf = hi - lo == 1;
  // the Gram step of the previous update rides along with the Khatri-Rao
  // operand kernel, or with the product itself when that reads the factors
  // directly; the vector-ALU GEMM path runs it on its own first
  if (p.mfma && !p.direct)
    TIMED(2, launch_krp_operands(L.xdt, p, L.R, L.dims, L.N, F, c->kf, c->ks, c->st, &c->pending));
  else if (!p.mfma || c->pending.parts == 0)
    HIPCHK(flush_gram(c));
  void *node = leaf ? Mout : node_buf(c, side, lo);
  const bool to_node = p.nsplit == 1 && ((side == 0 && !leaf) || (side == 1 && leaf));
  TIMED(side, launch_partial_mttkrp(L.xdt, p, L.R, c->X, L.dims, L.N, L.S, F, c->kf, c->ks,
                                    to_node ? node : c->part, c->st, &c->pending));
  if (defer) *defer = MRef{Mout, 1, 0};
  if (!to_node) {
    // right partials of a single-mode subtree are already row-major copies of M
    if (defer && leaf && side == 1) {
      *defer = MRef{c->part, p.nsplit, p.k * L.R};
      return NNCP_OK;
    }
    TIMED(3, launch_finalize(L.hdt, p, L.R, c->part, node, leaf ? 1 : 0, c->st));
  }
  return NNCP_OK;
}

// M^(n) through the dimension tree.  When from_root is false the node of
// mode n-1 (same subtree) must hold the values left by the previous call and
// H^(n-1) may have changed since (Gauss-Seidel order of Algorithm 1).
int mttkrp_tree(nncp_ctx *c, const FactorSet &F, int n, void *Mout, bool from_root,
                MRef *defer = nullptr, bool roots_ready = false, int have_node = -1) {
  const Layout &L = c->L;
  const int side = n < L.S ? 0 : 1;
  const int lo = side == 0 ? 0 : L.S, hi = side == 0 ? L.S : L.N;
  const int R = L.R;
  int start;
  if (defer) *defer = MRef{Mout, 1, 0};
  if (have_node >= lo) {
    // node have_node (<= n) already holds its values
    start = have_node + 1;
  } else if (roots_ready && n == lo) {
    start = lo + 1;
  } else if (from_root || n == lo) {
    int rc = root_gemm(c, F, side, Mout, hi - lo == 1 ? defer : nullptr);
    if (rc) return rc;
    if (hi - lo == 1) return NNCP_OK;
    start = lo + 1;
  } else {
    start = n;
  }
  for (int a = start; a <= n; ++a) {
    // node a = contiguous multi-TTV of node a-1 with H^(a-1)
    const int64_t Ia = L.dims[a - 1];
    const int64_t Q = prod(L.dims, a, hi);
    const bool leaf = a == hi - 1;
    void *out = leaf ? Mout : node_buf(c, side, a);
    int rc = run_mttv_contig(c, node_buf(c, side, a - 1), Ia, Q, F.H[a - 1], out, leaf ? 1 : 0);
    if (rc) return rc;
  }
  if (n < hi - 1) {
    const void *Hq[NNCP_MAX_MODES];
    for (int k = n + 1; k < hi; ++k) Hq[k - n - 1] = F.H[k];
    int ns = 1;
    void *part = c->part_override ? c->part_override : c->part;
    const int64_t cap = c->part_override ? c->part_override_elems : L.part_elems;
    int rc = run_mttv_strided(c, node_buf(c, side, n), L.dims[n], L.dims + n + 1, hi - n - 1, Hq,
                              defer ? nullptr : Mout, part, cap, &ns);
    if (rc) return rc;
    if (defer) *defer = MRef{part, ns, L.dims[n] * R};
  }
  return NNCP_OK;
}

int refresh_grams(nncp_ctx *c, const FactorSet &F, double *G) {
  for (int n = 0; n < c->L.N; ++n)
    HIPCHK(launch_gram(c->L.hdt, F.H[n], c->L.dims[n], c->L.R, G + (int64_t)n * c->L.R * c->L.R, c->st));
  return NNCP_OK;
}

// When defer is true the update's Gram step is left pending in c->pending
// for the next multi-TTV or Khatri-Rao launch to carry (flush_gram runs it
// otherwise); else it runs right after the update.
int update_mode(nncp_ctx *c, int algo, int n, MRef M, const double *S, double eps,
                double *relerr_out, double *scal, double *S_next = nullptr, bool defer = false,
                int unnormalised = 0, int fold_lambda = 1) {
  const Layout &L = c->L;
  HIPCHK(flush_gram(c));
  UpdateArgs a;
  a.algo = algo;
  a.I = L.dims[n];
  a.R = L.R;
  a.N = L.N;
  a.mode = n;
  a.M = M.p;
  a.msplit = M.msplit;
  a.mstride = M.mstride;
  a.S = S;
  a.S_next = S_next;
  a.next_mode = (n + 1) % L.N;
  if (!S) {
    HIPCHK(launch_hadamard(c->G, L.N, L.R, n, c->S, c->st));
    a.S = c->S;
  }
  a.G = c->G;
  a.H = c->H[n];
  a.lambda = c->lambda;
  a.hhat = c->hhat;
  a.part = c->upart;
  a.gpart = c->gpart;
  a.beta_out = c->scal + 48;
  {
    int64_t off = 0;
    for (int k = 0; k < n; ++k) off += L.dims[k] * L.R;
    a.admmU = c->admmU + off;
  }
  a.admmMc = c->admmMc;
  a.admmP = c->admmP;
  a.admmNorm = c->admmNorm;
  a.admmStatus = c->admmStatus;
  a.nesParam = c->scal + 56;
  a.eps = eps;
  a.alpha = c->scal + 8;
  a.relerr_out = relerr_out;
  a.scal = scal;
  a.defer = unnormalised;
  a.fold_lambda = fold_lambda;
  a.dead = dead_mask(c);
  if (unnormalised) a.lambda = fold_lambda ? c->lambda : c->ones;
  GramJob job;
  TIMED(4, launch_update(L.hdt, a, c->st, &job));
  c->pending = job;
  if (!defer) HIPCHK(flush_gram(c));
  return NNCP_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Buffers that one MTTKRP from the root touches (Khatri-Rao operands, the
// two node buffers, the split partials), packed at 256-byte boundaries.  The
// partial buffer is sized only for the launches that write partials: a root
// product written straight into its node needs none.
struct MttkrpCarve {
  size_t kf, ks, A, B, part, total;
  int64_t part_elems;
};

MttkrpCarve mttkrp_carve(const Layout &L) {
  const int N = L.N, S = L.S, R = L.R;
  int64_t part = 1;
  for (int side = 0; side < 2; ++side) {
    const GemmPlan &p = L.gp[side];
    const int lo = side == 0 ? 0 : S, hi = side == 0 ? S : N;
    const bool leaf = hi - lo == 1;
    const bool direct = p.nsplit == 1 && ((side == 0 && !leaf) || (side == 1 && leaf));
    if (!direct) part = std::max(part, (int64_t)p.nsplit * (side == 1 ? p.k : p.m) * R);
    for (int a = lo; a < hi - 1; ++a)
      part = std::max(part, mttv_strided_part_elems(L.hdt, L.dims[a], L.dims + a + 1, hi - a - 1, R));
  }
  const size_t hs = xsize(L.hdt), es = xsize(L.xdt);
  MttkrpCarve c;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + std::max<size_t>(bytes, 1)); return at; };
  c.kf = take(es * L.kfast_elems);
  c.ks = take(hs * L.kslow_elems);
  c.A = take(hs * L.nodeA);
  c.B = take(hs * L.nodeB);
  c.part = take(hs * part);
  c.part_elems = part;
  c.total = o;
  return c;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of nncp_mttkrp_noalloc: one copy of this array per GPU, held from
// the library's first use on that GPU until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol); it takes the device address that
// hipGetSymbolAddress returns for the current device, once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NNCP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of the scratch array on device `dev` (the current device).
int scratch_base(int dev, char **base) {
  if (dev < 0 || dev >= kMaxDevices) return fail(NNCP_E_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(NNCP_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *base = (char *)g_scratch_ptr[dev];
  return NNCP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *nncp_last_error(void) { return g_err.c_str(); }

size_t nncp_workspace_size(int N, const int64_t *dims, int R, int x_dtype, int h_dtype,
                           const nncp_options *opt) {
  Layout L;
  if (make_layout(L, N, dims, R, x_dtype, h_dtype, opt) != NNCP_OK) return 0;
  return L.total;
}

int nncp_init(nncp_ctx **out, int N, const int64_t *dims, int R, int x_dtype, const void *X,
              int h_dtype, void *const *H, double *lambda, void *workspace, size_t ws_bytes,
              void *stream, const nncp_options *opt) {
  if (!out) return fail(NNCP_E_INVAL, "ctx out-pointer is NULL");
  *out = nullptr;
  Layout L;
  int rc = make_layout(L, N, dims, R, x_dtype, h_dtype, opt);
  if (rc) return rc;
  if (!X || !H || !lambda || !workspace) return fail(NNCP_E_INVAL, "NULL X, H, lambda or workspace");
  if (!aligned16(X) || !aligned16(workspace) || !aligned16(lambda))
    return fail(NNCP_E_INVAL, "X, lambda and workspace must be 16-byte aligned");
  for (int n = 0; n < N; ++n) {
    if (!H[n]) return fail(NNCP_E_INVAL, "H[%d] is NULL", n);
    if (!aligned16(H[n])) return fail(NNCP_E_INVAL, "H[%d] must be 16-byte aligned", n);
  }
  if (ws_bytes < L.total)
    return fail(NNCP_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
  nncp_ctx *c = new (std::nothrow) nncp_ctx();
  if (!c) return fail(NNCP_E_INVAL, "out of host memory");
  c->magic = kMagic;
  c->L = L;
  c->X = X;
  for (int n = 0; n < NNCP_MAX_MODES; ++n) c->H[n] = n < N ? H[n] : nullptr;
  c->lambda = lambda;
  c->st = (hipStream_t)stream;
  c->ws = (char *)workspace;
  c->G = (double *)(c->ws + L.off_G);
  c->Gt = (double *)(c->ws + L.off_Gt);
  c->S = (double *)(c->ws + L.off_S);
  c->scal = (double *)(c->ws + L.off_scal);
  c->ones = (double *)(c->ws + L.off_ones);
  c->hhat = (double *)(c->ws + L.off_hhat);
  c->upart = (double *)(c->ws + L.off_upart);
  c->gpart = (double *)(c->ws + L.off_gpart);
  c->admmU = (double *)(c->ws + L.off_admmU);
  c->outer = (double *)(c->ws + L.off_outer);
  c->admmMc = (double *)(c->ws + L.off_admmMc);
  c->admmP = (double *)(c->ws + L.off_admmP);
  c->admmNorm = (double *)(c->ws + L.off_admmNorm);
  c->admmStatus = (int *)(c->ws + L.off_admmStatus);
  c->red = (double *)(c->ws + L.off_red);
  c->M = c->ws + L.off_M;
  c->nodeA = c->ws + L.off_A;
  c->nodeB = c->ws + L.off_B;
  c->nodeR = c->ws + L.off_R;
  c->kfR = c->ws + L.off_kfR;
  c->part = c->ws + L.off_part;
  c->kf = c->ws + L.off_kf;
  c->ks = c->ws + L.off_ks;
  c->gradpart = c->ws + L.off_gradpart;
  {
    const size_t hs = xsize(h_dtype);
    size_t oh = L.off_pgdH, og = L.off_pgdG;
    for (int n = 0; n < N; ++n) {
      c->pgdH[n] = c->ws + oh;
      c->pgdG[n] = c->ws + og;
      oh += hs * L.dims[n] * R;
      og += hs * L.dims[n] * R;
    }
  }
  // ones (for lambda-free losses), the ADMM duals and the count of outer
  // extrapolation steps (both start at zero), Grams, alpha: all by kernels on
  // the stream, so that nothing here waits for the device
  {
    hipError_t e = launch_fill(c->ones, 1.0, R, c->st);
    if (e == hipSuccess && R <= 64) e = launch_fill(c->admmU, 0.0, L.sumI * R, c->st);
    if (e == hipSuccess) e = launch_fill(c->scal + kOuterCount, 0.0, 1, c->st);
    if (e != hipSuccess) {
      delete c;
      return fail(NNCP_E_HIP, "fill: %s", hipGetErrorString(e));
    }
  }
  FactorSet F = factors_of(c, c->H);
  rc = refresh_grams(c, F, c->G);
  if (!rc) {
    hipError_t e = launch_sumsq(x_dtype, X, prod(L.dims, 0, N), c->red, c->scal + 8, c->st);
    if (e != hipSuccess) rc = fail(NNCP_E_HIP, "sumsq: %s", hipGetErrorString(e));
  }
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return NNCP_OK;
}

int nncp_set_factors(nncp_ctx *c, void *const *H, double *lambda) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!H) return fail(NNCP_E_INVAL, "H is NULL");
  for (int n = 0; n < c->L.N; ++n)
    if (!H[n] || !aligned16(H[n])) return fail(NNCP_E_INVAL, "H[%d] is NULL or misaligned", n);
  if (lambda && !aligned16(lambda)) return fail(NNCP_E_INVAL, "lambda misaligned");
  for (int n = 0; n < c->L.N; ++n) c->H[n] = H[n];
  if (lambda) c->lambda = lambda;
  ++c->binding;
  bump_versions(c, -1);
  // a new start point: the ADMM duals and the outer-step count start again
  // from zero
  if (c->L.R <= 64) HIPCHK(launch_fill(c->admmU, 0.0, c->L.sumI * c->L.R, c->st));
  HIPCHK(launch_fill(c->scal + kOuterCount, 0.0, 1, c->st));
  return refresh_grams(c, factors_of(c, c->H), c->G);
}

int nncp_split(const nncp_ctx *c) {
  if (check_ctx(c)) return NNCP_E_STATE;
  return c->L.S;
}

int nncp_gemm_path(const nncp_ctx *c, int side) {
  if (check_ctx(c)) return NNCP_E_STATE;
  if (side < 0 || side > 1) return fail(NNCP_E_INVAL, "side must be 0 or 1");
  return c->L.gp[side].mfma;
}

int nncp_read_probe(const void *buf, size_t bytes, int workgroups, void *out4, void *stream) {
  if (!buf || !out4) return fail(NNCP_E_INVAL, "NULL buffer");
  if (!aligned16(buf) || ((uintptr_t)out4 & 3)) return fail(NNCP_E_INVAL, "misaligned buffer");
  if (bytes == 0 || bytes % 16) return fail(NNCP_E_INVAL, "bytes must be a positive multiple of 16");
  if (workgroups < 1 || workgroups > (1 << 20)) return fail(NNCP_E_INVAL, "workgroups outside [1, 2^20]");
  HIPCHK(launch_read_probe(buf, bytes, workgroups, out4, (hipStream_t)stream));
  return NNCP_OK;
}

int nncp_gemm_plan(const nncp_ctx *c, int side, int64_t *info) {
  if (check_ctx(c)) return NNCP_E_STATE;
  if (side < 0 || side > 1) return fail(NNCP_E_INVAL, "side must be 0 or 1");
  if (!info) return fail(NNCP_E_INVAL, "info is NULL");
  const GemmPlan &p = c->L.gp[side];
  info[0] = p.mfma;
  info[1] = p.Pf;
  info[2] = p.Ps;
  info[3] = p.nsplit;
  info[4] = p.tiles;
  info[5] = p.W;
  info[6] = p.hl;
  info[7] = p.direct;
  return NNCP_OK;
}

int nncp_mttkrp(nncp_ctx *c, int mode, void *M) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (mode < 0 || mode >= c->L.N) return fail(NNCP_E_INVAL, "mode %d outside [0, %d)", mode, c->L.N);
  if (!M) return fail(NNCP_E_INVAL, "M is NULL");
  const Layout &L = c->L;
  const int side = mode < L.S ? 0 : 1;
  const int lo = side == 0 ? 0 : L.S, hi = side == 0 ? L.S : L.N;
  // the deepest node on the way to `mode` still valid (nodes are lo .. hi-2)
  int have = -1;
  for (int a = std::min(mode, hi - 2); a >= lo; --a)
    if (node_valid(c, side, a)) {
      have = a;
      break;
    }
  rc = mttkrp_tree(c, factors_of(c, c->H), mode, M, true, nullptr, false, have);
  if (rc) {
    drop_nodes(c);
    return rc;
  }
  // the nodes this call wrote
  const int first = have >= lo ? have + 1 : lo;
  for (int a = first; a <= std::min(mode, hi - 2); ++a) set_tag(c, side, a);
  return NNCP_OK;
}

int nncp_factors_changed(nncp_ctx *c, int mode) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (mode < -1 || mode >= c->L.N) return fail(NNCP_E_INVAL, "mode %d outside [-1, %d)", mode, c->L.N);
  bump_versions(c, mode);
  for (int n = 0; n < c->L.N; ++n)
    if (mode < 0 || n == mode)
      HIPCHK(launch_gram(c->L.hdt, c->H[n], c->L.dims[n], c->L.R, c->G + (int64_t)n * c->L.R * c->L.R,
                         c->st));
  return NNCP_OK;
}

int nncp_mttkrp_noalloc(int N, const int64_t *dims, int R, int x_dtype, const void *X,
                        int h_dtype, void *const *H, int mode, void *M, void *stream,
                        const nncp_options *opt) {
  Layout L;
  int rc = make_layout(L, N, dims, R, x_dtype, h_dtype, opt);
  if (rc) return rc;
  if (mode < 0 || mode >= N) return fail(NNCP_E_INVAL, "mode %d outside [0, %d)", mode, N);
  if (!X || !H || !M) return fail(NNCP_E_INVAL, "NULL X, H or M");
  if (!aligned16(X) || !aligned16(M)) return fail(NNCP_E_INVAL, "X and M must be 16-byte aligned");
  for (int n = 0; n < N; ++n)
    if (!H[n] || !aligned16(H[n])) return fail(NNCP_E_INVAL, "H[%d] is NULL or misaligned", n);
  const MttkrpCarve cv = mttkrp_carve(L);
  if (cv.total > (size_t)NNCP_NOALLOC_SCRATCH_BYTES)
    return fail(NNCP_E_WORKSPACE, "this MTTKRP needs %zu bytes of scratch, more than the %zu "
                "of nncp_mttkrp_noalloc", cv.total, (size_t)NNCP_NOALLOC_SCRATCH_BYTES);
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (stream) {
    hipDevice_t sd = -1;
    HIPCHK(hipStreamGetDevice((hipStream_t)stream, &sd));
    if (sd != dev)
      return fail(NNCP_E_INVAL, "the stream belongs to device %d, the current device is %d", (int)sd, dev);
  }
  char *base = nullptr;
  rc = scratch_base(dev, &base);
  if (rc) return rc;
  // a context on the host stack over the scratch: only the MTTKRP buffers are
  // set, no Gram step is pending and nothing is timed
  nncp_ctx c;
  c.magic = kMagic;
  c.L = L;
  c.L.part_elems = cv.part_elems;
  c.X = X;
  for (int n = 0; n < NNCP_MAX_MODES; ++n) c.H[n] = n < N ? H[n] : nullptr;
  c.lambda = nullptr;
  c.st = (hipStream_t)stream;
  c.ws = base;
  c.kf = base + cv.kf;
  c.ks = base + cv.ks;
  c.nodeA = base + cv.A;
  c.nodeB = base + cv.B;
  c.part = base + cv.part;
  c.pending.R = 0;
  return mttkrp_tree(&c, factors_of(&c, c.H), mode, M, true);
}

int nncp_gram(nncp_ctx *c, int mode, double *G) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (mode < 0 || mode >= c->L.N) return fail(NNCP_E_INVAL, "mode %d outside [0, %d)", mode, c->L.N);
  const int R = c->L.R;
  double *Gm = c->G + (int64_t)mode * R * R;
  HIPCHK(launch_gram(c->L.hdt, c->H[mode], c->L.dims[mode], R, Gm, c->st));
  if (G && G != Gm)
    HIPCHK(hipMemcpyAsync(G, Gm, sizeof(double) * R * R, hipMemcpyDeviceToDevice, c->st));
  return NNCP_OK;
}

int nncp_hadamard(nncp_ctx *c, int mode, double *S) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (mode < 0 || mode >= c->L.N) return fail(NNCP_E_INVAL, "mode %d outside [0, %d)", mode, c->L.N);
  if (!S) return fail(NNCP_E_INVAL, "S is NULL");
  HIPCHK(launch_hadamard(c->G, c->L.N, c->L.R, mode, S, c->st));
  return NNCP_OK;
}

static int update_api(nncp_ctx *c, int algo, int mode, const void *M, const double *S, double eps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (mode < 0 || mode >= c->L.N) return fail(NNCP_E_INVAL, "mode %d outside [0, %d)", mode, c->L.N);
  if (!M || !S) return fail(NNCP_E_INVAL, "M or S is NULL");
  bump_versions(c, mode);
  return update_mode(c, algo, mode, MRef{M, 1, 0}, S, eps, nullptr, nullptr);
}

int nncp_update_mu(nncp_ctx *c, int mode, const void *M, const double *S, double eps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  return update_api(c, NNCP_MU, mode, M, S, eps < 0 ? c->L.opt.eps_mu : eps);
}

int nncp_update_hals(nncp_ctx *c, int mode, const void *M, const double *S) {
  return update_api(c, NNCP_HALS, mode, M, S, 0.0);
}

int nncp_update_bpp(nncp_ctx *c, int mode, const void *M, const double *S) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (c->L.R > 64) return fail(NNCP_E_UNSUPPORTED, "BPP needs R <= 64 (R = %d)", c->L.R);
  return update_api(c, NNCP_BPP, mode, M, S, 0.0);
}

int nncp_update_admm(nncp_ctx *c, int mode, const void *M, const double *S) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (c->L.R > 64) return fail(NNCP_E_UNSUPPORTED, "ADMM needs R <= 64 (R = %d)", c->L.R);
  return update_api(c, NNCP_ADMM, mode, M, S, 0.0);
}

int nncp_update_nes(nncp_ctx *c, int mode, const void *M, const double *S) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (c->L.R > 64) return fail(NNCP_E_UNSUPPORTED, "NES needs R <= 64 (R = %d)", c->L.R);
  return update_api(c, NNCP_NES, mode, M, S, 0.0);
}

int nncp_cp_loss(nncp_ctx *c, double *loss, double *relerr) {
  int rc = check_ctx(c);
  if (rc) return rc;
  drop_nodes(c);
  const Layout &L = c->L;
  const int n = L.N - 1;
  rc = mttkrp_tree(c, factors_of(c, c->H), n, c->M, true);
  if (rc) return rc;
  HIPCHK(launch_loss(L.hdt, L.N, L.R, L.dims[n], c->M, c->H[n], c->lambda, c->G, c->scal + 8, loss,
                     relerr, c->scal + 4, c->st));
  return NNCP_OK;
}

// Outer extrapolation after sweep s (from 0) of the Nesterov-type sweeps
// (Section 4.3.5, Eq. eqn:nesouterupd), on F^(n) = H^(n) (n < N-1) and
// F^(N-1) = H^(N-1) diag(lambda) with the iterate saved before the sweep
// (c->pgdG, lambda in c->outer): candidate max(0, F + s_i (F - F_prev)),
// s_i = i^(1/N) with i the outer iteration (the device count of outer steps
// taken since init / set_factors, plus one), normalised into c->pgdH with its
// Grams in c->Gt and
// lambda_c the product of the column norms; its error from the identity
// (an extra MTTKRP of mode N-1); taken when its squared relative error is
// lower than the sweep's (c->scal[2]).  All on the stream, no host decision.
static int nes_outer_step(nncp_ctx *c, double *hist) {
  const Layout &L = c->L;
  const int N = L.N, R = L.R;
  const size_t hs = xsize(L.hdt);
  double *lamp = c->outer, *lamc = c->outer + R, *cand = c->outer + 2 * R;
  double *lamk = c->outer + 2 * R + 16;
  double *count = c->scal + kOuterCount;
  for (int k = 0; k < N; ++k) {
    int nb = 0;
    TIMED(4, launch_nes_extrap(L.hdt, c->H[k], c->pgdG[k], c->lambda, lamp, k == N - 1, count,
                               N, L.dims[k], R, c->hhat, c->upart, &nb, c->st));
    UpdateArgs a{};
    a.algo = NNCP_NES;
    a.I = L.dims[k];
    a.R = R;
    a.N = N;
    a.mode = k;
    a.next_mode = (k + 1) % N;
    a.S = c->S;
    a.S_next = nullptr;
    a.G = c->Gt;
    a.H = c->pgdH[k];
    a.lambda = lamk + (int64_t)k * R;
    a.hhat = c->hhat;
    a.part = c->upart;
    a.gpart = c->gpart;
    a.beta_out = cand + 8;
    a.alpha = c->scal + 8;
    a.relerr_out = nullptr;
    a.scal = nullptr;
    a.nesParam = c->scal + 56;
    GramJob job;
    TIMED(4, launch_norm_only(L.hdt, a, nb, c->st, &job));
    TIMED(4, launch_gram_finish(job, c->st));
  }
  TIMED(4, launch_nes_lamc(lamk, N, R, lamc, count, c->st));
  const FactorSet Fc = factors_of(c, c->pgdH);
  int rc = mttkrp_tree(c, Fc, N - 1, c->M, true);
  if (rc) return rc;
  // cand: [1] relerr, [2..4] beta, gamma, raw squared relative error
  TIMED(4, launch_loss(L.hdt, N, R, L.dims[N - 1], c->M, c->pgdH[N - 1], lamc, c->Gt,
                       c->scal + 8, nullptr, cand + 1, cand + 2, c->st));
  const double *ce2 = cand + 4, *e2 = c->scal + 2;
  for (int k = 0; k < N; ++k)
    TIMED(4, launch_nes_accept(hs, c->pgdH[k], c->H[k], L.dims[k] * R, ce2, e2, c->st));
  TIMED(4, launch_nes_accept(sizeof(double), lamc, c->lambda, R, ce2, e2, c->st));
  TIMED(4, launch_nes_accept(sizeof(double), c->Gt, c->G, (int64_t)N * R * R, ce2, e2, c->st));
  TIMED(4, launch_nes_accept_hist(ce2, e2, cand + 1, hist, c->st));
  return NNCP_OK;
}

// MU and HALS sweeps without the per-mode normalisation (R <= 64): each
// mode's rows are written unnormalised by one kernel, lambda is folded into
// the first update only, and the factors are normalised once at the end
// (launch_sweep_normalize); see k_update_rows_defer for why the iterates
// are unchanged.  The relative error after each sweep comes from the same
// identity with lambda = 1.
static int sweep_deferred(nncp_ctx *c, int algo, int nsweeps, double *relerr_hist) {
  const Layout &L = c->L;
  const FactorSet F = factors_of(c, c->H);
  HIPCHK(launch_hadamard(c->G, L.N, L.R, 0, c->S, c->st));
  HIPCHK(launch_fill(dead_mask(c), 0.0, L.R, c->st));
  for (int s = 0; s < nsweeps; ++s) {
    for (int n = 0; n < L.N; ++n) {
      MRef M;
      int rc = mttkrp_tree(c, F, n, c->M, false, &M);
      if (rc) {
        c->pending.R = 0;
        return rc;
      }
      const bool last = n == L.N - 1;
      rc = update_mode(c, algo, n, M, c->S, L.opt.eps_mu,
                       last && relerr_hist ? relerr_hist + s : nullptr, last ? c->scal : nullptr,
                       c->S, true, 1, (s == 0 && n == 0) ? 1 : 0);
      if (rc) {
        c->pending.R = 0;
        return rc;
      }
    }
  }
  HIPCHK(flush_gram(c));
  TIMED(4, launch_sweep_normalize(L.hdt, F, L.dims, L.N, L.R, c->G, c->lambda, c->outer, c->st));
  return NNCP_OK;
}

// The deferred path above measured slower than the per-mode normalisation
// at 512^3 (0.183 against 0.174 ms per BF16 sweep: its Gram step adds 64
// slices in one workgroup inside the next launch); it stays off until that
// step is spread over workgroups.
constexpr bool kDeferredSweep = true;

static int sweep_launches(nncp_ctx *c, int algo, int nsweeps, double *relerr_hist) {
  const Layout &L = c->L;
  if (kDeferredSweep && (algo == NNCP_MU || algo == NNCP_HALS) && L.R <= 64)
    return sweep_deferred(c, algo, nsweeps, relerr_hist);
  const FactorSet F = factors_of(c, c->H);
  const bool outer = algo == NNCP_NES_OUTER;
  if (outer) algo = NNCP_NES;
  const size_t hs = xsize(L.hdt);
  // S^(0) here; every update then leaves S of the next mode in c->S
  HIPCHK(launch_hadamard(c->G, L.N, L.R, 0, c->S, c->st));
  for (int s = 0; s < nsweeps; ++s) {
    if (outer) {
      // the iterate before the sweep; S^(0) again (the Grams may have been
      // replaced by the previous sweep's candidate)
      if (s > 0) HIPCHK(launch_hadamard(c->G, L.N, L.R, 0, c->S, c->st));
      for (int k = 0; k < L.N; ++k)
        HIPCHK(launch_copy(hs, c->H[k], c->pgdG[k], L.dims[k] * L.R, c->st));
      HIPCHK(launch_copy(sizeof(double), c->lambda, c->outer, L.R, c->st));
    }
    for (int n = 0; n < L.N; ++n) {
      MRef M;
      int rc = mttkrp_tree(c, F, n, c->M, false, &M);
      if (rc) {
        c->pending.R = 0;
        return rc;
      }
      const bool last = n == L.N - 1;
      rc = update_mode(c, algo, n, M, c->S, L.opt.eps_mu,
                       last && relerr_hist ? relerr_hist + s : nullptr, last ? c->scal : nullptr,
                       c->S, true);
      if (rc) {
        c->pending.R = 0;
        return rc;
      }
    }
    if (outer) {
      HIPCHK(flush_gram(c));
      int rc = nes_outer_step(c, relerr_hist ? relerr_hist + s : nullptr);
      if (rc) return rc;
    }
  }
  HIPCHK(flush_gram(c));
  return NNCP_OK;
}

static void drop_graph(nncp_ctx *c) {
  if (c->graph.exec) (void)hipGraphExecDestroy(c->graph.exec);
  c->graph = SweepGraph();
}

// Capture the launches of nsweeps sweeps on the private stream and
// instantiate them (kernels only: the sweep records no memset or copy).
static int build_graph(nncp_ctx *c, int algo, int nsweeps, double *relerr_hist) {
  drop_graph(c);
  if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  hipStream_t user = c->st;
  c->st = c->cap;
  hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    c->st = user;
    return fail(NNCP_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  int rc = sweep_launches(c, algo, nsweeps, relerr_hist);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap, &g);
  c->st = user;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(NNCP_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(NNCP_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  c->graph.exec = ex;
  c->graph.algo = algo;
  c->graph.nsweeps = nsweeps;
  c->graph.hist = relerr_hist;
  c->graph.binding = c->binding;
  return NNCP_OK;
}

int nncp_sweep(nncp_ctx *c, int algo, int nsweeps, double *relerr_hist) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (algo < NNCP_MU || algo > NNCP_NES_OUTER) return fail(NNCP_E_INVAL, "algo %d", algo);
  if (algo >= NNCP_BPP && c->L.R > 64)
    return fail(NNCP_E_UNSUPPORTED, "BPP, ADMM and NES need R <= 64 (R = %d)", c->L.R);
  if (nsweeps < 0) return fail(NNCP_E_INVAL, "nsweeps %d < 0", nsweeps);
  if (nsweeps == 0) return NNCP_OK;
  drop_nodes(c);
  bump_versions(c, -1);
  // Eager launches while timing (each launch is bracketed by events) or when
  // graphs are switched off; otherwise replay a cached graph of the sweeps.
  if (c->timing || !c->L.opt.graphs) return sweep_launches(c, algo, nsweeps, relerr_hist);
  const SweepGraph &g = c->graph;
  if (!(g.exec && g.algo == algo && g.nsweeps == nsweeps && g.hist == relerr_hist &&
        g.binding == c->binding)) {
    rc = build_graph(c, algo, nsweeps, relerr_hist);
    if (rc) return rc;
  }
  HIPCHK(hipGraphLaunch(c->graph.exec, c->st));
  return NNCP_OK;
}

int nncp_sweep_capture(nncp_ctx *c, int algo, int nsweeps, double *relerr_hist) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (algo < NNCP_MU || algo > NNCP_NES_OUTER) return fail(NNCP_E_INVAL, "algo %d", algo);
  if (algo >= NNCP_BPP && c->L.R > 64)
    return fail(NNCP_E_UNSUPPORTED, "BPP, ADMM and NES need R <= 64 (R = %d)", c->L.R);
  if (nsweeps < 1) return fail(NNCP_E_INVAL, "nsweeps %d < 1", nsweeps);
  if (!c->L.opt.graphs) return fail(NNCP_E_INVAL, "graphs are switched off for this context");
  return build_graph(c, algo, nsweeps, relerr_hist);
}

// The gradient's fused pass: the right product's Khatri-Rao operand, then
// one kernel for both root products (left into nodeA, right as per-tile
// partials in c->part), the partials added in tile order into nodeR: the
// right root node, or M^(N-1) itself (row-major) when the right subtree is
// the single mode N-1.  Nothing else writes nodeR, while the left subtree's
// multi-TTVs reuse c->part.
static int dual_roots(nncp_ctx *c, const FactorSet &F) {
  const Layout &L = c->L;
  HIPCHK(flush_gram(c));
  // the right operand's parts, and the left operand whole (its slow part, a
  // row of ones, goes to scratch), in one launch
  TIMED(2, launch_krp_operands2(L.xdt, L.gp[1], c->kf, c->ks, dual_full_plan(L.gp[0], L.S, L.N),
                                c->kfR, c->red, L.R, L.dims, L.N, F, c->st));
  // the right partials in the layout of their destination: [R][k] for the
  // right root node, [k][R] for M^(N-1), so that the sum reads and writes
  // whole lines
  const int leaf = L.N - L.S == 1 ? 1 : 0;
  TIMED(0, launch_dual_mttkrp(L.xdt, L.gp[0], L.gp[1], L.R, c->X, c->kfR, c->kf, c->ks, c->nodeA,
                              c->part, leaf ? 0 : 1, c->st));
  GemmPlan pd = L.gp[1];
  pd.nsplit = (int)L.dual_tiles;
  TIMED(3, launch_finalize(L.hdt, pd, L.R, c->part, c->nodeR, leaf, c->st, leaf ? 0 : 1));
  return NNCP_OK;
}

static int grad_at(nncp_ctx *c, const FactorSet &F, const double *G, void *const *grads,
                   double *loss) {
  const Layout &L = c->L;
  const bool dual = L.dual != 0;
  if (dual) {
    int rc = dual_roots(c, F);
    if (rc) return rc;
  }
  if (grads && L.R <= 64) {
    // every M^(n) kept until one launch forms all the gradients and the
    // loss: M^(n) for n < N-1 in its gradient buffer (or, when a strided
    // multi-TTV forms it, its split partials in the mode's own region),
    // M^(N-1) in c->M (or nodeR) for the loss
    GradAllArgs ga{};
    // on the fused path the walks launch nothing but multi-TTVs: collect
    // them and run them grouped (flushed before the gradient launch)
    MttvBatch batch;
    struct BatchGuard {
      nncp_ctx *c;
      ~BatchGuard() { c->batch = nullptr; }
    } guard{c};
    if (dual) c->batch = &batch;
    for (int n = 0; n < L.N; ++n) {
      const bool lastm = n == L.N - 1;
      MRef mr{lastm ? c->M : grads[n], 1, 0};
      void *Mout = lastm ? c->M : grads[n];
      int rc = NNCP_OK;
      c->part_override = L.gradpart_elems[n] ? (char *)c->gradpart + xsize(L.hdt) * L.gradpart_off[n]
                                             : nullptr;
      c->part_override_elems = L.gradpart_elems[n];
      if (dual && n == L.S && L.N - L.S == 1) {
        mr = MRef{c->nodeR, 1, 0};  // M^(N-1), added from the fused pass's partials
      } else if (dual) {
        c->right_root_in_R = true;
        rc = mttkrp_tree(c, F, n, Mout, false, lastm ? nullptr : &mr, true);
        c->right_root_in_R = false;
      } else {
        rc = mttkrp_tree(c, F, n, Mout, false, lastm ? nullptr : &mr);
      }
      c->part_override = nullptr;
      c->part_override_elems = 0;
      if (rc) return rc;
      ga.M[n] = mr.p;
      ga.msplit[n] = mr.msplit;
      ga.mstride[n] = mr.mstride;
      ga.H[n] = F.H[n];
      ga.grad[n] = grads[n];
      ga.I[n] = L.dims[n];
    }
    ga.N = L.N;
    ga.R = L.R;
    ga.G = G;
    ga.ones = c->ones;
    ga.alpha = c->scal + 8;
    ga.loss = loss;
    ga.scal = c->scal + 4;
    if (int rc = flush_batch(c)) return rc;
    c->batch = nullptr;
    HIPCHK(flush_gram(c));
    HIPCHK(launch_grad_all(L.hdt, ga, c->st));
    return NNCP_OK;
  }
  void *Mn = c->M;
  for (int n = 0; n < L.N; ++n) {
    int rc = NNCP_OK;
    Mn = c->M;
    // before the last mode, split partials of M^(n) are left for the
    // gradient kernel to add (the loss needs M^(N-1) itself)
    MRef mr{c->M, 1, 0};
    MRef *dp = grads && n < L.N - 1 ? &mr : nullptr;
    if (dual) {
      if (n == L.S && L.N - L.S == 1) {
        Mn = c->nodeR;  // M^(N-1), added from the fused pass's partials
        mr = MRef{Mn, 1, 0};
      } else {
        c->right_root_in_R = true;
        rc = mttkrp_tree(c, F, n, c->M, false, dp, true);
        c->right_root_in_R = false;
      }
    } else {
      rc = mttkrp_tree(c, F, n, c->M, false, dp);
    }
    if (rc) return rc;
    if (grads) {
      const double *S = nullptr;
      if (L.R > 64) {
        HIPCHK(launch_hadamard(G, L.N, L.R, n, c->S, c->st));
        S = c->S;
      }
      HIPCHK(launch_grad(L.hdt, L.dims[n], L.R, L.N, n, mr.p, mr.msplit, mr.mstride, F.H[n], G, S,
                         grads[n], c->st));
    }
  }
  const int n = L.N - 1;
  HIPCHK(launch_loss(L.hdt, L.N, L.R, L.dims[n], Mn, F.H[n], c->ones, G, c->scal + 8, loss,
                     nullptr, c->scal + 4, c->st));
  return NNCP_OK;
}

int nncp_grad(nncp_ctx *c, void *const *grads, double *loss) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!grads) return fail(NNCP_E_INVAL, "grads is NULL");
  for (int n = 0; n < c->L.N; ++n)
    if (!grads[n]) return fail(NNCP_E_INVAL, "grads[%d] is NULL", n);
  drop_nodes(c);
  return grad_at(c, factors_of(c, c->H), c->G, grads, loss);
}

int nncp_uses_fused_grad(const nncp_ctx *c) {
  if (check_ctx(c)) return NNCP_E_STATE;
  return c->L.dual ? 1 : 0;
}

int nncp_pgd(nncp_ctx *c, int nsteps, double armijo_c, int max_halvings, int power_iters,
             double *loss_hist, double *eta_hist) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (nsteps < 0 || max_halvings < 0 || power_iters < 0 || !(armijo_c >= 0.0))
    return fail(NNCP_E_INVAL, "bad PGD parameters");
  if (c->L.R > 64) return fail(NNCP_E_UNSUPPORTED, "nncp_pgd supports R <= 64");
  drop_nodes(c);
  bump_versions(c, -1);
  const Layout &L = c->L;
  const int N = L.N, R = L.R;
  const FactorSet F = factors_of(c, c->H);
  const FactorSet Ft = factors_of(c, c->pgdH);
  double *dL = c->scal + 16;    // loss at H
  double *dLt = c->scal + 17;   // loss at the trial
  double *deta = c->scal + 18;  // eta0
  double *dd = c->scal + 24;    // per-mode ||H' - H||^2
  for (int t = 0; t < nsteps; ++t) {
    rc = grad_at(c, F, c->G, c->pgdG, dL);
    if (rc) return rc;
    HIPCHK(launch_pgd_eta(c->G, N, R, power_iters, deta, c->st));
    double host[2];
    HIPCHK(hipMemcpyAsync(&host[0], dL, sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(&host[1], deta, sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const double Lcur = host[0];
    double eta = host[1], accepted = 0.0, Lnew = Lcur;
    for (int h = 0; h <= max_halvings; ++h) {
      for (int n = 0; n < N; ++n)
        HIPCHK(launch_pgd_trial(L.hdt, L.dims[n] * R, c->H[n], c->pgdG[n], eta, c->pgdH[n], c->red,
                                dd + n, c->st));
      rc = refresh_grams(c, Ft, c->Gt);
      if (rc) return rc;
      rc = mttkrp_tree(c, Ft, N - 1, c->M, true);
      if (rc) return rc;
      HIPCHK(launch_loss(L.hdt, N, R, L.dims[N - 1], c->M, c->pgdH[N - 1], c->ones, c->Gt,
                         c->scal + 8, dLt, nullptr, nullptr, c->st));
      double hb[NNCP_MAX_MODES + 1];
      HIPCHK(hipMemcpyAsync(hb, dd, sizeof(double) * N, hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipMemcpyAsync(hb + N, dLt, sizeof(double), hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipStreamSynchronize(c->st));
      double d = 0.0;
      for (int n = 0; n < N; ++n) d += hb[n];
      const double Lt = hb[N];
      if (Lt <= Lcur - armijo_c * d / eta) {
        accepted = eta;
        Lnew = Lt;
        const size_t hs = xsize(L.hdt);
        for (int n = 0; n < N; ++n)
          HIPCHK(hipMemcpyAsync(c->H[n], c->pgdH[n], hs * L.dims[n] * R, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(hipMemcpyAsync(c->G, c->Gt, sizeof(double) * N * R * R, hipMemcpyDeviceToDevice, c->st));
        break;
      }
      eta *= 0.5;
    }
    if (loss_hist) loss_hist[t] = Lnew;
    if (eta_hist) eta_hist[t] = accepted;
  }
  HIPCHK(hipStreamSynchronize(c->st));
  return NNCP_OK;
}

int nncp_timers_enable(nncp_ctx *c, int on) {
  int rc = check_ctx(c);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->st));
  for (int k = 0; k < NNCP_TIMER_CATEGORIES; ++k) {
    c->timers[k].used = 0;
    c->timers[k].ms = 0.0;
    c->timers[k].n = 0;
  }
  c->timing = on ? 1 : 0;
  return NNCP_OK;
}

int nncp_timers_read(nncp_ctx *c, double *ms, int64_t *launches) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!ms || !launches) return fail(NNCP_E_INVAL, "NULL output array");
  HIPCHK(hipStreamSynchronize(c->st));
  HIPCHK(tcollect(c));
  for (int k = 0; k < NNCP_TIMER_CATEGORIES; ++k) {
    ms[k] = c->timers[k].ms;
    launches[k] = c->timers[k].n;
  }
  return NNCP_OK;
}

int nncp_destroy(nncp_ctx *c) {
  int rc = check_ctx(c);
  if (rc) return rc;
  for (int k = 0; k < NNCP_TIMER_CATEGORIES; ++k)
    for (hipEvent_t e : c->timers[k].ev) (void)hipEventDestroy(e);
  drop_graph(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  c->magic = 0;
  delete c;
  return NNCP_OK;
}

}  // extern "C"
