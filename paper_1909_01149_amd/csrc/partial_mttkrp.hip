// Partial MTTKRP: the two GEMMs at the root of the dimension tree
// (Section 4.2.2, Algorithm 3, partial-MTTKRP lines), plus the partial
// Khatri-Rao operand (Algorithm 3, partial-KRP lines) and the deterministic
// split-reduction finalize.
//
// The tensor is read as a k x m row-major matrix Xr whose rows are the
// contiguous mode-0..S-1 fibres (m = I_0 ... I_{S-1}, k = I_S ... I_{N-1}).
//   left  (mode 0's subtree):  T^{0:S-1}(i, r)   = sum_j Xr[j, i] K^{S:N-1}(j, r)
//   right (mode S's subtree):  T^{S:N-1}(j, r)   = sum_i Xr[j, i] K^{0:S-1}(i, r)
// Both are 2 I R flops and one streaming pass over X; R is small, so they are
// HBM-bound streaming reductions that use the matrix cores only to keep the
// ALU cost per byte low (BF16/FP16 at R >= 32 needs more than the vector ALU
// can give at full HBM rate).
//
// Khatri-Rao operand.  K(rho, r) = prod over the reduced modes of
// H^(n)(digit_n(rho), r).  It is never formed in HBM: it factors as
// Kfast(rho mod Pf, r) * Kslow(rho / Pf, r) with "fast" a prefix of the
// reduced modes.  Kfast (Pf x Rpad) is staged once per workgroup in LDS in
// the tensor's own type, optionally as a hi + lo pair so the operand carries
// about 16 significant bits; each fast block's MFMA result is scaled by
// Kslow before it is added to the running sum.  For FP16 each Kfast column is
// scaled by a power of two into FP16's range and unscaled through Kslow.
//
// Matrix-core operand layouts (gfx950, wave64):
//   16x16x32 BF16/FP16: lane l holds A[l%16][8(l/16) .. +8] and
//                       B[8(l/16) .. +8][l%16]
//   16x16x4 FP32/FP64:  lane l holds A[l%16][l/16] and B[l/16][l%16]
//   result (all four):  lane l holds C[4(l/16) + v][l%16], v = 0..3
// The order of the reduction index inside a step is free as long as A and B
// agree, which lets every lane load 16 contiguous bytes of X.
#include "nncp_internal.h"

namespace nncp {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

template <typename T> __device__ __forceinline__ double to_d(T v) { return (double)v; }
template <> __device__ __forceinline__ double to_d<bf16_t>(bf16_t v) { return (double)(float)v; }
template <> __device__ __forceinline__ double to_d<f16_t>(f16_t v) { return (double)(float)v; }

template <typename T> __device__ __forceinline__ T from_d(double v) { return (T)v; }
template <> __device__ __forceinline__ bf16_t from_d<bf16_t>(double v) {
  // double -> float is exact for the products formed here up to rounding;
  // float -> bf16 rounds to nearest even.
  return (bf16_t)(float)v;
}
template <> __device__ __forceinline__ f16_t from_d<f16_t>(double v) { return (f16_t)(float)v; }

template <typename AT> struct CFrag;
template <> struct CFrag<float> { typedef f32x4 T; };
template <> struct CFrag<double> { typedef f64x4 T; };

// one matrix-core step on a 16-byte A chunk and a 16-byte B chunk
__device__ __forceinline__ void mma16(f32x4 &c, u32x4 a, u32x4 b, bf16_t *) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                              __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ __forceinline__ void mma16(f32x4 &c, u32x4 a, u32x4 b, f16_t *) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                             __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}
// FP32: the 16 bytes are 4 consecutive reduction indices, one MFMA each
__device__ __forceinline__ void mma16(f32x4 &c, u32x4 a, u32x4 b, float *) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
}
__device__ __forceinline__ double dbl_lo(u32x4 v) {
  return __builtin_bit_cast(double, ((uint64_t)v.y << 32) | v.x);
}
__device__ __forceinline__ double dbl_hi(u32x4 v) {
  return __builtin_bit_cast(double, ((uint64_t)v.w << 32) | v.z);
}
__device__ __forceinline__ void mma16(f64x4 &c, u32x4 a, u32x4 b, double *) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(dbl_lo(a), dbl_lo(b), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(dbl_hi(a), dbl_hi(b), c, 0, 0, 0);
}

// single-element MFMA (left kernel, FP32/FP64: one reduction index per lane)
__device__ __forceinline__ void mma1(f32x4 &c, float a, float b) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mma1(f64x4 &c, double a, double b) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// loads of X through the global (not flat) address space: gload marks them
// non-temporal, gload_c leaves them to the normal cache policy.  Normal loads
// let a tensor that fits the last-level cache stay there between the left
// and the right product; for much larger tensors the left kernel streams
// with non-temporal loads (measured faster there).
template <typename VT> __device__ __forceinline__ VT gload(const void *p) {
  typedef const __attribute__((address_space(1))) VT gvt;
  return __builtin_nontemporal_load((gvt *)p);
}
template <typename VT> __device__ __forceinline__ VT gload_c(const void *p) {
  typedef const __attribute__((address_space(1))) VT gvt;
  return *(gvt *)p;
}

template <bool NTL, typename VT> __device__ __forceinline__ VT xload(const void *p) {
  if constexpr (NTL) return gload<VT>(p);
  else return gload_c<VT>(p);
}

template <typename CT> __device__ __forceinline__ void czero(CT &c) {
  c[0] = 0; c[1] = 0; c[2] = 0; c[3] = 0;
}

// Result row held by lane group g in accumulator slot v: 4 g + v for the
// FP32-accumulating instructions, g + 4 v for the FP64 one.
template <typename AT> __device__ __forceinline__ int crow(int g, int v) {
  return sizeof(AT) == 8 ? g + 4 * v : 4 * g + v;
}

// LDS position of Kfast element (r, p).  Rows are ldk elements long; the
// 16-byte chunks of row r are XOR-swizzled with (r & swz) so that the 16
// lanes reading the same chunk index of 16 different rows hit 16 different
// bank groups (swz = 15 when a row has a multiple of 16 chunks, else 0 and
// the row is padded by one chunk instead).
template <typename XT>
__device__ __forceinline__ int kidx(int r, int p, int ldk, int swz) {
  constexpr int SV = 16 / (int)sizeof(XT);
  return r * ldk + (((p / SV) ^ (r & swz)) * SV) + (p % SV);
}

// ---------------------------------------------------------------------------
// Khatri-Rao operand: Kfast [hl][Rpad][Pf] in XT, Kslow [Ps][Rpad] in AT
// ---------------------------------------------------------------------------

struct KrpArgs {
  const void *H[NNCP_MAX_MODES];
  int64_t dims[NNCP_MAX_MODES];
  int fast_lo, fast_hi, slow_lo, slow_hi;
  int R, Rpad, hl, scale16;
  int64_t Pf, Ps;
};

template <typename HT>
__device__ double krp_entry(const KrpArgs &a, int lo, int hi, int64_t rho, int r) {
  double p = 1.0;
  const HT *const *H = (const HT *const *)a.H;
  for (int n = lo; n < hi; ++n) {
    const int64_t d = rho % a.dims[n];
    rho /= a.dims[n];
    p *= (double)H[n][d * a.R + r];
  }
  return p;
}

// Column r of the operand, the part that workgroup row by of gy forms.
template <typename XT, typename HT>
__device__ __forceinline__ void krp_column(const KrpArgs &a, XT *__restrict__ kfast,
                                           HT *__restrict__ kslow, int r, int by, int gy,
                                           double *red) {
  const bool live = r < a.R;
  double mx = 0.0;
  // the column maximum only matters for the FP16 scaling
  if (a.scale16) {
    if (live)
      for (int64_t p = threadIdx.x; p < a.Pf; p += 256) {
        const double v = krp_entry<HT>(a, a.fast_lo, a.fast_hi, p, r);
        mx = fmax(mx, fabs(v));
      }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
      __syncthreads();
    }
    mx = red[0];
  }
  int e = 0;
  if (a.scale16 && mx > 0.0) {
    int E;
    frexp(mx, &E);  // mx = f 2^E, f in [0.5, 1)
    e = 14 - E;     // max entry lands in [2^13, 2^14)
  }
  const double up = ldexp(1.0, e), down = ldexp(1.0, -e);
  // without the FP16 scaling the column is split over gy workgroups
  const int64_t t0 = threadIdx.x + 256 * (int64_t)by, ts = 256 * (int64_t)gy;
  for (int64_t p = t0; p < a.Pf; p += ts) {
    const double v = live ? krp_entry<HT>(a, a.fast_lo, a.fast_hi, p, r) * up : 0.0;
    const XT hi = from_d<XT>(v);
    kfast[(int64_t)r * a.Pf + p] = hi;
    if (a.hl) kfast[((int64_t)a.Rpad + r) * a.Pf + p] = from_d<XT>(v - to_d<XT>(hi));
  }
  for (int64_t q = t0; q < a.Ps; q += ts) {
    const double w = live ? krp_entry<HT>(a, a.slow_lo, a.slow_hi, q, r) * down : 0.0;
    kslow[q * a.Rpad + r] = (HT)w;
  }
}

template <typename XT, typename HT>
__global__ __launch_bounds__(256) void k_krp_operands(KrpArgs a, XT *__restrict__ kfast,
                                                      HT *__restrict__ kslow, GramJob job) {
  // extra columns of workgroups (blockIdx.x >= Rpad) when carrying the
  // Gram step of the previous update
  if (job.R && blockIdx.x >= a.Rpad) {
    gram_run(job, (blockIdx.x - a.Rpad) * gridDim.y + blockIdx.y);
    return;
  }
  __shared__ double red[256];
  krp_column<XT, HT>(a, kfast, kslow, blockIdx.x, blockIdx.y, gridDim.y, red);
}

// Two operands in one launch (columns of the first, then of the second), no
// FP16 scaling.
template <typename XT, typename HT>
__global__ __launch_bounds__(256) void k_krp_operands2(KrpArgs a0, XT *__restrict__ kf0,
                                                       HT *__restrict__ ks0, KrpArgs a1,
                                                       XT *__restrict__ kf1,
                                                       HT *__restrict__ ks1) {
  __shared__ double red[256];
  if ((int)blockIdx.x < a0.Rpad)
    krp_column<XT, HT>(a0, kf0, ks0, blockIdx.x, blockIdx.y, gridDim.y, red);
  else
    krp_column<XT, HT>(a1, kf1, ks1, blockIdx.x - a0.Rpad, blockIdx.y, gridDim.y, red);
}

// ---------------------------------------------------------------------------
// The Khatri-Rao operand as the matrix-core kernels read it.  Either the
// precomputed Kfast [hl][Rpad][Pf] and Kslow [Ps][Rpad] of k_krp_operands
// (hf == NULL, ldks = Rpad), or, when the fast part is a single mode and the
// slow part at most one (no FP16 scaling), the factors themselves: hf is the
// fast mode's factor [Pf][R], split into hi (+ lo) while it is staged with
// the same roundings as k_krp_operands, and kslow the slow mode's factor
// [Ps][R] (ldks = R) or NULL for no slow mode (a scale of one).  The direct
// form (R a multiple of 16, so R == Rpad) saves the operand kernel's launch.
// ---------------------------------------------------------------------------
template <typename XT> struct KOp {
  const XT *kfast;
  const typename XTraits<XT>::AT *kslow;
  const typename XTraits<XT>::AT *hf;
  int ldks;
};

template <typename XT> struct Chunk16 { XT v[16 / sizeof(XT)]; };

// Stage fast indices wbase .. wbase + W of Kfast into LDS rows of ldk
// elements (the hi rows 0 .. RP - 1, then the lo rows), 16-byte chunks
// XOR-swizzled with swz; nthr threads of the workgroup take part.
template <typename XT, bool HL>
__device__ __forceinline__ void stage_copy(const XT *kfast, XT *sk, int RP, int64_t Pf,
                                           int64_t wbase, int W, int ldk, int swz, int nthr) {
  constexpr int SV = 16 / (int)sizeof(XT);
  const int nv = W / SV;
  const int total = RP * nv * (HL ? 2 : 1);
  for (int e = threadIdx.x; e < total; e += nthr) {
    const int h = e / (RP * nv);
    const int rem = e - h * RP * nv;
    const int r = rem / nv, v = rem - r * nv;
    *reinterpret_cast<u32x4 *>(sk + h * RP * ldk + kidx<XT>(r, v * SV, ldk, swz)) =
        *reinterpret_cast<const u32x4 *>(kfast + ((int64_t)(h * RP + r)) * Pf + wbase + v * SV);
  }
}

template <typename XT, bool HL>
__device__ __forceinline__ void stage_kfast(const KOp<XT> &ko, XT *sk, int RP, int R, int64_t Pf,
                                            int64_t wbase, int W, int ldk, int swz, int nthr) {
  typedef typename XTraits<XT>::AT AT;
  constexpr int SV = 16 / (int)sizeof(XT);
  const int nv = W / SV;
  if (ko.hf == nullptr) {
    stage_copy<XT, HL>(ko.kfast, sk, RP, Pf, wbase, W, ldk, swz, nthr);
  } else if (R % (8 / (int)sizeof(AT) > 0 ? 8 / (int)sizeof(AT) : 1) == 0) {
    // thread e: columns r0 .. r0 + RV - 1 (r0 = RV (e % (RP / RV))) at fast
    // indices v SV .. v SV + SV - 1 (v = e / (RP / RV)): SV 16-byte loads of
    // factor rows (consecutive threads read consecutive pieces of a row),
    // RV 16-byte LDS chunks per half
    constexpr int RV = 8 / (int)sizeof(AT) > 0 ? 8 / (int)sizeof(AT) : 1;
    const int nrv = RP / RV;
    for (int e = threadIdx.x; e < nrv * nv; e += nthr) {
      const int r0 = RV * (e % nrv), v = e / nrv;
      AT x[SV][RV];
#pragma unroll
      for (int q = 0; q < SV; ++q) {
        typedef AT avec __attribute__((ext_vector_type(RV)));
        avec t;
        if (r0 < R) {
          t = *reinterpret_cast<const avec *>(ko.hf + (wbase + v * SV + q) * R + r0);
        } else {
#pragma unroll
          for (int u = 0; u < RV; ++u) t[u] = (AT)0;
        }
#pragma unroll
        for (int u = 0; u < RV; ++u) x[q][u] = t[u];
      }
#pragma unroll
      for (int u = 0; u < RV; ++u) {
        Chunk16<XT> hi, lo;
#pragma unroll
        for (int q = 0; q < SV; ++q) {
          const double xv = (double)x[q][u];
          hi.v[q] = from_d<XT>(xv);
          if (HL) lo.v[q] = from_d<XT>(xv - to_d<XT>(hi.v[q]));
        }
        XT *d = sk + kidx<XT>(r0 + u, v * SV, ldk, swz);
        *reinterpret_cast<u32x4 *>(d) = __builtin_bit_cast(u32x4, hi);
        if (HL) *reinterpret_cast<u32x4 *>(d + RP * ldk) = __builtin_bit_cast(u32x4, lo);
      }
    }
  } else {
    // thread e: column r = e % RP at fast indices v SV .. v SV + SV - 1 of
    // the window (consecutive threads read consecutive entries of a row)
    for (int e = threadIdx.x; e < RP * nv; e += nthr) {
      const int r = e % RP, v = e / RP;
      const int rc = r < R ? r : R - 1;
      Chunk16<XT> hi, lo;
#pragma unroll
      for (int q = 0; q < SV; ++q) {
        const double x = (double)ko.hf[(wbase + v * SV + q) * R + rc];
        const double xv = r < R ? x : 0.0;
        hi.v[q] = from_d<XT>(xv);
        if (HL) lo.v[q] = from_d<XT>(xv - to_d<XT>(hi.v[q]));
      }
      *reinterpret_cast<u32x4 *>(sk + kidx<XT>(r, v * SV, ldk, swz)) = __builtin_bit_cast(u32x4, hi);
      if (HL)
        *reinterpret_cast<u32x4 *>(sk + RP * ldk + kidx<XT>(r, v * SV, ldk, swz)) =
            __builtin_bit_cast(u32x4, lo);
    }
  }
}

// Kslow(b, r) where there is a slow part (r < Rpad: the direct form is used
// only when R == Rpad)
template <typename XT>
__device__ __forceinline__ typename XTraits<XT>::AT kslow_at(const KOp<XT> &ko, int64_t b, int r) {
  return ko.kslow[b * ko.ldks + r];
}
// the column scale of a product without slow modes: one, or the FP16 column
// scaling of the precomputed operand
template <typename XT>
__device__ __forceinline__ typename XTraits<XT>::AT kscale0(const KOp<XT> &ko, int r) {
  typedef typename XTraits<XT>::AT AT;
  return ko.kslow ? ko.kslow[r] : (AT)1;
}

// ---------------------------------------------------------------------------
// right partial MTTKRP on the matrix cores (reduction over the contiguous index)
//
// Workgroup = kRightWaves waves on the same 16*MT rows of Xr; the
// workgroup's share of the reduction (split blockIdx.y of nsplit) is cut into
// kRightWaves contiguous pieces, one per wave; the waves' sums are added
// through LDS in wave order.
// out: [nsplit][k][R] partial sums (factor type).
// ---------------------------------------------------------------------------

template <typename XT, int MT, int NT, bool HL, bool SLOW, int U, bool ILV>
__global__ __launch_bounds__(64 * kRightWaves) void k_gemm_right_mfma(
    const XT *__restrict__ X, int64_t m, int64_t k, KOp<XT> ko, int Pf, int64_t steps_total,
    int nsplit, int R, typename XTraits<XT>::AT *__restrict__ out, int ntx, GramJob job) {
  // workgroups past the product's ntx x nsplit (extra columns when nsplit is
  // 1, else extra rows: dispatched after every product workgroup) carry the
  // split Gram step of the previous update
  if (job.R) {
    const int lin = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (lin >= ntx * nsplit) {
      if (lin - ntx * nsplit < job.parts) gram_part(job, lin - ntx * nsplit);
      return;
    }
  }
  typedef typename XTraits<XT>::AT AT;
  typedef typename CFrag<AT>::T CT;
  constexpr int VEC = XTraits<XT>::VEC;
  constexpr int KSTEP = 4 * VEC;
  constexpr int RP = 16 * NT;
  extern __shared__ __align__(16) unsigned char smem[];
  XT *sk = reinterpret_cast<XT *>(smem);
  const int swz = ((Pf / VEC) % 16 == 0) ? 15 : 0;
  const int ldk = swz ? Pf : Pf + VEC;

  // stage Kfast (hi, then lo) into LDS
  stage_kfast<XT, HL>(ko, sk, RP, R, Pf, 0, Pf, ldk, swz, 64 * kRightWaves);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, g = lane >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * (16 * MT);
  const int64_t s_lo = steps_total * blockIdx.y / nsplit;
  const int64_t s_hi = steps_total * (blockIdx.y + 1) / nsplit;
  const int64_t w_lo = s_lo + (s_hi - s_lo) * wave / kRightWaves;
  const int64_t w_hi = s_lo + (s_hi - s_lo) * (wave + 1) / kRightWaves;
  const int spb = Pf / KSTEP;

  const XT *xp[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    int64_t jr = j0 + 16 * mt + row;
    if (jr > k - 1) jr = k - 1;
    xp[mt] = X + jr * m + g * VEC;
  }

  CT acc[MT][NT], blk[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) { czero(acc[mt][nt]); czero(blk[mt][nt]); }

  // Position in the fast block (pf) and fast-block index (bI) advance with
  // the steps; only the wave's starting position needs a division.
  int pf = (int)(w_lo % spb) * KSTEP;
  int64_t bI = w_lo / spb;
  auto flush = [&]() {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const AT s = kslow_at(ko, bI, 16 * nt + row);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[mt][nt][v] += blk[mt][nt][v] * s;
        czero(blk[mt][nt]);
      }
    }
  };
  auto step = [&](const u32x4 *va) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const XT *bp = sk + kidx<XT>(16 * nt + row, pf + g * VEC, ldk, swz);
      const u32x4 vb = *reinterpret_cast<const u32x4 *>(bp);
      u32x4 vbl;
      if (HL) vbl = *reinterpret_cast<const u32x4 *>(bp + RP * ldk);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        CT &c = SLOW ? blk[mt][nt] : acc[mt][nt];
        mma16(c, va[mt], vb, (XT *)nullptr);
        if (HL) mma16(c, va[mt], vbl, (XT *)nullptr);
      }
    }
    pf += KSTEP;
    if (pf == Pf) {
      if (SLOW) flush();
      pf = 0;
      ++bI;
    }
  };

  if constexpr (ILV) {
    // The workgroup's steps in batches of U, dealt to the waves in turn
    // (wave w takes batches w, w + kRightWaves, ...): at any time the waves
    // read neighbouring pieces of the same 16 MT rows (kRightWaves x U x 64
    // bytes of each row together, as the left kernel's waves do), instead
    // of kRightWaves distant ranges.  Current/next buffers; the batch after
    // the last re-reads the last one.  A block of the Khatri-Rao operand cut
    // by the end of a batch is flushed with its slow factor there; the
    // steps after the last full batch go to the wave next in turn.
    const int64_t nb = (s_hi - s_lo) / U;
    u32x4 cur[U][MT], nxt[U][MT];
    auto load = [&](u32x4 (&dst)[U][MT], int64_t b) {
      const int64_t t0 = s_lo + (b < nb ? b : nb - 1) * U;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) dst[u][mt] = gload_c<u32x4>(xp[mt] + (t0 + u) * KSTEP);
    };
    int64_t b = wave;
    if (b < nb) load(cur, b);
    for (; b < nb; b += kRightWaves) {
      load(nxt, b + kRightWaves);
      const int64_t t0 = s_lo + b * U;
      pf = (int)(t0 % spb) * KSTEP;
      bI = t0 / spb;
#pragma unroll
      for (int u = 0; u < U; ++u) step(cur[u]);
      if (SLOW && pf != 0) flush();
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) cur[u][mt] = nxt[u][mt];
    }
    if (wave == (int)(nb % kRightWaves) && s_lo + nb * U < s_hi) {
      const int64_t t0 = s_lo + nb * U;
      pf = (int)(t0 % spb) * KSTEP;
      bI = t0 / spb;
      for (int64_t tt = t0; tt < s_hi; ++tt) {
        u32x4 va[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) va[mt] = gload_c<u32x4>(xp[mt] + tt * KSTEP);
        step(va);
      }
      if (SLOW && pf != 0) flush();
    }
  } else {
  // batches of U steps, the next batch's loads issued before the current
  // batch is consumed.  16-bit and FP64 tensors: current/next buffers with a
  // copy (the last batch re-reads itself instead of running past the wave's
  // range).  FP32 tensors: two buffers used in turn with the loop unrolled
  // over them, so no copy waits for the loads (measured 5% faster for FP32,
  // slower for BF16); loads past the last full batch re-read it.
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) xp[mt] += w_lo * KSTEP;
  int64_t t = w_lo;
  const int64_t nb = (w_hi - w_lo) / U;
  if (nb > 0 && sizeof(XT) == 4) {
    u32x4 buf[2][U][MT];
    auto load = [&](u32x4 (&dst)[U][MT], int64_t bidx) {
      const int64_t bc = bidx < nb ? bidx : nb - 1;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          dst[u][mt] = gload_c<u32x4>(xp[mt] + (bc * U + u) * KSTEP);
    };
    load(buf[0], 0);
    for (int64_t b0 = 0; b0 < nb; b0 += 2) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t b = b0 + j;
        load(buf[j ^ 1], b + 1);
        if (b >= nb) break;
#pragma unroll
        for (int u = 0; u < U; ++u) step(buf[j][u]);
      }
    }
    t += nb * U;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) xp[mt] += nb * U * KSTEP;
  } else if (nb > 0) {
    u32x4 cur[U][MT], nxt[U][MT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        cur[u][mt] = gload_c<u32x4>(xp[mt] + u * KSTEP);
    for (int64_t b = 0; b < nb; ++b, t += U) {
      const int adv = b + 1 < nb ? U * KSTEP : 0;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          nxt[u][mt] = gload_c<u32x4>(xp[mt] + adv + u * KSTEP);
#pragma unroll
      for (int u = 0; u < U; ++u) step(cur[u]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) xp[mt] += U * KSTEP;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) cur[u][mt] = nxt[u][mt];
    }
  }
  for (; t < w_hi; ++t) {
    u32x4 va[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      va[mt] = gload_c<u32x4>(xp[mt]);
      xp[mt] += KSTEP;
    }
    step(va);
  }
  // a fast block cut by the end of the wave's range
  if (SLOW && pf != 0) flush();
  }
  if (!SLOW) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const AT s = kscale0(ko, 16 * nt + row);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[mt][nt][v] *= s;
    }
  }

  // add the waves' sums in wave order
  constexpr int NV = MT * NT * 4;
  __syncthreads();
  AT *red = reinterpret_cast<AT *>(smem);
  if (wave > 0) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          red[((wave - 1) * NV + (mt * NT + nt) * 4 + v) * 64 + lane] = acc[mt][nt][v];
  }
  __syncthreads();
  if (wave == 0) {
    AT *o = out + (int64_t)blockIdx.y * k * R;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int e = (mt * NT + nt) * 4 + v;
          AT s = acc[mt][nt][v];
#pragma unroll
          for (int w = 0; w < kRightWaves - 1; ++w) s += red[(w * NV + e) * 64 + lane];
          const int64_t j = j0 + 16 * mt + crow<AT>(g, v);
          const int r = 16 * nt + row;
          if (j < k && r < R) o[j * R + r] = s;
        }
  }
}

// ---------------------------------------------------------------------------
// left partial MTTKRP on the matrix cores (reduction over rows of Xr)
//
// A workgroup of left_waves() waves (eight in most cases: one workgroup per
// CU at the register use of these kernels) shares one LDS copy of the
// Khatri-Rao window; eight waves halve the staging traffic per byte of X
// against four, which measured 2-9% faster.  Each wave owns 16*QV consecutive columns i of Xr; lane (rho, g) loads QV
// consecutive columns from KL rows.  For BF16/FP16 the KL x QV block is
// transposed inside the lane (byte permutes) into QV A-operands of KL
// reduction elements each; for FP32/FP64 (KL = 1) every loaded element is
// an A-operand by itself.  out: [nsplit][R][m] (factor type), i.e. the node
// layout of the paper (column block r contiguous).
// ---------------------------------------------------------------------------

template <int BYTES> struct LoadT;
template <> struct LoadT<16> { typedef u32x4 T; };
template <> struct LoadT<8> { typedef u32x2 T; };

__device__ __forceinline__ uint32_t dw(const u32x4 &v, int i) { return v[i]; }
__device__ __forceinline__ uint32_t dw(const u32x2 &v, int i) { return v[i]; }

template <typename XT, int QV, int NT, bool HL, bool SLOW, bool NTL>
__global__ __launch_bounds__(64 * left_waves(sizeof(XT), QV, NT, SLOW)) void k_gemm_left_mfma(
    const XT *__restrict__ X, int64_t m, int64_t k, KOp<XT> ko, int Pf, int W,
    int64_t steps_total, int nsplit, int R, typename XTraits<XT>::AT *__restrict__ out, int ntx,
    GramJob job) {
  // workgroups past the product's ntx x nsplit (extra columns when nsplit is
  // 1, else extra rows: dispatched after every product workgroup) carry the
  // split Gram step of the previous update
  if (job.R) {
    const int lin = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (lin >= ntx * nsplit) {
      if (lin - ntx * nsplit < job.parts) gram_part(job, lin - ntx * nsplit);
      return;
    }
  }
  typedef typename XTraits<XT>::AT AT;
  typedef typename CFrag<AT>::T CT;
  constexpr int WV = left_waves(sizeof(XT), QV, NT, SLOW);
  constexpr int KL = XTraits<XT>::KL;
  constexpr int KSTEP = 4 * KL;  // rows per step
  constexpr int RP = 16 * NT;
  constexpr int LB = QV * (int)sizeof(XT);
  typedef typename LoadT<LB>::T LT;
  extern __shared__ __align__(16) unsigned char smem[];
  XT *sk = reinterpret_cast<XT *>(smem);
  constexpr int SVEC = 16 / (int)sizeof(XT);
  // LDS holds a window of W fast indices (W divides Pf); every wave walks the
  // same rows, so the window is re-staged between two barriers when the rows
  // cross into the next window (once per workgroup when W == Pf)
  const int swz = ((W / SVEC) % 16 == 0) ? 15 : 0;
  const int ldk = swz ? W : W + SVEC;
  // precomputed operand windows, staged inside the loop
  auto stage = [&](int wbase) { stage_copy<XT, HL>(ko.kfast, sk, RP, Pf, wbase, W, ldk, swz, 64 * WV); };
  int cur_w = -1;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rho = lane & 15, g = lane >> 4;
  const int64_t i0 = ((int64_t)blockIdx.x * WV + wave) * (16 * QV);
  const int64_t il = i0 + QV * rho;
  const bool valid = il < m;
  const XT *xp = X + (valid ? il : 0) + (int64_t)(g * KL) * m;
  const int64_t s_lo = steps_total * blockIdx.y / nsplit;
  const int64_t s_hi = steps_total * (blockIdx.y + 1) / nsplit;
  const int spb = Pf / KSTEP;

  CT acc[QV][NT], blk[QV][NT];
#pragma unroll
  for (int q = 0; q < QV; ++q)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) { czero(acc[q][nt]); czero(blk[q][nt]); }

  // Steps are taken in batches of SB (SB * KL rows per lane: 8 loads).  NB
  // batch buffers rotate with the loop unrolled over them, so the loads of
  // the next NB - 1 batches are in flight while a batch is consumed and no
  // register copy waits for them.  Steps past the end of the range re-load
  // the last valid step and are not computed.  Depths as measured best:
  // 16-bit tensors 4 (2 with a single 16-column tile), FP32 2, FP64 3.
  constexpr int SB = KL == 8 ? 1 : 8;
  constexpr int NB = KL == 8 ? (NT == 1 ? 2 : 4) : (sizeof(XT) == 4 ? 2 : 3);
  LT buf[NB][SB * KL];
  auto load_batch = [&](LT *dst, int64_t t0) {
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      const int64_t tt = t0 + b < s_hi ? t0 + b : s_hi - 1;
#pragma unroll
      for (int u = 0; u < KL; ++u)
        if constexpr (NTL) dst[b * KL + u] = gload<LT>(xp + (tt * KSTEP + u) * m);
        else dst[b * KL + u] = gload_c<LT>(xp + (tt * KSTEP + u) * m);
    }
  };
  if (s_lo < s_hi) {
#pragma unroll
    for (int j = 0; j < NB - 1; ++j) load_batch(buf[j], s_lo + j * SB);
  }
  if (ko.hf) {
    // the operand formed from the factors (one window, W == Pf), staged
    // while the first batches are in flight (outside the loop, where fewer
    // registers are live)
    stage_kfast<XT, HL>(ko, sk, RP, R, Pf, 0, W, ldk, swz, 64 * WV);
    __syncthreads();
    cur_w = 0;
  }
  // position in the fast block, window index and block index, advanced with
  // the steps (one division at the start)
  int pfa = (int)(s_lo % spb) * KSTEP;
  int64_t bI = s_lo / spb;
  for (int64_t t0 = s_lo; t0 < s_hi; t0 += NB * SB) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int64_t tb = t0 + j * SB;
      load_batch(buf[(j + NB - 1) % NB], tb + (NB - 1) * SB);
      if (tb >= s_hi) break;
#pragma unroll
      for (int b = 0; b < SB; ++b) {
        const int64_t t = tb + b;
        if (t >= s_hi) break;
        const LT *rw = buf[j] + b * KL;
        const int wi = W == Pf ? 0 : pfa / W;
        if (wi != cur_w) {
          __syncthreads();
          stage(wi * W);
          __syncthreads();
          cur_w = wi;
        }
        const int pf0 = pfa - wi * W;
        if constexpr (KL == 8) {
          u32x4 vb[NT], vbl[NT];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const XT *bp = sk + kidx<XT>(16 * nt + rho, pf0 + g * KL, ldk, swz);
            vb[nt] = *reinterpret_cast<const u32x4 *>(bp);
            if (HL) vbl[nt] = *reinterpret_cast<const u32x4 *>(bp + RP * ldk);
          }
#pragma unroll
          for (int q = 0; q < QV; ++q) {
            const uint32_t sel = (q & 1) ? 0x07060302u : 0x05040100u;
            u32x4 a;
            a.x = __builtin_amdgcn_perm(dw(rw[1], q >> 1), dw(rw[0], q >> 1), sel);
            a.y = __builtin_amdgcn_perm(dw(rw[3], q >> 1), dw(rw[2], q >> 1), sel);
            a.z = __builtin_amdgcn_perm(dw(rw[5], q >> 1), dw(rw[4], q >> 1), sel);
            a.w = __builtin_amdgcn_perm(dw(rw[7], q >> 1), dw(rw[6], q >> 1), sel);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
              CT &c = SLOW ? blk[q][nt] : acc[q][nt];
              mma16(c, a, vb[nt], (XT *)nullptr);
              if (HL) mma16(c, a, vbl[nt], (XT *)nullptr);
            }
          }
        } else {
          AT bb[NT];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) bb[nt] = (AT)sk[kidx<XT>(16 * nt + rho, pf0 + g, ldk, swz)];
          const AT *xv = reinterpret_cast<const AT *>(rw);
#pragma unroll
          for (int q = 0; q < QV; ++q)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) mma1(SLOW ? blk[q][nt] : acc[q][nt], xv[q], bb[nt]);
        }
        pfa += KSTEP;
        const bool wrap = pfa == Pf;
        if (SLOW && (wrap || t + 1 == s_hi)) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const AT sc = kslow_at(ko, bI, 16 * nt + rho);
#pragma unroll
            for (int q = 0; q < QV; ++q) {
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[q][nt][v] += blk[q][nt][v] * sc;
              czero(blk[q][nt]);
            }
          }
        }
        if (wrap) {
          pfa = 0;
          ++bI;
        }
      }
    }
  }

  // Epilogue: each group of 16 result columns r goes through LDS (the
  // operand's LDS, free after the barrier) so that every store writes whole
  // 16-byte pieces of the rows T(r, i0 ..) instead of scattered elements.
  constexpr int CW = 16 * QV;                // columns of T per wave
  constexpr int VE = 16 / (int)sizeof(AT);   // elements per 16-byte store
  constexpr int LDW = CW + VE;               // LDS row stride (elements)
  constexpr int LPR = CW / VE;               // lanes per row segment
  constexpr int RPI = 64 / LPR;              // rows per store instruction
  typedef AT avec __attribute__((ext_vector_type(VE)));
  AT *eb = reinterpret_cast<AT *>(smem) + wave * 16 * LDW;
  AT *o = out + (int64_t)blockIdx.y * R * m;
  const bool vec_ok = (m % VE) == 0;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const AT s = SLOW ? (AT)1 : kscale0(ko, 16 * nt + rho);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      AT *dst = eb + rho * LDW + QV * crow<AT>(g, v);
#pragma unroll
      for (int q0 = 0; q0 < QV; q0 += (VE < QV ? VE : QV)) {
        if constexpr (VE <= QV) {
          avec t;
#pragma unroll
          for (int e = 0; e < VE; ++e) t[e] = acc[q0 + e][nt][v] * s;
          *reinterpret_cast<avec *>(dst + q0) = t;
        } else {
#pragma unroll
          for (int e = 0; e < QV; ++e) dst[e] = acc[e][nt][v] * s;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r0 = 0; r0 < 16; r0 += RPI) {
      const int rr = r0 + lane / LPR, cc = (lane % LPR) * VE;
      const int r = 16 * nt + rr;
      const int64_t col = i0 + cc;
      if (r < R && col < m) {
        const AT *src = eb + rr * LDW + cc;
        AT *gd = o + (int64_t)r * m + col;
        if (vec_ok && col + VE <= m) {
          *reinterpret_cast<avec *>(gd) = *reinterpret_cast<const avec *>(src);
        } else {
#pragma unroll
          for (int e = 0; e < VE; ++e)
            if (col + e < m) gd[e] = src[e];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Both partial MTTKRPs of the root in one pass over X (the gradient, where
// every mode's MTTKRP is taken at the same factors):
//   left   T_L[i, r] = sum_j Xr[j, i] K_R(j, r)    (reduce over rows)
//   right  T_R[j, r] = sum_i Xr[j, i] K_L(i, r)    (reduce over columns)
// BF16 tensors, R <= 32.  A workgroup is kDualWaves waves on 128 consecutive
// columns each and walks every row in steps of 32; lane (rho, g) loads rows
// 8g .. 8g+7 of the step at columns 8 rho .. 8 rho+7 of its wave, eight
// 16-byte loads, as the left kernel does.
//  * T_L: the left kernel's in-lane transpose into A operands; the B operand
//    is K_R itself, the slow factor already folded in (formed once, whole,
//    by the Khatri-Rao operand kernel, hi + lo): its rows are staged in LDS a
//    window of kDualWin rows at a time between two barriers when the rows
//    cross into the next window, the next window's pieces loaded into
//    registers while the current one is in use.  No per-block accumulators
//    are needed.
//  * T_R: each lane also writes its eight 16-byte row pieces into a
//    wave-private LDS tile (16-byte chunks XOR-swizzled by row) and reads the
//    A operands (16 rows x 32 columns) back from it; the B operands are the
//    fast part of K_L (staged once); the product of each 32-column chunk is
//    scaled by the slow part of K_L at its columns (fixed for the wave, held
//    in registers) before it is added.  The waves' 32 x R results of a step
//    are added in wave order through LDS (two slot sets used in turn, one
//    barrier per step) and written as the workgroup's partial
//    out_r[tile][j][r]; the tiles' partials are added in tile order
//    afterwards by k_finalize.
// ---------------------------------------------------------------------------
constexpr int kDualWaves = 8;
constexpr int kDualWin = 128;

// Piece (16 bytes) of slot row sl that holds fragment c = h NT + nt.  With
// NT = 2 (four pieces a row) the pieces of any 16 consecutive lanes, and of
// any aligned 8 of them, land in distinct 16-byte bank groups, both for the
// writers (16 consecutive rows, one fragment) and for the readers (four
// consecutive columns r times q & 3, see the reduction); NT = 1 rotates by
// l / 16 only.
template <int NT>
__device__ __forceinline__ int dual_slot_piece(int sl, int c) {
  if constexpr (NT == 2) {
    const int f = 2 * (((sl >> 3) ^ (sl >> 1)) & 1) + ((sl >> 2) & 1);
    return c ^ f ^ ((sl >> 4) & 3);
  } else {
    return c ^ ((sl >> 4) & (2 * NT - 1));
  }
}

struct DualArgs {
  int64_t m, k;
  int PfL;             // fast length of K_L (a multiple of 32), staged whole
  int R;
  int rmaj;            // right partials [tile][R][k] (else [tile][k][R])
};

template <typename XT, int NT, bool HL, bool NTL>
__global__ __launch_bounds__(64 * kDualWaves) void k_gemm_dual_mfma(
    const XT *__restrict__ X, DualArgs a, const XT *__restrict__ kfr, const XT *__restrict__ kfl,
    const float *__restrict__ ksl, float *__restrict__ out_l, float *__restrict__ out_r) {
  typedef f32x4 CT;
  constexpr int WV = kDualWaves, QV = 8, KL = 8, KSTEP = 32, RP = 16 * NT;
  constexpr int SVEC = 8;  // elements per 16-byte chunk
  extern __shared__ __align__(16) unsigned char smem[];
  // LDS: K_R window [HL+1][RP][kDualWin] | K_L fast part [HL+1][RP][ldl] |
  //      X tiles [WV][32][128] | T_R slots [2][WV][64 * 4 * 2 * NT] floats
  const int ldl = ((a.PfL / SVEC) % 16 == 0) ? a.PfL : a.PfL + SVEC;
  const int swl = ((a.PfL / SVEC) % 16 == 0) ? 15 : 0;
  XT *skr = reinterpret_cast<XT *>(smem);
  XT *skl = skr + (HL ? 2 : 1) * RP * kDualWin;
  XT *sxt = skl + (HL ? 2 : 1) * RP * ldl;
  constexpr int SLOT = 64 * 4 * 2 * NT;  // floats per wave and step
  float *str = reinterpret_cast<float *>(sxt + WV * 32 * 128);
  const int m = (int)a.m;  // m < 2^31 (checked by the planner)
  const int64_t k = a.k;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rho = lane & 15, g = lane >> 4;
  const int64_t c0w = ((int64_t)blockIdx.x * WV + wave) * 128;  // the wave's first column
  const int64_t il = c0w + QV * rho;
  const bool valid = il < m;
  const XT *xp = X + (valid ? il : 0) + (int64_t)(g * KL) * m;

  // K_L fast part, staged once (the 16-byte chunks of row r XOR-swizzled with
  // r & swl, as in the other kernels)
  {
    const int nv = a.PfL / SVEC;
    const int total = RP * nv * (HL ? 2 : 1);
    for (int e = tid; e < total; e += 64 * WV) {
      const int h = e / (RP * nv);
      const int rem = e - h * RP * nv;
      const int r = rem / nv, v = rem - r * nv;
      *reinterpret_cast<u32x4 *>(skl + h * RP * ldl + kidx<XT>(r, v * SVEC, ldl, swl)) =
          *reinterpret_cast<const u32x4 *>(kfl + ((int64_t)(h * RP + r)) * a.PfL + v * SVEC);
    }
  }
  // the slow factor of K_L at the wave's four 32-column chunks, and the fast
  // offset of each chunk (a chunk never crosses a fast block: PfL % 32 == 0)
  float ks[4][NT];
  int pfl[4];
  bool cok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t col = c0w + 32 * c + 8 * g;  // this lane's 8 columns as an A operand
    cok[c] = col < m;
    const int64_t cc = c0w + 32 * c < m ? c0w + 32 * c : 0;
    pfl[c] = (int)(cc % a.PfL);
    const int64_t sidx = cc / a.PfL;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) ks[c][nt] = ksl[sidx * RP + 16 * nt + rho];
  }
  // K_R windows: rows wbase .. wbase + kDualWin of K_R ([HL+1][RP][k] in
  // global memory), fetched into registers (16-byte pieces) and stored to
  // LDS at the window boundary
  constexpr int WCH = kDualWin / SVEC;
  constexpr int WTOT = (HL ? 2 : 1) * RP * WCH;
  constexpr int WPT = (WTOT + 64 * WV - 1) / (64 * WV);
  u32x4 kwin[WPT];
  auto fetch_kr = [&](int64_t wbase) {
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int e = tid + q * 64 * WV;
      const int ec = e < WTOT ? e : WTOT - 1;
      const int h = ec / (RP * WCH), rem = ec - h * RP * WCH;
      const int r = rem / WCH, v = rem - r * WCH;
      const int64_t j = wbase + v * SVEC;
      kwin[q] = j < k ? *reinterpret_cast<const u32x4 *>(kfr + ((int64_t)(h * RP + r)) * k + j)
                      : u32x4{0u, 0u, 0u, 0u};
    }
  };
  auto store_kr = [&]() {
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int e = tid + q * 64 * WV;
      if (e >= WTOT) continue;
      const int h = e / (RP * WCH), rem = e - h * RP * WCH;
      const int r = rem / WCH, v = rem - r * WCH;
      *reinterpret_cast<u32x4 *>(skr + h * RP * kDualWin + kidx<XT>(r, v * SVEC, kDualWin, 15)) =
          kwin[q];
    }
  };
  fetch_kr(0);

  CT acc[QV][NT], cr[2][NT];
#pragma unroll
  for (int q = 0; q < QV; ++q)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) czero(acc[q][nt]);
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) czero(cr[h][nt]);

  XT *xt = sxt + wave * 32 * 128;
  const int64_t steps = k / KSTEP;
  constexpr int NB = 2;
  u32x4 buf[NB][KL];
  auto load_step = [&](u32x4 *dst, int64_t t) {
    const int64_t tt = t < steps ? t : steps - 1;
#pragma unroll
    for (int u = 0; u < KL; ++u) dst[u] = xload<NTL, u32x4>(xp + (tt * KSTEP + u) * (int64_t)m);
  };
  // step t + 2 is loaded into step t's registers as soon as step t has been
  // copied to the LDS tile (halfway through step t), so about a step and a
  // half of X is in flight per wave with two register buffers
  load_step(buf[0], 0);
  load_step(buf[1], 1);
  int64_t wcur = -1;
  for (int64_t t0 = 0; t0 < steps; t0 += NB) {
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      const int64_t t = t0 + jb;
      if (t >= steps) break;
      const u32x4 *rw = buf[jb];
      const int64_t j0 = t * KSTEP;
      const int64_t wb = j0 / kDualWin * kDualWin;
      if (wb != wcur) {
        __syncthreads();
        store_kr();
        __syncthreads();
        wcur = wb;
        fetch_kr(wb + kDualWin);
      }
      // ---- T_L: as the left kernel, B = K_R rows j0 - wb + 8g ..
      {
        u32x4 vb[NT], vbl[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const XT *bp = skr + kidx<XT>(16 * nt + rho, (int)(j0 - wb) + g * KL, kDualWin, 15);
          vb[nt] = *reinterpret_cast<const u32x4 *>(bp);
          if (HL) vbl[nt] = *reinterpret_cast<const u32x4 *>(bp + RP * kDualWin);
        }
#pragma unroll
        for (int q = 0; q < QV; ++q) {
          const uint32_t sel = (q & 1) ? 0x07060302u : 0x05040100u;
          u32x4 av;
          av.x = __builtin_amdgcn_perm(rw[1][q >> 1], rw[0][q >> 1], sel);
          av.y = __builtin_amdgcn_perm(rw[3][q >> 1], rw[2][q >> 1], sel);
          av.z = __builtin_amdgcn_perm(rw[5][q >> 1], rw[4][q >> 1], sel);
          av.w = __builtin_amdgcn_perm(rw[7][q >> 1], rw[6][q >> 1], sel);
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            mma16(acc[q][nt], av, vb[nt], (XT *)nullptr);
            if (HL) mma16(acc[q][nt], av, vbl[nt], (XT *)nullptr);
          }
        }
      }
      // ---- T_R: the step's 32 rows through the wave's LDS tile
      wave_sync_lds();
#pragma unroll
      for (int u = 0; u < KL; ++u) {
        const int row = 8 * g + u;
        *reinterpret_cast<u32x4 *>(xt + row * 128 + ((rho ^ (row & 15)) * SVEC)) = rw[u];
      }
      load_step(buf[jb], t + 2);
      wave_sync_lds();
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        u32x4 ar[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int row = 16 * h + rho;
          ar[h] = *reinterpret_cast<const u32x4 *>(xt + row * 128 + (((4 * c + g) ^ (row & 15)) * SVEC));
          if (!cok[c]) ar[h] = u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const XT *bp = skl + kidx<XT>(16 * nt + rho, pfl[c] + g * KL, ldl, swl);
          const u32x4 bh = *reinterpret_cast<const u32x4 *>(bp);
          u32x4 bl;
          if (HL) bl = *reinterpret_cast<const u32x4 *>(bp + RP * ldl);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            CT tmp;
            czero(tmp);
            mma16(tmp, ar[h], bh, (XT *)nullptr);
            if (HL) mma16(tmp, ar[h], bl, (XT *)nullptr);
#pragma unroll
            for (int v = 0; v < 4; ++v) cr[h][nt][v] += tmp[v] * ks[c][nt];
          }
        }
      }
      // ---- the waves' T_R results of this step, added in wave order.  Lane
      // l's fragment (h, nt) holds rows jj = 16 h + 4 (l / 16) + v (v < 4) of
      // the step at column r = 16 nt + l % 16; its 16-byte piece goes to
      // piece dual_slot_piece(l, h NT + nt) of the lane's slot row.
      float *slot = str + ((int)(t & 1) * WV + wave) * SLOT;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int ch = dual_slot_piece<NT>(lane, h * NT + nt);
          *reinterpret_cast<f32x4 *>(slot + lane * (8 * NT) + ch * 4) = cr[h][nt];
          czero(cr[h][nt]);
        }
      __syncthreads();
      // thread (r, q): rows 4 q .. 4 q + 3 of the step at column r, one
      // 16-byte piece per wave.  NT = 2: 16 consecutive threads take four
      // consecutive r times the four q & 3 (one h), a wave eight r times all
      // eight q (whole 128-byte row pieces of the result); NT = 1: q = tid % 8.
      if (tid < 8 * RP) {
        int q, r;
        if constexpr (NT == 2) {
          q = (tid & 3) + 4 * ((tid >> 4) & 1);
          r = ((tid >> 2) & 3) + 4 * (tid >> 5);
        } else {
          q = tid & 7;
          r = tid >> 3;
        }
        const int sl = (r & 15) + 16 * (q & 3);
        const int ch = dual_slot_piece<NT>(sl, (q >> 2) * NT + (r >> 4));
        const float *sb = str + (int)(t & 1) * WV * SLOT + sl * (8 * NT) + ch * 4;
        f32x4 s = *reinterpret_cast<const f32x4 *>(sb);
#pragma unroll 2
        for (int w = 1; w < WV; ++w) {
          const f32x4 v = *reinterpret_cast<const f32x4 *>(sb + w * SLOT);
          s[0] += v[0]; s[1] += v[1]; s[2] += v[2]; s[3] += v[3];
        }
        if (r < a.R) {
          const int64_t j = j0 + 4 * q;  // k is a multiple of 32
          if (a.rmaj) {
            *reinterpret_cast<f32x4 *>(out_r + ((int64_t)blockIdx.x * a.R + r) * k + j) = s;
          } else {
            float *o = out_r + ((int64_t)blockIdx.x * k + j) * a.R + r;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[(int64_t)v * a.R] = s[v];
          }
        }
      }
    }
  }

  // ---- T_L epilogue (as the left kernel): 16 result columns at a time
  // through LDS so that every store writes whole 16-byte pieces
  constexpr int CW = 16 * QV, VE = 4, LDW = CW + VE, LPR = CW / VE, RPI = 64 / LPR;
  float *eb = reinterpret_cast<float *>(smem) + wave * 16 * LDW;
  const bool vec_ok = (m % VE) == 0;
  const int64_t i0 = c0w;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float *dst = eb + rho * LDW + QV * (4 * g + v);
#pragma unroll
      for (int q0 = 0; q0 < QV; q0 += VE) {
        f32x4 tv;
#pragma unroll
        for (int e = 0; e < VE; ++e) tv[e] = acc[q0 + e][nt][v];
        *reinterpret_cast<f32x4 *>(dst + q0) = tv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r0 = 0; r0 < 16; r0 += RPI) {
      const int rr = r0 + lane / LPR, cc = (lane % LPR) * VE;
      const int r = 16 * nt + rr;
      const int64_t col = i0 + cc;
      if (r < a.R && col < m) {
        const float *src = eb + rr * LDW + cc;
        float *gd = out_l + (int64_t)r * m + col;
        if (vec_ok && col + VE <= m) {
          *reinterpret_cast<f32x4 *>(gd) = *reinterpret_cast<const f32x4 *>(src);
        } else {
#pragma unroll
          for (int e = 0; e < VE; ++e)
            if (col + e < m) gd[e] = src[e];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// portable vector-ALU partial MTTKRPs (any shape, any R; used when the
// matrix-core preconditions are not met, and as a forced path)
// ---------------------------------------------------------------------------

struct GenArgs {
  const void *H[NNCP_MAX_MODES];
  int64_t dims[NNCP_MAX_MODES];
  int red_lo, red_hi;  // reduced modes [lo, hi)
  int R;
  int64_t m, k;
  int nsplit;
};

template <typename HT>
__device__ __forceinline__ void krp_row(const GenArgs &a, int64_t rho, int r0, int rc, HT *out) {
  const HT *const *H = (const HT *const *)a.H;
  for (int c = 0; c < rc; ++c) out[c] = (HT)1;
  for (int n = a.red_lo; n < a.red_hi; ++n) {
    const int64_t d = rho % a.dims[n];
    rho /= a.dims[n];
    const HT *h = H[n] + d * a.R + r0;
    for (int c = 0; c < rc; ++c) out[c] *= h[c];
  }
}

// right: block per (row j, split); threads stride over i; 16-column chunks.
template <typename XT, typename HT>
__global__ __launch_bounds__(256) void k_gemm_right_generic(const XT *__restrict__ X, GenArgs a,
                                                            HT *__restrict__ out) {
  constexpr int RC = 16;
  __shared__ HT red[RC][257];
  const int64_t j = blockIdx.x;
  const int64_t lo = a.m * blockIdx.y / a.nsplit, hi = a.m * (blockIdx.y + 1) / a.nsplit;
  const XT *xr = X + j * a.m;
  for (int r0 = 0; r0 < a.R; r0 += RC) {
    const int rc = min(RC, a.R - r0);
    HT acc[RC];
    for (int c = 0; c < RC; ++c) acc[c] = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
      HT kv[RC];
      krp_row<HT>(a, i, r0, rc, kv);
      const HT x = (HT)to_d<XT>(xr[i]);
      for (int c = 0; c < rc; ++c) acc[c] += x * kv[c];
    }
    for (int c = 0; c < RC; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s)
        for (int c = 0; c < RC; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x < rc) out[((int64_t)blockIdx.y * a.k + j) * a.R + r0 + threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

// left: thread per column i, loop over the split's rows j.
template <typename XT, typename HT>
__global__ __launch_bounds__(256) void k_gemm_left_generic(const XT *__restrict__ X, GenArgs a,
                                                           HT *__restrict__ out) {
  constexpr int RC = 16;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t lo = a.k * blockIdx.y / a.nsplit, hi = a.k * (blockIdx.y + 1) / a.nsplit;
  if (i >= a.m) return;
  for (int r0 = 0; r0 < a.R; r0 += RC) {
    const int rc = min(RC, a.R - r0);
    HT acc[RC];
    for (int c = 0; c < RC; ++c) acc[c] = 0;
    for (int64_t j = lo; j < hi; ++j) {
      HT kv[RC];
      krp_row<HT>(a, j, r0, rc, kv);
      const HT x = (HT)to_d<XT>(X[j * a.m + i]);
      for (int c = 0; c < rc; ++c) acc[c] += x * kv[c];
    }
    for (int c = 0; c < rc; ++c) out[((int64_t)blockIdx.y * a.R + r0 + c) * a.m + i] = acc[c];
  }
}

// ---------------------------------------------------------------------------
// finalize: add the split partials in split order
//   right partials [s][rows][R]; left partials [s][R][rows]
//   node output [r][rows]; leaf output (M) [rows][r]
// ---------------------------------------------------------------------------

template <typename HT>
__global__ __launch_bounds__(256) void k_finalize(const HT *__restrict__ part, int64_t rows, int R,
                                                  int nsplit, int part_rmajor, int leaf,
                                                  HT *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * R) return;
  int64_t row, r;
  if (leaf) { row = e / R; r = e % R; } else { r = e / rows; row = e % rows; }
  const int64_t src = part_rmajor ? r * rows + row : row * R + r;
  const HT *p = part + src;
  const int64_t stride = rows * R;
  // added in split order; loads issued eight at a time
  HT s = p[0];
  int q = 1;
  for (; q + 8 <= nsplit; q += 8) {
    HT v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(q + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; q < nsplit; ++q) s += p[(int64_t)q * stride];
  out[e] = s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static KrpArgs make_krp_args(const GemmPlan &p, int R, const int64_t *dims, const FactorSet &F,
                             int N) {
  KrpArgs a;
  for (int n = 0; n < NNCP_MAX_MODES; ++n) {
    a.H[n] = n < N ? F.H[n] : nullptr;
    a.dims[n] = n < N ? dims[n] : 1;
  }
  a.fast_lo = p.fast_lo; a.fast_hi = p.fast_hi;
  a.slow_lo = p.slow_lo; a.slow_hi = p.slow_hi;
  a.R = R; a.Rpad = p.Rpad; a.hl = p.hl; a.scale16 = 0;
  a.Pf = p.Pf; a.Ps = p.Ps;
  return a;
}

hipError_t launch_krp_operands(int xdt, const GemmPlan &p, int R, const int64_t *dims, int N,
                               const FactorSet &F, void *kfast, void *kslow, hipStream_t st,
                               GramJob *carry) {
  KrpArgs a = make_krp_args(p, R, dims, F, N);
  const GramJob job = carry ? *carry : GramJob{};
  if (carry) carry->R = 0;
  // one workgroup per column and per 256 entries of the longer part (one per
  // column for FP16, whose scaling needs the column maximum)
  const int64_t longest = p.Pf > p.Ps ? p.Pf : p.Ps;
  int64_t chunks = (longest + 255) / 256;
  if (chunks > 64) chunks = 64;
  const unsigned gy = xdt == NNCP_F16 ? 1 : (unsigned)chunks;
  dim3 grid(p.Rpad + (gram_blocks(job) + gy - 1) / gy, gy), block(256);
  switch (xdt) {
    case NNCP_BF16:
      hipLaunchKernelGGL((k_krp_operands<bf16_t, float>), grid, block, 0, st, a, (bf16_t *)kfast, (float *)kslow, job);
      break;
    case NNCP_F16:
      a.scale16 = 1;
      hipLaunchKernelGGL((k_krp_operands<f16_t, float>), grid, block, 0, st, a, (f16_t *)kfast, (float *)kslow, job);
      break;
    case NNCP_F32:
      hipLaunchKernelGGL((k_krp_operands<float, float>), grid, block, 0, st, a, (float *)kfast, (float *)kslow, job);
      break;
    case NNCP_F64:
      hipLaunchKernelGGL((k_krp_operands<double, double>), grid, block, 0, st, a, (double *)kfast, (double *)kslow, job);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_krp_operands2(int xdt, const GemmPlan &p0, void *kf0, void *ks0,
                                const GemmPlan &p1, void *kf1, void *ks1, int R,
                                const int64_t *dims, int N, const FactorSet &F, hipStream_t st) {
  if (xdt == NNCP_F16) return hipErrorInvalidValue;
  const KrpArgs a0 = make_krp_args(p0, R, dims, F, N), a1 = make_krp_args(p1, R, dims, F, N);
  const int64_t longest = std::max(std::max(p0.Pf, p0.Ps), std::max(p1.Pf, p1.Ps));
  int64_t chunks = (longest + 255) / 256;
  if (chunks > 64) chunks = 64;
  const dim3 grid((unsigned)(p0.Rpad + p1.Rpad), (unsigned)chunks), block(256);
  switch (xdt) {
    case NNCP_BF16:
      hipLaunchKernelGGL((k_krp_operands2<bf16_t, float>), grid, block, 0, st, a0, (bf16_t *)kf0,
                         (float *)ks0, a1, (bf16_t *)kf1, (float *)ks1);
      break;
    case NNCP_F32:
      hipLaunchKernelGGL((k_krp_operands2<float, float>), grid, block, 0, st, a0, (float *)kf0,
                         (float *)ks0, a1, (float *)kf1, (float *)ks1);
      break;
    case NNCP_F64:
      hipLaunchKernelGGL((k_krp_operands2<double, double>), grid, block, 0, st, a0, (double *)kf0,
                         (double *)ks0, a1, (double *)kf1, (double *)ks1);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The operand of plan p: the factors themselves when p.direct, else the
// precomputed kf / ks.
template <typename XT>
static KOp<XT> make_kop(const GemmPlan &p, int R, const FactorSet &F, const void *kf,
                        const void *ks) {
  typedef typename XTraits<XT>::AT AT;
  KOp<XT> ko;
  if (p.direct) {
    ko.kfast = nullptr;
    ko.hf = (const AT *)F.H[p.fast_lo];
    ko.kslow = p.slow_hi > p.slow_lo ? (const AT *)F.H[p.slow_lo] : nullptr;
    ko.ldks = R;
  } else {
    ko.kfast = (const XT *)kf;
    ko.hf = nullptr;
    ko.kslow = (const AT *)ks;
    ko.ldks = p.Rpad;
  }
  return ko;
}

// grid of a product that carries a split Gram step: its workgroups come
// after the product's in dispatch order (extra columns when nsplit is 1,
// else extra rows), so that they never hold a CU a product workgroup waits for
static dim3 carry_grid(const GemmPlan &p, const GramJob &job) {
  const int gb = job.R ? job.parts : 0;
  if (p.nsplit == 1) return dim3((unsigned)(p.tiles + gb), 1);
  return dim3((unsigned)p.tiles, (unsigned)(p.nsplit + (gb + p.tiles - 1) / p.tiles));
}

template <typename XT, int MT, int NT, bool HL, bool SLOW>
static void run_right(const GemmPlan &p, int R, const void *X, const KOp<XT> &ko, void *out,
                      const GramJob &job, hipStream_t st) {
  typedef typename XTraits<XT>::AT AT;
  constexpr int KSTEP = 4 * XTraits<XT>::VEC;
  dim3 grid = carry_grid(p, job), block(64 * kRightWaves);
  // the waves take contiguous ranges (batches dealt in turn measured 1.5%
  // faster at 512^3 BF16 but 3% slower on the 256^4 tensor)
  constexpr bool ILV = false;
  hipLaunchKernelGGL((k_gemm_right_mfma<XT, MT, NT, HL, SLOW, 4, ILV>), grid, block, p.lds_bytes,
                     st, (const XT *)X, p.m, p.k, ko, (int)p.Pf, (p.m / KSTEP), p.nsplit, R,
                     (AT *)out, (int)p.tiles, job);
}

template <typename XT, int QV, int NT, bool HL, bool SLOW>
static void run_left(const GemmPlan &p, int R, const void *X, const KOp<XT> &ko, void *out,
                     const GramJob &job, hipStream_t st) {
  typedef typename XTraits<XT>::AT AT;
  constexpr int KSTEP = 4 * XTraits<XT>::KL;
  dim3 grid = carry_grid(p, job), block(64 * left_waves(sizeof(XT), QV, NT, SLOW));
  if (p.nt_loads)
    hipLaunchKernelGGL((k_gemm_left_mfma<XT, QV, NT, HL, SLOW, true>), grid, block, p.lds_bytes, st,
                       (const XT *)X, p.m, p.k, ko, (int)p.Pf, (int)p.W, (p.k / KSTEP), p.nsplit,
                       R, (AT *)out, (int)p.tiles, job);
  else
    hipLaunchKernelGGL((k_gemm_left_mfma<XT, QV, NT, HL, SLOW, false>), grid, block, p.lds_bytes, st,
                       (const XT *)X, p.m, p.k, ko, (int)p.Pf, (int)p.W, (p.k / KSTEP), p.nsplit,
                       R, (AT *)out, (int)p.tiles, job);
}

// NT dispatch (1..4) with the template flags fixed
#define NNCP_NT_SWITCH(NTV, CALL) \
  switch (NTV) {                  \
    case 1: { constexpr int NTC = 1; CALL; } break; \
    case 2: { constexpr int NTC = 2; CALL; } break; \
    case 3: { constexpr int NTC = 3; CALL; } break; \
    case 4: { constexpr int NTC = 4; CALL; } break; \
    default: return hipErrorInvalidValue;           \
  }
// the same for NT in 1..2 only
#define NNCP_NT_SWITCH12(NTV, CALL) \
  switch (NTV) {                    \
    case 1: { constexpr int NTC = 1; CALL; } break; \
    case 2: { constexpr int NTC = 2; CALL; } break; \
    default: return hipErrorInvalidValue;           \
  }

template <typename XT>
static hipError_t dispatch_mfma(const GemmPlan &p, int R, const void *X, const FactorSet &F,
                                const void *kf, const void *ks, void *out, const GramJob &job,
                                hipStream_t st) {
  constexpr bool IS16 = sizeof(XT) == 2;
  const KOp<XT> ko = make_kop<XT>(p, R, F, kf, ks);
  const bool slow = p.Ps > 1;
  if (p.side == 1) {
    constexpr int MT = sizeof(XT) == 8 ? 1 : 2;
    if (IS16 && p.hl) {
      if (slow) { NNCP_NT_SWITCH(p.NT, (run_right<XT, MT, NTC, IS16, true>(p, R, X, ko, out, job, st))) }
      else { NNCP_NT_SWITCH(p.NT, (run_right<XT, MT, NTC, IS16, false>(p, R, X, ko, out, job, st))) }
    } else {
      if (slow) { NNCP_NT_SWITCH(p.NT, (run_right<XT, MT, NTC, false, true>(p, R, X, ko, out, job, st))) }
      else { NNCP_NT_SWITCH(p.NT, (run_right<XT, MT, NTC, false, false>(p, R, X, ko, out, job, st))) }
    }
  } else {
    // columns per lane: 8 (16 B) for 16-bit types up to 32 columns of R, else 4
    if constexpr (IS16) {
      if (p.NT <= 2) {
        if (p.hl) {
          if (slow) { NNCP_NT_SWITCH12(p.NT, (run_left<XT, 8, NTC, IS16, true>(p, R, X, ko, out, job, st))) }
          else { NNCP_NT_SWITCH12(p.NT, (run_left<XT, 8, NTC, IS16, false>(p, R, X, ko, out, job, st))) }
        } else {
          if (slow) { NNCP_NT_SWITCH12(p.NT, (run_left<XT, 8, NTC, false, true>(p, R, X, ko, out, job, st))) }
          else { NNCP_NT_SWITCH12(p.NT, (run_left<XT, 8, NTC, false, false>(p, R, X, ko, out, job, st))) }
        }
      } else {
        if (p.hl) {
          if (slow) { NNCP_NT_SWITCH(p.NT, (run_left<XT, 4, NTC, IS16, true>(p, R, X, ko, out, job, st))) }
          else { NNCP_NT_SWITCH(p.NT, (run_left<XT, 4, NTC, IS16, false>(p, R, X, ko, out, job, st))) }
        } else {
          if (slow) { NNCP_NT_SWITCH(p.NT, (run_left<XT, 4, NTC, false, true>(p, R, X, ko, out, job, st))) }
          else { NNCP_NT_SWITCH(p.NT, (run_left<XT, 4, NTC, false, false>(p, R, X, ko, out, job, st))) }
        }
      }
    } else {
      constexpr int QV = 16 / sizeof(XT);
      if (slow) { NNCP_NT_SWITCH(p.NT, (run_left<XT, QV, NTC, false, true>(p, R, X, ko, out, job, st))) }
      else { NNCP_NT_SWITCH(p.NT, (run_left<XT, QV, NTC, false, false>(p, R, X, ko, out, job, st))) }
    }
  }
  return hipGetLastError();
}

template <typename XT, typename HT>
static hipError_t dispatch_generic(const GemmPlan &p, int R, const void *X, const int64_t *dims,
                                   int N, int S, const FactorSet &F, void *out, hipStream_t st) {
  GenArgs a;
  for (int n = 0; n < NNCP_MAX_MODES; ++n) {
    a.H[n] = n < N ? F.H[n] : nullptr;
    a.dims[n] = n < N ? dims[n] : 1;
  }
  a.R = R; a.m = p.m; a.k = p.k; a.nsplit = p.nsplit;
  if (p.side == 1) {
    a.red_lo = 0; a.red_hi = S;
    hipLaunchKernelGGL((k_gemm_right_generic<XT, HT>), dim3((unsigned)p.k, p.nsplit), dim3(256), 0, st,
                       (const XT *)X, a, (HT *)out);
  } else {
    a.red_lo = S; a.red_hi = N;
    hipLaunchKernelGGL((k_gemm_left_generic<XT, HT>), dim3((unsigned)((p.m + 255) / 256), p.nsplit),
                       dim3(256), 0, st, (const XT *)X, a, (HT *)out);
  }
  return hipGetLastError();
}

hipError_t launch_partial_mttkrp(int xdt, const GemmPlan &p, int R, const void *X,
                                 const int64_t *dims, int N, int S, const FactorSet &F,
                                 const void *kfast, const void *kslow, void *out,
                                 hipStream_t st, GramJob *carry) {
  if (p.mfma) {
    const GramJob job = carry ? *carry : GramJob{};
    // only a split Gram step rides along (its workgroups are light)
    if (job.R && job.parts == 0) return hipErrorInvalidValue;
    if (carry) carry->R = 0;
    if (p.direct && xdt == NNCP_F16) return hipErrorInvalidValue;  // needs the column scaling
    switch (xdt) {
      case NNCP_BF16: return dispatch_mfma<bf16_t>(p, R, X, F, kfast, kslow, out, job, st);
      case NNCP_F16: return dispatch_mfma<f16_t>(p, R, X, F, kfast, kslow, out, job, st);
      case NNCP_F32: return dispatch_mfma<float>(p, R, X, F, kfast, kslow, out, job, st);
      case NNCP_F64: return dispatch_mfma<double>(p, R, X, F, kfast, kslow, out, job, st);
    }
    return hipErrorInvalidValue;
  }
  if (carry && carry->R) return hipErrorInvalidValue;  // the caller runs it first
  switch (xdt) {
    case NNCP_BF16: return dispatch_generic<bf16_t, float>(p, R, X, dims, N, S, F, out, st);
    case NNCP_F16: return dispatch_generic<f16_t, float>(p, R, X, dims, N, S, F, out, st);
    case NNCP_F32: return dispatch_generic<float, float>(p, R, X, dims, N, S, F, out, st);
    case NNCP_F64: return dispatch_generic<double, double>(p, R, X, dims, N, S, F, out, st);
  }
  return hipErrorInvalidValue;
}

size_t dual_lds_bytes(int NT, int hl, int64_t PfL) {
  const int RP = 16 * NT;
  const int64_t ldl = ((PfL / 8) % 16 == 0) ? PfL : PfL + 8;
  const size_t main = (size_t)(hl ? 2 : 1) * RP * kDualWin * 2 + (size_t)(hl ? 2 : 1) * RP * ldl * 2 +
                      (size_t)kDualWaves * 32 * 128 * 2 + (size_t)2 * kDualWaves * 64 * 8 * NT * 4;
  const size_t epi = (size_t)kDualWaves * 16 * (16 * 8 + 4) * 4;
  return main > epi ? main : epi;
}

int64_t dual_tiles(int64_t m) { return (m + 128 * kDualWaves - 1) / (128 * kDualWaves); }

hipError_t launch_dual_mttkrp(int xdt, const GemmPlan &pl, const GemmPlan &pr, int R,
                              const void *X, const void *kfr, const void *kfl, const void *ksl,
                              void *out_l, void *out_r, int r_major, hipStream_t st) {
  if (xdt != NNCP_BF16 || pl.NT > 2 || pl.k % 32 != 0) return hipErrorInvalidValue;
  DualArgs a;
  a.m = pl.m;
  a.k = pl.k;
  a.PfL = (int)pr.Pf;
  a.R = R;
  a.rmaj = r_major ? 1 : 0;
  const size_t lds = dual_lds_bytes(pl.NT, pl.hl, pr.Pf);
  dim3 grid((unsigned)dual_tiles(pl.m)), block(64 * kDualWaves);
#define NNCP_DUAL(NTV, HLV, NTLV)                                                                 \
  hipLaunchKernelGGL((k_gemm_dual_mfma<bf16_t, NTV, HLV, NTLV>), grid, block, lds, st,          \
                     (const bf16_t *)X, a, (const bf16_t *)kfr, (const bf16_t *)kfl,             \
                     (const float *)ksl,                                                          \
                     (float *)out_l, (float *)out_r)
  const bool ntl = pl.nt_loads != 0;
  if (pl.NT == 1) {
    if (pl.hl) { if (ntl) NNCP_DUAL(1, true, true); else NNCP_DUAL(1, true, false); }
    else { if (ntl) NNCP_DUAL(1, false, true); else NNCP_DUAL(1, false, false); }
  } else {
    if (pl.hl) { if (ntl) NNCP_DUAL(2, true, true); else NNCP_DUAL(2, true, false); }
    else { if (ntl) NNCP_DUAL(2, false, true); else NNCP_DUAL(2, false, false); }
  }
#undef NNCP_DUAL
  return hipGetLastError();
}

hipError_t launch_finalize(int hdt, const GemmPlan &p, int R, const void *part, void *out,
                           int leaf, hipStream_t st, int part_rmajor) {
  const int64_t rows = p.side == 1 ? p.k : p.m;
  const int rmajor = part_rmajor >= 0 ? part_rmajor : p.side == 0;
  const int64_t n = rows * R;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (hdt == NNCP_F64)
    hipLaunchKernelGGL((k_finalize<double>), grid, block, 0, st, (const double *)part, rows, R,
                       p.nsplit, rmajor, leaf, (double *)out);
  else
    hipLaunchKernelGGL((k_finalize<float>), grid, block, 0, st, (const float *)part, rows, R,
                       p.nsplit, rmajor, leaf, (float *)out);
  return hipGetLastError();
}

}  // namespace nncp
