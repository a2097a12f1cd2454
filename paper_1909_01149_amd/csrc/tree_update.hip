// Dimension-tree multi-TTVs (Section 4.2, Algorithm 3 multi-TTV lines), Gram
// and Hadamard products (Algorithm 1), the per-mode factor update with
// column normalisation and the relative-error identity (Eqs. eqn:muupd,
// eqn:halsupd; Appendix B, Algorithm 4), the loss, the gradient of the loss
// and the projected-gradient helpers.
//
// Node layout (as in the paper's Figure 3): a node T over modes a..b is
// I_a x ... x I_b x R with column block r contiguous: entry (i_a, .., i_b, r)
// at r * P + i_a + I_a (i_{a+1} + ...), P = I_a ... I_b.
// Factors and M are I x R row-major.  Every reduction is done in a fixed order
// (no atomics), so results are bitwise reproducible run to run.
#include <type_traits>

#include "nncp_internal.h"

namespace nncp {

template <typename T> __device__ __forceinline__ double to_dd(T v) { return (double)v; }
template <> __device__ __forceinline__ double to_dd<bf16_t>(bf16_t v) { return (double)(float)v; }
template <> __device__ __forceinline__ double to_dd<f16_t>(f16_t v) { return (double)(float)v; }


// sum_{s < ns} p[s * stride] added in order s = 0, 1, ...; the loads are
// issued eight at a time so they overlap
template <typename HT>
__device__ __forceinline__ HT ordered_split_sum(const HT *__restrict__ p, int ns, int64_t stride) {
  HT acc = p[0];
  int sp = 1;
  for (; sp + 8 <= ns; sp += 8) {
    HT v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(sp + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; sp < ns; ++sp) acc += p[(int64_t)sp * stride];
  return acc;
}

// Same sum with every load issued before the first add when ns <= 32.
template <typename HT>
__device__ __forceinline__ HT ordered_split_sum_wide(const HT *__restrict__ p, int ns, int64_t stride) {
  if (ns > 32) return ordered_split_sum(p, ns, stride);
  HT v[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) v[k] = k < ns ? p[(int64_t)k * stride] : (HT)0;
  HT acc = v[0];
#pragma unroll
  for (int k = 1; k < 32; ++k)
    if (k < ns) acc += v[k];
  return acc;
}

// sum over the 64 lanes of a wave, fixed butterfly order
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// multi-TTV, contiguous reduction: out(q, r) = sum_i T[r][i + Ia q] H(i, r)
// G lanes per output (G = power of two <= 64), outputs ordered (r, q).
// ---------------------------------------------------------------------------
template <typename HT>
__global__ __launch_bounds__(256) void k_mttv_contig(const HT *__restrict__ T, int64_t Ia, int64_t Q,
                                                     int R, const HT *__restrict__ H,
                                                     HT *__restrict__ out, int leaf, int G) {
  const int64_t gt = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t o = gt / G;
  const int sub = (int)(gt % G);
  const int64_t total = Q * R;
  const bool live = o < total;
  const int64_t r = live ? o / Q : 0, q = live ? o % Q : 0;
  HT acc = 0;
  if (live) {
    const HT *t = T + r * (Ia * Q) + Ia * q;
    for (int64_t i = sub; i < Ia; i += G) acc += t[i] * H[i * R + r];
  }
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (live && sub == 0) {
    if (leaf) out[q * R + r] = acc;
    else out[r * Q + q] = acc;
  }
}

// Same reduction for 64 <= Ia <= 8192 with Ia % 4 == 0: a workgroup owns one
// column r (H(:, r) staged in LDS once) and a range of q; one wave per output,
// lanes stream T[r][Ia q ..] with 16-byte loads.
template <typename HT>
__global__ __launch_bounds__(256) void k_mttv_contig_wide(const HT *__restrict__ T, int64_t Ia,
                                                          int64_t Q, int R, const HT *__restrict__ H,
                                                          HT *__restrict__ out, int leaf,
                                                          int64_t qper) {
  __shared__ HT hs[8192];
  constexpr int V = 16 / (int)sizeof(HT);
  typedef HT vt __attribute__((ext_vector_type(V)));
  const int r = blockIdx.x;
  for (int64_t i = threadIdx.x; i < Ia; i += 256) hs[i] = H[i * R + r];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q0 = (int64_t)blockIdx.y * qper;
  const int64_t q1 = q0 + qper < Q ? q0 + qper : Q;
  const HT *Tr = T + (int64_t)r * Ia * Q;
  for (int64_t q = q0 + wave; q < q1; q += 4) {
    const vt *t = reinterpret_cast<const vt *>(Tr + Ia * q);
    HT acc = 0;
    for (int64_t c = lane; c < Ia / V; c += 64) {
      const vt x = t[c];
#pragma unroll
      for (int e = 0; e < V; ++e) acc += x[e] * hs[c * V + e];
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      if (leaf) out[q * R + r] = acc;
      else out[(int64_t)r * Q + q] = acc;
    }
  }
}

// Same reduction for Ia % V == 0 and Ia <= 64 V CPL: a wave owns QB = 8 / CPL
// outputs (q, r).  Each lane issues its loads of the QB rows of T first, the
// workgroup then stages H(:, r) in LDS, and the products are added in the
// order of the kernel above; a workgroup costs one memory round trip.
template <typename HT, int CPL>
__global__ __launch_bounds__(256) void k_mttv_contig_reg(const HT *__restrict__ T, int64_t Ia,
                                                         int64_t Q, int R, const HT *__restrict__ H,
                                                         HT *__restrict__ out, int leaf,
                                                         GramJob job) {
  constexpr int V = 16 / (int)sizeof(HT);
  constexpr int QB = 8 / CPL;
  typedef HT vt __attribute__((ext_vector_type(V)));
  __shared__ vt hs[64 * CPL];
  // extra columns of workgroups when carrying the Gram step
  if (job.R && blockIdx.x >= R) {
    gram_run(job, (blockIdx.x - R) * gridDim.y + blockIdx.y);
    return;
  }
  const int r = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t qb = ((int64_t)blockIdx.y * 4 + wave) * QB;
  const int64_t nv = Ia / V;
  const HT *Tr = T + (int64_t)r * Ia * Q;
  vt x[QB][CPL];
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    const int64_t q = qb + j < Q ? qb + j : Q - 1;
    const vt *t = reinterpret_cast<const vt *>(Tr + Ia * q);
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int64_t cv = lane + 64 * u;
      x[j][u] = t[cv < nv ? cv : 0];
    }
  }
  HT *hsf = reinterpret_cast<HT *>(hs);
  for (int64_t i = threadIdx.x; i < Ia; i += 256) hsf[i] = H[i * R + r];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    HT acc = 0;
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      if (lane + 64 * u < nv) {
        const vt hv = hs[lane + 64 * u];
#pragma unroll
        for (int e = 0; e < V; ++e) acc += x[j][u][e] * hv[e];
      }
    acc = wave_sum(acc);
    const int64_t q = qb + j;
    if (lane == 0 && q < Q) {
      if (leaf) out[q * R + r] = acc;
      else out[(int64_t)r * Q + q] = acc;
    }
  }
}

// Same reduction for Ia = GL V with GL < 64 a power of two: GL lanes per
// output, so that a wave's load takes 64 / GL whole consecutive rows of T
// (1 KB) instead of one row on GL of its 64 lanes; eight such loads per
// lane are issued first.  The pieces of an output are added by a butterfly
// over its GL lanes, which is the wave-wide butterfly of the kernel above
// with the stages that only add the idle lanes' zeros left out.
template <typename HT, int GL>
__device__ __forceinline__ void contig_pack_block(const HT *__restrict__ T, int64_t Ia, int64_t Q,
                                                  int R, const HT *__restrict__ H,
                                                  HT *__restrict__ out, int leaf, int r, int by,
                                                  HT *hs_lds) {
  constexpr int V = 16 / (int)sizeof(HT);
  constexpr int OPL = 64 / GL;  // outputs per load of a wave
  constexpr int NL = 8;         // loads per lane
  typedef HT vt __attribute__((ext_vector_type(V)));
  vt *hs = reinterpret_cast<vt *>(hs_lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / GL, sub = lane % GL;
  const int64_t qw = ((int64_t)by * 4 + wave) * (OPL * NL);
  const HT *Tr = T + (int64_t)r * Ia * Q;
  vt x[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int64_t q = qw + u * OPL + grp;
    x[u] = reinterpret_cast<const vt *>(Tr + Ia * (q < Q ? q : Q - 1))[sub];
  }
  for (int64_t i = threadIdx.x; i < Ia; i += 256) hs_lds[i] = H[i * R + r];
  __syncthreads();
  const vt hv = hs[sub];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    HT acc = 0;
#pragma unroll
    for (int e = 0; e < V; ++e) acc += x[u][e] * hv[e];
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    const int64_t q = qw + u * OPL + grp;
    if (sub == 0 && q < Q) {
      if (leaf) out[q * R + r] = acc;
      else out[(int64_t)r * Q + q] = acc;
    }
  }
}

template <typename HT, int GL>
__global__ __launch_bounds__(256) void k_mttv_contig_pack(const HT *__restrict__ T, int64_t Ia,
                                                          int64_t Q, int R,
                                                          const HT *__restrict__ H,
                                                          HT *__restrict__ out, int leaf,
                                                          GramJob job) {
  constexpr int V = 16 / (int)sizeof(HT);
  __shared__ __align__(16) HT hs[GL * V];
  // extra columns of workgroups when carrying the Gram step
  if (job.R && blockIdx.x >= R) {
    gram_run(job, (blockIdx.x - R) * gridDim.y + blockIdx.y);
    return;
  }
  contig_pack_block<HT, GL>(T, Ia, Q, R, H, out, leaf, blockIdx.x, blockIdx.y, hs);
}

// ---------------------------------------------------------------------------
// multi-TTV, strided reduction keeping the first mode:
//   part[z][i][r] = sum_{q in split z} T[r][i + Ia q] K(q, r),
//   K(q, r) = prod_k H^(k)(digit_k(q), r) over the node's remaining modes.
// Block = IT columns i x QS q-lanes; q-lanes added in order through LDS.
// ---------------------------------------------------------------------------
template <typename HT, int V>
__device__ __forceinline__ void strided_block(const HT *__restrict__ T, const StridedArgs &a,
                                              HT *__restrict__ part, int bx, int r, int64_t z,
                                              HT *red_lds, HT *kq) {
  typedef HT vt __attribute__((ext_vector_type(V)));
  vt *red = reinterpret_cast<vt *>(red_lds);
  const int il = threadIdx.x % a.IT, qs = threadIdx.x / a.IT;
  const int64_t i0 = ((int64_t)bx * a.IT + il) * V;
  const bool live = i0 < a.Ia;
  const int64_t q0 = a.Q * z / a.nsplit, q1 = a.Q * (z + 1) / a.nsplit;
  const HT *const *H = (const HT *const *)a.H;
  const HT *t = T + (int64_t)r * a.Ia * a.Q + (live ? i0 : 0);
  const int64_t Ia = a.Ia;
  const int QS = a.QS;
  vt acc = (vt)0;
  for (int64_t c0 = q0; c0 < q1; c0 += 1024) {
    const int cn = (int)(q1 - c0 < 1024 ? q1 - c0 : 1024);
    __syncthreads();
    for (int e = threadIdx.x; e < cn; e += 256) {
      HT kv = 1;
      int64_t rem = c0 + e;
      for (int n = 0; n < a.nq; ++n) {
        const int64_t d = rem % a.qd[n];
        rem /= a.qd[n];
        kv *= H[n][d * a.R + r];
      }
      kq[e] = kv;
    }
    __syncthreads();
    if (live) {
      // eight rows of T in flight, then their products in q order
      int e = qs;
      for (; e + 7 * QS < cn; e += 8 * QS) {
        vt x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = *reinterpret_cast<const vt *>(t + Ia * (c0 + e + u * QS));
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += x[u] * kq[e + u * QS];
      }
      for (; e < cn; e += QS) acc += *reinterpret_cast<const vt *>(t + Ia * (c0 + e)) * kq[e];
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (qs == 0 && live) {
    vt sum = red[il];
    for (int k = 1; k < QS; ++k) sum += red[k * a.IT + il];
#pragma unroll
    for (int v = 0; v < V; ++v) part[(z * Ia + i0 + v) * a.R + r] = sum[v];
  }
}

template <typename HT, int V>
__global__ __launch_bounds__(256) void k_mttv_strided(const HT *__restrict__ T, StridedArgs a,
                                                      HT *__restrict__ part, GramJob job) {
  __shared__ __align__(16) HT red[256 * V];
  __shared__ HT kq[1024];
  // extra rows of workgroups (blockIdx.y >= R) when carrying the Gram step
  if (job.R && blockIdx.y >= a.R) {
    gram_run(job, ((blockIdx.y - a.R) * gridDim.z + blockIdx.z) * gridDim.x + blockIdx.x);
    return;
  }
  strided_block<HT, V>(T, a, part, blockIdx.x, blockIdx.y, blockIdx.z, red, kq);
}

// ---------------------------------------------------------------------------
// Several independent multi-TTVs of the kinds above in one launch (the
// gradient's walks, where every M^(n) is taken at the same factors): job k
// owns workgroups start[k] .. start[k+1]-1, numbered as its own launch
// would number them (strided: x fastest, then r, then the split; contiguous:
// r fastest, then the q-block).
// ---------------------------------------------------------------------------
constexpr int kMttvGroupMax = 4;
struct MttvGroup {
  MttvJob j[kMttvGroupMax];
  int64_t start[kMttvGroupMax + 1];
  int n;
};

template <typename HT, int V, int GL>
__global__ __launch_bounds__(256) void k_mttv_group(MttvGroup g) {
  constexpr int VC = 16 / (int)sizeof(HT);
  __shared__ __align__(16) HT red[256 * V];
  __shared__ HT kq[1024];
  __shared__ __align__(16) HT hs[GL * VC];
  const int64_t b = blockIdx.x;
  int k = 0;
#pragma unroll
  for (int q = 1; q < kMttvGroupMax; ++q)
    if (q < g.n && b >= g.start[q]) k = q;
  const MttvJob &j = g.j[k];
  const int64_t lb = b - g.start[k];
  if (j.kind == 0) {
    const int64_t bx = lb % j.gx, rest = lb / j.gx;
    strided_block<HT, V>((const HT *)j.T, j.sa, (HT *)j.out, (int)bx, (int)(rest % j.R),
                         rest / j.R, red, kq);
  } else {
    contig_pack_block<HT, GL>((const HT *)j.T, j.Ia, j.Q, j.R, (const HT *)j.H, (HT *)j.out, j.leaf,
                              (int)(lb % j.R), (int)(lb / j.R), hs);
  }
}

template <typename HT>
__global__ __launch_bounds__(256) void k_sum_splits(const HT *__restrict__ part, int64_t n, int ns,
                                                    HT *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  out[e] = ordered_split_sum(part + e, ns, n);
}


// acc + sum over rows i = s, s+ns, ... < rows of chunk[i][x] * chunk[i][y], in
// row order; eight rows' operands are read before their products are added
__device__ __forceinline__ double gram_rows(const double *chunk, int R, int x, int y, int s,
                                            int rows, int ns, double acc) {
  int i = s;
  for (; i + 7 * ns < rows; i += 8 * ns) {
    double u[8], w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      u[k] = chunk[(i + k * ns) * R + x];
      w[k] = chunk[(i + k * ns) * R + y];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += u[k] * w[k];
  }
  for (; i < rows; i += ns) acc += chunk[i * R + x] * chunk[i * R + y];
  return acc;
}

// ---------------------------------------------------------------------------
// Gram G = H^T H, FP64, one workgroup of 1024 threads.  Rows are staged in LDS
// in chunks of CH rows (coalesced loads, converted to FP64 once); thread
// (pair p, slice s) accumulates the chunk rows i = s (mod ns) from LDS; the
// slices are added in order at the end.
// ---------------------------------------------------------------------------
template <typename HT>
__device__ void gram_block(const HT *__restrict__ H, int64_t I, int R, double *__restrict__ G,
                           double *lds /* >= 1024 doubles */, double *chunk /* >= 4096 doubles */) {
  const int npairs = R * (R + 1) / 2;
  int ns = 1;
  while (ns * 2 * npairs <= 1024) ns *= 2;
  const int per_round = 1024 / ns;
  const int CH = 4096 / R;  // rows per LDS chunk
  for (int base = 0; base < npairs; base += per_round) {
    const int pl = threadIdx.x / ns, s = threadIdx.x % ns;
    const int p = base + pl;
    const bool live = pl < per_round && p < npairs;
    int a = 0, b = 0;
    if (live) {
      int rem = p;
      while (rem >= R - a) { rem -= R - a; ++a; }
      b = a + rem;
    }
    double acc = 0.0;
    for (int64_t i0 = 0; i0 < I; i0 += CH) {
      const int rows = (int)(I - i0 < CH ? I - i0 : CH);
      __syncthreads();
      {
        const int ne = rows * R;
        int e = threadIdx.x;
        for (; e + 3 * 1024 < ne; e += 4 * 1024) {
          HT v0 = H[i0 * R + e], v1 = H[i0 * R + e + 1024], v2 = H[i0 * R + e + 2048],
             v3 = H[i0 * R + e + 3072];
          chunk[e] = (double)v0;
          chunk[e + 1024] = (double)v1;
          chunk[e + 2048] = (double)v2;
          chunk[e + 3072] = (double)v3;
        }
        for (; e < ne; e += 1024) chunk[e] = (double)H[i0 * R + e];
      }
      __syncthreads();
      if (live) acc = gram_rows(chunk, R, a, b, s, rows, ns, acc);
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    if (s == 0 && live) {
      double v = lds[threadIdx.x];
      for (int k = 1; k < ns; ++k) v += lds[threadIdx.x + k];
      G[a * R + b] = v;
      G[b * R + a] = v;
    }
    __syncthreads();
  }
}

template <typename HT>
__global__ __launch_bounds__(1024) void k_gram(const HT *__restrict__ H, int64_t I, int R,
                                               double *__restrict__ G) {
  __shared__ double lds[1024];
  __shared__ double chunk[4096];
  gram_block<HT>(H, I, R, G, lds, chunk);
}

__global__ __launch_bounds__(256) void k_hadamard(const double *__restrict__ G, int N, int R,
                                                  int mode, double *__restrict__ S) {
  for (int e = threadIdx.x; e < R * R; e += 256) {
    double s = 1.0;
    for (int k = 0; k < N; ++k)
      if (k != mode) s *= G[(int64_t)k * R * R + e];
    S[e] = s;
  }
}

// ---------------------------------------------------------------------------
// ||X||^2: grid-stride FP64 partial sums, then one block adds them in order
// ---------------------------------------------------------------------------
template <typename XT>
__global__ __launch_bounds__(256) void k_sumsq_part(const XT *__restrict__ X, int64_t n,
                                                    double *__restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += stride) {
    const double v = to_dd<XT>(X[e]);
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_final(const double *__restrict__ part, int np,
                                                   double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int e = threadIdx.x; e < np; e += 256) acc += part[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// per-mode update, in two launches:
//   k_update_rows    (one workgroup per 4*rpw rows): Hhat = H diag(lambda);
//                    MU or HALS on each row; Hhat (FP64) stored; per-workgroup
//                    column sums of squares and <M, Hhat> partials
//   k_update_finish  (one workgroup): lambda = column norms (partials added in
//                    workgroup order); H = Hhat / lambda; G^(mode) = H^T H;
//                    after the last mode beta, gamma and the relative error.
// A row of Hhat is held by LPR lanes (LPR = power of two >= R, at most 64),
// lane `sub` owning columns sub + LPR u, u < CPL.  HALS keeps the residual
// g = M - Hhat S of the row and, column by column in order, broadcasts the
// change of column r from its owner lane and updates g; this is the same
// arithmetic as forming (Hhat S)(:, r) afresh from the latest Hhat.
// ---------------------------------------------------------------------------
int update_rows_per_block(int R) { (void)R; return 4; }

__device__ __forceinline__ double bcast(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One row per wave, R > 64: lane c owns columns c + 64 u (u < CPL); S is
// read from global memory (L2-resident).
template <typename HT, int CPL>
__global__ __launch_bounds__(256) void k_update_rows(UpdateArgs a) {
  __shared__ double hrow[4][256];
  __shared__ double wred[4][256];
  __shared__ double bred[4];
  __shared__ double sdiag[256];
  const int R = a.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const HT *M = (const HT *)a.M;
  const HT *H = (const HT *)a.H;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  const bool live = i < a.I;
  // every global load is issued before its first use: lambda, the row of H
  // and the row of M
  double hraw[CPL], lamv[CPL];
  HT mraw[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int c = lane + 64 * u;
    const bool ok = live && c < R;
    hraw[u] = ok ? (double)H[i * R + c] : 0.0;
    lamv[u] = c < R ? a.lambda[c] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int c = lane + 64 * u;
    mraw[u] = (live && c < R) ? ordered_split_sum_wide(M + i * R + c, a.msplit, a.mstride) : (HT)0;
  }
  const double *Sg = a.S;
  auto Sv = [&](int c, int r) -> double { return Sg[c * R + r]; };
  // HALS divisors S(r, r), read once
  for (int c = threadIdx.x; c < R; c += 256) sdiag[c] = Sv(c, c);
  double h[CPL], m[CPL], g[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int c = lane + 64 * u;
    h[u] = hraw[u] * lamv[u];
    m[u] = (double)mraw[u];
    if (c < R) hrow[wave][c] = h[u];
  }
  __syncthreads();
  // g = (Hhat S)(i, :) from the row in LDS, j in order, eight j's operands
  // read before their products are added
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int c = lane + 64 * u;
    double acc = 0.0;
    if (c < R) {
      int j = 0;
      for (; j + 8 <= R; j += 8) {
        double hv[8], sv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          hv[k] = hrow[wave][j + k];
          sv[k] = Sv(j + k, c);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += hv[k] * sv[k];
      }
      for (; j < R; ++j) acc += hrow[wave][j] * Sv(j, c);
    }
    g[u] = acc;
  }
  if (a.algo == NNCP_MU) {
#pragma unroll
    for (int u = 0; u < CPL; ++u) h[u] = h[u] * m[u] / (g[u] + a.eps);
  } else {
#pragma unroll
    for (int u = 0; u < CPL; ++u) g[u] = m[u] - g[u];
    for (int r = 0; r < R; ++r) {
      const double d = sdiag[r];
      if (!(d > 0.0)) continue;
      const int ur = r >> 6, owner = r & 63;
      double hs = h[0], gs = g[0];
#pragma unroll
      for (int u = 1; u < CPL; ++u)
        if (ur == u) { hs = h[u]; gs = g[u]; }
      const double hr = bcast(hs, owner), gr = bcast(gs, owner);
      double v = hr + gr / d;
      v = v > 0.0 ? v : 0.0;
      const double delta = v - hr;
#pragma unroll
      for (int u = 0; u < CPL; ++u) {
        const int c = lane + 64 * u;
        if (c < R) g[u] -= delta * Sv(r, c);
        if (u == ur && lane == owner) h[u] = v;
      }
    }
  }
  double beta = 0.0;
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int c = lane + 64 * u;
    double sq = 0.0;
    if (live && c < R) {
      a.hhat[i * R + c] = h[u];
      sq = h[u] * h[u];
      beta += m[u] * h[u];
    }
    if (c < R) wred[wave][c] = sq;
  }
  beta = wave_sum(beta);
  if (lane == 0) bred[wave] = beta;
  __syncthreads();
  // per-workgroup partials (the 4 rows added in wave order)
  double *cpart = a.part + (int64_t)blockIdx.x * (R + 1);
  for (int c = threadIdx.x; c < R; c += 256)
    cpart[c] = wred[0][c] + wred[1][c] + wred[2][c] + wred[3][c];
  if (threadIdx.x == 0) cpart[R] = bred[0] + bred[1] + bred[2] + bred[3];
}

template <typename HT>
__device__ void finish_generic(const UpdateArgs &a, int nblocks, double (*wred)[2], double *lam_s,
                               double *lds, double *chunk) {
  const int R = a.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // column norms and beta: one wave per column, lanes over the workgroup
  // partials, then a fixed butterfly
  for (int c = wave; c <= R; c += 16) {
    double sum = 0.0;
    for (int b = lane; b < nblocks; b += 64) sum += a.part[(int64_t)b * (R + 1) + c];
    sum = wave_sum(sum);
    if (lane == 0) {
      if (c < R) lam_s[c] = sqrt(sum);
      else wred[0][0] = sum;
    }
  }
  __syncthreads();
  const double beta = wred[0][0];
  for (int c = threadIdx.x; c < R; c += 1024) a.lambda[c] = lam_s[c];
  HT *H = (HT *)a.H;
  double *Gm = a.G + (int64_t)a.mode * R * R;
  for (int64_t e = threadIdx.x; e < a.I * R; e += 1024) {
    const double l = lam_s[e % R];
    H[e] = (HT)(l > 0.0 ? a.hhat[e] / l : 0.0);
  }
  __syncthreads();
  gram_block<HT>(H, a.I, R, Gm, lds, chunk);
  __syncthreads();
  if (a.relerr_out || a.scal) {
    double gsum = 0.0;
    for (int e = threadIdx.x; e < R * R; e += 1024) {
      const int r = e / R, c = e % R;
      double sv;
      if (a.S) sv = a.S[e];
      else {
        sv = 1.0;
        for (int k = 0; k < a.N; ++k)
          if (k != a.mode) sv *= a.G[(int64_t)k * R * R + e];
      }
      gsum += lam_s[r] * sv * Gm[e] * lam_s[c];
    }
    const double v = wave_sum(gsum);
    if (lane == 0) wred[wave][1] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double gamma = 0.0;
      for (int w = 0; w < 16; ++w) gamma += wred[w][1];
      const double alpha = a.alpha ? a.alpha[0] : 0.0;
      const double e2 = (alpha - 2.0 * beta + gamma) / alpha;
      if (a.scal) {
        a.scal[0] = beta;
        a.scal[1] = gamma;
        a.scal[2] = e2;
      }
      if (a.relerr_out) a.relerr_out[0] = sqrt(e2 > 0.0 ? e2 : 0.0);
    }
  }
  if (a.S_next) {
    // S for the next mode (every Gram is current now); written after gamma
    // has used S of this mode, which may live in the same buffer
    __syncthreads();
    for (int e = threadIdx.x; e < R * R; e += 1024) {
      double v = 1.0;
      for (int q = 0; q < a.N; ++q)
        if (q != a.next_mode) v *= a.G[(int64_t)q * R * R + e];
      a.S_next[e] = v;
    }
  }
}


// Single-workgroup finish, used for R > 64.
template <typename HT>
__global__ __launch_bounds__(1024) void k_update_finish(UpdateArgs a, int nblocks) {
  __shared__ double wred[16][2];
  __shared__ double lam_s[256];
  __shared__ double lds[1024];
  __shared__ double chunk[4096];
  finish_generic<HT>(a, nblocks, wred, lam_s, lds, chunk);
}

// ---------------------------------------------------------------------------
// Row update for R <= RB <= 64: one row per wave, lane c owns column c and
// keeps column c of S in registers.  HALS (Eq. eqn:halsupd) visits the columns in
// order; at step r every lane forms its candidate, the value of lane r is
// broadcast and every lane folds the change into its entry of the gradient,
// so a step costs a few dependent instructions.  The HALS quotient uses the
// reciprocal of S(r, r) (within one rounding of the quotient).
template <typename HT, int RB, bool NES, bool FULL>
__global__ __launch_bounds__(256) void k_update_rows_small(UpdateArgs a) {
  __shared__ double wred[4][64];
  __shared__ double bred[4];
  const int R = FULL ? RB : a.R;  // FULL: R == RB, known when compiling
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const HT *M = (const HT *)a.M;
  const HT *H = (const HT *)a.H;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  const bool live = i < a.I;
  const bool own = lane < R;
  const int c = own ? lane : 0;
  const int64_t ir = live ? i : a.I - 1;
  // every load is issued before any value is used (addresses clamped into
  // range instead of branching): the split partials of M, column c of S,
  // S(c, c), lambda and the entry of H
  const int ns = a.msplit;
  const HT *mp = M + ir * R + c;
  HT mv[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) mv[k] = k < ns ? mp[(int64_t)k * a.mstride] : (HT)0;
  double sc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) sc[r] = r < R ? a.S[r * R + c] : 0.0;
  const double d_raw = a.S[c * R + c];
  const double lam_raw = a.lambda[c];
  const HT h_raw = H[ir * R + c];
  const double nes_lam = NES ? a.nesParam[2] : 0.0, nes_alpha = NES ? a.nesParam[3] : 0.0;
  const double nes_beta = NES ? a.nesParam[4] : 0.0;
  const bool nes_ok = NES && a.nesParam[5] > 0.0;
  HT macc = mv[0];
#pragma unroll
  for (int k = 1; k < 32; ++k)
    if (k < ns) macc += mv[k];
  for (int k = 32; k < ns; ++k) macc += mp[(int64_t)k * a.mstride];
  const bool ok = live && own;
  if (!own) {
#pragma unroll
    for (int r = 0; r < RB; ++r) sc[r] = 0.0;
  }
  const double d = own ? d_raw : 0.0;
  double h = ok ? (double)h_raw * lam_raw : 0.0;
  const double m = ok ? (double)macc : 0.0;
  if constexpr (NES) {
    // Nesterov-type steps (Section 4.3.5) from x* = Hhat, the gradient of
    // the proximal objective y S - m + lam (y - x*) with y S in order
    if (nes_ok) {
      const double xs = h;
      double x = h, y = h;
      for (int k = 0; k < kNesIters; ++k) {
        double gy = 0.0;
#pragma unroll
        for (int j = 0; j < RB; ++j)
          if (j < R) gy += bcast(y, j) * sc[j];
        gy = gy - m + nes_lam * (y - xs);
        const double v = y - nes_alpha * gy;
        const double xn = v > 0.0 ? v : 0.0;
        y = xn + nes_beta * (xn - x);
        x = xn;
      }
      h = x;
    }
  } else {
  // g = (Hhat S)(i, c), j in order
  double g = 0.0;
#pragma unroll
  for (int j = 0; j < RB; ++j)
    if (j < R) g += bcast(h, j) * sc[j];
  if (a.algo == NNCP_MU) {
    h = h * m / (g + a.eps);
  } else {
    g = m - g;
    const bool pos = d > 0.0;
    const double invd = pos ? 1.0 / d : 0.0;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (r < R) {
        double v = h + g * invd;
        v = v > 0.0 ? v : 0.0;
        const double dl = pos ? v - h : 0.0;
        const double delta = bcast(dl, r);
        if (lane == r && pos) h = v;
        g -= delta * sc[r];
      }
    }
  }
  }
  double sq = 0.0, beta = 0.0;
  if (live && own) {
    a.hhat[i * R + c] = h;
    sq = h * h;
    beta = m * h;
  }
  wred[wave][lane] = sq;
  beta = wave_sum(beta);
  if (lane == 0) bred[wave] = beta;
  __syncthreads();
  // per-workgroup partials (the 4 rows added in wave order)
  double *cpart = a.part + (int64_t)blockIdx.x * (R + 1);
  if (threadIdx.x < R)
    cpart[threadIdx.x] = wred[0][threadIdx.x] + wred[1][threadIdx.x] + wred[2][threadIdx.x] +
                         wred[3][threadIdx.x];
  if (threadIdx.x == 0) cpart[R] = bred[0] + bred[1] + bred[2] + bred[3];
}

// Cross-lane exchange through LDS inside one wave: a wave's LDS accesses are
// performed in order, so a compiler barrier with wavefront-scope fences is
// all that orders a write by one lane before a read by another.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Step parameters of the Nesterov-type update (Section 4.3.5), one wave, lane
// i holding row i of S: L = the largest eigenvalue of S and L - mu the
// largest of L I - S, each by kNesPower power steps from the all-ones vector
// (the vector goes through LDS for the matrix-vector product, four partial
// sums per lane; norms by a wave reduction), then
// lam = max(0, (L - kappa mu) / (kappa - 1)), alpha = 1 / (L + lam) and the
// constant momentum beta = (1 - sqrt(q)) / (1 + sqrt(q)), q = (mu + lam) /
// (L + lam).  Writes [L, mu, lam, alpha, beta, ok]; ok = 0 when L <= 0.
// ---------------------------------------------------------------------------
template <int RB>
__device__ double nes_power(const double (&sr)[RB], int R, int lane, double shift, double sgn,
                            double *vs) {
  const bool own = lane < R;
  // row `lane` of shift I + sgn S, times the vector in vs
  auto matvec = [&](double v) {
    vs[lane] = v;
    wave_sync();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < R) acc[j & 3] += ((j == lane ? shift : 0.0) + sgn * sr[j]) * vs[j];
    wave_sync();
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
  };
  double v = own ? 1.0 / sqrt((double)R) : 0.0;
  for (int t = 0; t < kNesPower; ++t) {
    const double w = matvec(v);
    const double nrm = sqrt(wave_sum(own ? w * w : 0.0));
    if (!(nrm > 0.0)) break;
    v = own ? w / nrm : 0.0;
  }
  const double sv = matvec(v);
  return wave_sum(own ? v * sv : 0.0);
}

template <int RB, bool FULL>
__global__ __launch_bounds__(64) void k_nes_prep(UpdateArgs a) {
  __shared__ double vs[64];
  const int R = FULL ? RB : a.R, lane = threadIdx.x;
  const bool own = lane < R;
  double sr[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) sr[j] = (own && j < R) ? a.S[lane * R + j] : 0.0;
  if (!own) {
#pragma unroll
    for (int j = 0; j < RB; ++j) sr[j] = 0.0;
  }
  const double L = nes_power<RB>(sr, R, lane, 0.0, 1.0, vs);
  const double lt = nes_power<RB>(sr, R, lane, L, -1.0, vs);
  double mu = L - lt;
  if (!(mu > 0.0)) mu = 0.0;
  double lam = (L - kNesKappa * mu) / (kNesKappa - 1.0);
  if (!(lam > 0.0)) lam = 0.0;
  double alpha = 0.0, beta = 0.0, ok = 0.0;
  if (L > 0.0) {
    const double q = sqrt((mu + lam) / (L + lam));
    alpha = 1.0 / (L + lam);
    beta = (1.0 - q) / (1.0 + q);
    ok = 1.0;
  }
  if (lane < 6) {
    const double vals[6] = {L, mu, lam, alpha, beta, ok};
    double v = vals[0];
#pragma unroll
    for (int k = 1; k < 6; ++k)
      if (lane == k) v = vals[k];
    a.nesParam[lane] = v;
  }
}

// BPP rows for R <= RB <= 64 (Section 4.3.3, Eq. eqn:snls): every row x of
// Hhat becomes the exact solution of min_{x >= 0} 1/2 x^T S x - m^T x, whose
// KKT conditions are x >= 0, y = S x - m >= 0, x_i y_i = 0.  One wave per row;
// lane c owns index c.  The passive set F is a ballot mask; the indices that
// break the conditions (x < 0 on F, y < 0 off F) switch sets while their
// count keeps falling, then three more full switches are allowed, then only
// the largest index switches (block principal pivoting).  The search starts
// from the support of the row's current value H diag(lambda).  Each switch solves
// S_FF x_F = m_F by a left-looking Cholesky factorisation in the wave's LDS
// (lane p owns row p of the factor) and two triangular solves, and forms
// y = S x - m off F.  The search ends when no index breaks the conditions,
// after 5 R + 10 solves, or when S_FF is not positive definite (the last x,
// clipped at 0, is kept).  All arithmetic is FP64.
template <typename HT, int RB>
__global__ __launch_bounds__(RB <= 32 ? 256 : 64) void k_update_bpp(UpdateArgs a) {
  constexpr int WPB = RB <= 32 ? 4 : 1;  // rows (waves) per workgroup
  constexpr bool S_LDS = RB <= 32;
  constexpr int LD = RB + 1;             // LDS row stride of the factor
  __shared__ double sS[S_LDS ? RB * RB : 1];
  __shared__ double sL[WPB][RB * LD];
  __shared__ double wred[WPB][64];
  __shared__ double bred[WPB];
  const int R = a.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const HT *M = (const HT *)a.M;
  const int64_t i = (int64_t)blockIdx.x * WPB + wave;
  const bool live = i < a.I;
  const bool own = lane < R;
  const int c = own ? lane : 0;
  const int64_t ir = live ? i : a.I - 1;
  // M row (split partials added in order), then S staged for the workgroup
  const int ns = a.msplit;
  const HT *mp = M + ir * R + c;
  HT mv[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) mv[k] = k < ns ? mp[(int64_t)k * a.mstride] : (HT)0;
  if constexpr (S_LDS) {
    for (int e = threadIdx.x; e < R * R; e += 64 * WPB) sS[e] = a.S[e];
  }
  HT macc = mv[0];
#pragma unroll
  for (int k = 1; k < 32; ++k)
    if (k < ns) macc += mv[k];
  for (int k = 32; k < ns; ++k) macc += mp[(int64_t)k * a.mstride];
  const double m = (live && own) ? (double)macc : 0.0;
  const double h0 = (live && own) ? (double)((const HT *)a.H)[ir * R + c] * a.lambda[c] : 0.0;
  __syncthreads();
  auto Sat = [&](int r, int q) -> double { return S_LDS ? sS[r * R + q] : a.S[r * R + q]; };
  double *L = sL[wave];

  // One solve on the passive set Fm: S_FF = L L^T (left-looking; lane p
  // owns row p of L in the wave's LDS and its diagonal in a register, column
  // k from columns 0..k-1 with eight products' operands read before they are
  // added), L z = m_F and L^T x_F = z with the pivots and the running values
  // broadcast by v_readlane, then y = S x - m off F.  The only cross-lane
  // LDS reads are of rows of L finished at an earlier step, so one wave
  // barrier per column suffices.  Returns false (leaving x and y) when S_FF
  // is not positive definite.
  auto solve = [&](bool pas, uint64_t Fm, double &x, double &y) -> bool {
    const int f = __popcll(Fm);
    const int pos = __popcll(Fm & ((1ull << lane) - 1));
    wave_sync();
    if (pas) {
      uint64_t t = Fm;
      for (int q = 0; q <= pos; ++q) {
        const int c2 = __ffsll((unsigned long long)t) - 1;
        t &= t - 1;
        L[pos * LD + q] = Sat(c, c2);
      }
    }
    double dk = 0.0;  // L(pos, pos) on the lane that owns row pos
    {
      uint64_t t = Fm;
      for (int k = 0; k < f; ++k) {
        const int lk = __ffsll((unsigned long long)t) - 1;  // lane of row k
        t &= t - 1;
        wave_sync();
        double v = 0.0;
        if (pas && pos >= k) {
          v = L[pos * LD + k];
          const double *lp = L + pos * LD, *lkr = L + k * LD;
          int j = 0;
          for (; j + 8 <= k; j += 8) {
            double u[8], w[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              u[e] = lp[j + e];
              w[e] = lkr[j + e];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) v -= u[e] * w[e];
          }
          for (; j < k; ++j) v -= lp[j] * lkr[j];
        }
        const double piv = bcast(v, lk);
        if (!(piv > 0.0)) return false;
        const double d = sqrt(piv);
        if (pas && pos == k) dk = d;
        if (pas && pos > k) L[pos * LD + k] = v / d;
      }
    }
    wave_sync();
    // L z = m_F: column by column, z_k broadcast from the lane of row k
    double b = pas ? m : 0.0, zz = 0.0;
    {
      uint64_t t = Fm;
      for (int k = 0; k < f; ++k) {
        const int lk = __ffsll((unsigned long long)t) - 1;
        t &= t - 1;
        const double zk = bcast(b, lk) / bcast(dk, lk);
        if (pas && pos == k) zz = zk;
        if (pas && pos > k) b -= L[pos * LD + k] * zk;
      }
    }
    // L^T x_F = z: rows from the last, x_k broadcast from the lane of row k
    double xr = 0.0;
    {
      // lanes of rows f-1 .. 0: the set bits of Fm from the highest
      uint64_t t = Fm;
      for (int k = f - 1; k >= 0; --k) {
        const int lk = 63 - __clzll(t);
        t &= ~(1ull << lk);
        const double xk = bcast(zz, lk) / bcast(dk, lk);
        if (pas && pos == k) xr = xk;
        if (pas && pos < k) zz -= L[k * LD + pos] * xk;
      }
    }
    x = pas ? xr : 0.0;
    double yv = 0.0;
    {
      if (own && !pas) yv = -m;
      uint64_t t = Fm;
      for (int q = 0; q < f; ++q) {
        const int lq = __ffsll((unsigned long long)t) - 1;
        t &= t - 1;
        const double xq = bcast(xr, lq);
        if (own && !pas) yv += Sat(c, lq) * xq;
      }
    }
    y = yv;
    return true;
  };

  // start from the row's current support (H diag(lambda) > 0), solved once
  bool pas = own && live && h0 > 0.0;
  double x = 0.0, y = -m;
  int ninf = R + 1, backup = 3, solves = 0;
  const int maxsolves = 5 * R + 10;
  {
    const uint64_t F0 = __ballot(pas);
    bool started = false;
    if (F0) {
      ++solves;
      started = solve(pas, F0, x, y);
    }
    if (!started) {
      pas = false;
      x = 0.0;
      y = -m;
    }
  }
  for (;;) {
    const bool bad = own && (pas ? (x < 0.0) : (y < 0.0));
    const uint64_t V = __ballot(bad);
    const int nv = __popcll(V);
    if (nv == 0 || solves >= maxsolves) break;
    bool full;
    if (nv < ninf) { ninf = nv; backup = 3; full = true; }
    else if (backup >= 1) { --backup; full = true; }
    else full = false;
    const int last = 63 - __clzll(V);
    if (bad && (full || lane == last)) pas = !pas;
    ++solves;
    if (!solve(pas, __ballot(pas), x, y)) break;
  }
  const double h = (own && x > 0.0) ? x : 0.0;
  double sq = 0.0, beta = 0.0;
  if (live && own) {
    a.hhat[i * R + c] = h;
    sq = h * h;
    beta = m * h;
  }
  wred[wave][lane] = sq;
  beta = wave_sum(beta);
  if (lane == 0) bred[wave] = beta;
  __syncthreads();
  // per-workgroup partials (the WPB rows added in wave order)
  double *cpart = a.part + (int64_t)blockIdx.x * (R + 1);
  if (threadIdx.x < R) {
    double v = wred[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < WPB; ++w) v += wred[w][threadIdx.x];
    cpart[threadIdx.x] = v;
  }
  if (threadIdx.x == 0) {
    double v = bred[0];
#pragma unroll
    for (int w = 1; w < WPB; ++w) v += bred[w];
    cpart[R] = v;
  }
}

// ---------------------------------------------------------------------------
// ADMM (Section 4.3.4, Eqs. eqn:admmnls and eqn:admmupd), for the factor
// (H = X^T, A^T A = S, A^T B = M^T) with the scaled dual U of the mode:
//   rho = trace(S) / R,  Ht = (M + rho (H + U)) (S + rho I)^-1,
//   H = max(0, Ht - U),  U = U + H - Ht,
// at most kAdmmMaxit passes, stopped after a pass once
//   ||H - Ht||^2 / ||H||^2 < tol  and  ||H - H_prev||^2 / ||U||^2 < tol
// over the whole factor.  The Cholesky factor of S + rho I is cached (here as
// the inverse P = L^-T L^-1, formed once per update: S + rho I has condition
// number at most R + 1, so a pass is one row-times-P product).

// P = (S + rho I)^-1 and rho in one workgroup: in-place Gauss-Jordan
// elimination without pivoting (the pivots of a symmetric positive definite
// matrix are its positive Schur complements; the condition number here is at
// most R + 1), each thread owning entries of the R x R array in LDS, two
// barriers per pivot.  A pivot that is not positive marks the update as
// singular (the start value is then kept).
template <int RB>
__global__ __launch_bounds__(1024) void k_admm_prep(UpdateArgs a) {
  constexpr int EPT = (RB * RB + 1023) / 1024;  // entries per thread
  __shared__ double A[RB * RB];
  __shared__ double red[16];
  __shared__ int bad_s;
  const int R = a.R, RR = R * R;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // rho = trace(S) / R
  const double sd = tid < R ? a.S[tid * R + tid] : 0.0;
  const double ws = wave_sum(sd);
  if (lane == 0) red[wave] = ws;
  if (tid == 0) bad_s = 0;
  __syncthreads();
  double tr = 0.0;
  for (int w = 0; w < 16; ++w) tr += red[w];
  const double rho = tr / R;
  for (int e = tid; e < RR; e += 1024) A[e] = a.S[e] + ((e / R) == (e % R) ? rho : 0.0);
  __syncthreads();
  for (int k = 0; k < R; ++k) {
    const double piv = A[k * R + k];
    double nv[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + 1024 * q;
      nv[q] = 0.0;
      if (e < RR) {
        const int i = e / R, j = e % R;
        const double p = 1.0 / piv;
        const double akj = j == k ? p : A[k * R + j] * p;   // new row k
        nv[q] = i == k ? akj : (j == k ? 0.0 : A[e]) - A[i * R + k] * akj;
      }
    }
    if (tid == 0 && !(piv > 0.0)) bad_s = 1;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + 1024 * q;
      if (e < RR) A[e] = nv[q];
    }
    __syncthreads();
  }
  for (int e = tid; e < RR; e += 1024) a.admmP[e] = A[e];
  if (tid == 0) {
    a.admmP[RR] = rho;
    a.admmP[RR + 1] = bad_s ? 1.0 : 0.0;
  }
}

// One ADMM pass over every row: one row per wave, lane c owns column c and
// keeps column c of P in registers.  Pass 0 starts from H diag(lambda) and
// the split partials of M (added in order; their sum is kept for the later
// passes); a later pass first takes the stopping test on the previous pass's
// per-workgroup norms (every workgroup adds them in the same order, so all
// agree) and does nothing once the updates have stopped.  Each pass leaves
// the row kernel's partials (column sums of squares and beta) of its result.
template <typename HT, int RB, bool FULL>
__global__ __launch_bounds__(256) void k_admm_pass(UpdateArgs a, int pass, int nblocks) {
  __shared__ double wred[4][64];
  __shared__ double nred[4][4];
  __shared__ double bred[4];
  __shared__ double tred[256][4];
  __shared__ int run_s;
  const int R = FULL ? RB : a.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  const bool live = i < a.I;
  const bool own = lane < R;
  const int c = own ? lane : 0;
  const int64_t ir = live ? i : a.I - 1;
  const double rho = a.admmP[R * R];
  const bool singular = a.admmP[R * R + 1] != 0.0;
  // ---- the stopping test on the previous pass
  if (threadIdx.x == 0) run_s = 1;
  if (pass > 0) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double *np = a.admmNorm + (int64_t)(pass - 1) * nblocks * 4;
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += np[(int64_t)b * 4 + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) tred[threadIdx.x][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
      double t[4] = {0.0, 0.0, 0.0, 0.0};
      for (int q = 0; q < 256; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] += tred[q][k];
      const double nd = t[0], nh = t[1], nc = t[2], nu = t[3];
      const bool rok = nh > 0.0 ? nd / nh < kAdmmTol : nd == 0.0;
      const bool sok = nu > 0.0 ? nc / nu < kAdmmTol : nc == 0.0;
      run_s = (a.admmStatus[pass - 1] != 0 && !(rok && sok)) ? 1 : 0;
    }
  }
  __syncthreads();
  const bool run = run_s != 0 && !singular;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.admmStatus[pass] = run ? 1 : 0;
  // a singular S + rho I leaves the start value (pass 0 writes it back)
  if (!run && !(pass == 0 && singular)) return;
  // ---- loads: column c of P, the row of M (or its kept sum), H, U
  double pc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) pc[r] = (own && r < R && run) ? a.admmP[r * R + c] : 0.0;
  double m, h;
  if (pass == 0) {
    const HT *M = (const HT *)a.M;
    const HT *mp = M + ir * R + c;
    const int ns = a.msplit;
    HT mv[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) mv[k] = k < ns ? mp[(int64_t)k * a.mstride] : (HT)0;
    HT macc = mv[0];
#pragma unroll
    for (int k = 1; k < 32; ++k)
      if (k < ns) macc += mv[k];
    for (int k = 32; k < ns; ++k) macc += mp[(int64_t)k * a.mstride];
    m = (live && own) ? (double)macc : 0.0;
    h = (live && own) ? (double)((const HT *)a.H)[ir * R + c] * a.lambda[c] : 0.0;
    if (live && own) a.admmMc[i * R + c] = m;
  } else {
    m = (live && own) ? a.admmMc[i * R + c] : 0.0;
    h = (live && own) ? a.hhat[i * R + c] : 0.0;
  }
  const double u = (live && own) ? a.admmU[i * R + c] : 0.0;
  double hn = h, un = u, t = h;
  if (run) {
    // Ht(c) = sum_j (m + rho (h + u))_j P(j, c), j in order
    const double bj = m + rho * (h + u);
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < R) acc += bcast(bj, j) * pc[j];
    t = acc;
    hn = t - u > 0.0 ? t - u : 0.0;
    un = u + hn - t;
  }
  double sq = 0.0, beta = 0.0, nd = 0.0, nh = 0.0, nc = 0.0, nu = 0.0;
  if (live && own) {
    a.hhat[i * R + c] = hn;
    a.admmU[i * R + c] = un;
    sq = hn * hn;
    beta = m * hn;
    nd = (hn - t) * (hn - t);
    nh = hn * hn;
    nc = (hn - h) * (hn - h);
    nu = un * un;
  }
  wred[wave][lane] = sq;
  beta = wave_sum(beta);
  nd = wave_sum(nd);
  nh = wave_sum(nh);
  nc = wave_sum(nc);
  nu = wave_sum(nu);
  if (lane == 0) {
    bred[wave] = beta;
    nred[wave][0] = nd;
    nred[wave][1] = nh;
    nred[wave][2] = nc;
    nred[wave][3] = nu;
  }
  __syncthreads();
  double *cpart = a.part + (int64_t)blockIdx.x * (R + 1);
  if (threadIdx.x < R)
    cpart[threadIdx.x] = wred[0][threadIdx.x] + wred[1][threadIdx.x] + wred[2][threadIdx.x] +
                         wred[3][threadIdx.x];
  if (threadIdx.x == 0) cpart[R] = bred[0] + bred[1] + bred[2] + bred[3];
  if (threadIdx.x < 4)
    a.admmNorm[((int64_t)pass * nblocks + blockIdx.x) * 4 + threadIdx.x] =
        nred[0][threadIdx.x] + nred[1][threadIdx.x] + nred[2][threadIdx.x] + nred[3][threadIdx.x];
}

// Upper tiles (tx <= ty) of the T x T grid of 16 x 16 tiles of an R x R
// matrix, T = ceil(R / 16), in row-major order.
__device__ __forceinline__ void tile_pair(int t, int T, int &tx, int &ty) {
  int q = t, r = 0;
  while (q >= T - r) { q -= T - r; ++r; }
  tx = r;
  ty = r + q;
}

int norm_gpart_elems(int R) { return (int)norm_pn_offset(R) + R * R; }

// Finish of the update for R <= RB <= 64, spread over a few workgroups.
// Every workgroup adds the row kernel's per-workgroup partials itself (the
// same order everywhere, so all hold the same lambda and beta), normalises
// its slice of rows and writes the Gram of that slice (FP64 MFMA over the
// stored, rounded values; upper 16 x 16 tiles).  When the next mode's S is
// asked for, the workgroups also write the product of the Grams other than
// mode and next_mode (256 entries each, in turn).  Adding the slices, gamma
// and the next mode's S are left to the Gram step (gram_finish), which a
// later kernel runs once these are complete.
template <typename HT, int RB, bool FULL>
__global__ __launch_bounds__(256) void k_update_norm(UpdateArgs a, int nblocks, int64_t rpw) {
  constexpr int TB = RB / 16;                     // tile grid bound
  constexpr int TW = (TB * (TB + 1) / 2 + 3) / 4; // tiles per wave
  __shared__ double rowbuf[4096];
  __shared__ double colsum[256];
  __shared__ double lam_s[64];
  const int R = FULL ? RB : a.R;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nct = R + 1, tpc = 256 / nct;
  const int pc = tid % nct, pj = tid / nct;
  const bool pl = pj < tpc;
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = a.I < r0 + rpw ? a.I : r0 + rpw;
  const int CHR = 4096 / R;
  const int T = (R + 15) / 16, ntile = T * (T + 1) / 2;
  // ---- loads first: the row kernel's partials (consecutive threads read
  // consecutive entries) and the first chunk of Hhat
  // (addresses clamped, so that every load is issued unconditionally)
  double pp[32], hv[16];
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int b = pj + k * tpc;
    pp[k] = a.part[(int64_t)(b < nblocks ? b : nblocks - 1) * nct + pc];
  }
  const int rows0 = (int)(r1 - r0 < CHR ? r1 - r0 : CHR);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = tid + 256 * k;
    hv[k] = a.hhat[r0 * R + (e < rows0 * R ? e : rows0 * R - 1)];
  }
  // ---- the product of the Grams other than mode and next_mode (independent
  // of this update), 256 entries per workgroup in turn; its loads go out
  // behind the ones above
  auto gram_product = [&](int e) {
    const int ec = e < R * R ? e : R * R - 1;
    double g[NNCP_MAX_MODES];
#pragma unroll
    for (int q = 0; q < NNCP_MAX_MODES; ++q)
      g[q] = (q < a.N && q != a.mode && q != a.next_mode) ? a.G[(int64_t)q * R * R + ec] : 1.0;
    double p = 1.0;
#pragma unroll
    for (int q = 0; q < NNCP_MAX_MODES; ++q) p *= g[q];
    if (e < R * R) a.gpart[norm_pn_offset(R) + e] = p;
  };
  if (a.S_next && blockIdx.x * 256 < R * R) {
    // the first chunk straight-line, the rest (few workgroups) in a loop
    gram_product(blockIdx.x * 256 + tid);
    for (int e0 = (blockIdx.x + gridDim.x) * 256; e0 < R * R; e0 += gridDim.x * 256)
      gram_product(e0 + tid);
  }
  // ---- lambda (column norms) and beta
  {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if (pl && pj + k * tpc < nblocks) acc += pp[k];
    for (int b = pj + 32 * tpc; pl && b < nblocks; b += tpc) acc += a.part[(int64_t)b * nct + pc];
    colsum[tid] = acc;
  }
  __syncthreads();
  if (tid < nct) {
    double sum = 0.0;
    for (int j = 0; j < tpc; ++j) sum += colsum[j * nct + tid];
    if (tid < R) {
      lam_s[tid] = sqrt(sum);
      if (blockIdx.x == 0) a.lambda[tid] = lam_s[tid];
    } else if (blockIdx.x == 0) {
      a.beta_out[0] = sum;
    }
  }
  __syncthreads();
  // ---- normalise the slice chunk by chunk; Gram tiles of the stored values
  HT *H = (HT *)a.H;
  f64x4 acc[TW];
  int tx[TW], ty[TW];
#pragma unroll
  for (int s = 0; s < TW; ++s) {
    acc[s][0] = acc[s][1] = acc[s][2] = acc[s][3] = 0.0;
    tx[s] = ty[s] = -1;
    const int t = wave + 4 * s;
    if (t < ntile) tile_pair(t, T, tx[s], ty[s]);
  }
  const int lr = lane >> 4, lc = lane & 15;
  for (int64_t c0 = r0; c0 < r1; c0 += CHR) {
    const int rows = (int)(r1 - c0 < CHR ? r1 - c0 : CHR);
    const int ne = rows * R;
    if (c0 != r0) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = tid + 256 * k;
        hv[k] = a.hhat[c0 * R + (e < ne ? e : ne - 1)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = tid + 256 * k;
      if (e < ne) {
        const double l = lam_s[e % R];
        const HT h = (HT)(l > 0.0 ? hv[k] / l : 0.0);
        H[c0 * R + e] = h;
        rowbuf[e] = (double)h;
      }
    }
    __syncthreads();
    // C(x, y) += sum_k rowbuf(k, 16 tx + x) rowbuf(k, 16 ty + y), four rows a
    // step; the operands of eight steps are read before their products
#pragma unroll
    for (int s = 0; s < TW; ++s) {
      if (tx[s] < 0) continue;
      const int cx = 16 * tx[s] + lc, cy = 16 * ty[s] + lc;
      for (int k0 = 0; k0 < rows; k0 += 32) {
        double av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int kr = k0 + 4 * u + lr;
          av[u] = (kr < rows && cx < R) ? rowbuf[kr * R + cx] : 0.0;
          bv[u] = (kr < rows && cy < R) ? rowbuf[kr * R + cy] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc[s], 0, 0, 0);
      }
    }
  }
  // result entry (lr + 4 v, lc) of each tile
  double *gp = a.gpart + (int64_t)blockIdx.x * ntile * 256;
#pragma unroll
  for (int s = 0; s < TW; ++s) {
    if (tx[s] < 0) continue;
    const int t = wave + 4 * s;
#pragma unroll
    for (int v = 0; v < 4; ++v) gp[t * 256 + (lr + 4 * v) * 16 + lc] = acc[s][v];
  }
}

// Row update of the sweep's MU/HALS path without normalisation.  MU
// (Eq. eqn:muupd) and HALS (Eq. eqn:halsupd) commute with column scalings
// of the other factors (M and S scale with them and the update scales back),
// so the factors can stay unnormalised through the sweeps and be normalised
// once at the end of the call (k_norm_scales, k_apply_scales): the iterates
// are those of the normalised iteration up to rounding.  The kernel writes
// the rows straight into H; there is no separate normalisation launch.
// kDeferWaves rows per pass (one row per wave, lane c owns column c and
// keeps column c of S in registers), row blocks gridDim.x apart.  The stored
// (rounded) rows also feed the workgroup's slice of the Gram of the new
// factor (upper 16 x 16 tiles on FP64 MFMA, four rows a step; wave w owns
// tiles w, w + kDeferWaves) and its shares of beta = <M, Hhat> and
// of gamma = sum_i hs_i S hs_i^T (hs the stored row), which the relative
// error identity needs with lambda = 1; both added in row-block and wave
// order.  The arithmetic of a row is that of k_update_rows_small.
template <typename HT, int RB, bool FULL>
__global__ __launch_bounds__(64 * kDeferWaves) void k_update_rows_defer(UpdateArgs a) {
  constexpr int WV = kDeferWaves, TQ = (10 + WV - 1) / WV;  // at most 10 upper tiles
  __shared__ double rows[WV][RB];
  __shared__ double bred[WV][2];
  // FULL: R == RB, known when compiling (no per-column bound tests)
  const int R = FULL ? RB : a.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int T = (R + 15) / 16, ntile = T * (T + 1) / 2;
  int tx[TQ], ty[TQ];
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    tx[q] = ty[q] = -1;
    if (wave + WV * q < ntile) tile_pair(wave + WV * q, T, tx[q], ty[q]);
  }
  const int lr = lane >> 4, lc = lane & 15;
  f64x4 gacc[TQ];
#pragma unroll
  for (int q = 0; q < TQ; ++q) gacc[q][0] = gacc[q][1] = gacc[q][2] = gacc[q][3] = 0.0;
  double bsum = 0.0, gsum = 0.0;
  const HT *M = (const HT *)a.M;
  HT *H = (HT *)a.H;
  const bool own = lane < R;
  const int c = own ? lane : 0;
  double sc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) sc[r] = (own && r < R) ? a.S[r * R + c] : 0.0;
  const double d = own ? a.S[c * R + c] : 0.0;
  // the start value: lambda folded in (first update of the call), or zero
  // in a dead column (as lambda_r = 0 would make it), else the row as stored
  const double lam = a.fold_lambda ? a.lambda[c] : (a.dead[c] != 0.0 ? 0.0 : 1.0);
  const int ns = a.msplit;
  // beta and gamma feed only the relative error (asked for after the last
  // mode of a sweep)
  const bool want = a.relerr_out != nullptr || a.scal != nullptr;
  for (int64_t blk = blockIdx.x; blk * WV < a.I; blk += gridDim.x) {
    const int64_t i = blk * WV + wave;
    const bool live = i < a.I;
    const int64_t ir = live ? i : a.I - 1;
    const HT *mp = M + ir * R + c;
    // the split partials in split order, NL loads issued together (indices
    // clamped, so that none waits on a bound test)
    auto msum = [&](auto nl) -> HT {
      constexpr int NL = decltype(nl)::value;
      HT mv[NL];
#pragma unroll
      for (int k = 0; k < NL; ++k) mv[k] = mp[(int64_t)(k < ns ? k : ns - 1) * a.mstride];
      HT sum = mv[0];
#pragma unroll
      for (int k = 1; k < NL; ++k)
        if (k < ns) sum += mv[k];
      return sum;
    };
    HT macc;
    if (ns == 1) {
      macc = mp[0];
    } else if (ns <= 8) {
      macc = msum(std::integral_constant<int, 8>{});
    } else if (ns <= 16) {
      macc = msum(std::integral_constant<int, 16>{});
    } else {
      macc = msum(std::integral_constant<int, 32>{});
      for (int k = 32; k < ns; ++k) macc += mp[(int64_t)k * a.mstride];
    }
    const HT h_raw = H[ir * R + c];
    const bool ok = live && own;
    double h = ok ? (double)h_raw * lam : 0.0;
    const double m = ok ? (double)macc : 0.0;
    double g = 0.0;
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < R) g += bcast(h, j) * sc[j];
    if (a.algo == NNCP_MU) {
      h = h * m / (g + a.eps);
    } else {
      g = m - g;
      const bool pos = d > 0.0;
      const double invd = pos ? 1.0 / d : 0.0;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (r < R) {
          double v = h + g * invd;
          v = v > 0.0 ? v : 0.0;
          const double dl = pos ? v - h : 0.0;
          const double delta = bcast(dl, r);
          if (lane == r && pos) h = v;
          g -= delta * sc[r];
        }
      }
    }
    const HT hst = (HT)h;
    if (ok) H[i * R + c] = hst;
    const double hs = ok ? (double)hst : 0.0;
    if (lane < RB) rows[wave][lane] = hs;
    if (want) {
      // (hs S)(c), j in order
      double gs = 0.0;
#pragma unroll
      for (int j = 0; j < RB; ++j)
        if (j < R) gs += bcast(hs, j) * sc[j];
      const double beta = wave_sum(ok ? m * h : 0.0);
      const double gam = wave_sum(ok ? hs * gs : 0.0);
      if (lane == 0) {
        bred[wave][0] = beta;
        bred[wave][1] = gam;
      }
    }
    __syncthreads();
    // the pass's rows four at a time (the K of one 16x16x4 step)
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      if (tx[q] < 0) continue;
#pragma unroll
      for (int k0 = 0; k0 < WV; k0 += 4) {
        const double av = rows[k0 + lr][16 * tx[q] + lc];
        const double bv = rows[k0 + lr][16 * ty[q] + lc];
        gacc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, gacc[q], 0, 0, 0);
      }
    }
    if (want && threadIdx.x == 0) {
#pragma unroll
      for (int w = 0; w < WV; ++w) {
        bsum += bred[w][0];
        gsum += bred[w][1];
      }
    }
    __syncthreads();
  }
  // this workgroup's slice: entry (lr + 4 v, lc) of tile t, as the finish
  // kernel writes its slices
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    if (tx[q] < 0) continue;
    double *gp = a.gpart + ((int64_t)blockIdx.x * ntile + wave + WV * q) * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) gp[(lr + 4 * v) * 16 + lc] = gacc[q][v];
  }
  if (want && threadIdx.x == 0) {
    a.part[blockIdx.x] = bsum;
    a.part[gridDim.x + blockIdx.x] = gsum;
  }
}

// End of the deferred path, step 1 (one workgroup): the column norms of
// every factor from its Gram, s_k(r) = sqrt(G^(k)(r, r)), and
// lambda_r = prod_k s_k(r) (modes in order).  scale = [N][R] norms, then R
// lambdas.
__global__ __launch_bounds__(256) void k_norm_scales(const double *__restrict__ G, int N, int R,
                                                     double *__restrict__ lambda,
                                                     double *__restrict__ scale) {
  for (int r = threadIdx.x; r < R; r += 256) {
    double l = 1.0;
    for (int k = 0; k < N; ++k) {
      const double sk = sqrt(G[((int64_t)k * R + r) * R + r]);
      scale[k * R + r] = sk;
      l *= sk;
    }
    scale[N * R + r] = l;
    lambda[r] = l;
  }
}

struct ScaleArgs {
  void *H[NNCP_MAX_MODES];
  int64_t off[NNCP_MAX_MODES + 1];  // prefix sums of I_k R
  int N, R;
};

// Step 2: H^(k)(i, r) /= s_k(r) and G^(k)(a, b) /= s_k(a) s_k(b), zero where
// lambda is zero; one thread per entry (the factors' entries first, then the
// N Grams).
template <typename HT>
__global__ __launch_bounds__(256) void k_apply_scales(ScaleArgs a, double *__restrict__ G,
                                                      const double *__restrict__ scale) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int N = a.N, R = a.R;
  const double *lam = scale + N * R;
  if (e < a.off[N]) {
    int k = 0;
    while (e >= a.off[k + 1]) ++k;
    const int r = (int)((e - a.off[k]) % R);
    HT *H = (HT *)a.H[k];
    const int64_t idx = e - a.off[k];
    const double s = scale[k * R + r];
    H[idx] = lam[r] > 0.0 ? (HT)((double)H[idx] / s) : (HT)0;
    return;
  }
  const int64_t f = e - a.off[N];
  if (f >= (int64_t)N * R * R) return;
  const int k = (int)(f / ((int64_t)R * R));
  const int x = (int)((f / R) % R), y = (int)(f % R);
  const double sx = scale[k * R + x], sy = scale[k * R + y];
  G[f] = (lam[x] > 0.0 && lam[y] > 0.0) ? G[f] / (sx * sy) : 0.0;
}

// the Gram step as a kernel of its own (gram_blocks(j) workgroups)
__global__ __launch_bounds__(256) void k_gram_finish(GramJob j) { gram_run<3>(j, blockIdx.x); }

// ---------------------------------------------------------------------------
// loss of [[lambda; H]] given M^(N-1) at the current factors
// ---------------------------------------------------------------------------
// one workgroup of NT threads: beta = <M, H diag(lambda)>, gamma =
// lambda^T (prod_k G^(k)) lambda, the loss 0.5 (alpha - 2 beta + gamma)
template <typename HT, int NT>
__device__ __forceinline__ void loss_block(int N, int R, int64_t In, const HT *__restrict__ M,
                                           const HT *__restrict__ H,
                                           const double *__restrict__ lambda,
                                           const double *__restrict__ G,
                                           const double *__restrict__ alpha, double *loss,
                                           double *relerr, double *scal,
                                           double (*wred)[2] /* LDS, NT / 64 rows */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // beta: the thread's entries e = t, t + NT, ... in order, eight at a time
  // with their loads issued together (the column e % R kept incrementally)
  double beta = 0.0;
  {
    const int64_t n = In * R;
    const int rstep = NT % R;
    int r = (int)(threadIdx.x % R);
    int64_t e = threadIdx.x;
    for (; e + 7 * NT < n; e += 8 * NT) {
      HT mv[8], hv[8];
      double lv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        mv[u] = M[e + u * NT];
        hv[u] = H[e + u * NT];
        lv[u] = lambda[r];
        r += rstep;
        if (r >= R) r -= R;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) beta += (double)mv[u] * (double)hv[u] * lv[u];
    }
    for (; e < n; e += NT) {
      beta += (double)M[e] * (double)H[e] * lambda[r];
      r += rstep;
      if (r >= R) r -= R;
    }
  }
  // gamma: the N Gram entries of an e loaded together (N <= 8), multiplied
  // in mode order (the unused slots are 1)
  double gamma = 0.0;
  for (int e = threadIdx.x; e < R * R; e += NT) {
    double s = 1.0;
    if (N <= 8) {
      double gv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double v = G[(int64_t)(k < N ? k : N - 1) * R * R + e];
        gv[k] = k < N ? v : 1.0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) s *= gv[k];
    } else {
      for (int k = 0; k < N; ++k) s *= G[(int64_t)k * R * R + e];
    }
    gamma += lambda[e / R] * s * lambda[e % R];
  }
  beta = wave_sum(beta);
  gamma = wave_sum(gamma);
  if (lane == 0) { wred[wave][0] = beta; wred[wave][1] = gamma; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0, g = 0.0;
    for (int w = 0; w < NT / 64; ++w) { b += wred[w][0]; g += wred[w][1]; }
    const double al = alpha[0];
    const double r2 = al - 2.0 * b + g;
    if (loss) loss[0] = 0.5 * r2;
    if (relerr) relerr[0] = sqrt((r2 > 0.0 ? r2 : 0.0) / al);
    if (scal) { scal[0] = b; scal[1] = g; scal[2] = r2 / al; }
  }
}

template <typename HT>
__global__ __launch_bounds__(1024) void k_loss(int N, int R, int64_t In, const HT *__restrict__ M,
                                               const HT *__restrict__ H,
                                               const double *__restrict__ lambda,
                                               const double *__restrict__ G,
                                               const double *__restrict__ alpha, double *loss,
                                               double *relerr, double *scal) {
  __shared__ double wred[16][2];
  loss_block<HT, 1024>(N, R, In, M, H, lambda, G, alpha, loss, relerr, scal, wred);
}

// ---------------------------------------------------------------------------
// gradient of 0.5 ||X - [[H]]||^2 for one mode: grad = H S - M
// ---------------------------------------------------------------------------
// grad = H S - M for the entries of workgroup `blk` of one mode
template <typename HT>
__device__ __forceinline__ void grad_block(int64_t blk, int64_t I, int R, int N, int mode,
                                           const HT *__restrict__ M, int msplit, int64_t mstride,
                                           const HT *__restrict__ H, const double *__restrict__ G,
                                           const double *__restrict__ Sg, HT *__restrict__ grad,
                                           double *sS /* LDS, 64 x 64 */) {
  // S in LDS for R <= 64, else read from the global Hadamard product Sg
  const bool lds = R <= 64;
  if (lds) {
    for (int e = threadIdx.x; e < R * R; e += 256) {
      double s = 1.0;
      for (int k = 0; k < N; ++k)
        if (k != mode) s *= G[(int64_t)k * R * R + e];
      sS[e] = s;
    }
  }
  __syncthreads();
  const int64_t e = blk * 256 + threadIdx.x;
  if (e >= I * R) return;
  const int64_t i = e / R;
  const int r = (int)(e % R);
  // the split partials of M in split order (one load each, issued together)
  const HT m = ordered_split_sum_wide(M + e, msplit, mstride);
  double s = 0.0;
  for (int c = 0; c < R; ++c) s += (double)H[i * R + c] * (lds ? sS[c * R + r] : Sg[c * R + r]);
  grad[e] = (HT)(s - (double)m);
}

template <typename HT>
__global__ __launch_bounds__(256) void k_grad(int64_t I, int R, int N, int mode,
                                              const HT *__restrict__ M, int msplit,
                                              int64_t mstride, const HT *__restrict__ H,
                                              const double *__restrict__ G,
                                              const double *__restrict__ Sg, HT *__restrict__ grad) {
  __shared__ double sS[64 * 64];
  grad_block<HT>(blockIdx.x, I, R, N, mode, M, msplit, mstride, H, G, Sg, grad, sS);
}

// Every mode's gradient in one launch (R <= 64): workgroups wg0[n] ..
// wg0[n + 1] - 1 take mode n (M^(n) as a.M[n], msplit partial copies; a
// mode's M may be its gradient buffer itself: each entry is read before the
// same thread overwrites it), and workgroup wg0[N] the loss from M^(N-1)
// (which must not be a gradient buffer).
template <typename HT>
__global__ __launch_bounds__(256) void k_grad_all(GradAllArgs a) {
  __shared__ double sS[64 * 64];
  const int b = blockIdx.x;
  if (b == a.wg0[a.N]) {
    const int n = a.N - 1;
    loss_block<HT, 256>(a.N, a.R, a.I[n], (const HT *)a.M[n], (const HT *)a.H[n], a.ones, a.G,
                        a.alpha, a.loss, nullptr, a.scal, reinterpret_cast<double (*)[2]>(sS));
    return;
  }
  int n = 0;
  while (n + 1 < a.N && b >= a.wg0[n + 1]) ++n;
  grad_block<HT>(b - a.wg0[n], a.I[n], a.R, a.N, n, (const HT *)a.M[n], a.msplit[n],
                 a.mstride[n], (const HT *)a.H[n], a.G, nullptr, (HT *)a.grad[n], sS);
}

// ---------------------------------------------------------------------------
// projected gradient helpers
// ---------------------------------------------------------------------------
// Step size of the projected gradient: 1 / max_n lambda_max(S^(n)), each
// lambda_max by `iters` power steps from the normalised all-ones vector and a
// final Rayleigh quotient.  One wave per mode (modes n, n + 8, ... for wave
// n of eight): lane i < R keeps row i of S^(n) = prod_{k != n} G^(k) in
// registers; the iterate goes through the wave's LDS row, read as a
// broadcast by every lane, and the norm is a wave reduction.  w_i = sum_j
// S(i, j) v_j is added in j order.
template <int RB, bool FULL>
__global__ __launch_bounds__(512) void k_pgd_eta(const double *__restrict__ G, int N, int Rin,
                                                 int iters, double *__restrict__ eta) {
  __shared__ double vs[8][RB];
  __shared__ double lm[8];
  const int R = FULL ? RB : Rin;  // FULL: R == RB, known when compiling
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool own = lane < R;
  const int i = own ? lane : 0;
  double lmax = 0.0;
  for (int n = wave; n < N; n += 8) {
    // row i of S^(n): the other modes' Gram rows one mode at a time, each
    // row's loads issued together (indices clamped), multiplied in mode order
    double srow[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) srow[j] = 1.0;
    for (int k = 0; k < N; ++k) {
      if (k == n) continue;
      const double *gk = G + (int64_t)k * R * R + (int64_t)i * R;
      double gv[RB];
#pragma unroll
      for (int j = 0; j < RB; ++j) gv[j] = gk[j < R ? j : R - 1];
#pragma unroll
      for (int j = 0; j < RB; ++j) srow[j] *= gv[j];
    }
#pragma unroll
    for (int j = 0; j < RB; ++j) srow[j] = (own && j < R) ? srow[j] : 0.0;
    if (lane < RB) vs[wave][lane] = lane < R ? 1.0 / sqrt((double)R) : 0.0;
    wave_sync_lds();
    auto matvec = [&]() {
      double w = 0.0;
#pragma unroll
      for (int j = 0; j < RB; ++j)
        if (j < R) w += srow[j] * vs[wave][j];
      return w;
    };
    for (int t = 0; t < iters; ++t) {
      const double w = matvec();
      const double nrm = sqrt(wave_sum(own ? w * w : 0.0));
      if (!(nrm > 0.0)) break;
      wave_sync_lds();
      if (own) vs[wave][lane] = w / nrm;
      wave_sync_lds();
    }
    const double w = matvec();
    const double rq = wave_sum(own ? vs[wave][lane] * w : 0.0);
    if (rq > lmax) lmax = rq;
    wave_sync_lds();
  }
  if (lane == 0) lm[wave] = lmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double l = lm[0];
    for (int w = 1; w < 8; ++w) l = lm[w] > l ? lm[w] : l;
    eta[0] = l > 0.0 ? 1.0 / l : 1.0;
  }
}

template <typename HT>
__global__ __launch_bounds__(256) void k_pgd_trial(int64_t n, const HT *__restrict__ H,
                                                   const HT *__restrict__ g, double eta,
                                                   HT *__restrict__ Hn, double *__restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += stride) {
    const double h = (double)H[e];
    double v = h - eta * (double)g[e];
    v = v > 0.0 ? v : 0.0;
    const HT vn = (HT)v;
    Hn[e] = vn;
    const double d = (double)vn - h;
    acc += d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_mttv_contig(int hdt, const void *T, int64_t Ia, int64_t Q, int R, const void *H,
                              void *out, int leaf, hipStream_t st, GramJob *carry) {
  const int V = hdt == NNCP_F64 ? 2 : 4;
  GramJob job = carry ? *carry : GramJob{};
  if (carry) carry->R = 0;
  const int64_t gl = Ia / V;
  if (Ia % V == 0 && gl < 64 && (gl & (gl - 1)) == 0) {
    const unsigned gy = (unsigned)((Q + 4 * (64 / gl) * 8 - 1) / (4 * (64 / gl) * 8));
    dim3 grid((unsigned)R + (gram_blocks(job) + gy - 1) / gy, gy), block(256);
#define NNCP_CONTIG_PACK(HTV, GLV)                                                            \
  hipLaunchKernelGGL((k_mttv_contig_pack<HTV, GLV>), grid, block, 0, st, (const HTV *)T, Ia, Q, \
                     R, (const HTV *)H, (HTV *)out, leaf, job)
#define NNCP_CONTIG_PACK_GL(HTV)       \
  switch (gl) {                        \
    case 1: NNCP_CONTIG_PACK(HTV, 1); break;   \
    case 2: NNCP_CONTIG_PACK(HTV, 2); break;   \
    case 4: NNCP_CONTIG_PACK(HTV, 4); break;   \
    case 8: NNCP_CONTIG_PACK(HTV, 8); break;   \
    case 16: NNCP_CONTIG_PACK(HTV, 16); break; \
    default: NNCP_CONTIG_PACK(HTV, 32); break; \
  }
    if (hdt == NNCP_F64) { NNCP_CONTIG_PACK_GL(double) }
    else { NNCP_CONTIG_PACK_GL(float) }
#undef NNCP_CONTIG_PACK_GL
#undef NNCP_CONTIG_PACK
    return hipGetLastError();
  }
  if (Ia % V == 0 && Ia <= 8 * 64 * V) {
    const int CPL = Ia <= 64 * V ? 1 : Ia <= 128 * V ? 2 : Ia <= 256 * V ? 4 : 8;
    const int QB = 8 / CPL;
    const unsigned gy = (unsigned)((Q + 4 * QB - 1) / (4 * QB));
    dim3 grid((unsigned)R + (gram_blocks(job) + gy - 1) / gy, gy), block(256);
#define NNCP_CONTIG_REG(HTV, C)                                                            \
  hipLaunchKernelGGL((k_mttv_contig_reg<HTV, C>), grid, block, 0, st, (const HTV *)T, Ia, Q, R, \
                     (const HTV *)H, (HTV *)out, leaf, job)
    if (hdt == NNCP_F64) {
      switch (CPL) {
        case 1: NNCP_CONTIG_REG(double, 1); break;
        case 2: NNCP_CONTIG_REG(double, 2); break;
        case 4: NNCP_CONTIG_REG(double, 4); break;
        default: NNCP_CONTIG_REG(double, 8); break;
      }
    } else {
      switch (CPL) {
        case 1: NNCP_CONTIG_REG(float, 1); break;
        case 2: NNCP_CONTIG_REG(float, 2); break;
        case 4: NNCP_CONTIG_REG(float, 4); break;
        default: NNCP_CONTIG_REG(float, 8); break;
      }
    }
#undef NNCP_CONTIG_REG
    return hipGetLastError();
  }
  // the other variants do not carry the Gram step: run it first
  if (job.R) {
    const hipError_t e = launch_gram_finish(job, st);
    if (e != hipSuccess) return e;
  }
  if (Ia >= 64 && Ia <= 8192 && Ia % V == 0 && (hdt != NNCP_F64 || Ia <= 4096)) {
    // about 2048 workgroups, at least 4 outputs (one per wave) each
    int64_t qper = (Q * R + 2047) / 2048;
    if (qper < 4) qper = 4;
    const int64_t gy = (Q + qper - 1) / qper;
    dim3 grid((unsigned)R, (unsigned)gy), block(256);
    if (hdt == NNCP_F64)
      hipLaunchKernelGGL(k_mttv_contig_wide<double>, grid, block, 0, st, (const double *)T, Ia, Q,
                         R, (const double *)H, (double *)out, leaf, qper);
    else
      hipLaunchKernelGGL(k_mttv_contig_wide<float>, grid, block, 0, st, (const float *)T, Ia, Q,
                         R, (const float *)H, (float *)out, leaf, qper);
    return hipGetLastError();
  }
  int G = 1;
  while (G < 64 && G < Ia) G *= 2;
  const int64_t threads = Q * R * G;
  dim3 grid((unsigned)((threads + 255) / 256)), block(256);
  if (hdt == NNCP_F64)
    hipLaunchKernelGGL(k_mttv_contig<double>, grid, block, 0, st, (const double *)T, Ia, Q, R,
                       (const double *)H, (double *)out, leaf, G);
  else
    hipLaunchKernelGGL(k_mttv_contig<float>, grid, block, 0, st, (const float *)T, Ia, Q, R,
                       (const float *)H, (float *)out, leaf, G);
  return hipGetLastError();
}

// vector width of the strided kernel: 16-byte loads when Ia allows them
static int strided_vec(int hdt, int64_t Ia) {
  const int V = hdt == NNCP_F64 ? 2 : 4;
  return Ia % V == 0 ? V : 1;
}

static void strided_shape(int64_t Ia, int V, int64_t Q, int R, int &IT, int &QS, int &ns,
                          int64_t &gx) {
  // at most 64 column threads, so at least 4 q-lanes per workgroup (the two
  // multi-TTVs of a 512^3 sweep took 19.0 us against 20.4 us with 128 x 2)
  IT = 1;
  while (IT < 64 && IT * V < Ia) IT *= 2;
  QS = 256 / IT;
  gx = (Ia + (int64_t)IT * V - 1) / ((int64_t)IT * V);
  int64_t want = (512 + gx * R - 1) / (gx * R);
  int64_t maxs = (Q + QS - 1) / QS;
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  if (want > 4096) want = 4096;
  ns = (int)want;
}

int64_t mttv_strided_part_elems(int hdt, int64_t Ia, const int64_t *qdims, int nq, int R) {
  int64_t Q = 1;
  for (int k = 0; k < nq; ++k) Q *= qdims[k];
  int IT, QS, ns;
  int64_t gx;
  strided_shape(Ia, strided_vec(hdt, Ia), Q, R, IT, QS, ns, gx);
  return (int64_t)ns * Ia * R;
}

hipError_t launch_mttv_strided(int hdt, const void *T, int64_t Ia, const int64_t *qdims, int nq,
                               const void *const *Hq, int R, void *M, void *part,
                               int64_t part_elems, hipStream_t st, int *nsplit_out,
                               GramJob *carry) {
  StridedArgs a;
  GramJob job = carry ? *carry : GramJob{};
  int64_t Q = 1;
  for (int k = 0; k < NNCP_MAX_MODES; ++k) {
    a.H[k] = k < nq ? Hq[k] : nullptr;
    a.qd[k] = k < nq ? qdims[k] : 1;
    if (k < nq) Q *= qdims[k];
  }
  a.nq = nq; a.Ia = Ia; a.Q = Q; a.R = R;
  int64_t gx;
  const int V = strided_vec(hdt, Ia);
  strided_shape(Ia, V, Q, R, a.IT, a.QS, a.nsplit, gx);
  if ((int64_t)a.nsplit * Ia * R > part_elems) return hipErrorInvalidValue;
  if (carry) carry->R = 0;
  const int64_t per_row = gx * (int64_t)a.nsplit;
  dim3 grid((unsigned)gx, R + (unsigned)((gram_blocks(job) + per_row - 1) / per_row), a.nsplit),
      block(256);
  const int64_t n = Ia * R;
  dim3 g2((unsigned)((n + 255) / 256));
  if (nsplit_out) *nsplit_out = a.nsplit;
  if (hdt == NNCP_F64) {
    if (V == 2)
      hipLaunchKernelGGL((k_mttv_strided<double, 2>), grid, block, 0, st, (const double *)T, a, (double *)part, job);
    else
      hipLaunchKernelGGL((k_mttv_strided<double, 1>), grid, block, 0, st, (const double *)T, a, (double *)part, job);
    if (M)
      hipLaunchKernelGGL(k_sum_splits<double>, g2, dim3(256), 0, st, (const double *)part, n, a.nsplit, (double *)M);
  } else {
    if (V == 4)
      hipLaunchKernelGGL((k_mttv_strided<float, 4>), grid, block, 0, st, (const float *)T, a, (float *)part, job);
    else
      hipLaunchKernelGGL((k_mttv_strided<float, 1>), grid, block, 0, st, (const float *)T, a, (float *)part, job);
    if (M)
      hipLaunchKernelGGL(k_sum_splits<float>, g2, dim3(256), 0, st, (const float *)part, n, a.nsplit, (float *)M);
  }
  return hipGetLastError();
}

bool plan_mttv_contig(int hdt, const void *T, int64_t Ia, int64_t Q, int R, const void *H,
                      void *out, int leaf, MttvJob *j) {
  const int V = hdt == NNCP_F64 ? 2 : 4;
  const int64_t gl = Ia / V;
  if (Ia % V != 0 || gl >= 64 || (gl & (gl - 1)) != 0) return false;
  const size_t hs = hdt == NNCP_F64 ? 8 : 4;
  const int64_t gy = (Q + 4 * (64 / gl) * 8 - 1) / (4 * (64 / gl) * 8);
  *j = MttvJob{};
  j->kind = 1;
  j->T = T;
  j->out = out;
  j->Ia = Ia;
  j->Q = Q;
  j->R = R;
  j->leaf = leaf;
  j->H = H;
  j->blocks = (int64_t)R * gy;
  j->vec = (int)gl;
  j->rd0 = (const char *)T;
  j->rd1 = j->rd0 + hs * (size_t)(R * Ia * Q);
  j->wr0 = (const char *)out;
  j->wr1 = j->wr0 + hs * (size_t)(Q * R);
  return true;
}

bool plan_mttv_strided(int hdt, const void *T, int64_t Ia, const int64_t *qdims, int nq,
                       const void *const *Hq, int R, void *part, int64_t part_elems, MttvJob *j,
                       int *nsplit_out) {
  StridedArgs a;
  int64_t Q = 1;
  for (int k = 0; k < NNCP_MAX_MODES; ++k) {
    a.H[k] = k < nq ? Hq[k] : nullptr;
    a.qd[k] = k < nq ? qdims[k] : 1;
    if (k < nq) Q *= qdims[k];
  }
  a.nq = nq; a.Ia = Ia; a.Q = Q; a.R = R;
  int64_t gx;
  const int V = strided_vec(hdt, Ia);
  strided_shape(Ia, V, Q, R, a.IT, a.QS, a.nsplit, gx);
  if ((int64_t)a.nsplit * Ia * R > part_elems) return false;
  const size_t hs = hdt == NNCP_F64 ? 8 : 4;
  *j = MttvJob{};
  j->kind = 0;
  j->T = T;
  j->out = part;
  j->sa = a;
  j->gx = gx;
  j->Ia = Ia;
  j->Q = Q;
  j->R = R;
  j->blocks = gx * R * a.nsplit;
  j->vec = V;
  j->rd0 = (const char *)T;
  j->rd1 = j->rd0 + hs * (size_t)(R * Ia * Q);
  j->wr0 = (const char *)part;
  j->wr1 = j->wr0 + hs * (size_t)(a.nsplit * Ia * R);
  if (nsplit_out) *nsplit_out = a.nsplit;
  return true;
}

static bool overlap(const char *a0, const char *a1, const char *b0, const char *b1) {
  return a0 < b1 && b0 < a1;
}

template <typename HT>
static hipError_t launch_group(const MttvGroup &g, int sv, int cv, hipStream_t st) {
  const dim3 grid((unsigned)g.start[g.n]), block(256);
#define NNCP_GROUP(VV, GLV) hipLaunchKernelGGL((k_mttv_group<HT, VV, GLV>), grid, block, 0, st, g)
#define NNCP_GROUP_GL(VV)                   \
  switch (cv) {                             \
    case 1: NNCP_GROUP(VV, 1); break;       \
    case 2: NNCP_GROUP(VV, 2); break;       \
    case 4: NNCP_GROUP(VV, 4); break;       \
    case 8: NNCP_GROUP(VV, 8); break;       \
    case 16: NNCP_GROUP(VV, 16); break;     \
    case 32: NNCP_GROUP(VV, 32); break;     \
    default: return hipErrorInvalidValue;   \
  }
  constexpr int VW = sizeof(HT) == 8 ? 2 : 4;
  if (sv == VW) {
    NNCP_GROUP_GL(VW)
  } else if (sv == 1) {
    NNCP_GROUP_GL(1)
  } else {
    return hipErrorInvalidValue;
  }
#undef NNCP_GROUP_GL
#undef NNCP_GROUP
  return hipGetLastError();
}

hipError_t launch_mttv_jobs(int hdt, const MttvJob *jobs, int n, hipStream_t st) {
  constexpr int kMax = 64;
  if (n < 0 || n > kMax) return hipErrorInvalidValue;
  int level[kMax];
  int top = -1;
  for (int b = 0; b < n; ++b) {
    const MttvJob &y = jobs[b];
    level[b] = 0;
    for (int a = 0; a < b; ++a) {
      const MttvJob &x = jobs[a];
      if (overlap(x.wr0, x.wr1, y.rd0, y.rd1) || overlap(x.wr0, x.wr1, y.wr0, y.wr1) ||
          overlap(x.rd0, x.rd1, y.wr0, y.wr1))
        level[b] = level[b] > level[a] + 1 ? level[b] : level[a] + 1;
    }
    top = top > level[b] ? top : level[b];
  }
  for (int lv = 0; lv <= top; ++lv) {
    // the level's jobs in order, a launch per run of matching variants
    MttvGroup g{};
    int sv = 0, cv = 0;
    auto flush = [&]() -> hipError_t {
      if (g.n == 0) return hipSuccess;
      hipError_t e = hdt == NNCP_F64 ? launch_group<double>(g, sv ? sv : 1, cv ? cv : 1, st)
                                     : launch_group<float>(g, sv ? sv : 1, cv ? cv : 1, st);
      g = MttvGroup{};
      sv = cv = 0;
      return e;
    };
    for (int b = 0; b < n; ++b) {
      if (level[b] != lv) continue;
      const MttvJob &y = jobs[b];
      const bool fits = g.n < kMttvGroupMax && (y.kind == 0 ? (sv == 0 || sv == y.vec)
                                                            : (cv == 0 || cv == y.vec));
      if (!fits) {
        const hipError_t e = flush();
        if (e != hipSuccess) return e;
      }
      if (y.kind == 0) sv = y.vec;
      else cv = y.vec;
      g.j[g.n] = y;
      g.start[g.n + 1] = g.start[g.n] + y.blocks;
      ++g.n;
    }
    const hipError_t e = flush();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gram(int hdt, const void *H, int64_t I, int R, double *G, hipStream_t st) {
  if (hdt == NNCP_F64)
    hipLaunchKernelGGL(k_gram<double>, dim3(1), dim3(1024), 0, st, (const double *)H, I, R, G);
  else
    hipLaunchKernelGGL(k_gram<float>, dim3(1), dim3(1024), 0, st, (const float *)H, I, R, G);
  return hipGetLastError();
}

hipError_t launch_hadamard(const double *G, int N, int R, int mode, double *S, hipStream_t st) {
  hipLaunchKernelGGL(k_hadamard, dim3(1), dim3(256), 0, st, G, N, R, mode, S);
  return hipGetLastError();
}

hipError_t launch_sumsq(int xdt, const void *X, int64_t n, double *part, double *out,
                        hipStream_t st) {
  const int nb = 1024;
  dim3 grid(nb), block(256);
  switch (xdt) {
    case NNCP_F64: hipLaunchKernelGGL(k_sumsq_part<double>, grid, block, 0, st, (const double *)X, n, part); break;
    case NNCP_F32: hipLaunchKernelGGL(k_sumsq_part<float>, grid, block, 0, st, (const float *)X, n, part); break;
    case NNCP_BF16: hipLaunchKernelGGL(k_sumsq_part<bf16_t>, grid, block, 0, st, (const bf16_t *)X, n, part); break;
    case NNCP_F16: hipLaunchKernelGGL(k_sumsq_part<f16_t>, grid, block, 0, st, (const f16_t *)X, n, part); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, part, nb, out);
  return hipGetLastError();
}

int defer_workgroups(int64_t I) {
  const int64_t blocks = (I + kDeferWaves - 1) / kDeferWaves;
  return (int)(blocks < kGramSlices ? blocks : kGramSlices);
}

template <typename HT>
static hipError_t update_dispatch(const UpdateArgs &a, hipStream_t st, GramJob *job) {
  const int rpb = update_rows_per_block(a.R);
  const int nb = (int)((a.I + rpb - 1) / rpb);
  dim3 grid(nb), block(256);
  *job = GramJob{};
  job->R = 0;
  if (a.defer) {
    if (a.R > 64 || (a.algo != NNCP_MU && a.algo != NNCP_HALS)) return hipErrorInvalidValue;
    const int nw = defer_workgroups(a.I);
    job->gpart = a.gpart;
    job->G = a.G;
    job->S = a.S;
    job->S_next = a.S_next;
    job->lambda = a.lambda;   // the ones vector on this path
    job->beta = a.part;       // any valid address; beta comes from beta_part
    job->beta_part = a.part;
    job->gamma_part = a.part + nw;
    job->nbeta = nw;
    job->pn_inline = 1;
    job->dead = const_cast<double *>(a.dead);
    {
      const int T = (a.R + 15) / 16;
      job->parts = (T * (T + 1) / 2) * 8;  // 32 upper-tile entries each
    }
    job->alpha = a.alpha;
    job->relerr_out = a.relerr_out;
    job->scal = a.scal;
    job->R = a.R;
    job->N = a.N;
    job->mode = a.mode;
    job->next_mode = a.next_mode;
    job->nw = nw;
    const dim3 blk(64 * kDeferWaves);
#define NNCP_DEFER(RBV)                                                                     \
  if (a.R == RBV) hipLaunchKernelGGL((k_update_rows_defer<HT, RBV, true>), dim3(nw), blk, 0, st, a); \
  else hipLaunchKernelGGL((k_update_rows_defer<HT, RBV, false>), dim3(nw), blk, 0, st, a);
    if (a.R <= 16) {
      NNCP_DEFER(16)
    } else if (a.R <= 32) {
      NNCP_DEFER(32)
    } else {
      NNCP_DEFER(64)
    }
#undef NNCP_DEFER
    return hipGetLastError();
  }
  if (a.R <= 64) {
    int64_t rpw;
    const int nw = norm_workgroups(a.I, &rpw);
    job->gpart = a.gpart;
    job->pn = a.gpart + norm_pn_offset(a.R);
    job->G = a.G;
    job->S = a.S;
    job->S_next = a.S_next;
    job->lambda = a.lambda;
    job->beta = a.beta_out;
    job->alpha = a.alpha;
    job->relerr_out = a.relerr_out;
    job->scal = a.scal;
    job->R = a.R;
    job->N = a.N;
    job->mode = a.mode;
    job->next_mode = a.next_mode;
    job->nw = nw;
#define NNCP_UPDATE_SMALL(RBV, FV)                                                         \
  if (a.algo == NNCP_NES) {                                                               \
    hipLaunchKernelGGL((k_nes_prep<RBV, FV>), dim3(1), dim3(64), 0, st, a);               \
    hipLaunchKernelGGL((k_update_rows_small<HT, RBV, true, FV>), grid, block, 0, st, a);  \
    hipLaunchKernelGGL((k_update_norm<HT, RBV, FV>), dim3(nw), dim3(256), 0, st, a, nb, rpw); \
  } else if (a.algo == NNCP_ADMM) {                                                       \
    hipLaunchKernelGGL((k_admm_prep<RBV>), dim3(1), dim3(1024), 0, st, a);                \
    for (int p = 0; p < kAdmmMaxit; ++p)                                                  \
      hipLaunchKernelGGL((k_admm_pass<HT, RBV, FV>), grid, block, 0, st, a, p, nb);       \
    hipLaunchKernelGGL((k_update_norm<HT, RBV, FV>), dim3(nw), dim3(256), 0, st, a, nb, rpw); \
  } else if (a.algo == NNCP_BPP) {                                                        \
    constexpr int WPB = RBV <= 32 ? 4 : 1;                                                \
    const int nbb = (int)((a.I + WPB - 1) / WPB);                                         \
    hipLaunchKernelGGL((k_update_bpp<HT, RBV>), dim3(nbb), dim3(64 * WPB), 0, st, a);     \
    hipLaunchKernelGGL((k_update_norm<HT, RBV, FV>), dim3(nw), dim3(256), 0, st, a, nbb, rpw); \
  } else {                                                                                 \
    hipLaunchKernelGGL((k_update_rows_small<HT, RBV, false, FV>), grid, block, 0, st, a); \
    hipLaunchKernelGGL((k_update_norm<HT, RBV, FV>), dim3(nw), dim3(256), 0, st, a, nb, rpw); \
  }
    // R equal to the tile width (compiled without per-column bound tests),
    // or below it
#define NNCP_UPDATE_SMALL_R(RBV)   \
  if (a.R == RBV) {                \
    NNCP_UPDATE_SMALL(RBV, true)   \
  } else {                         \
    NNCP_UPDATE_SMALL(RBV, false)  \
  }
    if (a.R <= 16) {
      NNCP_UPDATE_SMALL_R(16)
    } else if (a.R <= 32) {
      NNCP_UPDATE_SMALL_R(32)
    } else {
      NNCP_UPDATE_SMALL_R(64)
    }
#undef NNCP_UPDATE_SMALL_R
#undef NNCP_UPDATE_SMALL
  } else {
    if (a.algo == NNCP_BPP || a.algo == NNCP_ADMM || a.algo == NNCP_NES) return hipErrorInvalidValue;
    if (a.R <= 128) hipLaunchKernelGGL((k_update_rows<HT, 2>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_update_rows<HT, 4>), grid, block, 0, st, a);
    hipLaunchKernelGGL((k_update_finish<HT>), dim3(1), dim3(1024), 0, st, a, nb);
  }
  return hipGetLastError();
}

int norm_workgroups(int64_t I, int64_t *rows_per_wg) {
  int64_t nw = (I + 15) / 16;
  nw = nw < 1 ? 1 : (nw > kNormWG ? kNormWG : nw);
  const int64_t rpw = (I + nw - 1) / nw;
  if (rows_per_wg) *rows_per_wg = rpw;
  return (int)((I + rpw - 1) / rpw);
}

hipError_t launch_update(int hdt, const UpdateArgs &a, hipStream_t st, GramJob *job) {
  return hdt == NNCP_F64 ? update_dispatch<double>(a, st, job) : update_dispatch<float>(a, st, job);
}

hipError_t launch_sweep_normalize(int hdt, const FactorSet &F, const int64_t *dims, int N, int R,
                                  double *G, double *lambda, double *scale, hipStream_t st) {
  ScaleArgs a;
  a.N = N;
  a.R = R;
  a.off[0] = 0;
  for (int k = 0; k < NNCP_MAX_MODES; ++k) {
    a.H[k] = k < N ? const_cast<void *>(F.H[k]) : nullptr;
    if (k < N) a.off[k + 1] = a.off[k] + dims[k] * R;
  }
  hipLaunchKernelGGL(k_norm_scales, dim3(1), dim3(256), 0, st, G, N, R, lambda, scale);
  const int64_t total = a.off[N] + (int64_t)N * R * R;
  dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (hdt == NNCP_F64)
    hipLaunchKernelGGL(k_apply_scales<double>, grid, block, 0, st, a, G, scale);
  else
    hipLaunchKernelGGL(k_apply_scales<float>, grid, block, 0, st, a, G, scale);
  return hipGetLastError();
}

hipError_t launch_gram_finish(const GramJob &j, hipStream_t st) {
  if (j.R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_finish, dim3(gram_blocks(j)), dim3(256), 0, st, j);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Outer extrapolation of the Nesterov-type sweeps (Section 4.3.5, Eq.
// eqn:nesouterupd): the candidate F + s (F - F_prev), clipped at 0, for
// F = H (and H diag(lambda) for the last mode), its normalisation and Gram
// through the update's norm kernel and Gram step, then an accept step that
// takes the candidate only when its squared relative error is lower.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T *__restrict__ src, T *__restrict__ dst,
                                              int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

// one row per wave, 4 rows per workgroup; lane c owns entry c.  Writes the
// clipped candidate (FP64) and, per workgroup, the column sums of squares of
// its rows added in wave order (the row kernel's partial layout, beta = 0).
template <typename HT>
__global__ __launch_bounds__(256) void k_nes_extrap(const HT *__restrict__ H,
                                                    const HT *__restrict__ Hp,
                                                    const double *__restrict__ lam,
                                                    const double *__restrict__ lamp, int last,
                                                    const double *__restrict__ count, double invN,
                                                    int64_t I, int R,
                                                    double *__restrict__ raw,
                                                    double *__restrict__ part) {
  __shared__ double wred[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  const bool ok = i < I && lane < R;
  // s_i = i^(1/N) for outer iteration i = (outer steps taken so far) + 1
  const double s = pow(count[0] + 1.0, invN);
  double sq = 0.0;
  if (ok) {
    const double f = (double)H[i * R + lane] * (last ? lam[lane] : 1.0);
    const double fp = (double)Hp[i * R + lane] * (last ? lamp[lane] : 1.0);
    double v = f + s * (f - fp);
    v = v > 0.0 ? v : 0.0;
    raw[i * R + lane] = v;
    sq = v * v;
  }
  wred[wave][lane] = sq;
  __syncthreads();
  double *cpart = part + (int64_t)blockIdx.x * (R + 1);
  if (threadIdx.x < R)
    cpart[threadIdx.x] = wred[0][threadIdx.x] + wred[1][threadIdx.x] + wred[2][threadIdx.x] +
                         wred[3][threadIdx.x];
  if (threadIdx.x == 0) cpart[R] = 0.0;
}

// lambda_c(r) = prod over modes of the candidate's column norms, in mode order;
// also counts the outer step (every extrapolation kernel of this step has run)
__global__ __launch_bounds__(64) void k_nes_lamc(const double *__restrict__ lamk, int N, int R,
                                                 double *__restrict__ lamc,
                                                 double *__restrict__ count) {
  const int r = threadIdx.x;
  if (r == 0) count[0] += 1.0;
  if (r >= R) return;
  double p = 1.0;
  for (int k = 0; k < N; ++k) p *= lamk[(int64_t)k * R + r];
  lamc[r] = p;
}

// every thread takes the same decision from the two squared errors
template <typename T>
__global__ __launch_bounds__(256) void k_nes_accept(const T *__restrict__ src, T *__restrict__ dst,
                                                    int64_t n, const double *__restrict__ cand_e2,
                                                    const double *__restrict__ cur_e2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n && cand_e2[0] < cur_e2[0]) dst[e] = src[e];
}

__global__ __launch_bounds__(256) void k_nes_accept_hist(const double *__restrict__ cand_e2,
                                                         const double *__restrict__ cur_e2,
                                                         const double *__restrict__ cand_rel,
                                                         double *__restrict__ hist) {
  if (threadIdx.x == 0 && cand_e2[0] < cur_e2[0]) hist[0] = cand_rel[0];
}

hipError_t launch_copy(size_t elem_bytes, const void *src, void *dst, int64_t n, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (n <= 0) return hipSuccess;
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_copy<double>, grid, block, 0, st, (const double *)src, (double *)dst, n);
  else
    hipLaunchKernelGGL(k_copy<float>, grid, block, 0, st, (const float *)src, (float *)dst, n);
  return hipGetLastError();
}

hipError_t launch_nes_extrap(int hdt, const void *H, const void *Hp, const double *lam,
                             const double *lamp, int last, const double *count, int N, int64_t I,
                             int R, double *raw, double *part, int *nblocks, hipStream_t st) {
  if (R > 64) return hipErrorInvalidValue;
  const int nb = (int)((I + 3) / 4);
  *nblocks = nb;
  const double invN = 1.0 / N;
  if (hdt == NNCP_F64)
    hipLaunchKernelGGL(k_nes_extrap<double>, dim3(nb), dim3(256), 0, st, (const double *)H,
                       (const double *)Hp, lam, lamp, last, count, invN, I, R, raw, part);
  else
    hipLaunchKernelGGL(k_nes_extrap<float>, dim3(nb), dim3(256), 0, st, (const float *)H,
                       (const float *)Hp, lam, lamp, last, count, invN, I, R, raw, part);
  return hipGetLastError();
}

hipError_t launch_nes_lamc(const double *lamk, int N, int R, double *lamc, double *count,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_nes_lamc, dim3(1), dim3(64), 0, st, lamk, N, R, lamc, count);
  return hipGetLastError();
}

// p[0 .. n) = v
__global__ __launch_bounds__(256) void k_fill(double *__restrict__ p, double v, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = v;
}

hipError_t launch_fill(double *p, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_nes_accept(size_t elem_bytes, const void *src, void *dst, int64_t n,
                             const double *cand_e2, const double *cur_e2, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_nes_accept<double>, grid, block, 0, st, (const double *)src,
                       (double *)dst, n, cand_e2, cur_e2);
  else
    hipLaunchKernelGGL(k_nes_accept<float>, grid, block, 0, st, (const float *)src, (float *)dst,
                       n, cand_e2, cur_e2);
  return hipGetLastError();
}

hipError_t launch_nes_accept_hist(const double *cand_e2, const double *cur_e2,
                                  const double *cand_rel, double *hist, hipStream_t st) {
  if (!hist) return hipSuccess;
  hipLaunchKernelGGL(k_nes_accept_hist, dim3(1), dim3(64), 0, st, cand_e2, cur_e2, cand_rel, hist);
  return hipGetLastError();
}

// The norm kernel and Gram job alone (R <= 64), for rows given as Hhat and
// per-workgroup partials from another kernel.
hipError_t launch_norm_only(int hdt, const UpdateArgs &a, int nblocks, hipStream_t st,
                            GramJob *job) {
  if (a.R > 64) return hipErrorInvalidValue;
  int64_t rpw;
  const int nw = norm_workgroups(a.I, &rpw);
  *job = GramJob{};
  job->gpart = a.gpart;
  job->pn = a.gpart + norm_pn_offset(a.R);
  job->G = a.G;
  job->S = a.S;
  job->S_next = a.S_next;
  job->lambda = a.lambda;
  job->beta = a.beta_out;
  job->alpha = a.alpha;
  job->relerr_out = a.relerr_out;
  job->scal = a.scal;
  job->R = a.R;
  job->N = a.N;
  job->mode = a.mode;
  job->next_mode = a.next_mode;
  job->nw = nw;
#define NNCP_NORM_ONLY(HTV, RBV)                                                                     \
  {                                                                                                  \
    if (a.R == RBV)                                                                                  \
      hipLaunchKernelGGL((k_update_norm<HTV, RBV, true>), dim3(nw), dim3(256), 0, st, a, nblocks, rpw); \
    else                                                                                             \
      hipLaunchKernelGGL((k_update_norm<HTV, RBV, false>), dim3(nw), dim3(256), 0, st, a, nblocks, rpw); \
  }
  if (hdt == NNCP_F64) {
    if (a.R <= 16) NNCP_NORM_ONLY(double, 16)
    else if (a.R <= 32) NNCP_NORM_ONLY(double, 32)
    else NNCP_NORM_ONLY(double, 64)
  } else {
    if (a.R <= 16) NNCP_NORM_ONLY(float, 16)
    else if (a.R <= 32) NNCP_NORM_ONLY(float, 32)
    else NNCP_NORM_ONLY(float, 64)
  }
#undef NNCP_NORM_ONLY
  return hipGetLastError();
}

int64_t update_part_elems(int64_t I, int R) {
  // one row per workgroup at the most (the BPP kernel at R > 32)
  return I * (int64_t)(R + 1);
}

hipError_t launch_loss(int hdt, int N, int R, int64_t In, const void *M, const void *H,
                       const double *lambda, const double *G, const double *alpha, double *loss,
                       double *relerr, double *scal, hipStream_t st) {
  if (hdt == NNCP_F64)
    hipLaunchKernelGGL(k_loss<double>, dim3(1), dim3(1024), 0, st, N, R, In, (const double *)M,
                       (const double *)H, lambda, G, alpha, loss, relerr, scal);
  else
    hipLaunchKernelGGL(k_loss<float>, dim3(1), dim3(1024), 0, st, N, R, In, (const float *)M,
                       (const float *)H, lambda, G, alpha, loss, relerr, scal);
  return hipGetLastError();
}

hipError_t launch_grad_all(int hdt, GradAllArgs a, hipStream_t st) {
  if (a.R > 64 || a.N < 2 || a.N > NNCP_MAX_MODES) return hipErrorInvalidValue;
  a.wg0[0] = 0;
  for (int n = 0; n < a.N; ++n) a.wg0[n + 1] = a.wg0[n] + (int)((a.I[n] * a.R + 255) / 256);
  dim3 grid((unsigned)a.wg0[a.N] + 1), block(256);
  if (hdt == NNCP_F64) hipLaunchKernelGGL(k_grad_all<double>, grid, block, 0, st, a);
  else hipLaunchKernelGGL(k_grad_all<float>, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_grad(int hdt, int64_t I, int R, int N, int mode, const void *M, int msplit,
                       int64_t mstride, const void *H, const double *G, const double *S,
                       void *grad, hipStream_t st) {
  const int64_t n = I * R;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (R > 64 && !S) return hipErrorInvalidValue;
  if (hdt == NNCP_F64)
    hipLaunchKernelGGL(k_grad<double>, grid, block, 0, st, I, R, N, mode, (const double *)M, msplit, mstride,
                       (const double *)H, G, S, (double *)grad);
  else
    hipLaunchKernelGGL(k_grad<float>, grid, block, 0, st, I, R, N, mode, (const float *)M, msplit, mstride,
                       (const float *)H, G, S, (float *)grad);
  return hipGetLastError();
}

hipError_t launch_pgd_eta(const double *G, int N, int R, int iters, double *eta, hipStream_t st) {
  if (R > 64) return hipErrorInvalidValue;
#define NNCP_PGD_ETA(RBV)                                                                           \
  {                                                                                                 \
    if (R == RBV)                                                                                   \
      hipLaunchKernelGGL((k_pgd_eta<RBV, true>), dim3(1), dim3(512), 0, st, G, N, R, iters, eta);  \
    else                                                                                            \
      hipLaunchKernelGGL((k_pgd_eta<RBV, false>), dim3(1), dim3(512), 0, st, G, N, R, iters, eta); \
  }
  if (R <= 16) NNCP_PGD_ETA(16)
  else if (R <= 32) NNCP_PGD_ETA(32)
  else NNCP_PGD_ETA(64)
#undef NNCP_PGD_ETA
  return hipGetLastError();
}

hipError_t launch_pgd_trial(int hdt, int64_t n, const void *H, const void *g, double eta, void *Hn,
                            double *part, double *d_out, hipStream_t st) {
  const int nb = 256;
  if (hdt == NNCP_F64)
    hipLaunchKernelGGL(k_pgd_trial<double>, dim3(nb), dim3(256), 0, st, n, (const double *)H,
                       (const double *)g, eta, (double *)Hn, part);
  else
    hipLaunchKernelGGL(k_pgd_trial<float>, dim3(nb), dim3(256), 0, st, n, (const float *)H,
                       (const float *)g, eta, (float *)Hn, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, part, nb, d_out);
  return hipGetLastError();
}

}  // namespace nncp
