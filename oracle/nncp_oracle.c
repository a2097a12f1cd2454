/*
 * nncp_oracle.c -- reference implementation of dense nonnegative CP (NNCP)
 * by alternating updates, in plain C and FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and the GPU library never calls it.
 *
 * Everything is computed from the plain definitions in the paper (PLANC,
 * arXiv 1909.01149), with no blocking, fusion or dimension tree:
 *   - the objective, Eq. (eqn:nncp), Section 1;
 *   - the alternating-update outer/inner iteration, Algorithm 1 (alg:nncp);
 *   - MTTKRP M^(n) = X_(n) (H^(N) kr ... kr H^(n+1) kr H^(n-1) kr ... kr H^(1)),
 *     Appendix "Factor Matrix Normalization" and Section 4.2.1 (3-way example);
 *   - Gram G^(n) = H^(n)^T H^(n) and S^(n) = Hadamard product of the other
 *     Grams, Algorithm 1;
 *   - MU rule, Eq. (eqn:muupd); HALS rule, Eq. (eqn:halsupd), Section 4.3;
 *   - BPP (exact NNLS per row, Eq. (eqn:snls) and its KKT conditions),
 *     Section 4.3.3, with the pivoting rule of the method the paper cites;
 *   - ADMM, Eqs. (eqn:admmnls), (eqn:admmupd), Section 4.3.4 (at most 5
 *     passes, rho = trace(S)/R, the stopping test of the cited method);
 *   - the Nesterov-type update, Eqs. (eqn:nesnls), (eqn:nesinnerupd),
 *     Section 4.3.5 (20 steps, with the step parameters read below);
 *   - column normalisation with weights lambda, Appendix "Factor Matrix
 *     Normalization" and Algorithm 4 (alg:Par-NNCP-long);
 *   - relative error through the identity
 *     ||X-M||^2 = ||X||^2 - 2<M^(N), Hhat^(N)> + lambda^T (S^(N) * G^(N)) lambda,
 *     Appendix "Relative Error Computation" and Algorithm 4.
 *
 * Readings where the paper is silent or inconsistent (each one is listed in
 * the design notes of the repository):
 *   - lambda is folded into the factor being updated before the update,
 *     because the appendix states that the solve actually computes H^(n) Lambda;
 *   - MU adds eps (default 1e-16) to the denominator; the paper only asks
 *     for some small positive guard;
 *   - HALS divides by S(r,r) as in Eq. (eqn:halsupd) and skips a column whose
 *     S(r,r) is 0; columns are updated in order 1..R using the latest values;
 *   - HALS normalisation happens once after the whole update (Algorithm 4),
 *     not after every column;
 *   - all N factors are given as the start iterate (Algorithm 1 initialises
 *     only modes 2..N, but MU and HALS need a start value for mode 1 as well);
 *   - a zero column stays zero with lambda_r = 0;
 *   - the ADMM dual U of each mode starts at zero and is kept from one
 *     update of that mode to the next (it lives with the solver, like the
 *     auxiliary variables the paper's solver classes hold);
 *   - the Nesterov-type update: the gradient's sign is that of the objective
 *     (the printed one is flipped); lambda, alpha, beta follow the rule in
 *     orc_nes_params; every update takes exactly 20 steps;
 *   - the outer extrapolation of Eq. (eqn:nesouterupd) (sweeps with
 *     ORC_NES_OUTER) acts on H^(n) for n < N-1 and H^(N-1) diag(lambda),
 *     clips the candidate at 0 and normalises it, uses s_i = i^(1/N) with
 *     i the outer-iteration number (1 for the first sweep from a fresh
 *     start; a caller continuing an earlier run passes its next number),
 *     and compares squared relative errors;
 *   - the squared relative error is clamped at 0 before the square root.
 *
 * Layouts: the tensor is stored with mode 0 varying fastest (the local
 * storage order of Section 4.1.2, column-major carried to N modes), so the
 * linear index of (i_0, ..., i_{N-1}) is i_0 + I_0 (i_1 + I_1 (i_2 + ...)).
 * A factor H^(n) is I_n x R, row-major (entry (i, r) at i*R + r).  Modes are
 * 0-based here; the paper numbers them from 1.
 *
 * Parity status: every function here is pinned by CPU tests against closed
 * forms, brute force (explicit unfolding times explicit Khatri-Rao product),
 * invariants or finite differences; see tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 16

/* ------------------------------------------------------------------ */
/* helpers: multi-index bookkeeping                                     */
/* ------------------------------------------------------------------ */

static int64_t prod_dims(int N, const int64_t *dims) {
  int64_t p = 1;
  for (int k = 0; k < N; ++k) p *= dims[k];
  return p;
}

/* linear index -> multi-index, mode 0 fastest */
static void unravel(int N, const int64_t *dims, int64_t lin, int64_t *idx) {
  for (int k = 0; k < N; ++k) {
    idx[k] = lin % dims[k];
    lin /= dims[k];
  }
}

/* advance a multi-index by one position in memory order */
static void advance(int N, const int64_t *dims, int64_t *idx) {
  for (int k = 0; k < N; ++k) {
    if (++idx[k] < dims[k]) return;
    idx[k] = 0;
  }
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* MTTKRP by its definition                                             */
/* ------------------------------------------------------------------ */

/*
 * M^(n)[i_n, r] = sum over every entry of X whose mode-n index is i_n of
 *                 X[i_0..i_{N-1}] * prod_{k != n} H^(k)[i_k, r].
 * This is the mode-n matricized tensor times the Khatri-Rao product of all
 * other factors, written entrywise (Section 4.2.1; Appendix, normalisation
 * paragraph).  One pass over X in memory order; when nthreads > 1 the pass is
 * cut into nthreads contiguous ranges, each thread accumulates into its own
 * copy of M, and the copies are added in thread order (so a given nthreads
 * always gives the same bits).
 */
int orc_mttkrp(int N, const int64_t *dims, int R, const double *X,
               const double *const *H, int mode, double *M, int nthreads) {
  if (N < 1 || N > ORC_MAXN || R < 1 || mode < 0 || mode >= N) return -1;
  const int64_t I = prod_dims(N, dims);
  const int64_t In = dims[mode];
  if (nthreads < 1) nthreads = 1;
  double *priv = (double *)calloc((size_t)nthreads * (size_t)(In * R), sizeof(double));
  if (!priv) return -2;

#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
#endif
  for (int t = 0; t < nthreads; ++t) {
    const int64_t lo = I * t / nthreads, hi = I * (t + 1) / nthreads;
    double *Mt = priv + (size_t)t * (size_t)(In * R);
    int64_t idx[ORC_MAXN];
    if (lo < hi) unravel(N, dims, lo, idx);
    for (int64_t lin = lo; lin < hi; ++lin) {
      const double x = X[lin];
      for (int r = 0; r < R; ++r) {
        double p = x;
        for (int k = 0; k < N; ++k)
          if (k != mode) p *= H[k][idx[k] * R + r];
        Mt[idx[mode] * R + r] += p;
      }
      advance(N, dims, idx);
    }
  }
  for (int64_t e = 0; e < In * R; ++e) {
    double s = 0.0;
    for (int t = 0; t < nthreads; ++t) s += priv[(size_t)t * (size_t)(In * R) + e];
    M[e] = s;
  }
  free(priv);
  return 0;
}

/*
 * Selected rows of M^(n): for each requested i_n, sum over the (I / I_n)
 * entries whose mode-n index is i_n.  Same definition as orc_mttkrp, used to
 * check full-size problems row by row.
 */
int orc_mttkrp_rows(int N, const int64_t *dims, int R, const double *X,
                    const double *const *H, int mode, const int64_t *rows,
                    int nrows, double *out, int nthreads) {
  if (N < 1 || N > ORC_MAXN || R < 1 || mode < 0 || mode >= N) return -1;
  /* the other modes, in memory order */
  int64_t odims[ORC_MAXN];
  int omodes[ORC_MAXN], no = 0;
  for (int k = 0; k < N; ++k)
    if (k != mode) { odims[no] = dims[k]; omodes[no] = k; ++no; }
  int64_t stride[ORC_MAXN];
  stride[0] = 1;
  for (int k = 1; k < N; ++k) stride[k] = stride[k - 1] * dims[k - 1];
  const int64_t J = prod_dims(no, odims);
  if (nthreads < 1) nthreads = 1;

  for (int q = 0; q < nrows; ++q) {
    const int64_t in = rows[q];
    if (in < 0 || in >= dims[mode]) return -1;
    double *priv = (double *)calloc((size_t)nthreads * (size_t)R, sizeof(double));
    if (!priv) return -2;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
#endif
    for (int t = 0; t < nthreads; ++t) {
      const int64_t lo = J * t / nthreads, hi = J * (t + 1) / nthreads;
      double *acc = priv + (size_t)t * R;
      int64_t oidx[ORC_MAXN];
      if (lo < hi) unravel(no, odims, lo, oidx);
      for (int64_t j = lo; j < hi; ++j) {
        int64_t lin = in * stride[mode];
        for (int a = 0; a < no; ++a) lin += oidx[a] * stride[omodes[a]];
        const double x = X[lin];
        for (int r = 0; r < R; ++r) {
          double p = x;
          for (int a = 0; a < no; ++a) p *= H[omodes[a]][oidx[a] * R + r];
          acc[r] += p;
        }
        advance(no, odims, oidx);
      }
    }
    for (int r = 0; r < R; ++r) {
      double s = 0.0;
      for (int t = 0; t < nthreads; ++t) s += priv[(size_t)t * R + r];
      out[(size_t)q * R + r] = s;
    }
    free(priv);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Gram, Hadamard of Grams, sum of squares                              */
/* ------------------------------------------------------------------ */

/* G = H^T H for an I x R row-major H (Algorithm 1, Gram lines). */
void orc_gram(int64_t I, int R, const double *H, double *G) {
  for (int a = 0; a < R; ++a)
    for (int b = 0; b < R; ++b) {
      double s = 0.0;
      for (int64_t i = 0; i < I; ++i) s += H[i * R + a] * H[i * R + b];
      G[a * R + b] = s;
    }
}

/* S = Hadamard product of G[k] over k != mode (Algorithm 1, S^(n) line). */
void orc_hadamard_except(int N, int R, const double *const *G, int mode, double *S) {
  for (int e = 0; e < R * R; ++e) {
    double s = 1.0;
    for (int k = 0; k < N; ++k)
      if (k != mode) s *= G[k][e];
    S[e] = s;
  }
}

double orc_sumsq(int64_t n, const double *X) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += X[i] * X[i];
  return s;
}

/* ------------------------------------------------------------------ */
/* factor updates on Hhat = H^(n) diag(lambda)                          */
/* ------------------------------------------------------------------ */

/*
 * Multiplicative update, Eq. (eqn:muupd) written for the factor matrix
 * (X = H^T, A^T B = M^T, A^T A = S):
 *   Hhat[i,r] <- Hhat[i,r] * M[i,r] / ((Hhat S)[i,r] + eps).
 * All entries use the Hhat from before the update.
 */
void orc_update_mu(int64_t I, int R, double *Hhat, const double *M,
                   const double *S, double eps) {
  double *old = (double *)malloc(sizeof(double) * (size_t)R);
  for (int64_t i = 0; i < I; ++i) {
    for (int c = 0; c < R; ++c) old[c] = Hhat[i * R + c];
    for (int r = 0; r < R; ++r) {
      double hs = 0.0;
      for (int c = 0; c < R; ++c) hs += old[c] * S[c * R + r];
      Hhat[i * R + r] = old[r] * M[i * R + r] / (hs + eps);
    }
  }
  free(old);
}

/*
 * HALS, Eq. (eqn:halsupd) written for the factor matrix: for r = 0..R-1 in
 * order, column r of Hhat becomes
 *   max(0, Hhat[:,r] + (M[:,r] - (Hhat S)[:,r]) / S[r,r]),
 * where Hhat already holds the new columns 0..r-1.  A column with S[r,r] = 0
 * is left unchanged.
 */
void orc_update_hals(int64_t I, int R, double *Hhat, const double *M, const double *S) {
  for (int r = 0; r < R; ++r) {
    const double d = S[r * R + r];
    if (!(d > 0.0)) continue;
    for (int64_t i = 0; i < I; ++i) {
      double hs = 0.0;
      for (int c = 0; c < R; ++c) hs += Hhat[i * R + c] * S[c * R + r];
      const double v = Hhat[i * R + r] + (M[i * R + r] - hs) / d;
      Hhat[i * R + r] = v > 0.0 ? v : 0.0;
    }
  }
}

/*
 * BPP, Section 4.3.3 with Eq. (eqn:snls): each row x of Hhat becomes the
 * exact solution of the single right-hand-side NNLS problem
 *   min_{x >= 0} 1/2 x^T S x - m^T x      (A^T A = S, A^T b = m = row of M),
 * whose KKT conditions are x >= 0, y = S x - m >= 0, x_i y_i = 0.  The
 * active set is found by block principal pivoting (Kim and Park, 2011): with
 * a passive set F, x_F solves S_FF x_F = m_F by a Cholesky factorisation of
 * S_FF, x is 0 off F and y = S x - m off F (0 on F).  The search starts from
 * the support of the row's current value (F = {i : x_i > 0}, solved once; an
 * empty F starts from x = 0, y = -m), as alternating NNLS solvers do between
 * outer iterations.  Every index breaking the conditions (x_i < 0 on F,
 * y_i < 0 off F) switches sets while their count keeps falling; after the
 * count stops falling three more full switches are allowed, then only the
 * largest such index switches until the count falls again.  The search ends
 * when no index breaks the conditions, after 5 R + 10 solves, or when S_FF
 * is not positive definite (then the last x, clipped at 0, is kept; a start
 * set that fails this way is replaced by the empty set).  x is the start
 * value on entry and the solution on exit.  Returns the number of solves,
 * or -1 if the search ended without meeting the conditions.
 * work: R*R + 4*R doubles.
 */
static int bpp_solve(int R, const double *S, const double *m, const double *passive,
                     double *x, double *y, double *L, double *z, double *idx) {
  int f = 0;
  for (int i = 0; i < R; ++i)
    if (passive[i] != 0.0) idx[f++] = (double)i;
  /* S_FF = L L^T, then L z = m_F and L^T x_F = z */
  for (int a = 0; a < f; ++a) {
    const int ia = (int)idx[a];
    for (int b = 0; b <= a; ++b) {
      const int ib = (int)idx[b];
      double v = S[ia * R + ib];
      for (int c = 0; c < b; ++c) v -= L[a * R + c] * L[b * R + c];
      if (b == a) {
        if (!(v > 0.0)) return 0;
        L[a * R + a] = sqrt(v);
      } else {
        L[a * R + b] = v / L[b * R + b];
      }
    }
  }
  for (int a = 0; a < f; ++a) {
    double v = m[(int)idx[a]];
    for (int c = 0; c < a; ++c) v -= L[a * R + c] * z[c];
    z[a] = v / L[a * R + a];
  }
  for (int a = f - 1; a >= 0; --a) {
    double v = z[a];
    for (int c = a + 1; c < f; ++c) v -= L[c * R + a] * z[c];
    z[a] = v / L[a * R + a];
  }
  for (int i = 0; i < R; ++i) x[i] = 0.0;
  for (int a = 0; a < f; ++a) x[(int)idx[a]] = z[a];
  for (int i = 0; i < R; ++i) {
    if (passive[i] != 0.0) { y[i] = 0.0; continue; }
    double v = -m[i];
    for (int a = 0; a < f; ++a) v += S[i * R + (int)idx[a]] * z[a];
    y[i] = v;
  }
  return 1;
}

int orc_bpp_row(int R, const double *S, const double *m, double *x, double *work) {
  double *L = work;            /* R x R, row-major, lower triangle */
  double *y = L + R * R;
  double *z = y + R;
  double *passive = z + R;     /* 1.0 on F, 0.0 off F */
  double *idx = passive + R;   /* F's indices in increasing order */
  int f0 = 0, solves = 0;
  for (int i = 0; i < R; ++i) {
    passive[i] = x[i] > 0.0 ? 1.0 : 0.0;
    f0 += x[i] > 0.0;
  }
  if (f0 > 0) {
    ++solves;
    if (!bpp_solve(R, S, m, passive, x, y, L, z, idx)) f0 = 0;
  }
  if (f0 == 0) {
    for (int i = 0; i < R; ++i) {
      x[i] = 0.0;
      y[i] = -m[i];
      passive[i] = 0.0;
    }
  }
  int ninf = R + 1, backup = 3;
  const int maxsolves = 5 * R + 10;
  for (;;) {
    int nv = 0, last = -1;
    for (int i = 0; i < R; ++i) {
      const int bad = passive[i] != 0.0 ? (x[i] < 0.0) : (y[i] < 0.0);
      if (bad) { ++nv; last = i; }
    }
    if (nv == 0) return solves;
    if (solves >= maxsolves) break;
    int full;
    if (nv < ninf) { ninf = nv; backup = 3; full = 1; }
    else if (backup >= 1) { --backup; full = 1; }
    else full = 0;
    for (int i = 0; i < R; ++i) {
      const int bad = passive[i] != 0.0 ? (x[i] < 0.0) : (y[i] < 0.0);
      if (bad && (full || i == last)) passive[i] = passive[i] != 0.0 ? 0.0 : 1.0;
    }
    ++solves;
    if (!bpp_solve(R, S, m, passive, x, y, L, z, idx)) break;
  }
  for (int i = 0; i < R; ++i) x[i] = x[i] > 0.0 ? x[i] : 0.0;
  return -1;
}

/* BPP for every row of Hhat, each search starting from the row's current
 * support.  Returns the number of rows whose search ended without meeting
 * the KKT conditions. */
int64_t orc_update_bpp(int64_t I, int R, double *Hhat, const double *M, const double *S) {
  double *work = (double *)malloc(sizeof(double) * (size_t)(R * R + 4 * R));
  int64_t failed = 0;
  for (int64_t i = 0; i < I; ++i)
    if (orc_bpp_row(R, S, M + i * R, Hhat + i * R, work) < 0) ++failed;
  free(work);
  return failed;
}

/*
 * ADMM, Section 4.3.4 with Eqs. (eqn:admmnls) and (eqn:admmupd), written for
 * the factor (H = X^T, A^T A = S, A^T B = M^T), with the scaled dual U:
 *   rho   = trace(S) / R                     (||A||_F^2 / R)
 *   Ht    = (M + rho (H + U)) (S + rho I)^-1  (Cholesky of S + rho I, once)
 *   H     = max(0, Ht - U)
 *   U     = U + H - Ht
 * repeated at most maxit times; after each pass the stopping test of the
 * cited method is taken on the whole factor:
 *   r = ||H - Ht||_F^2 / ||H||_F^2 < tol  and  s = ||H - H_prev||_F^2 / ||U||_F^2 < tol
 * (a zero denominator counts as passing only when its numerator is 0).
 * Hhat (the start value) and U are updated in place.  Returns the number of
 * passes, or -1 if S + rho I is not positive definite (Hhat unchanged).
 */
int orc_update_admm(int64_t I, int R, double *Hhat, double *U, const double *M,
                    const double *S, int maxit, double tol) {
  double tr = 0.0;
  for (int r = 0; r < R; ++r) tr += S[r * R + r];
  const double rho = tr / R;
  double *L = (double *)malloc(sizeof(double) * (size_t)R * R);
  double *z = (double *)malloc(sizeof(double) * (size_t)R);
  double *Ht = (double *)malloc(sizeof(double) * (size_t)(I * R));
  double *Hp = (double *)malloc(sizeof(double) * (size_t)(I * R));
  int rc = 0;
  /* S + rho I = L L^T */
  for (int a = 0; a < R && rc == 0; ++a) {
    for (int b = 0; b <= a; ++b) {
      double v = S[a * R + b] + (a == b ? rho : 0.0);
      for (int c = 0; c < b; ++c) v -= L[a * R + c] * L[b * R + c];
      if (b == a) {
        if (!(v > 0.0)) { rc = -1; break; }
        L[a * R + a] = sqrt(v);
      } else {
        L[a * R + b] = v / L[b * R + b];
      }
    }
  }
  int pass = 0;
  while (rc == 0 && pass < maxit) {
    ++pass;
    double nd = 0.0, nh = 0.0, nc = 0.0, nu = 0.0;
    for (int64_t i = 0; i < I; ++i) {
      double *h = Hhat + i * R, *u = U + i * R, *t = Ht + i * R;
      /* (S + rho I) t^T = (m + rho (h + u))^T: L z = ., L^T t = z */
      for (int a = 0; a < R; ++a) {
        double v = M[i * R + a] + rho * (h[a] + u[a]);
        for (int c = 0; c < a; ++c) v -= L[a * R + c] * z[c];
        z[a] = v / L[a * R + a];
      }
      for (int a = R - 1; a >= 0; --a) {
        double v = z[a];
        for (int c = a + 1; c < R; ++c) v -= L[c * R + a] * z[c];
        z[a] = v / L[a * R + a];
      }
      for (int a = 0; a < R; ++a) {
        t[a] = z[a];
        Hp[i * R + a] = h[a];
        const double hn = t[a] - u[a] > 0.0 ? t[a] - u[a] : 0.0;
        h[a] = hn;
        u[a] += hn - t[a];
      }
    }
    for (int64_t e = 0; e < I * R; ++e) {
      const double d = Hhat[e] - Ht[e], c = Hhat[e] - Hp[e];
      nd += d * d;
      nh += Hhat[e] * Hhat[e];
      nc += c * c;
      nu += U[e] * U[e];
    }
    const int rok = nh > 0.0 ? nd / nh < tol : nd == 0.0;
    const int sok = nu > 0.0 ? nc / nu < tol : nc == 0.0;
    if (rok && sok) break;
  }
  free(L);
  free(z);
  free(Ht);
  free(Hp);
  return rc == 0 ? pass : -1;
}

/* largest eigenvalue of a symmetric matrix by power steps (defined below) */
double orc_power_lmax(int R, const double *A, int iters);

/*
 * Step parameters of the Nesterov-type update (Section 4.3.5).  The paper
 * ties lambda, alpha and beta to the singular values of A (here the
 * eigenvalues of S = A^T A) and leaves the rule to the method it cites; the
 * reading used here:
 *   L  = largest eigenvalue of S, by `power` power steps from the all-ones
 *        vector (orc_power_lmax),
 *   mu = L minus the largest eigenvalue of L I - S found the same way,
 *        at least 0 (an estimate of the smallest eigenvalue of S from above),
 *   lam = max(0, (L - kappa mu) / (kappa - 1)), the smallest proximal weight
 *        that brings the condition number of S + lam I down to kappa,
 *   alpha = 1 / (L + lam),
 *   beta = (1 - sqrt(q)) / (1 + sqrt(q)), q = (mu + lam) / (L + lam), the
 *        constant momentum of the accelerated gradient method for a
 *        strongly convex objective.
 * out: [L, mu, lam, alpha, beta].  Returns 0, or -1 when L is not positive
 * (out[3] = out[4] = 0).
 */
int orc_nes_params(int R, const double *S, int power, double kappa, double *out) {
  const double L = orc_power_lmax(R, S, power);
  double *T = (double *)malloc(sizeof(double) * (size_t)R * R);
  for (int a = 0; a < R; ++a)
    for (int b = 0; b < R; ++b) T[a * R + b] = (a == b ? L : 0.0) - S[a * R + b];
  const double lt = orc_power_lmax(R, T, power);
  free(T);
  double mu = L - lt;
  if (!(mu > 0.0)) mu = 0.0;
  double lam = (L - kappa * mu) / (kappa - 1.0);
  if (!(lam > 0.0)) lam = 0.0;
  out[0] = L;
  out[1] = mu;
  out[2] = lam;
  if (!(L > 0.0)) {
    out[3] = out[4] = 0.0;
    return -1;
  }
  const double q = sqrt((mu + lam) / (L + lam));
  out[3] = 1.0 / (L + lam);
  out[4] = (1.0 - q) / (1.0 + q);
  return 0;
}

/*
 * Nesterov-type update, Section 4.3.5 with Eqs. (eqn:nesnls) and
 * (eqn:nesinnerupd), written for the rows x of the factor (A^T A = S,
 * A^T B = M^T) with x* the start value of the row:
 *   grad(y) = y S - m + lam (y - x*)
 * (the gradient of 1/2 ||A x - b||^2 + lam/2 ||x - x*||^2; the sign printed
 * in the paper is flipped), and
 *   x_0 = y_0 = x*,
 *   x_{k+1} = max(0, y_k - alpha grad(y_k)),
 *   y_{k+1} = x_{k+1} + beta (x_{k+1} - x_k),
 * for exactly `iters` steps (the paper's cap is 20; the stopping tests of the
 * cited method are not used), with the parameters of orc_nes_params.
 * Hhat holds the start value on entry and the result on exit.  Returns 0, or
 * -1 when L is not positive (Hhat unchanged).
 */
int orc_update_nes(int64_t I, int R, double *Hhat, const double *M, const double *S, int iters,
                   int power, double kappa) {
  double prm[5];
  if (orc_nes_params(R, S, power, kappa, prm) != 0) return -1;
  const double lam = prm[2], alpha = prm[3], beta = prm[4];
  double *xs = (double *)malloc(sizeof(double) * (size_t)R);
  double *x = (double *)malloc(sizeof(double) * (size_t)R);
  double *y = (double *)malloc(sizeof(double) * (size_t)R);
  double *xn = (double *)malloc(sizeof(double) * (size_t)R);
  for (int64_t i = 0; i < I; ++i) {
    double *h = Hhat + i * R;
    const double *m = M + i * R;
    for (int c = 0; c < R; ++c) xs[c] = x[c] = y[c] = h[c];
    for (int k = 0; k < iters; ++k) {
      for (int c = 0; c < R; ++c) {
        double g = 0.0;
        for (int r = 0; r < R; ++r) g += y[r] * S[r * R + c];
        g = g - m[c] + lam * (y[c] - xs[c]);
        const double v = y[c] - alpha * g;
        xn[c] = v > 0.0 ? v : 0.0;
      }
      for (int c = 0; c < R; ++c) {
        y[c] = xn[c] + beta * (xn[c] - x[c]);
        x[c] = xn[c];
      }
    }
    for (int c = 0; c < R; ++c) h[c] = x[c];
  }
  free(xs);
  free(x);
  free(y);
  free(xn);
  return 0;
}

/*
 * Column normalisation (Algorithm 4, column-norm and column-scale lines):
 * lambda_r = ||Hhat[:,r]||_2 and H[:,r] = Hhat[:,r] / lambda_r, or a zero
 * column with lambda_r = 0.
 */
void orc_normalize(int64_t I, int R, const double *Hhat, double *H, double *lambda) {
  for (int r = 0; r < R; ++r) {
    double s = 0.0;
    for (int64_t i = 0; i < I; ++i) s += Hhat[i * R + r] * Hhat[i * R + r];
    const double l = sqrt(s);
    lambda[r] = l;
    for (int64_t i = 0; i < I; ++i) H[i * R + r] = l > 0.0 ? Hhat[i * R + r] / l : 0.0;
  }
}

/* ------------------------------------------------------------------ */
/* alternating-update sweeps                                            */
/* ------------------------------------------------------------------ */

enum { ORC_MU = 0, ORC_HALS = 1, ORC_BPP = 2, ORC_ADMM = 3, ORC_NES = 4, ORC_NES_OUTER = 5 };
#define ORC_ADMM_MAXIT 5
#define ORC_ADMM_TOL 0.01
#define ORC_NES_ITERS 20
#define ORC_NES_POWER 20
#define ORC_NES_KAPPA 100.0

/*
 * The candidate of the outer extrapolation, Eq. (eqn:nesouterupd), from the
 * iterate after a sweep (H, lambda) and the iterate before it (Hp, lamp),
 * with step s_i: on F^(n) = H^(n) for n < N-1 and F^(N-1) = H^(N-1)
 * diag(lambda) (the same model with one set of weights),
 *   Fc^(n) = max(0, F^(n) + s_i (F^(n) - F_prev^(n))),
 * each Fc^(n) normalised into Hc[n] with its column norms multiplied into
 * lamc (so [[lamc; Hc]] = [[Fc]]).  Returns the candidate's squared relative
 * error through the identity of the appendix (one MTTKRP of mode N-1 and the
 * Grams of the candidate), alpha = ||X||^2.
 */
double orc_nes_outer_candidate(int N, const int64_t *dims, int R, const double *X,
                               const double *const *H, const double *lambda,
                               const double *const *Hp, const double *lamp, double si,
                               double alpha, double *const *Hc, double *lamc, int nthreads) {
  int64_t maxI = 0;
  for (int k = 0; k < N; ++k)
    if (dims[k] > maxI) maxI = dims[k];
  double *nrm = (double *)malloc(sizeof(double) * (size_t)R);
  double *Gc[ORC_MAXN];
  for (int r = 0; r < R; ++r) lamc[r] = 1.0;
  for (int k = 0; k < N; ++k) {
    const int last = k == N - 1;
    for (int64_t i = 0; i < dims[k]; ++i)
      for (int r = 0; r < R; ++r) {
        const double f = H[k][i * R + r] * (last ? lambda[r] : 1.0);
        const double fp = Hp[k][i * R + r] * (last ? lamp[r] : 1.0);
        const double v = f + si * (f - fp);
        Hc[k][i * R + r] = v > 0.0 ? v : 0.0;
      }
    orc_normalize(dims[k], R, Hc[k], Hc[k], nrm);
    for (int r = 0; r < R; ++r) lamc[r] *= nrm[r];
    Gc[k] = (double *)malloc(sizeof(double) * (size_t)R * R);
    orc_gram(dims[k], R, Hc[k], Gc[k]);
  }
  const int n = N - 1;
  const int64_t In = dims[n];
  double *M = (double *)malloc(sizeof(double) * (size_t)(maxI * R));
  orc_mttkrp(N, dims, R, X, (const double *const *)Hc, n, M, nthreads);
  double bc = 0.0, gc = 0.0;
  for (int64_t i = 0; i < In; ++i)
    for (int r = 0; r < R; ++r) bc += M[i * R + r] * Hc[n][i * R + r] * lamc[r];
  for (int a = 0; a < R; ++a)
    for (int b = 0; b < R; ++b) {
      double p = 1.0;
      for (int k = 0; k < N; ++k) p *= Gc[k][a * R + b];
      gc += lamc[a] * p * lamc[b];
    }
  for (int k = 0; k < N; ++k) free(Gc[k]);
  free(M);
  free(nrm);
  return (alpha - 2.0 * bc + gc) / alpha;
}

/*
 * nsweeps outer iterations of Algorithm 1 with the local steps of
 * Algorithm 4 (normalisation and relative error).  H[n] (I_n x R) and
 * lambda (R) are the start iterate on entry and the result on exit.
 * algo: ORC_MU, ORC_HALS, ORC_BPP, ORC_ADMM, ORC_NES, or ORC_NES_OUTER (the
 * Nesterov-type updates plus the outer extrapolation after every sweep).
 * relerr[s] receives the relative error after sweep s from the identity;
 * relerr2_raw[s] (may be NULL) the unclamped squared relative error.
 * first_sweep is the outer-iteration number i of the first of these sweeps
 * (1 for a fresh start); only the outer extrapolation uses it.
 * Returns 0, or a negative value on bad arguments.
 */
int orc_sweeps_from(int N, const int64_t *dims, int R, const double *X, double *const *H,
                    double *lambda, int algo, double eps_mu, int nsweeps, int64_t first_sweep,
                    double *relerr, double *relerr2_raw, int nthreads) {
  if (N < 2 || N > ORC_MAXN || R < 1 || nsweeps < 0 || first_sweep < 1) return -1;
  if (algo < ORC_MU || algo > ORC_NES_OUTER) return -1;
  const int64_t I = prod_dims(N, dims);
  double *G[ORC_MAXN];
  int64_t maxI = 0;
  for (int k = 0; k < N; ++k) {
    G[k] = (double *)malloc(sizeof(double) * (size_t)R * R);
    orc_gram(dims[k], R, H[k], G[k]);
    if (dims[k] > maxI) maxI = dims[k];
  }
  double *M = (double *)malloc(sizeof(double) * (size_t)(maxI * R));
  double *Hhat = (double *)malloc(sizeof(double) * (size_t)(maxI * R));
  /* ADMM duals, one per mode, zero at the start and kept across sweeps */
  double *Ud[ORC_MAXN];
  for (int k = 0; k < N; ++k)
    Ud[k] = algo == ORC_ADMM ? (double *)calloc((size_t)(dims[k] * R), sizeof(double)) : NULL;
  double *S = (double *)malloc(sizeof(double) * (size_t)R * R);
  const double alpha = orc_sumsq(I, X);
  /* outer extrapolation: the iterate before the sweep and the candidate */
  const int outer = algo == ORC_NES_OUTER;
  double *Hp[ORC_MAXN], *Hc[ORC_MAXN];
  double *lamp = (double *)malloc(sizeof(double) * (size_t)R);
  double *lamc = (double *)malloc(sizeof(double) * (size_t)R);
  for (int k = 0; k < N; ++k) {
    Hp[k] = outer ? (double *)malloc(sizeof(double) * (size_t)(dims[k] * R)) : NULL;
    Hc[k] = outer ? (double *)malloc(sizeof(double) * (size_t)(dims[k] * R)) : NULL;
  }

  for (int s = 0; s < nsweeps; ++s) {
    double beta = 0.0, gamma = 0.0;
    if (outer) {
      for (int k = 0; k < N; ++k) memcpy(Hp[k], H[k], sizeof(double) * (size_t)(dims[k] * R));
      memcpy(lamp, lambda, sizeof(double) * (size_t)R);
    }
    for (int n = 0; n < N; ++n) {
      const int64_t In = dims[n];
      orc_mttkrp(N, dims, R, X, (const double *const *)H, n, M, nthreads);
      orc_hadamard_except(N, R, (const double *const *)G, n, S);
      for (int64_t i = 0; i < In; ++i)
        for (int r = 0; r < R; ++r) Hhat[i * R + r] = H[n][i * R + r] * lambda[r];
      if (algo == ORC_MU)
        orc_update_mu(In, R, Hhat, M, S, eps_mu);
      else if (algo == ORC_HALS)
        orc_update_hals(In, R, Hhat, M, S);
      else if (algo == ORC_BPP)
        orc_update_bpp(In, R, Hhat, M, S);
      else if (algo == ORC_ADMM)
        orc_update_admm(In, R, Hhat, Ud[n], M, S, ORC_ADMM_MAXIT, ORC_ADMM_TOL);
      else
        orc_update_nes(In, R, Hhat, M, S, ORC_NES_ITERS, ORC_NES_POWER, ORC_NES_KAPPA);
      orc_normalize(In, R, Hhat, H[n], lambda);
      orc_gram(In, R, H[n], G[n]);
      if (n == N - 1) {
        /* beta = <M^(N), Hhat^(N)>, gamma = lambda^T (S^(N) * G^(N)) lambda */
        for (int64_t e = 0; e < In * R; ++e) beta += M[e] * Hhat[e];
        for (int a = 0; a < R; ++a)
          for (int b = 0; b < R; ++b)
            gamma += lambda[a] * S[a * R + b] * G[n][a * R + b] * lambda[b];
      }
    }
    double e2 = (alpha - 2.0 * beta + gamma) / alpha;
    if (outer) {
      /* s_i = i^(1/N) for outer iteration i; the candidate replaces the
       * iterate (and its Grams) when its squared relative error is lower */
      const double si = pow((double)(first_sweep + s), 1.0 / N);
      const double e2c = orc_nes_outer_candidate(N, dims, R, X, (const double *const *)H, lambda,
                                                 (const double *const *)Hp, lamp, si, alpha, Hc,
                                                 lamc, nthreads);
      if (e2c < e2) {
        for (int k = 0; k < N; ++k) {
          memcpy(H[k], Hc[k], sizeof(double) * (size_t)(dims[k] * R));
          orc_gram(dims[k], R, H[k], G[k]);
        }
        memcpy(lambda, lamc, sizeof(double) * (size_t)R);
        e2 = e2c;
      }
    }
    if (relerr2_raw) relerr2_raw[s] = e2;
    relerr[s] = sqrt(e2 > 0.0 ? e2 : 0.0);
  }
  for (int k = 0; k < N; ++k) {
    free(Hp[k]);
    free(Hc[k]);
  }
  free(lamp);
  free(lamc);
  for (int k = 0; k < N; ++k) {
    free(G[k]);
    free(Ud[k]);
  }
  free(M);
  free(Hhat);
  free(S);
  return 0;
}

/* orc_sweeps_from from a fresh start (outer iteration 1) */
int orc_sweeps(int N, const int64_t *dims, int R, const double *X, double *const *H,
               double *lambda, int algo, double eps_mu, int nsweeps,
               double *relerr, double *relerr2_raw, int nthreads) {
  return orc_sweeps_from(N, dims, R, X, H, lambda, algo, eps_mu, nsweeps, 1, relerr, relerr2_raw,
                         nthreads);
}

/* ------------------------------------------------------------------ */
/* direct residual, loss and gradient                                   */
/* ------------------------------------------------------------------ */

/*
 * E = [[lambda; H]] - X written out entry by entry (lambda may be NULL for
 * all ones); returns 0.5 * ||E||^2.  If E is not NULL the residual is stored.
 */
double orc_residual(int N, const int64_t *dims, int R, const double *X,
                    const double *const *H, const double *lambda, double *E) {
  const int64_t I = prod_dims(N, dims);
  int64_t idx[ORC_MAXN];
  for (int k = 0; k < N; ++k) idx[k] = 0;
  double s = 0.0;
  for (int64_t lin = 0; lin < I; ++lin) {
    double m = 0.0;
    for (int r = 0; r < R; ++r) {
      double p = lambda ? lambda[r] : 1.0;
      for (int k = 0; k < N; ++k) p *= H[k][idx[k] * R + r];
      m += p;
    }
    const double e = m - X[lin];
    if (E) E[lin] = e;
    s += e * e;
    advance(N, dims, idx);
  }
  return 0.5 * s;
}

/*
 * Gradient of L = 0.5 ||X - [[H]]||^2 (all lambda = 1) with respect to every
 * factor: dL/dH^(n) = MTTKRP(E, n) with E = [[H]] - X the explicit residual
 * tensor.  grads[n] is I_n x R.  Returns L.
 */
double orc_grad(int N, const int64_t *dims, int R, const double *X,
                const double *const *H, double *const *grads, int nthreads) {
  const int64_t I = prod_dims(N, dims);
  double *E = (double *)malloc(sizeof(double) * (size_t)I);
  const double L = orc_residual(N, dims, R, X, H, NULL, E);
  for (int n = 0; n < N; ++n) orc_mttkrp(N, dims, R, E, H, n, grads[n], nthreads);
  free(E);
  return L;
}

/* ------------------------------------------------------------------ */
/* projected gradient with Armijo backtracking                          */
/* ------------------------------------------------------------------ */

/* largest eigenvalue of a symmetric R x R matrix by `iters` power steps from
 * the all-ones vector (the matrices used here are entrywise nonnegative). */
double orc_power_lmax(int R, const double *A, int iters) {
  double *v = (double *)malloc(sizeof(double) * R), *w = (double *)malloc(sizeof(double) * R);
  for (int i = 0; i < R; ++i) v[i] = 1.0 / sqrt((double)R);
  double lam = 0.0;
  for (int t = 0; t < iters; ++t) {
    double nrm = 0.0;
    for (int i = 0; i < R; ++i) {
      double s = 0.0;
      for (int j = 0; j < R; ++j) s += A[i * R + j] * v[j];
      w[i] = s;
      nrm += s * s;
    }
    nrm = sqrt(nrm);
    if (!(nrm > 0.0)) { lam = 0.0; break; }
    for (int i = 0; i < R; ++i) v[i] = w[i] / nrm;
  }
  {
    double num = 0.0;
    for (int i = 0; i < R; ++i) {
      double s = 0.0;
      for (int j = 0; j < R; ++j) s += A[i * R + j] * v[j];
      num += v[i] * s;
    }
    lam = num;
  }
  free(v);
  free(w);
  return lam;
}

/*
 * nsteps projected-gradient steps on L = 0.5 ||X - [[H]]||^2 (lambda = 1,
 * no normalisation).  Each step: gradients at the current point; step
 * eta0 = 1 / max_n lmax(S^(n)) (lmax by `power_iters` power steps);
 * trial H' = max(0, H - eta grad) for all modes at once; accept when
 * L(H') <= L(H) - armijo_c * sum_n ||H' - H||^2 / eta, otherwise halve eta,
 * at most max_halvings times; if no trial is accepted H is left unchanged.
 * loss_hist[t] is L after step t, eta_hist[t] (may be NULL) the accepted eta
 * (0 if rejected).
 */
int orc_pgd(int N, const int64_t *dims, int R, const double *X, double *const *H,
            int nsteps, double armijo_c, int max_halvings, int power_iters,
            double *loss_hist, double *eta_hist, int nthreads) {
  if (N < 2 || N > ORC_MAXN || R < 1) return -1;
  double *grads[ORC_MAXN], *Hn[ORC_MAXN], *G[ORC_MAXN];
  for (int k = 0; k < N; ++k) {
    grads[k] = (double *)malloc(sizeof(double) * (size_t)(dims[k] * R));
    Hn[k] = (double *)malloc(sizeof(double) * (size_t)(dims[k] * R));
    G[k] = (double *)malloc(sizeof(double) * (size_t)R * R);
  }
  double *S = (double *)malloc(sizeof(double) * (size_t)R * R);
  for (int t = 0; t < nsteps; ++t) {
    const double L = orc_grad(N, dims, R, X, (const double *const *)H, grads, nthreads);
    double lmax = 0.0;
    for (int k = 0; k < N; ++k) orc_gram(dims[k], R, H[k], G[k]);
    for (int n = 0; n < N; ++n) {
      orc_hadamard_except(N, R, (const double *const *)G, n, S);
      const double l = orc_power_lmax(R, S, power_iters);
      if (l > lmax) lmax = l;
    }
    double eta = lmax > 0.0 ? 1.0 / lmax : 1.0;
    double accepted = 0.0, Lnew = L;
    for (int h = 0; h <= max_halvings; ++h) {
      double d = 0.0;
      for (int k = 0; k < N; ++k)
        for (int64_t e = 0; e < dims[k] * R; ++e) {
          const double v = H[k][e] - eta * grads[k][e];
          Hn[k][e] = v > 0.0 ? v : 0.0;
          d += (Hn[k][e] - H[k][e]) * (Hn[k][e] - H[k][e]);
        }
      const double Lt = orc_residual(N, dims, R, X, (const double *const *)Hn, NULL, NULL);
      if (Lt <= L - armijo_c * d / eta) {
        accepted = eta;
        Lnew = Lt;
        for (int k = 0; k < N; ++k)
          memcpy(H[k], Hn[k], sizeof(double) * (size_t)(dims[k] * R));
        break;
      }
      eta *= 0.5;
    }
    loss_hist[t] = Lnew;
    if (eta_hist) eta_hist[t] = accepted;
  }
  for (int k = 0; k < N; ++k) { free(grads[k]); free(Hn[k]); free(G[k]); }
  free(S);
  return 0;
}
