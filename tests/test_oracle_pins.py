"""Pins for the CPU oracle: checks against things other than the oracle itself.

Each pin is a closed form, a textbook/library routine on explicitly formed
matrices, an invariant the paper states, brute force on tiny inputs, or a
hand-worked fixture under tests/golden/.  A plausible mistake in the oracle
(a dropped factor, a wrong index order, a missing lambda fold, a sign) fails
at least one of them.
"""
import itertools
import os

import numpy as np
import pytest
from scipy.optimize import nnls

import nncp_inputs as gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# independent constructions used by the pins (numpy only)
# ---------------------------------------------------------------------------

def unfold(X, dims, n):
    """Mode-n matricization X_(n): I_n x prod(other), column index with the
    lowest remaining mode fastest (the layout the paper's KRP order matches)."""
    N = len(dims)
    T = np.asarray(X, dtype=np.float64).reshape(dims[::-1])   # axes (i_{N-1}, ..., i_0)
    axis_of = lambda k: N - 1 - k
    order = [axis_of(n)] + [axis_of(k) for k in reversed(range(N)) if k != n]
    return T.transpose(order).reshape(dims[n], -1)


def khatri_rao_excluding(factors, n):
    """H^(N) kr ... kr H^(n+1) kr H^(n-1) kr ... kr H^(1), column r being the
    Kronecker product of the columns (textbook definition, via np.kron)."""
    mats = [factors[k] for k in reversed(range(len(factors))) if k != n]
    R = factors[0].shape[1]
    cols = []
    for r in range(R):
        v = np.ones(1)
        for A in mats:
            v = np.kron(v, A[:, r])
        cols.append(v)
    return np.stack(cols, axis=1)


def reconstruct(factors, lam=None):
    """[[lam; H]] as a flat memory-order tensor via explicit outer products."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    out = np.zeros(dims[::-1])
    for r in range(R):
        t = np.ones(())
        for k in reversed(range(len(factors))):
            t = np.multiply.outer(t, factors[k][:, r])
        out += (1.0 if lam is None else lam[r]) * t
    return out.reshape(-1)


def subproblem_objective(Hhat, M, S):
    """0.5 tr(H S H^T) - tr(H^T M): the mode-n least-squares objective up to a
    constant (A^T A = S, A^T B = M^T in Eq. eqn:nls)."""
    return 0.5 * np.sum((Hhat @ S) * Hhat) - np.sum(Hhat * M)


SHAPES = [
    [3, 4],
    [2, 3, 4],
    [3, 1, 5],
    [5, 4, 3, 2],
    [2, 3, 2, 3, 2],
    [7, 1, 1],
]


# ---------------------------------------------------------------------------
# MTTKRP
# ---------------------------------------------------------------------------

def test_mttkrp_hand_worked_fixture():
    rows = {}
    for line in open(os.path.join(GOLDEN, "mttkrp_2x2x2_hand.txt")):
        line = line.split("#")[0].split()
        if line:
            rows.setdefault(line[0], []).append([float(v) for v in line[1:]])
    X = np.array(rows["X"][0])
    H = [np.array(rows[k]) for k in ("U", "V", "W")]
    for n, key in enumerate(("M1", "M2", "M3")):
        np.testing.assert_array_equal(oracle.mttkrp(X, H, n), np.array(rows[key]))


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("R", [1, 3])
def test_mttkrp_equals_unfolding_times_khatri_rao(dims, R):
    """Small integers: both sides are exact in FP64, so equality is bitwise."""
    seed = 11 + len(dims) * 7 + R
    X = gen.integer_tensor(dims, seed)
    H = gen.integer_factors(dims, R, seed + 1)
    for n in range(len(dims)):
        ref = unfold(X, dims, n) @ khatri_rao_excluding(H, n)
        np.testing.assert_array_equal(oracle.mttkrp(X, H, n), ref)


def test_mttkrp_rank_one_closed_form():
    """X = a o b o c gives M^(1)(:,r) = a (b^T H2(:,r)) (c^T H3(:,r))."""
    rng = np.random.default_rng(5)
    a, b, c = rng.random(4), rng.random(5), rng.random(6)
    X = np.multiply.outer(np.multiply.outer(c, b), a).reshape(-1)   # memory order
    H = [rng.random((4, 3)), rng.random((5, 3)), rng.random((6, 3))]
    np.testing.assert_allclose(oracle.mttkrp(X, H, 0), np.outer(a, (b @ H[1]) * (c @ H[2])), rtol=1e-14)
    np.testing.assert_allclose(oracle.mttkrp(X, H, 1), np.outer(b, (a @ H[0]) * (c @ H[2])), rtol=1e-14)
    np.testing.assert_allclose(oracle.mttkrp(X, H, 2), np.outer(c, (a @ H[0]) * (b @ H[1])), rtol=1e-14)


@pytest.mark.parametrize("dims", [[3, 4, 5], [2, 2, 3, 2]])
def test_mttkrp_all_ones(dims):
    I = int(np.prod(dims))
    H = [np.ones((d, 2)) for d in dims]
    for n in range(len(dims)):
        np.testing.assert_array_equal(oracle.mttkrp(np.ones(I), H, n), np.full((dims[n], 2), I / dims[n]))


def test_mttkrp_multilinear():
    dims = [4, 3, 5]
    rng = np.random.default_rng(1)
    X1, X2 = rng.random(60), rng.random(60)
    H = [rng.random((d, 2)) for d in dims]
    for n in range(3):
        lhs = oracle.mttkrp(2.0 * X1 - 3.0 * X2, H, n)
        rhs = 2.0 * oracle.mttkrp(X1, H, n) - 3.0 * oracle.mttkrp(X2, H, n)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-13)
        for k in range(3):
            Hs = [h.copy() for h in H]
            Hs[k] *= 2.5
            expect = oracle.mttkrp(X1, H, n) * (1.0 if k == n else 2.5)
            np.testing.assert_allclose(oracle.mttkrp(X1, Hs, n), expect, rtol=1e-14)


def test_mttkrp_mode_permutation_covariance():
    """Permuting the modes of X and the factor list permutes the results."""
    dims = [3, 4, 5]
    rng = np.random.default_rng(2)
    X = rng.random(60)
    H = [rng.random((d, 2)) for d in dims]
    perm = [2, 0, 1]
    T = X.reshape(dims[::-1])                                 # axes (i2, i1, i0)
    # new mode q is old mode perm[q]; new array axes (q2, q1, q0)
    Tp = T.transpose([2 - perm[2], 2 - perm[1], 2 - perm[0]])
    Xp = np.ascontiguousarray(Tp).reshape(-1)
    Hp = [H[p] for p in perm]
    for q in range(3):
        np.testing.assert_allclose(oracle.mttkrp(Xp, Hp, q), oracle.mttkrp(X, H, perm[q]), rtol=1e-13)


def test_mttkrp_three_way_dimension_tree_identities():
    """Section 4.2.1: with T = X x_3 W (I x J x R), M^(1) = sum_j V T and
    M^(2) = sum_i U T (formed here with einsum, independently)."""
    I, J, K, R = 5, 4, 6, 3
    rng = np.random.default_rng(3)
    X = rng.random(I * J * K)
    U, V, W = rng.random((I, R)), rng.random((J, R)), rng.random((K, R))
    Xa = X.reshape(K, J, I)
    T = np.einsum("kji,kr->ijr", Xa, W)
    np.testing.assert_allclose(oracle.mttkrp(X, [U, V, W], 0), np.einsum("jr,ijr->ir", V, T), rtol=1e-13)
    np.testing.assert_allclose(oracle.mttkrp(X, [U, V, W], 1), np.einsum("ir,ijr->jr", U, T), rtol=1e-13)


def test_mttkrp_threads_and_rows_agree():
    dims = [5, 6, 7]
    X = gen.integer_tensor(dims, 9)
    H = gen.integer_factors(dims, 4, 10)
    for n in range(3):
        full = oracle.mttkrp(X, H, n, nthreads=1)
        np.testing.assert_array_equal(oracle.mttkrp(X, H, n, nthreads=3), full)
        rows = [0, dims[n] - 1, 2]
        np.testing.assert_array_equal(oracle.mttkrp_rows(X, H, n, rows, nthreads=2), full[rows])


# ---------------------------------------------------------------------------
# Gram, Hadamard, normalisation
# ---------------------------------------------------------------------------

def test_gram_and_hadamard():
    rng = np.random.default_rng(4)
    Hs = [rng.random((d, 5)) for d in (7, 3, 4)]
    Gs = [oracle.gram(h) for h in Hs]
    for h, g in zip(Hs, Gs):
        np.testing.assert_allclose(g, h.T @ h, rtol=1e-14)
        np.testing.assert_array_equal(g, g.T)
    for n in range(3):
        others = [Gs[k] for k in range(3) if k != n]
        np.testing.assert_allclose(oracle.hadamard_except(Gs, n), others[0] * others[1], rtol=1e-15)
    # S^(n) = A^T A for the explicit Khatri-Rao product A (Eq. eqn:nls)
    for n in range(3):
        A = khatri_rao_excluding(Hs, n)
        np.testing.assert_allclose(oracle.hadamard_except(Gs, n), A.T @ A, rtol=1e-13)


def test_normalize():
    rng = np.random.default_rng(6)
    Hhat = rng.random((6, 4))
    Hhat[:, 2] = 0.0
    H, lam = oracle.normalize(Hhat)
    np.testing.assert_allclose(np.linalg.norm(H[:, [0, 1, 3]], axis=0), 1.0, rtol=1e-14)
    assert lam[2] == 0.0 and np.all(H[:, 2] == 0.0)
    np.testing.assert_allclose(H * lam[None, :], Hhat, rtol=1e-14)
    # the model [[lambda; H]] is unchanged by normalisation
    others = [rng.random((3, 4)), rng.random((5, 4))]
    np.testing.assert_allclose(reconstruct([H] + others, lam), reconstruct([Hhat] + others), rtol=1e-13)


# ---------------------------------------------------------------------------
# updates
# ---------------------------------------------------------------------------

def _subproblem(dims, R, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.random(int(np.prod(dims)))
    H = [rng.random((d, R)) for d in dims]
    A = khatri_rao_excluding(H, n)
    M = unfold(X, dims, n) @ A
    S = A.T @ A
    return X, H, A, M, S


def test_hals_rank_one_is_exact_nnls():
    """R = 1: one HALS step solves every row's NNLS exactly (scipy nnls on the
    explicit Khatri-Rao product and unfolding)."""
    dims = [5, 4, 3]
    X, H, A, M, S = _subproblem(dims, 1, 0, 7)
    B = unfold(X, dims, 0)
    B[1] *= -1.0  # make one row's solution hit the bound
    M = B @ A
    out = oracle.update_hals(H[0], M, S)
    for i in range(dims[0]):
        x, _ = nnls(A, B[i])
        np.testing.assert_allclose(out[i], x, rtol=1e-12, atol=1e-14)


def test_hals_repeated_converges_to_nnls():
    """HALS is exact block-coordinate descent on a strictly convex problem:
    repeating it converges to the NNLS solution of every row."""
    dims = [6, 5, 4]
    X, H, A, M, S = _subproblem(dims, 3, 1, 8)
    B = unfold(X, dims, 1) - 0.3  # some negative data so constraints bind
    M = B @ A
    Hh = H[1].copy()
    for _ in range(3000):
        Hh = oracle.update_hals(Hh, M, S)
    for i in range(dims[1]):
        x, _ = nnls(A, B[i])
        np.testing.assert_allclose(Hh[i], x, rtol=1e-8, atol=1e-10)


def test_hals_last_column_kkt_and_monotone():
    dims = [7, 4, 5]
    X, H, A, M, S = _subproblem(dims, 4, 0, 9)
    M = M - 0.2 * M.mean()
    Hh = H[0] * 3.0
    out = oracle.update_hals(Hh, M, S)
    assert np.all(out >= 0)
    g = out @ S - M                      # gradient of the subproblem
    r = S.shape[0] - 1                   # the last column was updated last
    pos = out[:, r] > 0
    np.testing.assert_allclose(g[pos, r], 0.0, atol=1e-12)
    assert np.all(g[~pos, r] >= -1e-12)
    assert subproblem_objective(out, M, S) <= subproblem_objective(Hh, M, S) + 1e-12


# ---------------------------------------------------------------------------
# BPP (Section 4.3.3): exact NNLS per row
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("R", [1, 3, 8, 17, 32, 64])
def test_bpp_matches_scipy_nnls(R):
    """min ||A x - b|| over x >= 0 from scipy's active-set solver (Lawson and
    Hanson), an independent implementation, against BPP on S = A^T A, m = A^T b."""
    rng = np.random.default_rng(100 + R)
    for t in range(20):
        n = int(rng.integers(R, 3 * R + 5))
        A = rng.standard_normal((n, R))
        b = rng.standard_normal(n)
        x, solves = oracle.bpp_row(A.T @ A, A.T @ b)
        xs, _ = nnls(A, b, maxiter=50 * R)
        assert solves >= 0
        np.testing.assert_allclose(x, xs, rtol=1e-9, atol=1e-12 * max(1.0, np.abs(xs).max()))


def test_bpp_kkt_and_special_cases():
    rng = np.random.default_rng(7)
    R = 12
    A = rng.random((30, R))
    S = A.T @ A
    # KKT on a general right-hand side
    m = 5.0 * rng.standard_normal(R)
    assert (m > 0).any() and (m < 0).any()
    x, solves = oracle.bpp_row(S, m)
    y = S @ x - m
    assert solves >= 1 and np.all(x >= 0)
    assert np.all(y >= -1e-10 * np.abs(m).max())
    assert np.abs(x * y).max() <= 1e-10 * np.abs(m).max() ** 2
    # interior solution: the unconstrained solve is already nonnegative
    xt = rng.random(R) + 0.1
    x, _ = oracle.bpp_row(S, S @ xt)
    np.testing.assert_allclose(x, np.linalg.solve(S, S @ xt), rtol=1e-10)
    np.testing.assert_allclose(x, xt, rtol=1e-8)
    # m <= 0 (S has nonnegative entries): x = 0 satisfies KKT at once
    x, solves = oracle.bpp_row(S, -rng.random(R))
    assert solves == 0 and np.all(x == 0)
    # R = 1 closed form max(0, m / s)
    x, _ = oracle.bpp_row(np.array([[4.0]]), np.array([3.0]))
    assert x[0] == 0.75


def test_bpp_warm_start():
    """The solution does not depend on the start support; started from the
    solution's own support the search needs one solve."""
    rng = np.random.default_rng(8)
    for R in (5, 16, 40):
        A = rng.random((2 * R, R)) + 0.05 * rng.standard_normal((2 * R, R))
        m = 3.0 * rng.standard_normal(R)
        S = A.T @ A
        xc, nc = oracle.bpp_row(S, m)
        xr, nr = oracle.bpp_row(S, m, x0=rng.random(R) * (rng.random(R) < 0.5))
        xw, nw = oracle.bpp_row(S, m, x0=xc)
        assert nc >= 1 and nr >= 1 and nw == 1
        np.testing.assert_allclose(xr, xc, rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(xw, xc, rtol=1e-10, atol=1e-13)


def test_bpp_update_is_the_limit_of_hals():
    """Repeated HALS sweeps over the columns converge to the exact per-row
    NNLS solution, which BPP computes directly (the start values do not
    matter to BPP)."""
    dims = [7, 4, 5]
    X, H, A, M, S = _subproblem(dims, 4, 1, 12)
    M = M - 0.3 * M.mean()
    Hb, failed = oracle.update_bpp(M, S)
    assert failed == 0 and np.all(Hb >= 0)
    Hh = H[1].copy()
    for _ in range(3000):
        Hh = oracle.update_hals(Hh, M, S)
    np.testing.assert_allclose(Hb, Hh, rtol=1e-8, atol=1e-10)
    assert subproblem_objective(Hb, M, S) <= subproblem_objective(Hh, M, S) + 1e-12


# ---------------------------------------------------------------------------
# ADMM (Section 4.3.4)
# ---------------------------------------------------------------------------

def test_admm_single_pass_is_regularised_least_squares():
    """One pass from (H, U): Ht minimises ||A t - b||^2 + rho ||t - (h + u)||^2,
    solved here as a stacked least-squares problem with lstsq (no normal
    equations), rho = ||A||_F^2 / R; then H = max(0, Ht - U), U += H - Ht."""
    dims = [6, 5, 4]
    R, n = 3, 1
    X, H, A, M, S = _subproblem(dims, R, n, 13)
    B = unfold(X, dims, n)                  # I_n x J, so M = B A
    rng = np.random.default_rng(14)
    H0 = rng.random((dims[n], R))
    U0 = 0.1 * rng.standard_normal((dims[n], R))
    rho = np.linalg.norm(A) ** 2 / R
    Ht = np.zeros_like(H0)
    for i in range(dims[n]):
        lhs = np.vstack([A, np.sqrt(rho) * np.eye(R)])
        rhs = np.concatenate([B[i], np.sqrt(rho) * (H0[i] + U0[i])])
        Ht[i] = np.linalg.lstsq(lhs, rhs, rcond=None)[0]
    Hn = np.maximum(0.0, Ht - U0)
    Un = U0 + Hn - Ht
    Ho, Uo, passes = oracle.update_admm(H0, U0, M, S, maxit=1)
    assert passes == 1
    np.testing.assert_allclose(Ho, Hn, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(Uo, Un, rtol=1e-10, atol=1e-12)


def test_admm_fixed_point_and_limit_are_the_nnls_solution():
    rng = np.random.default_rng(15)
    R = 6
    A = rng.random((20, R))
    Bm = rng.standard_normal((9, 20)) + 0.5
    S = A.T @ A
    M = Bm @ A
    Xs = np.stack([nnls(A, b)[0] for b in Bm])          # scipy NNLS per row
    rho = np.trace(S) / R
    Us = (Xs @ S - M) / rho                               # scaled dual at the optimum
    Ho, Uo, passes = oracle.update_admm(Xs, Us, M, S, maxit=5)
    assert passes == 1                                    # stops at once: r = s = 0
    np.testing.assert_allclose(Ho, Xs, rtol=1e-9, atol=1e-12)
    # from a cold start many passes reach the same solution
    Ho, Uo, passes = oracle.update_admm(np.zeros_like(Xs), np.zeros_like(Xs), M, S, maxit=3000,
                                        tol=1e-30)
    np.testing.assert_allclose(Ho, Xs, rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------------------
# Nesterov-type update (Section 4.3.5)
# ---------------------------------------------------------------------------

def test_nes_params_against_eigvalsh():
    """L from power steps is the largest eigenvalue (LAPACK, an independent
    routine) when the leading eigenvalue is well separated; mu is an estimate
    of the smallest from above; the proximal weight caps the condition number
    of S + lam I at kappa."""
    rng = np.random.default_rng(31)
    for R in (1, 4, 8, 16):
        A = rng.random((3 * R + 10, R))
        S = A.T @ A
        ev = np.linalg.eigvalsh(S)
        L, mu, lam, alpha, beta, ok = oracle.nes_params(S, power=20, kappa=100.0)
        assert ok
        np.testing.assert_allclose(L, ev[-1], rtol=1e-9)
        assert ev[0] - 1e-9 * ev[-1] <= mu <= L * (1 + 1e-12)
        assert lam >= 0.0
        assert (L + lam) / (mu + lam) <= 100.0 * (1 + 1e-9)
        assert 0.0 <= beta < 1.0 and alpha > 0.0
    # a scaled identity: L = mu = s exactly, no momentum, no proximal term
    L, mu, lam, alpha, beta, ok = oracle.nes_params(2.5 * np.eye(6))
    assert (L, mu, lam, beta) == (2.5, 2.5, 0.0, 0.0)
    np.testing.assert_allclose(alpha, 1 / 2.5, rtol=1e-15)
    # S = 0: no step is defined, the start value is kept
    H0 = np.random.default_rng(2).random((3, 4))
    Ho, ok = oracle.update_nes(H0, np.ones((3, 4)), np.zeros((4, 4)))
    assert not ok
    np.testing.assert_array_equal(Ho, H0)


def test_nes_diagonal_s_solves_in_one_step():
    """For S = s I the subproblem separates and its solution is max(0, m / s);
    with alpha = 1/s and no momentum one step reaches it, and it is a fixed
    point afterwards."""
    rng = np.random.default_rng(32)
    M = rng.standard_normal((7, 5))
    S = 3.0 * np.eye(5)
    H0 = rng.random((7, 5))
    want = np.maximum(0.0, M / 3.0)
    for iters in (1, 20):
        Ho, ok = oracle.update_nes(H0, M, S, iters=iters)
        assert ok
        np.testing.assert_allclose(Ho, want, rtol=1e-15, atol=1e-15)


def test_nes_limit_is_the_nnls_solution():
    """Without the proximal term (kappa large enough that lam = 0) many steps
    reach the NNLS solution (scipy's active-set solver per row)."""
    rng = np.random.default_rng(33)
    R = 6
    A = rng.random((20, R))
    Bm = rng.standard_normal((9, 20)) + 0.5
    S = A.T @ A
    M = Bm @ A
    L, mu, lam, alpha, beta, ok = oracle.nes_params(S, kappa=1e12)
    assert lam == 0.0
    Xs = np.stack([nnls(A, b)[0] for b in Bm])
    Ho, ok = oracle.update_nes(np.zeros_like(Xs) + 0.1, M, S, iters=4000, kappa=1e12)
    assert ok
    np.testing.assert_allclose(Ho, Xs, rtol=1e-8, atol=1e-10)


def test_nes_limit_with_the_proximal_term():
    """With lam > 0 the fixed point minimises ||A x - b||^2 + lam ||x - x*||^2
    over x >= 0, i.e. the NNLS solution of the stacked system
    [A; sqrt(lam) I] x = [b; sqrt(lam) x*] (scipy, per row)."""
    rng = np.random.default_rng(34)
    R = 6
    A = rng.random((20, R))
    Bm = rng.standard_normal((9, 20)) + 0.5
    S = A.T @ A
    M = Bm @ A
    X0 = rng.random((9, R))
    L, mu, lam, alpha, beta, ok = oracle.nes_params(S, kappa=3.0)
    assert lam > 0.0
    want = np.stack([nnls(np.vstack([A, np.sqrt(lam) * np.eye(R)]),
                          np.concatenate([b, np.sqrt(lam) * x0]))[0] for b, x0 in zip(Bm, X0)])
    Ho, ok = oracle.update_nes(X0, M, S, iters=4000, kappa=3.0)
    assert ok
    np.testing.assert_allclose(Ho, want, rtol=1e-8, atol=1e-10)


def test_nes_lowers_the_proximal_objective():
    """Twenty steps from x* lower f_p below its value at x* (where the
    proximal term is 0), for a general subproblem."""
    dims = [6, 5, 4]
    X, H, A, M, S = _subproblem(dims, 3, 1, 35)
    Hh = H[1] * 1.7
    Ho, ok = oracle.update_nes(Hh, M, S)
    assert ok and np.all(Ho >= 0)
    L, mu, lam, alpha, beta, _ = oracle.nes_params(S)
    fp = subproblem_objective(Ho, M, S) + 0.5 * lam * np.sum((Ho - Hh) ** 2)
    assert fp < subproblem_objective(Hh, M, S)


def test_nes_outer_extrapolation_never_raises_the_error():
    """The first sweep of NES with the outer step starts like plain NES; the
    candidate is taken only when its error is lower, so the error after the
    sweep is at most the plain one, and equal when the candidate is refused.
    Over several sweeps the candidate is accepted at least once here, and
    every reported error is that of the returned factors (the identity test
    above covers the latter for NES_OUTER as well)."""
    dims = [12, 10, 9]
    X, H0 = gen.small_lowrank(dims, 4, 4, 36, noise=0.02)
    lam0 = np.ones(4)
    _, _, rel_plain, _ = oracle.sweeps(X, H0, lam0, oracle.NES, 1)
    _, _, rel_outer, _ = oracle.sweeps(X, H0, lam0, oracle.NES_OUTER, 1)
    assert rel_outer[0] <= rel_plain[0]
    _, _, rp, _ = oracle.sweeps(X, H0, lam0, oracle.NES, 12)
    Ho, lo, ro, _ = oracle.sweeps(X, H0, lam0, oracle.NES_OUTER, 12)
    assert not np.array_equal(ro, rp)                    # some candidate was taken
    direct = np.linalg.norm(X - reconstruct(Ho, lo)) / np.linalg.norm(X)
    np.testing.assert_allclose(ro[-1], direct, rtol=1e-8)


def test_mu_invariants():
    dims = [6, 5, 4]
    X, H, A, M, S = _subproblem(dims, 3, 2, 10)
    Hh = H[2].copy()
    Hh[0, 1] = 0.0
    f0 = subproblem_objective(Hh, M, S)
    out = oracle.update_mu(Hh, M, S, 1e-16)
    assert np.all(out >= 0)
    assert out[0, 1] == 0.0                      # zeros stay zero
    assert subproblem_objective(out, M, S) <= f0 + 1e-12 * abs(f0)   # Lee-Seung descent
    # a positive exact solution of H S = M is a fixed point
    Hstar = np.random.default_rng(3).random((4, 3)) + 0.5
    np.testing.assert_allclose(oracle.update_mu(Hstar, Hstar @ S, S, 0.0), Hstar, rtol=1e-12)


# ---------------------------------------------------------------------------
# sweeps: identity, monotonicity, exact low rank, KKT
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("algo", [oracle.MU, oracle.HALS, oracle.BPP, oracle.ADMM, oracle.NES,
                                  oracle.NES_OUTER])
@pytest.mark.parametrize("dims", [[6, 5, 4], [4, 3, 5, 2]])
def test_sweep_relerr_identity_matches_direct_residual(algo, dims):
    X, H0 = gen.small_lowrank(dims, 3, 3, 21, noise=0.05)
    lam0 = np.ones(3)
    prev = None
    for s in range(1, 6):
        Hs, lam, rel, raw = oracle.sweeps(X, H0, lam0, algo, s)
        direct = np.linalg.norm(X - reconstruct(Hs, lam)) / np.linalg.norm(X)
        np.testing.assert_allclose(rel[-1], direct, rtol=1e-8, atol=1e-10)
        if prev is not None:
            np.testing.assert_allclose(rel[:-1], prev, rtol=0, atol=0)   # deterministic prefix
        prev = rel
        for h in Hs:
            assert np.all(h >= 0)
            n = np.linalg.norm(h, axis=0)
            np.testing.assert_allclose(n[n > 0], 1.0, rtol=1e-13)


@pytest.mark.parametrize("algo", [oracle.MU, oracle.HALS, oracle.BPP])
def test_objective_nonincreasing_after_every_mode(algo):
    """With lambda folded into the updated factor, each mode update can only
    lower ||X - [[lambda; H]]|| (MU: Lee-Seung; HALS: exact coordinate steps;
    BPP: the exact block minimiser)."""
    dims = [5, 4, 6]
    X, H = gen.small_lowrank(dims, 3, 3, 31, noise=0.1)
    lam = np.ones(3)
    Hs = [h.copy() for h in H]
    f = np.linalg.norm(X - reconstruct(Hs, lam))
    for sweep in range(4):
        for n in range(3):
            Gs = [oracle.gram(h) for h in Hs]
            M = oracle.mttkrp(X, Hs, n)
            S = oracle.hadamard_except(Gs, n)
            Hhat = Hs[n] * lam[None, :]
            if algo == oracle.MU:
                Hhat = oracle.update_mu(Hhat, M, S)
            elif algo == oracle.HALS:
                Hhat = oracle.update_hals(Hhat, M, S)
            else:
                Hhat, failed = oracle.update_bpp(M, S)
                assert failed == 0
            Hs[n], lam = oracle.normalize(Hhat)
            fn = np.linalg.norm(X - reconstruct(Hs, lam))
            assert fn <= f * (1 + 1e-12)
            f = fn
    # and the oracle's own sweep loop follows the same trajectory
    Ho, lo, rel, _ = oracle.sweeps(X, H, np.ones(3), algo, 4)
    for a, b in zip(Ho, Hs):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rel[-1], f / np.linalg.norm(X), rtol=1e-9)


def test_exact_low_rank_converges_to_zero():
    """Exact nonnegative low-rank data, no noise: HALS drives the error to ~0
    from a random start (the paper's synthetic sets are exact low rank)."""
    dims = [7, 6, 5]
    X, H0 = gen.small_lowrank(dims, 2, 2, 41)
    Hs, lam, rel, raw = oracle.sweeps(X, H0, np.ones(2), oracle.HALS, 400)
    direct = np.linalg.norm(X - reconstruct(Hs, lam)) / np.linalg.norm(X)
    assert direct < 1e-6
    assert rel[-1] < 1e-6
    # monotone until the identity reaches its cancellation floor (~sqrt(u))
    above = rel > 1e-6
    k = int(np.argmin(above)) if not above.all() else len(rel)
    assert np.all(np.diff(rel[:k]) <= 1e-12)


def test_kkt_residual_shrinks():
    dims = [6, 5, 4]
    X, H0 = gen.small_lowrank(dims, 3, 3, 51, noise=0.02)

    def kkt(Hs, lam):
        worst = 0.0
        for n in range(3):
            Hh = [h.copy() for h in Hs]
            Hh[n] = Hh[n] * lam[None, :]
            Gs = [oracle.gram(h) for h in Hh]
            M = oracle.mttkrp(X, Hh, n)
            S = oracle.hadamard_except(Gs, n)
            g = Hh[n] @ S - M
            worst = max(worst, np.linalg.norm(np.minimum(Hh[n], g)) / np.linalg.norm(M))
        return worst

    k = []
    for s in (2, 20, 200):
        Hs, lam, _, _ = oracle.sweeps(X, H0, np.ones(3), oracle.HALS, s)
        k.append(kkt(Hs, lam))
    assert k[1] < k[0] and k[2] < k[1] and k[2] < 1e-3


# ---------------------------------------------------------------------------
# gradient and projected gradient
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [[3, 4, 2], [2, 3, 2, 2, 3]])
def test_gradient_central_differences(dims):
    """L is quadratic in each single entry, so a central difference with
    h = 1e-3 is exact up to rounding."""
    rng = np.random.default_rng(61)
    R = 2
    X = rng.random(int(np.prod(dims)))
    H = [rng.random((d, R)) for d in dims]
    L, gs = oracle.grad(X, H)

    def loss(Hs):
        return 0.5 * np.sum((X - reconstruct(Hs)) ** 2)

    np.testing.assert_allclose(L, loss(H), rtol=1e-13)
    h = 1e-3
    for n in range(len(dims)):
        fd = np.zeros_like(H[n])
        for i, r in itertools.product(range(dims[n]), range(R)):
            Hp = [a.copy() for a in H]
            Hm = [a.copy() for a in H]
            Hp[n][i, r] += h
            Hm[n][i, r] -= h
            fd[i, r] = (loss(Hp) - loss(Hm)) / (2 * h)
        np.testing.assert_allclose(gs[n], fd, rtol=1e-7, atol=1e-9)
        # closed form of the adjoint: H S - M
        Gs = [a.T @ a for a in H]
        S = np.prod([Gs[k] for k in range(len(dims)) if k != n], axis=0)
        M = unfold(X, dims, n) @ khatri_rao_excluding(H, n)
        np.testing.assert_allclose(gs[n], H[n] @ S - M, rtol=1e-11, atol=1e-12)


def test_gradient_zero_at_exact_fit():
    dims = [4, 3, 5]
    H = gen.uniform_factors(dims, 2, 71)
    X = reconstruct(H)
    L, gs = oracle.grad(X, H)
    assert L < 1e-28
    for g in gs:
        assert np.max(np.abs(g)) < 1e-12


def test_power_iteration_matches_eigvalsh():
    rng = np.random.default_rng(81)
    for R in (1, 4, 16):
        B = rng.random((20, R))
        A = B.T @ B
        np.testing.assert_allclose(oracle.power_lmax(A, 200), np.linalg.eigvalsh(A)[-1], rtol=1e-10)


def test_pgd_monotone_and_nonnegative():
    dims = [5, 4, 3]
    X, H0 = gen.small_lowrank(dims, 2, 2, 91, noise=0.05)
    Hs, lh, eh = oracle.pgd(X, H0, 30)
    L0 = 0.5 * np.sum((X - reconstruct(H0)) ** 2)
    assert np.all(np.diff(np.concatenate([[L0], lh])) <= 1e-12 * L0)
    assert lh[-1] < 0.5 * L0
    for h in Hs:
        assert np.all(h >= 0)
    np.testing.assert_allclose(lh[-1], 0.5 * np.sum((X - reconstruct(Hs)) ** 2), rtol=1e-12)


# ---------------------------------------------------------------------------
# planted mistakes: each must be caught by one of the pins above
# ---------------------------------------------------------------------------

def test_planted_mistakes_are_caught():
    """Perturbations of the MTTKRP definition that a buggy oracle could make
    (transposed KRP order, a dropped factor) disagree with the brute force."""
    dims = [3, 4, 5]
    X = gen.integer_tensor(dims, 101)
    H = gen.integer_factors(dims, 2, 102, hi=5)
    good = unfold(X, dims, 0) @ khatri_rao_excluding(H, 0)
    # KRP in the wrong order (H^(1) slowest instead of fastest)
    wrong_order = unfold(X, dims, 0) @ khatri_rao_excluding([H[0], H[2], H[1]], 0)
    assert not np.array_equal(wrong_order, good)
    # dropped factor
    dropped = [H[0], H[1], np.ones_like(H[2])]
    assert not np.array_equal(oracle.mttkrp(X, dropped, 0), good)
    np.testing.assert_array_equal(oracle.mttkrp(X, H, 0), good)
