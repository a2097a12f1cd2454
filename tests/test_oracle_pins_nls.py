"""Pins for the oracle's NES momentum, NES outer extrapolation and ADMM
stopping test (Sections 4.3.4 and 4.3.5), each with planted mistakes.

Every pin is a check against something other than the oracle: the
convergence-rate guarantee of the accelerated gradient method, a direct
residual built in NumPy from Eq. (eqn:nesouterupd), or ADMM passes solved
independently as stacked least-squares problems.  The planted-mistake tests
compile an altered copy of the oracle's C source (one textual change each),
route the oracle through it, and require the pin to fail.
"""
import os

import numpy as np
import pytest
from scipy.optimize import nnls

import nncp_inputs as gen
import oracle


# ---------------------------------------------------------------------------
# planted mistakes: altered builds of the oracle source
# ---------------------------------------------------------------------------

def _mutant(tmp_path, name, old, new):
    """Build the oracle with `old` replaced by `new` (which must occur once)."""
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    return oracle.build_variant(str(tmp_path / f"liboracle_{name}.so"), src.replace(old, new))


def _assert_pin_catches(tmp_path, name, old, new, check):
    path = _mutant(tmp_path, name, old, new)
    with oracle.using_library(path):
        with pytest.raises(AssertionError):
            check()


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


# ---------------------------------------------------------------------------
# NES momentum (Section 4.3.5, Eq. eqn:nesinnerupd): a rate pin
# ---------------------------------------------------------------------------

def _nes_rate_instance():
    """A strongly convex subproblem with condition number exactly 100
    (eigenvalues 100, 50, 1 of S), an interior NNLS optimum and a start
    whose error has equal weight on every eigenvector, close enough to the
    optimum that no projection is ever active."""
    rng = np.random.default_rng(4101)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    ev = np.array([100.0, 50.0, 1.0])
    S = (Q * ev) @ Q.T
    S = 0.5 * (S + S.T)
    x_opt = np.array([1.5, 1.25, 1.75])
    m = x_opt @ S
    x0 = x_opt + 0.05 * Q @ np.ones(3) / np.sqrt(3.0)
    return S, m, x0, x_opt, ev


def _check_nes_rate(k=200):
    """Nesterov's constant-momentum scheme on an L-smooth, mu-strongly convex
    objective guarantees (Nesterov 2004, Thm 2.2.3 with
    ||x - x*||^2 <= 2 (f(x) - f*) / mu)
        ||x_k - x*|| <= sqrt((L + mu) / mu) (1 - sqrt(mu / L))^(k/2) ||x_0 - x*||.
    Plain projected gradient (no momentum) only reaches (1 - mu/L)^k, and a
    momentum computed from mu/L instead of its square root oscillates with
    modulus about sqrt(beta); both miss this bound by orders of magnitude."""
    S, m, x0, x_opt, ev = _nes_rate_instance()
    L, mu = ev[0], ev[-1]
    pL, pmu, lam, alpha, beta, ok = oracle.nes_params(S)
    assert ok
    assert lam < 1e-9 * L                  # kappa(S) = 100: no proximal term
    x, ok = oracle.update_nes(x0[None, :], m[None, :], S, iters=k)
    assert ok
    err = np.linalg.norm(x[0] - x_opt)
    bound = np.sqrt((L + mu) / mu) * (1.0 - np.sqrt(mu / L)) ** (k / 2) * np.linalg.norm(x0 - x_opt)
    assert err <= bound, (err, bound)
    assert np.all(x >= 0.0)


def test_nes_momentum_meets_the_accelerated_rate():
    S, m, x0, x_opt, ev = _nes_rate_instance()
    np.testing.assert_allclose(np.linalg.eigvalsh(S)[::-1], ev, rtol=1e-12)
    assert np.all(x_opt @ S == m)
    _check_nes_rate()


def test_nes_rate_pin_catches_planted_momentum(tmp_path):
    # beta from q instead of sqrt(q)
    _assert_pin_catches(tmp_path, "beta_q", "const double q = sqrt((mu + lam) / (L + lam));",
                        "const double q = (mu + lam) / (L + lam);", _check_nes_rate)
    # no momentum at all
    _assert_pin_catches(tmp_path, "beta_0", "out[4] = (1.0 - q) / (1.0 + q);", "out[4] = 0.0;",
                        _check_nes_rate)


# ---------------------------------------------------------------------------
# NES outer extrapolation (Eq. eqn:nesouterupd)
# ---------------------------------------------------------------------------

def _outer_instance():
    dims = [12, 10, 9]
    X, H0 = gen.small_lowrank(dims, 4, 4, 36, noise=0.02)
    return dims, X, H0, np.ones(4)


def _candidate_direct(X, H, lam, Hp, lamp, si):
    """The candidate written out from Eq. (eqn:nesouterupd) in NumPy: the step
    acts on F^(n) = H^(n) for n < N-1 and F^(N-1) = H^(N-1) diag(lambda);
    Fc = max(0, F + s_i (F - F_prev)); squared relative error of the
    unweighted model [[Fc]] by explicit reconstruction."""
    N = len(H)
    F = [H[k] * (lam[None, :] if k == N - 1 else 1.0) for k in range(N)]
    Fp = [Hp[k] * (lamp[None, :] if k == N - 1 else 1.0) for k in range(N)]
    Fc = [np.maximum(0.0, F[k] + si * (F[k] - Fp[k])) for k in range(N)]
    model = reconstruct(Fc)
    return Fc, model, np.sum((X - model) ** 2) / np.sum(X ** 2)


def _check_outer_candidate():
    dims, X, H0, lam0 = _outer_instance()
    H1, lam1, _, _ = oracle.sweeps(X, H0, lam0, oracle.NES, 1)
    H2, lam2, _, _ = oracle.sweeps(X, H1, lam1, oracle.NES, 1)
    for (H, lam, Hp, lamp) in ((H1, lam1, H0, lam0), (H2, lam2, H1, lam1)):
        for i in (1, 2, 5):
            si = i ** (1.0 / len(dims))
            Hc, lamc, e2c = oracle.nes_outer_candidate(X, H, lam, Hp, lamp, si)
            Fc, model, e2_direct = _candidate_direct(X, H, lam, Hp, lamp, si)
            # the identity-based error of the oracle equals the direct one
            assert abs(e2c - e2_direct) <= 1e-10, (e2c, e2_direct)
            # same model, normalised factors
            assert np.allclose(reconstruct(Hc, lamc), model, rtol=1e-12, atol=1e-13)
            for h in Hc:
                nrm = np.linalg.norm(h, axis=0)
                assert np.allclose(nrm[nrm > 0], 1.0, rtol=1e-13)


def test_nes_outer_candidate_matches_the_direct_residual():
    _check_outer_candidate()


def _check_outer_sweeps(nsweeps=6):
    """NES_OUTER sweeps equal the composition written out here: a plain NES
    sweep, then the candidate with s_i = i^(1/N) for outer iteration i from
    the iterate before that sweep, taken when its squared error is lower.
    A candidate must be taken at some i >= 2 (where s_i != 1)."""
    dims, X, H0, lam0 = _outer_instance()
    N = len(dims)
    H, lam = [h.copy() for h in H0], lam0.copy()
    taken, want_rel = [], []
    for i in range(1, nsweeps + 1):
        Hn, lamn, _, raw = oracle.sweeps(X, H, lam, oracle.NES, 1)
        Hc, lamc, e2c = oracle.nes_outer_candidate(X, Hn, lamn, H, lam, i ** (1.0 / N))
        if e2c < raw[0]:
            H, lam, e2 = Hc, lamc, e2c
            taken.append(i)
        else:
            H, lam, e2 = Hn, lamn, raw[0]
        want_rel.append(np.sqrt(max(e2, 0.0)))
    assert any(i >= 2 for i in taken), taken
    Ho, lo, ro, _ = oracle.sweeps(X, H0, lam0, oracle.NES_OUTER, nsweeps)
    np.testing.assert_allclose(ro, want_rel, rtol=1e-12, atol=0)
    np.testing.assert_allclose(lo, lam, rtol=1e-12)
    for a, b in zip(Ho, H):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)
    # continuing a run: the outer-iteration number carries over
    Ha, la, ra, _ = oracle.sweeps(X, H0, lam0, oracle.NES_OUTER, 2)
    Hb, lb, rb, _ = oracle.sweeps(X, Ha, la, oracle.NES_OUTER, nsweeps - 2, first_sweep=3)
    np.testing.assert_allclose(np.concatenate([ra, rb]), ro, rtol=1e-12)


def test_nes_outer_sweeps_compose_sweep_and_candidate():
    _check_outer_sweeps()


def test_nes_outer_pins_catch_planted_mistakes(tmp_path):
    # flipped sign of the extrapolation step
    _assert_pin_catches(tmp_path, "outer_sign", "const double v = f + si * (f - fp);",
                        "const double v = f - si * (f - fp);", _check_outer_candidate)
    # exponent N instead of 1/N in s_i
    _assert_pin_catches(tmp_path, "outer_exp", "pow((double)(first_sweep + s), 1.0 / N)",
                        "pow((double)(first_sweep + s), (double)N)", _check_outer_sweeps)
    # the iteration number restarting at 0 instead of 1 (s_1 = 0: no step)
    _assert_pin_catches(tmp_path, "outer_index", "pow((double)(first_sweep + s), 1.0 / N)",
                        "pow((double)(first_sweep + s - 1), 1.0 / N)", _check_outer_sweeps)


# ---------------------------------------------------------------------------
# ADMM stopping test (Section 4.3.4): both residuals below the tolerance
# ---------------------------------------------------------------------------

def _admm_passes_lstsq(A, B, H0, U0, maxit):
    """ADMM passes solved independently of the oracle: each row's Ht
    minimises ||A t - b||^2 + rho ||t - (h + u)||^2 as a stacked least-squares
    problem (lstsq, no normal equations), rho = ||A||_F^2 / R; then
    H = max(0, Ht - U), U += H - Ht.  Returns per pass (H, U, r, s) with the
    squared-norm ratios r = ||H - Ht||^2 / ||H||^2, s = ||H - H_prev||^2 / ||U||^2."""
    R = A.shape[1]
    rho = np.linalg.norm(A) ** 2 / R
    lhs = np.vstack([A, np.sqrt(rho) * np.eye(R)])
    H, U = H0.copy(), U0.copy()
    out = []
    for _ in range(maxit):
        T = np.stack([np.linalg.lstsq(lhs, np.concatenate([b, np.sqrt(rho) * (h + u)]),
                                      rcond=None)[0] for b, h, u in zip(B, H, U)])
        Hn = np.maximum(0.0, T - U)
        Un = U + Hn - T
        r = np.sum((Hn - T) ** 2) / np.sum(Hn ** 2)
        s = np.sum((Hn - H) ** 2) / np.sum(Un ** 2)
        out.append((Hn, Un, r, s))
        H, U = Hn, Un
    return out


def _admm_stop_instance():
    """An instance near the NNLS optimum where, after the first pass, only r
    is below the tolerance: a test that stops when either is below it ends
    after 1 pass, the test of both after 2, and a test on unsquared norms
    (sqrt(r), sqrt(s) < tol) runs all 5 passes."""
    rng = np.random.default_rng(41)
    R = 4
    A = rng.random((30, R))
    B = rng.random((8, 30)) + 0.3 * rng.standard_normal((8, 30))
    S, M = A.T @ A, B @ A
    Xs = np.stack([nnls(A, b)[0] for b in B])
    rho = np.trace(S) / R
    Us = (Xs @ S - M) / rho
    e1 = 10 ** rng.uniform(-4, -1)
    e2 = 10 ** rng.uniform(-4, -1)
    H0 = np.maximum(Xs + e1 * rng.standard_normal(Xs.shape), 0.0)
    U0 = Us + e2 * rng.standard_normal(Xs.shape)
    return A, B, S, M, H0, U0


def _check_admm_stop():
    A, B, S, M, H0, U0 = _admm_stop_instance()
    tol = 0.01
    ref = _admm_passes_lstsq(A, B, H0, U0, 5)

    def stop_after(test):
        return next((k + 1 for k, (_, _, r, s) in enumerate(ref) if test(r, s)), 5)

    both = stop_after(lambda r, s: r < tol and s < tol)
    assert (both, stop_after(lambda r, s: r < tol or s < tol),
            stop_after(lambda r, s: r ** 0.5 < tol and s ** 0.5 < tol)) == (2, 1, 5)
    # no ratio within 20% of the tolerance, so rounding cannot flip a test
    for _, _, r, s in ref:
        for v in (r, s, r ** 0.5, s ** 0.5):
            assert abs(np.log10(v / tol)) > 0.08
    Ho, Uo, passes = oracle.update_admm(H0, U0, M, S, maxit=5, tol=tol)
    assert passes == both, passes
    np.testing.assert_allclose(Ho, ref[both - 1][0], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Uo, ref[both - 1][1], rtol=1e-9, atol=1e-12)


def test_admm_stops_when_both_residuals_are_small():
    _check_admm_stop()


def test_admm_stop_pin_catches_planted_mistakes(tmp_path):
    # either residual instead of both
    _assert_pin_catches(tmp_path, "admm_or", "if (rok && sok) break;", "if (rok || sok) break;",
                        _check_admm_stop)
    # unsquared norm ratios
    _assert_pin_catches(tmp_path, "admm_unsquared",
                        "const int rok = nh > 0.0 ? nd / nh < tol : nd == 0.0;\n"
                        "    const int sok = nu > 0.0 ? nc / nu < tol : nc == 0.0;",
                        "const int rok = nh > 0.0 ? sqrt(nd / nh) < tol : nd == 0.0;\n"
                        "    const int sok = nu > 0.0 ? sqrt(nc / nu) < tol : nc == 0.0;",
                        _check_admm_stop)
