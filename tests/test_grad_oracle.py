"""Pins of the gradient references (oracle/grad.py) -- CPU only.

The hand-written adjoint of eq. (hpcp3) and of the initial guess of eqs.
(dmguess),(pmcpguess) is checked against things it does not compute itself:
  * central finite differences of the forward recursion at a fixed number of
    updates (every term of the step adjoint, the c-term and both branches of
    the beta(mu) min enter at first order, so a dropped term, a sign or a
    transposed product fails);
  * the Daleckii-Krein derivative of the exact ground-state projector, which
    the recursion's gradient reaches at convergence;
  * the degenerate fillings N = 0 and N = M, where D_0 does not depend on H.
"""
import numpy as np
import pytest

import oracle
from oracle import grad
import workloads as W


def _case(M, N, seed):
    H = W.sym_gaussian(M, seed)
    lo, hi = oracle.gershgorin(H)
    return H, lo, hi


def test_forward_iterates_match_oracle(oracle_lib):
    H, lo, hi = _case(20, 7, 1)
    for p in (0, 1, 5):
        Ds, cs, t12, mu, beta = grad.forward_iterates(H, 7, lo, hi, p)
        r = oracle.purify(H, 7, lo, hi, tol_ddbar=0.0, max_iter=p)
        assert r.iters == p
        np.testing.assert_allclose(Ds[-1], r.D, atol=1e-13, rtol=0)
        if p:
            np.testing.assert_allclose(cs, r.col("c")[:p], atol=1e-12, rtol=0)
        assert mu == pytest.approx(r.mu, abs=1e-15) and beta == pytest.approx(r.beta, rel=1e-15)


@pytest.mark.parametrize("M,N,p", [(16, 5, 0), (16, 5, 1), (16, 5, 4), (24, 20, 6), (20, 2, 5),
                                   (18, 9, 3)])
def test_adjoint_matches_finite_differences(oracle_lib, M, N, p):
    H, lo, hi = _case(M, N, 11 + M + N)
    P = W.sym_gaussian(M, 12)
    g = grad.adjoint(H, N, lo, hi, p, P)
    assert np.allclose(g, g.T, atol=0, rtol=0)
    for t in range(3):
        dH = W.sym_gaussian(M, 100 + t)
        fd = grad.loss_fd(H, N, lo, hi, p, P, dH, h=1e-5)
        an = float(np.sum(g * dH))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (t, fd, an)


def test_adjoint_single_element_direction(oracle_lib):
    """A symmetric unit perturbation of one off-diagonal pair and one diagonal
    element: catches a transposed or mis-indexed term that a random direction
    might average out."""
    M, N, p = 12, 4, 3
    H, lo, hi = _case(M, N, 5)
    # a non-symmetric dL/dD: the adjoint takes its symmetric part
    Gp = np.random.default_rng(9).standard_normal((M, M))
    g = grad.adjoint(H, N, lo, hi, p, Gp)
    for (i, j) in [(2, 7), (5, 5)]:
        dH = np.zeros((M, M))
        dH[i, j] = dH[j, i] = 1.0
        fd = grad.loss_fd(H, N, lo, hi, p, Gp, dH, h=1e-5)
        an = float(np.sum(g * dH))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_adjoint_both_beta_branches(oracle_lib):
    """beta = min(theta/(emax-mu), (1-theta)/(mu-emin)): bounds placed so that
    each branch is active in turn, with the other's derivative being wrong."""
    M, N, p = 14, 6, 2
    H = W.sym_gaussian(M, 21)
    mu = np.trace(H) / M
    lo, hi = oracle.gershgorin(H)
    for emin, emax in [(lo, hi + 10.0), (lo - 10.0, hi)]:
        theta = N / M
        first = theta / (emax - mu) <= (1 - theta) / (mu - emin)
        P = W.sym_gaussian(M, 22)
        g = grad.adjoint(H, N, emin, emax, p, P)
        dH = np.eye(M)          # shifts mu only: isolates the beta'(mu) term
        fd = grad.loss_fd(H, N, emin, emax, p, P, dH, h=1e-5)
        an = float(np.sum(g * dH))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (first, fd, an)


@pytest.mark.parametrize("N", [0, 10])
def test_adjoint_degenerate_filling_is_zero(oracle_lib, N):
    """D_0 = 0 or I is already idempotent: the forward stops before any update
    (p = 0) and D_0 does not depend on H (beta = 0)."""
    M = 10
    H, lo, hi = _case(M, N, 3)
    r = oracle.purify(H, N, lo, hi)
    assert r.iters == 0 and r.beta == 0.0
    g = grad.adjoint(H, N, lo, hi, 0, W.sym_gaussian(M, 4))
    assert np.all(g == 0.0)


@pytest.mark.parametrize("M,N,gap,seed", [(64, 20, 0.4, 7), (96, 48, 0.1, 8)])
def test_converged_adjoint_matches_daleckii_krein(oracle_lib, M, N, gap, seed):
    """At convergence D_p is the projector onto the N lowest eigenvectors, so
    the gradient of Tr(D_p P) approaches the exact projector derivative."""
    w = W.spectral(M, N, gap, seed)
    r = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=1e-12)
    assert r.status == oracle.OK
    P = W.sym_gaussian(M, seed + 1)
    g = grad.adjoint(w.H, w.N, w.emin, w.emax, r.iters, P)
    dk = grad.daleckii_krein(w.lam, w.Q, w.N, P)
    assert np.abs(g - dk).max() <= 1e-8 * np.abs(dk).max()


def test_daleckii_krein_matches_finite_differences_of_projector(oracle_lib):
    """The closed form itself, against FD of the eigendecomposition-based projector."""
    M, N = 10, 4
    H = W.sym_gaussian(M, 31)
    P = W.sym_gaussian(M, 32)
    w, V, _ = oracle.jacobi_eigh(H)
    dk = grad.daleckii_krein(w, V, N, P)
    dH = W.sym_gaussian(M, 33)
    h = 1e-6

    def L(Hx):
        ww, VV, _ = oracle.jacobi_eigh(Hx)
        return float(np.sum(oracle.projector(VV, N) * P))

    fd = (L(H + h * dH) - L(H - h * dH)) / (2 * h)
    assert abs(fd - np.sum(dk * dH)) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("alpha", [0.0, 0.5, 0.8])
def test_adjoint_hole_particle_guess_matches_finite_differences(oracle_lib, alpha):
    """The fixed-alpha hole-particle guess: the slope alpha beta_min +
    (1 - alpha) beta_max moves with mu through both branches."""
    M, N, p = 16, 7, 3
    H, lo, hi = _case(M, N, 41)
    P = W.sym_gaussian(M, 42)
    g = grad.adjoint(H, N, lo, hi, p, P, alpha=alpha)
    for dH in (W.sym_gaussian(M, 43), np.eye(M)):
        fd = grad.loss_fd(H, N, lo, hi, p, P, dH, h=1e-5, alpha=alpha)
        an = float(np.sum(g * dH))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (alpha, fd, an)


@pytest.mark.parametrize("M,N,p", [(16, 5, 4), (20, 14, 5), (18, 9, 6)])
def test_pmcp_adjoint_matches_finite_differences(oracle_lib, M, N, p):
    """The PMCP recursion, eqs. (pm1a)/(pm1b): both coefficient branches
    (c <= 1/2 and c > 1/2) appear among the cases, and each enters through
    its coefficients and their c-derivatives."""
    H, lo, hi = _case(M, N, 61 + M + N)
    P = W.sym_gaussian(M, 62)
    _, cs, *_ = grad.forward_iterates(H, N, lo, hi, p, method="pmcp")
    g = grad.adjoint(H, N, lo, hi, p, P, method="pmcp")
    for t in range(3):
        dH = W.sym_gaussian(M, 200 + t)
        fd = grad.loss_fd(H, N, lo, hi, p, P, dH, h=1e-5, method="pmcp")
        an = float(np.sum(g * dH))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (t, fd, an, cs)


def test_pmcp_cases_cover_both_branches(oracle_lib):
    seen = set()
    for M, N, p in ((16, 5, 4), (20, 14, 5), (18, 9, 6)):
        H, lo, hi = _case(M, N, 61 + M + N)
        _, cs, *_ = grad.forward_iterates(H, N, lo, hi, p, method="pmcp")
        seen |= {bool(c > 0.5) for c in cs}
    assert seen == {False, True}


def test_pmcp_forward_iterates_match_oracle(oracle_lib):
    H, lo, hi = _case(20, 14, 95)
    Ds, cs, *_ = grad.forward_iterates(H, 14, lo, hi, 5, method="pmcp")
    r = oracle.purify_ex(H, 14, lo, hi, method="pmcp", init="pmcp", tol_ddbar=0.0, max_iter=5)
    assert r.iters == 5
    np.testing.assert_allclose(Ds[-1], r.D, atol=1e-13, rtol=0)


@pytest.mark.parametrize("M,N", [(20, 3), (20, 17), (24, 5)])
def test_alpha_search_adjoint_matches_finite_differences(oracle_lib, M, N):
    """The alpha search of eq. (hpcpguessalpha): the slope follows
    ||mu I - H||_F, so the gradient gains a term along mu I - H.  Directions:
    random, the identity (no change of S), and mu I - H itself (all of the
    change of S)."""
    H, lo, hi = _case(M, N, 71 + M + N)
    P = W.sym_gaussian(M, 72)
    *_, alpha, searched = grad.guess(H, N, lo, hi, init="search")
    assert searched and 0.0 < alpha < 1.0
    p = 4
    for method in ("hpcp", "pmcp"):
        g = grad.adjoint(H, N, lo, hi, p, P, method=method, init="search")
        mu = np.trace(H) / M
        for dH in (W.sym_gaussian(M, 73), np.eye(M), mu * np.eye(M) - H):
            fd = grad.loss_fd(H, N, lo, hi, p, P, dH, h=1e-5, method=method, init="search")
            an = float(np.sum(g * dH))
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (method, fd, an)


def test_alpha_search_term_is_needed(oracle_lib):
    """Dropping the search term (treating the searched alpha as fixed) breaks
    the finite-difference agreement along mu I - H."""
    M, N, p = 20, 3, 4
    H, lo, hi = _case(M, N, 71 + M + N)
    P = W.sym_gaussian(M, 72)
    *_, alpha, _ = grad.guess(H, N, lo, hi, init="search")
    g_fixed = grad.adjoint(H, N, lo, hi, p, P, alpha=alpha)
    dH = np.trace(H) / M * np.eye(M) - H
    fd = grad.loss_fd(H, N, lo, hi, p, P, dH, h=1e-5, init="search")
    assert abs(fd - float(np.sum(g_fixed * dH))) > 1e-4 * max(1.0, abs(fd))
