"""Gradient references for the purification (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

The loss is any L(D_p) of the final iterate; the caller supplies
Gbar_p = dL/dD_p.  Every update is differentiated by hand.  Both recursions
are D' = a D + b D^2 + e D^3 with coefficients of c = (T2 - T3)/(T1 - T2),
T_k = Tr D^k:
    HPCP, eq. (hpcp3):            a = 1 - 2c, b = 2 + 2c, e = -2;
    PMCP, eq. (pm1a), c <= 1/2:   a = (1 - 2c)/(1 - c), b = (1 + c)/(1 - c),
                                  e = -1/(1 - c);
    PMCP, eq. (pm1b), c > 1/2:    a = 0, b = (1 + c)/c, e = -1/c.
For symmetric D and Gbar' (= dL/dD'):

    A     = Gbar' D
    Gbar  = a Gbar' + b (A + A^T) + e (A D + (A D)^T + D A) + kappa grad_c
    kappa = <Gbar', dD'/dc> = <Gbar', a'(c) D + b'(c) D^2 + e'(c) D^3>
    grad_c = [(2 D - 3 D^2) - c (I - 2 D)] / (T1 - T2)

The initial guess D0 = theta I + beta (mu I - H), mu = Tr(H)/M, with the
bounds held fixed: eqs. (dmguess),(pmcpguess) take beta = beta_min, the
hole-particle guess of eq. (hpcpguess) beta = alpha beta_min + (1 - alpha)
beta_max with a fixed alpha, and

    dL/dH = -beta Gbar0 + (I/M) [beta Tr Gbar0 + beta'(mu) <Gbar0, mu I - H>],

where beta' is that of the active branch of the min: theta/(emax - mu)^2 or
-(1-theta)/(mu - emin)^2 (for the hole-particle guess, alpha times the min
branch's plus 1 - alpha times the max branch's).  The alpha search of eq.
(hpcpguessalpha) picks the slope at which Tr D0^2 = Mtheta^2 + beta^2 S hits
its target, S = ||mu I - H||_F^2: beta = sqrt((target - M theta^2)/S), which
depends on H only through S (not on mu or the bounds, while alpha stays
inside (0, 1)).  With g = mu I - H (Tr g = 0), d beta = (beta/S) <g, dH>, so

    dL/dH = -beta Gbar0 + (beta Tr Gbar0 / M) I + (beta <Gbar0, g> / S) g.

``adjoint`` is written in FP64 numpy with library matmuls.  It is pinned by
central finite differences of the oracle's forward recursion, at a fixed
number of updates, and by the Daleckii-Krein formula at convergence
(``daleckii_krein``).
"""
from __future__ import annotations

import numpy as np

from . import initial_guess, initial_guess_hp


def coefficients(c: float, method: str = "hpcp"):
    """(a, b, e) of D' = a D + b D^2 + e D^3 and their derivatives in c."""
    if method == "hpcp":
        return (1 - 2 * c, 2 + 2 * c, -2.0), (-2.0, 2.0, 0.0)
    if c <= 0.5:
        r = 1.0 / (1.0 - c)
        return ((1 - 2 * c) * r, (1 + c) * r, -r), (-r * r, 2 * r * r, -r * r)
    r = 1.0 / c
    return (0.0, (1 + c) * r, -r), (0.0, -r * r, r * r)


def guess(H: np.ndarray, N: int, emin: float, emax: float, alpha: float = 1.0,
          init: str | None = None):
    """D0, mu, slope beta, alpha and whether alpha came from the search
    (strictly inside (0, 1)).  init None: alpha = 1 is the PMCP guess, other
    alpha the fixed hole-particle guess; init "search": the alpha search."""
    if init == "search":
        D, mu, beta, a = initial_guess_hp(H, N, emin, emax, "search")
        M = H.shape[0]
        theta = N / M
        delta = 2.0 / 3.0
        has_target = theta < 1.0 - delta or theta > delta
        return D, mu, beta, a, bool(has_target and 0.0 < a < 1.0 and 0 < N < M)
    if alpha == 1.0:
        D, mu, beta = initial_guess(H, N, emin, emax)
        return D, mu, beta, 1.0, False
    D, mu, beta, a = initial_guess_hp(H, N, emin, emax, "hp", alpha=alpha)
    return D, mu, beta, a, False


def forward_iterates(H: np.ndarray, N: int, emin: float, emax: float, p: int,
                     alpha: float = 1.0, method: str = "hpcp", init: str | None = None):
    """D_0..D_p of the recursion (plain FP64, symmetrised each step) and
    c_0..c_{p-1}; see ``guess`` for alpha and init."""
    D, mu, beta, _, _ = guess(H, N, emin, emax, alpha, init)
    Ds, cs, t12 = [D], [], []
    for _ in range(p):
        X2 = D @ D
        X3 = X2 @ D
        t1, t2, t3 = np.trace(D), np.trace(X2), np.trace(X3)
        c = (t2 - t3) / (t1 - t2)
        (a, b, e), _ = coefficients(c, method)
        Dn = a * D + b * X2 + e * X3
        D = 0.5 * (Dn + Dn.T)
        Ds.append(D)
        cs.append(c)
        t12.append(t1 - t2)
    return Ds, np.array(cs), np.array(t12), mu, beta


def adjoint(H: np.ndarray, N: int, emin: float, emax: float, p: int, Gbar_p: np.ndarray,
            alpha: float = 1.0, method: str = "hpcp", init: str | None = None):
    """dL/dH for L(D_p), given Gbar_p = dL/dD_p (symmetrised here); alpha and
    init select the guess as in ``guess``, method the recursion."""
    M = H.shape[0]
    Ds, cs, t12, mu, beta = forward_iterates(H, N, emin, emax, p, alpha, method, init)
    _, _, _, alpha_used, searched = guess(H, N, emin, emax, alpha, init)
    G = 0.5 * (Gbar_p + Gbar_p.T)
    I = np.eye(M)
    for n in range(p - 1, -1, -1):
        D, c = Ds[n], cs[n]
        (a, b, e), (da, db, de) = coefficients(c, method)
        X2 = D @ D
        A = G @ D
        AD = A @ D
        DA = D @ A
        kappa = da * np.sum(G * D) + db * np.sum(G * X2) + de * np.sum(G * (X2 @ D))
        grad_c = ((2 * D - 3 * X2) - c * (I - 2 * D)) / t12[n]
        G = a * G + b * (A + A.T) + e * (AD + AD.T + DA) + kappa * grad_c
        G = 0.5 * (G + G.T)
    theta = N / M
    g = mu * I - H
    if searched:
        S = float(np.sum(g * g))
        dH = -beta * G + I / M * (beta * np.trace(G)) + (beta * np.sum(G * g) / S) * g
        return 0.5 * (dH + dH.T)
    if 0 < N < M:
        bt, bb = theta / (emax - mu), (1 - theta) / (mu - emin)
        dbt, dbb = theta / (emax - mu) ** 2, -(1 - theta) / (mu - emin) ** 2
        dmin, dmax = (dbt, dbb) if bt <= bb else (dbb, dbt)
        dbeta = alpha_used * dmin + (1 - alpha_used) * dmax
    else:
        dbeta = 0.0
    dH = -beta * G + I / M * (beta * np.trace(G) + dbeta * np.sum(G * g))
    return 0.5 * (dH + dH.T)


def loss_fd(H, N, emin, emax, p, P, dH, h=1e-6, alpha=1.0, method="hpcp", init=None):
    """Central difference of L = Tr(D_p P) along the symmetric direction dH
    (the bounds fixed; the alpha search, if any, redone at H +- h dH)."""
    def L(Hx):
        Ds, *_ = forward_iterates(Hx, N, emin, emax, p, alpha, method, init)
        return float(np.sum(Ds[-1] * P))
    return (L(H + h * dH) - L(H - h * dH)) / (2 * h)


def daleckii_krein(eps: np.ndarray, V: np.ndarray, N: int, P: np.ndarray) -> np.ndarray:
    """Gradient of L = Tr(D P) with D the projector onto the N lowest
    eigenvectors of H = V diag(eps) V^T:
        dL/dH = V (F o (V^T Psym V)) V^T,  F_ij = (n_i - n_j)/(eps_i - eps_j)
    (0 when n_i = n_j), n = occupations.  Returned symmetric."""
    order = np.argsort(eps, kind="stable")
    n = np.zeros_like(eps)
    n[order[:N]] = 1.0
    dn = n[:, None] - n[None, :]
    de = eps[:, None] - eps[None, :]
    F = np.where(dn != 0, dn / np.where(de == 0, 1.0, de), 0.0)
    Ps = 0.5 * (P + P.T)
    G = V @ (F * (V.T @ Ps @ V)) @ V.T
    return 0.5 * (G + G.T)
