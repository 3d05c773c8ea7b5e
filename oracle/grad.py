"""Gradient references for the purification (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

The loss is any L(D_p) of the final iterate; the caller supplies
Gbar_p = dL/dD_p.  Every step of eq. (hpcp3) is differentiated by hand,
D' = a D + b D^2 - 2 D^3 with a = 1 - 2c, b = 2 + 2c and
c = (T2 - T3)/(T1 - T2), T_k = Tr D^k.  For symmetric D and Gbar':

    A     = Gbar' D
    Gbar  = a Gbar' + b (A + A^T) - 2 (A D + (A D)^T + D A) + kappa grad_c
    kappa = <Gbar', dD'/dc> = 2 (<Gbar', D^2> - <Gbar', D>)
    grad_c = [(2 D - 3 D^2) - c (I - 2 D)] / (T1 - T2)

The initial guess of eqs. (dmguess),(pmcpguess) has D0 = theta I + beta(mu)
(mu I - H), with mu = Tr(H)/M and the bounds held fixed (the hole-particle
guess of eq. (hpcpguess) with a fixed alpha has the same form with
beta = alpha beta_min + (1 - alpha) beta_max):

    dL/dH = -beta Gbar0 + (I/M) [beta Tr Gbar0 + beta'(mu) <Gbar0, mu I - H>],

where beta' is that of the active branch of the min:
theta/(emax - mu)^2 or -(1-theta)/(mu - emin)^2 (for the hole-particle guess,
alpha times the min branch's plus 1 - alpha times the max branch's).

``adjoint`` is written in FP64 numpy with library matmuls.  It is pinned by
central finite differences of the oracle's forward recursion, at a fixed
number of updates, and by the Daleckii-Krein formula at convergence
(``daleckii_krein``).
"""
from __future__ import annotations

import numpy as np

from . import initial_guess, initial_guess_hp


def forward_iterates(H: np.ndarray, N: int, emin: float, emax: float, p: int,
                     alpha: float = 1.0):
    """D_0..D_p of eq. (hpcp3) (plain FP64, symmetrised each step) and c_0..c_{p-1};
    alpha < 1 starts from the hole-particle guess of eq. (hpcpguess)."""
    if alpha == 1.0:
        D, mu, beta = initial_guess(H, N, emin, emax)
    else:
        D, mu, beta, _ = initial_guess_hp(H, N, emin, emax, "hp", alpha=alpha)
    Ds, cs, t12 = [D], [], []
    for _ in range(p):
        X2 = D @ D
        X3 = X2 @ D
        t1, t2, t3 = np.trace(D), np.trace(X2), np.trace(X3)
        c = (t2 - t3) / (t1 - t2)
        Dn = (1 - 2 * c) * D + (2 + 2 * c) * X2 - 2 * X3
        D = 0.5 * (Dn + Dn.T)
        Ds.append(D)
        cs.append(c)
        t12.append(t1 - t2)
    return Ds, np.array(cs), np.array(t12), mu, beta


def adjoint(H: np.ndarray, N: int, emin: float, emax: float, p: int, Gbar_p: np.ndarray,
            alpha: float = 1.0):
    """dL/dH for L(D_p), given Gbar_p = dL/dD_p (symmetrised here).  alpha < 1:
    the hole-particle guess, slope alpha beta_min + (1 - alpha) beta_max with
    alpha fixed."""
    M = H.shape[0]
    Ds, cs, t12, mu, beta = forward_iterates(H, N, emin, emax, p, alpha)
    G = 0.5 * (Gbar_p + Gbar_p.T)
    I = np.eye(M)
    for n in range(p - 1, -1, -1):
        D, c = Ds[n], cs[n]
        a, b = 1 - 2 * c, 2 + 2 * c
        X2 = D @ D
        A = G @ D
        AD = A @ D
        DA = D @ A
        kappa = 2.0 * (np.sum(G * X2) - np.sum(G * D))
        grad_c = ((2 * D - 3 * X2) - c * (I - 2 * D)) / t12[n]
        G = a * G + b * (A + A.T) - 2 * (AD + AD.T + DA) + kappa * grad_c
        G = 0.5 * (G + G.T)
    theta = N / M
    if 0 < N < M:
        bt, bb = theta / (emax - mu), (1 - theta) / (mu - emin)
        dbt, dbb = theta / (emax - mu) ** 2, -(1 - theta) / (mu - emin) ** 2
        dmin, dmax = (dbt, dbb) if bt <= bb else (dbb, dbt)
        dbeta = alpha * dmin + (1 - alpha) * dmax
    else:
        dbeta = 0.0
    dH = -beta * G + I / M * (beta * np.trace(G) + dbeta * np.sum(G * (mu * I - H)))
    return 0.5 * (dH + dH.T)


def loss_fd(H, N, emin, emax, p, P, dH, h=1e-6, alpha=1.0):
    """Central difference of L = Tr(D_p P) along the symmetric direction dH."""
    def L(Hx):
        Ds, *_ = forward_iterates(Hx, N, emin, emax, p, alpha)
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
