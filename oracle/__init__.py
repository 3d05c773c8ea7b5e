"""CPU oracle for generalized canonical purification (test infrastructure).

TEST INFRASTRUCTURE ONLY: the slow, obviously-correct FP64 reference the GPU
library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
library (``paper_1512_07236_amd``) and never imports it.

Parts:
  * ``purify``            -- the recursion of eq. (hpcp3) step by step, plain C
                             loops in FP64 (``gcp_oracle.c``), from the
                             canonical initial guess of eqs. (dmguess)+(pmcpguess).
  * ``jacobi_eigh`` / ``projector`` -- the definition of the result: the
                             projector onto the N lowest eigenvectors of H
                             (cyclic Jacobi, plain C).
  * ``projector_from_spectrum`` -- the same definition when H = Q diag(lam) Q^T
                             is known by construction (one library matmul).
  * ``scalar_map``        -- the recursion acting on eigenvalues: because every
                             iterate is a polynomial in H, eq. (hpcp3) maps each
                             eigenvalue of D0 by x -> x + 2(x^2(1-x) - c x(1-x))
                             with c formed from power sums of the eigenvalues.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gcp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, BREAKDOWN, INVALID = 0, 1, 2, -1
HIST_COLS = 9
HIST_FIELDS = ("n", "t1", "t2", "t3", "c", "omega", "gamma", "lagrangian", "step")
METHODS = {"hpcp": 0, "pmcp": 1}           # eq. (hpcp3) / eqs. (pm1a),(pm1b)
INITS = {"pmcp": 0, "hp": 1, "search": 2}  # eq. (pmcpguess) / eq. (hpcpguess) / its alpha search


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        i64, dbl, cint = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        L.oracle_matmul.argtypes = [i64, P, P, P]
        L.oracle_matmul_rows.argtypes = [i64, i64, i64, P, P, P]
        L.oracle_gershgorin.argtypes = [i64, P, P, P]
        L.oracle_initial_guess.argtypes = [i64, i64, P, dbl, dbl, P, P, P]
        L.oracle_initial_guess.restype = cint
        L.oracle_purify_from.argtypes = [i64, i64, P, dbl, dbl, cint, P, ctypes.POINTER(cint)]
        L.oracle_purify_from.restype = cint
        L.oracle_purify_from_m.argtypes = [i64, i64, P, cint, dbl, dbl, cint, P,
                                           ctypes.POINTER(cint)]
        L.oracle_purify_from_m.restype = cint
        L.oracle_purify.argtypes = [i64, i64, P, dbl, dbl, dbl, dbl, cint, P, P,
                                    ctypes.POINTER(cint), P]
        L.oracle_purify.restype = cint
        L.oracle_purify_ex.argtypes = [i64, i64, P, dbl, dbl, cint, cint, dbl, dbl, cint, dbl,
                                       dbl, cint, P, P, ctypes.POINTER(cint), P]
        L.oracle_purify_ex.restype = cint
        L.oracle_initial_guess_hp.argtypes = [i64, i64, P, dbl, dbl, cint, dbl, dbl, P, P]
        L.oracle_initial_guess_hp.restype = cint
        L.oracle_jacobi_eigh.argtypes = [i64, P, P, P, dbl, cint]
        L.oracle_jacobi_eigh.restype = cint
        L.oracle_projector.argtypes = [i64, i64, P, P]
        L.oracle_update_at.argtypes = [i64, P, dbl, cint, P, P]
        L.oracle_update_at.restype = cint
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def matmul(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A, B = _f64(A), _f64(B)
    M = A.shape[0]
    C = np.empty((M, M))
    lib().oracle_matmul(M, _p(A), _p(B), _p(C))
    return C


def matmul_rows(A: np.ndarray, B: np.ndarray, r0: int, r1: int) -> np.ndarray:
    A, B = _f64(A), _f64(B)
    M = A.shape[0]
    C = np.empty((r1 - r0, M))
    lib().oracle_matmul_rows(M, r0, r1, _p(A), _p(B), _p(C))
    return C


def gershgorin(H: np.ndarray):
    H = _f64(H)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    lib().oracle_gershgorin(H.shape[0], _p(H), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def initial_guess(H: np.ndarray, N: int, emin: float, emax: float):
    """Returns (D0, mu, beta); raises ValueError on invalid input."""
    H = _f64(H)
    M = H.shape[0]
    D0 = np.empty((M, M))
    mu, beta = ctypes.c_double(), ctypes.c_double()
    st = lib().oracle_initial_guess(M, N, _p(H), emin, emax, _p(D0), ctypes.byref(mu),
                                    ctypes.byref(beta))
    if st != OK:
        raise ValueError("invalid purification input (N out of range or bounds do not bracket mu)")
    return D0, mu.value, beta.value


@dataclass
class Result:
    D: np.ndarray
    status: int
    iters: int
    history: np.ndarray      # (iters+1, HIST_COLS)
    mu: float = float("nan")
    beta: float = float("nan")
    emin: float = float("nan")
    emax: float = float("nan")

    def col(self, name: str) -> np.ndarray:
        return self.history[:, HIST_FIELDS.index(name)]


def purify(H: np.ndarray, N: int, emin: float = float("nan"), emax: float = float("nan"),
           tol_ddbar: float = 1e-6, tol_idem: float = 0.0, max_iter: int = 100) -> Result:
    """Initial guess + HPCP recursion in FP64 (plain C).  NaN bounds -> Gershgorin."""
    H = _f64(H)
    M = H.shape[0]
    D = np.empty((M, M))
    hist = np.full((max_iter + 1, HIST_COLS), np.nan)
    iters = ctypes.c_int()
    scal = np.empty(4)
    st = lib().oracle_purify(M, N, _p(H), emin, emax, tol_ddbar, tol_idem, max_iter, _p(D),
                             _p(hist), ctypes.byref(iters), _p(scal))
    if st == INVALID:
        raise ValueError("invalid purification input")
    n = iters.value
    return Result(D, st, n, hist[: n + 1].copy(), *scal)


def purify_ex(H: np.ndarray, N: int, emin: float = float("nan"), emax: float = float("nan"),
              method: str = "hpcp", init: str = "pmcp", alpha: float = 0.5,
              delta: float = 2.0 / 3.0, tol_ddbar: float = 1e-6, tol_idem: float = 0.0,
              max_iter: int = 100, hole: bool = False) -> Result:
    """purify with a choice of recursion (HPCP eq. (hpcp3) or PMCP eqs.
    (pm1a)/(pm1b)) and initial guess (PMCP guess, hole-particle mix with alpha,
    or the alpha search); hole=True purifies I - D0 and returns I - Dbar_p (the
    history is Dbar's).  Result.alpha is the alpha used (1 = PMCP guess)."""
    H = _f64(H)
    M = H.shape[0]
    D = np.empty((M, M))
    hist = np.full((max_iter + 1, HIST_COLS), np.nan)
    iters = ctypes.c_int()
    scal = np.empty(5)
    st = lib().oracle_purify_ex(M, N, _p(H), emin, emax, METHODS[method], INITS[init], alpha,
                                delta, 1 if hole else 0, tol_ddbar, tol_idem, max_iter, _p(D),
                                _p(hist), ctypes.byref(iters), _p(scal))
    if st == INVALID:
        raise ValueError("invalid purification input")
    n = iters.value
    r = Result(D, st, n, hist[: n + 1].copy(), *scal[:4])
    r.alpha = float(scal[4])
    return r


def initial_guess_hp(H: np.ndarray, N: int, emin: float, emax: float, init: str = "hp",
                     alpha: float = 0.5, delta: float = 2.0 / 3.0):
    """Hole-particle guess of eq. (hpcpguess) as a matrix: (D0+, mu, slope, alpha)."""
    H = _f64(H)
    M = H.shape[0]
    D0 = np.empty((M, M))
    scal = np.empty(3)
    st = lib().oracle_initial_guess_hp(M, N, _p(H), emin, emax, INITS[init], alpha, delta,
                                       _p(D0), _p(scal))
    if st != OK:
        raise ValueError("invalid purification input")
    return D0, float(scal[0]), float(scal[1]), float(scal[2])


def purify_from(D0: np.ndarray, N: int, tol_ddbar: float = 1e-6, tol_idem: float = 0.0,
                max_iter: int = 100, method: str = "hpcp") -> Result:
    """The recursion (HPCP, or PMCP with method="pmcp") from a given symmetric
    D0 (copied)."""
    D = _f64(D0).copy()
    M = D.shape[0]
    hist = np.full((max_iter + 1, HIST_COLS), np.nan)
    iters = ctypes.c_int()
    st = lib().oracle_purify_from_m(M, N, _p(D), METHODS[method], tol_ddbar, tol_idem, max_iter,
                                    _p(hist), ctypes.byref(iters))
    n = iters.value
    return Result(D, st, n, hist[: n + 1].copy())


def update_at(D: np.ndarray, c: float = float("nan"), method: str = "hpcp"):
    """One update of the recursion from the symmetric D at the given c (plain
    C, FP64): eq. (hpcp3) for method "hpcp", eqs. (pm1a)/(pm1b) for "pmcp";
    c = NaN uses the coefficient eq. (hpcp3) forms from D itself.  Returns
    (D', (Tr D, Tr D^2, Tr D^3, c_own)) with c_own = Tr(D^2 Dbar)/Tr(D Dbar)
    from the same products."""
    D = _f64(D)
    M = D.shape[0]
    out = np.empty((M, M))
    tr = np.empty(4)
    if lib().oracle_update_at(M, _p(D), float(c), METHODS[method], _p(out), _p(tr)) != OK:
        raise MemoryError("update_at: allocation failed")
    return out, tuple(float(x) for x in tr)


def power_traces(D: np.ndarray):
    """Tr D, Tr D^2, Tr D^3 and c = (Tr D^2 - Tr D^3)/(Tr D - Tr D^2) of a
    symmetric D by their definitions (FP64; Tr D^2 = sum of D o D and
    Tr D^3 = sum of (D D) o D, one library matmul), for sizes where the plain
    C product would be slow."""
    D = _f64(D)
    X2 = D @ D
    t1, t2, t3 = float(np.trace(D)), float(np.sum(D * D)), float(np.sum(X2 * D))
    return t1, t2, t3, (t2 - t3) / (t1 - t2)


def jacobi_eigh(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Cyclic Jacobi: returns (w ascending, V with eigenvectors as columns, sweeps)."""
    A = _f64(A)
    M = A.shape[0]
    w = np.empty(M)
    V = np.empty((M, M))
    sweeps = lib().oracle_jacobi_eigh(M, _p(A), _p(w), _p(V), tol, max_sweeps)
    if sweeps < 0:
        raise MemoryError("jacobi_eigh: allocation failed")
    return w, V, sweeps


def projector(V: np.ndarray, N: int) -> np.ndarray:
    """Sum of v_i v_i^T over the first N columns of V (eigenvalues ascending)."""
    V = _f64(V)
    M = V.shape[0]
    P = np.empty((M, M))
    lib().oracle_projector(M, N, _p(V), _p(P))
    return P


def ground_state_jacobi(H: np.ndarray, N: int):
    """Definition of the result: projector onto the N lowest eigenvectors of H.
    Returns (P, eigenvalues ascending)."""
    w, V, _ = jacobi_eigh(H)
    return projector(V, N), w


def projector_from_spectrum(Q: np.ndarray, lam: np.ndarray, N: int) -> np.ndarray:
    """Definition of the result for H = Q diag(lam) Q^T: Q_occ Q_occ^T with occ
    the indices of the N smallest lam (library matmul)."""
    occ = np.argsort(lam, kind="stable")[:N]
    Qo = np.ascontiguousarray(Q[:, occ])
    return Qo @ Qo.T


def verify_quantities(D: np.ndarray, H: np.ndarray) -> dict:
    """The acceptance quantities of a density matrix, by their definitions
    (FP64, library matmuls): Tr D, ||D||_F^2, ||D^2 - D||_F, Tr(DH) and
    ||HD - DH||_F, for the symmetric parts of D and H."""
    D = 0.5 * (_f64(D) + _f64(D).T)
    H = 0.5 * (_f64(H) + _f64(H).T)
    return {"trace": float(np.trace(D)), "fro2": float(np.sum(D * D)),
            "idem": float(np.linalg.norm(D @ D - D)), "energy": float(np.sum(D * H)),
            "comm": float(np.linalg.norm(H @ D - D @ H))}


def scalar_map(eps: np.ndarray, N: int, emin: float, emax: float, mu: Optional[float] = None,
               tol_ddbar: float = 1e-6, tol_idem: float = 0.0, max_iter: int = 100,
               method: str = "hpcp", init: str = "pmcp", alpha: float = 0.5,
               delta: float = 2.0 / 3.0, c_given=None):
    """The recursion on eigenvalues (H with known spectrum eps).

    Every iterate is a polynomial in H, so D_n has the eigenvectors of H and
    eigenvalues obtained from x0 = theta + beta (mu - eps) by repeatedly applying
    eq. (hpcp3) to numbers: x <- x + 2 (x^2 (1-x) - c x (1-x)),
    c = sum x^2(1-x) / sum x(1-x).  Returns dict(status, iters, c, t1, t2, t3,
    omega, x) with per-iterate arrays; the same termination rule as ``purify``.

    method "pmcp" maps by eqs. (pm1a)/(pm1b) instead; init "hp" / "search" use
    the hole-particle guess of eq. (hpcpguess) with the given alpha or the
    alpha of the search of eq. (hpcpguessalpha), on eigenvalues (the same
    readings as the C oracle, including the fall-back to the PMCP guess when
    c_0 is outside [0, 1]).

    c_given: update n applies c_given[n] (while there is one) instead of the c
    of the iterate, which is still what the "c" column records: the map then
    follows another solver's trajectory, whose c_n carry that solver's
    rounding, and its traces differ from that solver's by trace rounding only.
    """
    eps = np.asarray(eps, dtype=np.float64)
    M = eps.size
    theta = N / M
    if mu is None:
        mu = float(np.sum(eps)) / M
    beta = 0.0
    alpha_used = 1.0
    if 0 < N < M:
        bt, bb = theta / (emax - mu), (1 - theta) / (mu - emin)
        bmin, bmax = min(bt, bb), max(bt, bb)
        beta = bmin
        if init != "pmcp":
            a = alpha
            if init == "search":
                if theta < 1 - delta:
                    target = N - delta * N
                elif theta > delta:
                    target = N - delta * (M - N)
                else:
                    target = None
                if target is None:
                    a = 0.5
                else:
                    f = [float(np.sum((theta + (t * bmin + (1 - t) * bmax) * (mu - eps)) ** 2))
                         for t in (0.0, 0.5, 1.0)]
                    qa = 2 * f[2] - 4 * f[1] + 2 * f[0]
                    qb = f[2] - f[0] - qa
                    roots = np.roots([qa, qb, f[0] - target]) if qa != 0 else np.array([])
                    roots = [r.real for r in roots if abs(r.imag) == 0]
                    inside = [r for r in roots if 0.0 <= r <= 1.0]
                    if inside:
                        a = inside[0] if len(inside) == 1 else min(inside)
                    elif roots:
                        a = min(roots, key=lambda r: abs(r - 0.5))
                    else:
                        a = 1.0 if f[2] > target else 0.0
                    a = min(1.0, max(0.0, a))
            bhp = a * bmin + (1 - a) * bmax
            x = theta + bhp * (mu - eps)
            t1, t2, t3 = x.sum(), (x * x).sum(), (x ** 3).sum()
            c0 = (t2 - t3) / (t1 - t2) if t1 > t2 else float("nan")
            if 0.0 <= c0 <= 1.0:
                beta, alpha_used = bhp, a
    x = theta + beta * (mu - eps)
    out = {k: [] for k in ("t1", "t2", "t3", "c", "omega")}
    status = NOT_CONVERGED
    n = 0
    while True:
        t1, t2 = x.sum(), (x * x).sum()
        omega = ((x * x - x) ** 2).sum()
        out["t1"].append(t1); out["t2"].append(t2); out["omega"].append(omega)
        if abs(t1 - t2) <= tol_ddbar or np.sqrt(omega) <= tol_idem:
            status = OK
            break
        if n >= max_iter:
            break
        if t1 - t2 <= 0:
            status = BREAKDOWN
            break
        t3 = (x ** 3).sum()
        c = (t2 - t3) / (t1 - t2)
        out["t3"].append(t3); out["c"].append(c)
        if not (0.0 <= c <= 1.0):
            status = BREAKDOWN
            break
        if c_given is not None and n < len(c_given):
            c = float(c_given[n])
        if method == "hpcp":
            x = x + 2.0 * (x * x * (1 - x) - c * x * (1 - x))
        elif c <= 0.5:
            x = ((1 - 2 * c) * x + (1 + c) * x * x - x ** 3) / (1 - c)
        else:
            x = ((1 + c) * x * x - x ** 3) / c
        n += 1
    res = {k: np.array(v) for k, v in out.items()}
    res.update(status=status, iters=n, x=x, beta=beta, mu=mu, alpha=alpha_used)
    return res
