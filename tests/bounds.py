"""Rounding-error bounds of the GPU purification's arithmetic (test helper).

The bounds are derived from the unit roundoff of each operand encoding and of
the FP32 (or FP64) accumulation of the matrix products, never from a
measurement.  They are used by the element-wise parity tests, which check the
GPU one update at a time: from the GPU's own iterate D_n (its master values,
returned exactly in FP64) and its own coefficient c_n, the oracle's update in
FP64 must agree with the GPU's D_{n+1} within the bound, element by element.

Notation: u32 = 2^-24, u64 = 2^-53.  For one output element of a product
X = A B (A, B symmetric masters), P_ij = sum_k |A_ik| |B_kj|.

Worst-case model (bounds "det"):
  * every FP32 addition of the accumulation, and every rounded product, has
    relative error at most 2 u32 of the running value (the factor 2 also
    covers round-toward-zero); the running value never exceeds P_ij, so
    |error| <= 2 u32 kappa P_ij with kappa the number of rounding steps a term
    passes through (recursive-summation bound, first order);
  * 16-bit products: each K stage adds `terms` products (K values per stage x
    split products), a chunk accumulator holds `fold` stages, and the chunk
    is added into a running total: kappa = terms*fold + ceil(stages/fold) + 2
    (the 2 covers the K-split partial sum rounded once to FP32);
    FP32 products: the same with 32 K values per stage;
    FP64 products: one accumulator over K, kappa = K + 1;
  * split encodings drop the small cross products (lo*lo; for three planes
    mid*lo, lo*mid, lo*lo): at most u_drop P_ij;
  * encoding an element x to its planes errs by at most u_enc |x| + a_enc
    (a_enc: the float16 subnormal floor).

Statistical model (bounds "sigma"), for sums of many element errors such as
the traces: the rounding errors are independent and zero-mean with
|delta| <= r uniformly distributed (variance <= r^2/3); a sum is then bounded
by 6 standard deviations.
"""
from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53

# float16 encodings store 2^10 x (subnormal half-spacing 2^-25 in those units)
F16_SCALE = 1024.0
_F16_ABS = 2.0 ** -25 / F16_SCALE

_E_BF = 2.0 ** -8 + 2.0 ** -24    # float -> bfloat16 (8-bit significand) after double -> float
_E_H = 2.0 ** -11 + 2.0 ** -24    # float -> float16 (11-bit significand) after double -> float

PLANES = {"fp64": 1, "fp32": 1, "bf16": 1, "fp16": 1, "bf16x3": 2, "fp16x3": 2, "bf16x6": 3}
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16": 1, "fp16": 1, "bf16x3": 3, "fp16x3": 3, "bf16x6": 6}


def encoding(precision: str):
    """(u_enc, a_enc, u_drop) of an encoding.

    u_enc/a_enc bound |x - dec(enc(x))| <= u_enc |x| + a_enc.  Split planes
    are formed from exact residuals (x - hi is exact by Sterbenz's lemma), so
    each level multiplies the relative error by the level's roundoff.
    u_drop bounds the dropped cross products relative to |a||b|."""
    if precision == "fp64":
        return U64, 0.0, 0.0
    if precision == "fp32":
        return U32, 2.0 ** -150, 0.0
    if precision == "bf16":
        return _E_BF, 2.0 ** -134, 0.0
    if precision == "fp16":
        return _E_H, _F16_ABS, 0.0
    if precision == "bf16x3":
        e = _E_BF
        return e * e, 2.0 ** -134, (e * (1 + e)) ** 2
    if precision == "fp16x3":
        e = _E_H
        return e * e, (1 + e) * _F16_ABS, (e * (1 + e)) ** 2
    if precision == "bf16x6":
        e = _E_BF
        lvl = e * (1 + e)
        return e ** 3, 2.0 ** -134, 2 * lvl ** 3 + lvl ** 4
    raise ValueError(precision)


def padded(M: int) -> int:
    return (M + 255) // 256 * 256


def accumulation_kappa(M: int, precision: str, fold_every: int = 0, ksplit: int = 0) -> int:
    """Rounding steps a product term passes through in the library's
    accumulation scheme (worst case), for the launch configuration the
    library chooses at size M.  ksplit >= 2 (16-bit encodings): every block
    accumulates stages / ksplit and the blocks' totals meet in FP64, whose
    rounding is below first order here."""
    Mp = padded(M)
    if precision == "fp64":
        return Mp + 1
    if precision == "fp32":
        # stages of 32 K values, 8 MFMA steps each; default fold sqrt(stages / 8)
        stages = Mp // 32
        fold = fold_every if fold_every > 0 else max(1, int(math.sqrt(stages / 8) + 0.5))
        fold = min(fold, stages)
        return 32 * fold + math.ceil(stages / fold) + 2
    np_ = PLANES[precision]
    # K per stage: 64 values of one plane, or 32 values of every plane
    stages = Mp * np_ // 64 if np_ <= 2 else Mp // 32
    per_stage = 2 if np_ == 1 else PRODUCTS[precision]   # products per stage and element
    ks = min(ksplit, stages) if ksplit >= 2 else 1
    # the library rounds half away from zero (lround)
    fold = fold_every if fold_every > 0 else max(1, int(math.floor(math.sqrt(stages / ks / per_stage) + 0.5)))
    own = -(-stages // ks)   # stages of the longest split
    fold = min(fold, own)
    terms = 32 * per_stage
    return terms * fold + math.ceil(own / fold) + 2


def unit(precision: str) -> float:
    return U64 if precision == "fp64" else U32


def product_bound(A: np.ndarray, B: np.ndarray, M: int, precision: str, fold_every: int = 0,
                  ksplit: int = 0):
    """Element-wise bound on |fl(A B) - A B| for the GPU product of two
    masters (off-diagonal elements), and P = |A| |B|."""
    u_enc, a_enc, u_drop = encoding(precision)
    P = np.abs(A) @ np.abs(B)
    kappa = accumulation_kappa(M, precision, fold_every, ksplit)
    # 1.01: the split terms sum to at most (1 + 3 u_lvl) |a||b|
    rel = 1.01 * (2.0 * unit(precision) * kappa + u_drop)
    K = A.shape[0]
    absd = 0.0
    if precision in ("fp16x3",):
        # float16 subnormal floors of the dropped lo*lo terms
        e = _E_H * (1 + _E_H)
        f = 2.0 * _F16_ABS * F16_SCALE
        absd = (e * f / F16_SCALE) * (np.abs(A).sum(1)[:, None] + np.abs(B).sum(0)[None, :]) \
            + K * (f / F16_SCALE) ** 2
    return rel * P + absd, P


def step_bounds(D: np.ndarray, c: float, precision: str, fold_every: int = 0,
                method: str = "hpcp", ksplit: int = 0):
    """Bounds for one GPU update from the master D (FP64) at coefficient c.

    Returns a dict with
      dD   : element-wise bound on |D'_gpu - D'_oracle| (the oracle's update
             at the same c from the same D),
      T3_det, T3_sig : bounds on |T3_gpu - Tr(D^3)| (worst case, and 6 sigma
             of the statistical model),
      T2, T1 : bounds on the FP64 trace sums,
    all first order in the roundoff."""
    M = D.shape[0]
    u = unit(precision)
    u_enc, a_enc, u_drop = encoding(precision)
    A = np.abs(D)
    off = ~np.eye(M, dtype=bool)
    X2 = D @ D
    # K1: X2 = D D, then encoded (off-diagonal); diagonal from FP64 row sums
    dP1, P1 = product_bound(D, D, M, precision, fold_every, ksplit)
    rowsq = (D * D).sum(1)
    E1 = np.where(off, dP1 + u_enc * (np.abs(X2) + dP1) + a_enc, 0.0)
    E1[np.diag_indices(M)] = 2 * M * U64 * rowsq + 4 * M * U64 * np.diag(P1)
    # the oracle's own FP64 products
    E1 = E1 + 2 * M * U64 * P1
    X2m = X2   # master of X2 to first order
    # K2: X3 = X2 D (product of the masters)
    dP2, P2 = product_bound(X2m, D, M, precision, fold_every, ksplit)
    if method == "hpcp":
        a, b, e = 1 - 2 * c, 2 + 2 * c, -2.0
    elif c <= 0.5:
        a, b, e = (1 - 2 * c) / (1 - c), (1 + c) / (1 - c), -1 / (1 - c)
    else:
        a, b, e = 0.0, (1 + c) / c, -1 / c
    X3 = X2 @ D
    Dn = a * D + b * X2 + e * X3
    dX3 = E1 @ A + dP2 + 2 * M * U64 * P2
    fp64 = 16 * U64 * (np.abs(a * D) + np.abs(b * X2) + np.abs(e * X3))
    dD = np.abs(b) * E1 + np.abs(e) * dX3 + fp64
    # diagonal: FP64 from d2 (row sums) and d3 = sum_k X2m_ik D_ik
    d3err = (E1 * A).sum(1) + 2 * M * U64 * (np.abs(X2) * A).sum(1)
    dD[np.diag_indices(M)] = (np.abs(b) * np.diag(E1) + np.abs(e) * d3err + np.diag(fp64))
    # the new off-diagonal master is encoded
    dD = dD + np.where(off, u_enc * (np.abs(Dn) + dD) + a_enc, 0.0)
    # traces
    T1 = 4 * M * U64 * np.abs(np.diag(D)).sum()
    T2 = 4 * M * U64 * (D * D).sum()
    T3_det = (E1 * A).sum() + 4 * M * U64 * (np.abs(X2) * A).sum()
    # statistical: Var E1_ij <= (2 u)^2 kappa P1^2 / 3 + (u_enc X2)^2 / 3 + u_drop^2 sum a^2 b^2 / 9;
    # each off-diagonal pair enters T3 twice with the same (mirrored) error
    kappa = accumulation_kappa(M, precision, fold_every, ksplit)
    D2sq = D * D
    var = ((2 * u) ** 2 * kappa * (1.01 * P1) ** 2 / 3 + (u_enc * X2) ** 2 / 3
           + (u_drop ** 2 / 9) * (D2sq @ D2sq) + a_enc ** 2 / 3)
    var_T3 = 2.0 * float((D2sq * var)[off].sum())
    T3_sig = 6.0 * math.sqrt(var_T3) + 4 * M * U64 * (np.abs(X2) * A).sum() \
        + float((np.diag(E1) * np.diag(A)).sum())
    return {"dD": dD, "T1": T1, "T2": T2, "T3_det": T3_det, "T3_sig": T3_sig}


def c_bound(t1: float, t2: float, t3: float, dT1: float, dT2: float, dT3: float) -> float:
    """First-order bound on |c - c_exact| for c = (T2 - T3)/(T1 - T2) given
    bounds on the traces' errors."""
    dd = abs(t1 - t2)
    return (dT2 + dT3) / dd + abs(t2 - t3) * (dT1 + dT2) / dd ** 2 + 8 * U64 * (1 + abs(t2 - t3) / dd)


def max_abs_bound(fro_err: float, M: int, nsigma: float = 10.0) -> float:
    """Largest element of an error matrix E = Q F Q^T whose basis Q is a
    random orthogonal matrix: its entries are close to Gaussian with standard
    deviation at most sqrt(2) ||E||_F / M (the diagonal ones have twice the
    variance of the off-diagonal ones), so no entry exceeds nsigma of that
    (probability below 1e-15 per entry at 10 sigma).  A single misplaced or
    wrongly stored element shows up as an outlier far above it."""
    return nsigma * math.sqrt(2.0) * fro_err / M
