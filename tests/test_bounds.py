"""CPU checks of the element-wise rounding bounds (tests/bounds.py).

An emulation of one FP16X3 update in numpy follows the arithmetic the bounds
model: the off-diagonal iterate split into float16 hi/lo planes of 2^10 x,
the three products hi*hi, hi*lo, lo*hi accumulated term by term in float32
(chunk accumulator folded into a float32 total), the diagonal kept in FP64
with the residual correction, the update formed in FP64 and encoded again.
The bound must hold for it, and a single planted error of the size a wrong
or misplaced element would have must break it.
"""
import math

import numpy as np
import pytest

import oracle
from bounds import accumulation_kappa, encoding, step_bounds


def enc_fp16x3(x):
    y = (x * 1024.0)
    hi = y.astype(np.float32).astype(np.float16)
    lo = (y - hi.astype(np.float64)).astype(np.float32).astype(np.float16)
    return hi, lo


def dec_fp16x3(hi, lo):
    return (hi.astype(np.float64) + lo.astype(np.float64)) / 1024.0


def emulated_product(Ah, Al, Bh, Bl, fold, stage=32):
    """sum over K of hi*hi + hi*lo + lo*hi, term by term in float32, a chunk
    accumulator of `fold` stages added into a float32 total; 2^-20 scale."""
    M = Ah.shape[0]
    tot = np.zeros((M, M), np.float32)
    acc = np.zeros((M, M), np.float32)
    nst = M // stage
    for s in range(nst):
        for k in range(s * stage, (s + 1) * stage):
            for a, b in ((Ah, Bh), (Ah, Bl), (Al, Bh)):
                acc = (acc + np.outer(a[:, k].astype(np.float32), b[k, :].astype(np.float32))
                       .astype(np.float32)).astype(np.float32)
        if (s + 1) % fold == 0 or s == nst - 1:
            tot = (tot + acc).astype(np.float32)
            acc[:] = 0
    return tot.astype(np.float64) / 1024.0 ** 2


def emulated_step(D, c, fold):
    M = D.shape[0]
    off = ~np.eye(M, dtype=bool)
    dg = np.diag(D).copy()
    hi, lo = enc_fp16x3(D)
    Dm = np.where(off, dec_fp16x3(hi, lo), D)
    r = dg - np.diag(dec_fp16x3(hi, lo))
    # K1
    v = emulated_product(hi, lo, hi.T, lo.T, fold)   # B rows of D = columns (symmetric)
    x2 = v + Dm * (r[:, None] + r[None, :])
    d2 = (Dm * Dm).sum(1)
    h2, l2 = enc_fp16x3(x2)
    X2m = np.where(off, dec_fp16x3(h2, l2), 0.0)
    X2m[np.diag_indices(M)] = d2
    s2 = d2 - np.diag(dec_fp16x3(h2, l2))
    d3 = (X2m * Dm).sum(1)
    # K2
    h2[np.diag_indices(M)], l2[np.diag_indices(M)] = enc_fp16x3(d2)
    s2 = d2 - dec_fp16x3(*enc_fp16x3(d2))
    v3 = emulated_product(h2, l2, hi.T, lo.T, fold)
    x3 = v3 + X2m * r[None, :] + s2[:, None] * Dm
    a, b, e = 1 - 2 * c, 2 + 2 * c, -2.0
    dn = a * Dm + b * X2m + e * x3
    hn, ln = enc_fp16x3(dn)
    out = np.where(off, dec_fp16x3(hn, ln), 0.0)
    out[np.diag_indices(M)] = a * dg + b * d2 + e * d3
    out = np.triu(out) + np.triu(out, 1).T    # upper tiles mirrored
    return out, float(d3.sum())


@pytest.fixture(scope="module")
def iterate():
    import workloads
    w = workloads.spectral(256, 97, gap=0.1, seed=77)
    D0, _, _ = oracle.initial_guess(w.H, w.N, w.emin, w.emax)
    hi, lo = enc_fp16x3(D0)
    off = ~np.eye(256, dtype=bool)
    return np.where(off, dec_fp16x3(hi, lo), D0)   # a master iterate


def test_emulated_fp16x3_step_within_bound_and_planted_error_caught(oracle_lib, iterate):
    D = iterate
    _, (t1, t2, t3, c) = oracle.update_at(D)
    stages = 256 * 2 // 64
    fold = max(1, int(round(math.sqrt(stages / 3))))
    assert accumulation_kappa(256, "fp16x3") == 96 * fold + math.ceil(stages / fold) + 2
    got, t3_emu = emulated_step(D, c, fold)
    ref, _ = oracle.update_at(D, c)
    bb = step_bounds(D, c, "fp16x3")
    b = bb["dD"]
    # T3 from the emulated epilogue sums, within both trace bounds
    assert abs(t3_emu - t3) <= bb["T3_sig"] <= bb["T3_det"]
    diff = np.abs(got - ref)
    assert np.all(diff <= b), float((diff / b).max())
    # the bound is not vacuous: it sits far below the size of an element
    off = ~np.eye(256, dtype=bool)
    assert np.median(b[off] / np.abs(ref[off])) < 5e-3
    for (i, j), delta in (((3, 7), 5e-5), ((100, 30), 1e-4), ((5, 5), 2e-4)):
        bad = got.copy()
        bad[i, j] += delta
        assert not np.all(np.abs(bad - ref) <= b), (i, j, delta)
    # an element stored from its neighbour (a misplaced mirror or tile store)
    for (i, j) in ((3, 7), (200, 17), (128, 127)):
        bad = got.copy()
        bad[i, j] = got[i, j + 1]
        assert not np.all(np.abs(bad - ref) <= b), (i, j)


def test_wrong_sign_of_the_cubic_term_is_caught(oracle_lib, iterate):
    """Forming the update with +2 D^3 instead of -2 D^3 exceeds the bound."""
    D = iterate
    _, (_, _, _, c) = oracle.update_at(D)
    ref, _ = oracle.update_at(D, c)
    b = step_bounds(D, c, "fp16x3")["dD"]
    wrong = ref + 4.0 * (D @ D @ D)
    assert not np.all(np.abs(wrong - ref) <= b)
