"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own code: alternative forms of the update
that the paper derives (gradient form, Palser-Manolopoulos appendix form,
McWeeny special case), closed forms (2x2, diagonal H, known spectra),
invariants (trace conservation, fixed points), a library eigensolver, Ky Fan's
minimum principle, and the convergence properties the paper states.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_sym_spectrum(M, lam, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), Q


def one_step(D, N):
    """One application of the oracle's recursion (max_iter=1, no tolerance)."""
    r = oracle.purify_from(D, N, tol_ddbar=-np.inf, tol_idem=-np.inf, max_iter=1)
    assert r.status == oracle.NOT_CONVERGED and r.iters == 1
    return r.D, r.history[0]


@pytest.fixture(scope="module", autouse=True)
def _build(oracle_lib):
    return oracle_lib


# ---------------------------------------------------------------- update form

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_update_equals_lagrangian_gradient_step(seed):
    """eq. (hpcp3) == D - 1/2 grad L (eq. hpcp1a) with grad Omega of eq. (mcw2b),
    grad L of eq. (mcwgrada) and gamma = 1/3 - 2c/3 (eq. mcwgama, d = 0)."""
    M = 12
    rng = np.random.default_rng(seed)
    D, _ = rand_sym_spectrum(M, rng.uniform(0.02, 0.98, M), seed)
    N = int(round(np.trace(D)))
    D1, row = one_step(D, N)
    D2, D3 = D @ D, D @ D @ D
    c = np.trace(D2 - D3) / np.trace(D - D2)
    gamma = 1.0 / 3.0 - 2.0 / 3.0 * c
    grad_omega = 2.0 * (2.0 * D3 - 3.0 * D2 + D)
    grad_L = grad_omega - 6.0 * gamma * (D - D2)
    ref = D - 0.5 * grad_L
    assert np.abs(D1 - ref).max() < 1e-13
    assert abs(row[4] - c) < 1e-13
    assert abs(row[6] - gamma) < 1e-13


@pytest.mark.parametrize("lo,hi", [(0.02, 0.6), (0.4, 0.98), (0.05, 0.95)])
def test_update_equals_pm_appendix_combination(lo, hi):
    """Appendix: (1-c) x eq.(pm1a) + c x eq.(pm3a) for c <= 1/2, and
    c x eq.(pm1b) + (1-c) x eq.(pm3b) for c > 1/2, both equal eq. (hpcp3)."""
    M = 10
    rng = np.random.default_rng(7)
    D, _ = rand_sym_spectrum(M, rng.uniform(lo, hi, M), 3)
    D1, row = one_step(D, int(round(np.trace(D))))
    c = row[4]
    I = np.eye(M)
    Db = I - D
    P = np.linalg.matrix_power
    if c <= 0.5:
        pm1a = -P(D, 3) / (1 - c) + (1 + c) / (1 - c) * P(D, 2) + (1 - 2 * c) / (1 - c) * D
        pm3a = I - (-P(Db, 3) / c + (2 - c) / c * P(Db, 2) - (1 - 2 * c) / c * Db)
        ref = (1 - c) * pm1a + c * pm3a
    else:
        pm1b = -P(D, 3) / c + (1 + c) / c * P(D, 2)
        pm3b = I - (-P(Db, 3) / (1 - c) + (2 - c) / (1 - c) * P(Db, 2))
        ref = c * pm1b + (1 - c) * pm3b
    assert np.abs(D1 - ref).max() < 1e-12


def test_mcweeny_special_case():
    """A spectrum symmetric about 1/2 gives c = 1/2 and the update reduces to
    McWeeny's 3D^2 - 2D^3 (eq. mcweeny3)."""
    M = 10
    half = np.random.default_rng(3).uniform(0.05, 0.45, M // 2)
    lam = np.concatenate([half, 1.0 - half])
    D, _ = rand_sym_spectrum(M, lam, 4)
    D1, row = one_step(D, M // 2)
    assert abs(row[4] - 0.5) < 1e-13
    assert np.abs(D1 - (3 * D @ D - 2 * D @ D @ D)).max() < 1e-13


def test_eigenvalues_follow_scalar_map():
    """Every iterate is a polynomial in D0: the eigenvalues of one step equal
    x + 2(x^2(1-x) - c x(1-x)) applied to the eigenvalues x (sorted)."""
    M = 16
    x = np.random.default_rng(11).uniform(0.01, 0.99, M)
    D, Q = rand_sym_spectrum(M, x, 5)
    D1, row = one_step(D, int(round(x.sum())))
    c = row[4]
    fx = x + 2 * (x * x * (1 - x) - c * x * (1 - x))
    assert np.allclose(np.sort(np.linalg.eigvalsh(D1)), np.sort(fx), atol=1e-13)
    # and D1 keeps D's eigenvectors
    assert np.abs(Q.T @ D1 @ Q - np.diag(fx)).max() < 1e-13


@pytest.mark.parametrize("method,c", [("hpcp", 0.3), ("hpcp", 0.8), ("pmcp", 0.2), ("pmcp", 0.7)])
def test_update_at_given_c_follows_the_eigenvalue_map(method, c):
    """update_at(D, c) at a coefficient c chosen from outside: the eigenvalues
    of D = Q diag(x) Q^T map by eq. (hpcp3) on numbers, x + 2(x^2(1-x) -
    c x(1-x)) (or eqs. (pm1a)/(pm1b) on numbers for PMCP), the eigenvectors
    are kept, the returned traces are the power sums of x, and the trace
    moves by exactly 2(T2 - T3) - 2c(T1 - T2) for HPCP (zero only at the
    coefficient the recursion forms itself)."""
    M = 14
    x = np.random.default_rng(21).uniform(0.02, 0.98, M)
    D, Q = rand_sym_spectrum(M, x, 9)
    D1, (t1, t2, t3, c_own) = oracle.update_at(D, c, method=method)
    if method == "hpcp":
        fx = x + 2 * (x * x * (1 - x) - c * x * (1 - x))
    elif c <= 0.5:
        fx = ((1 - 2 * c) * x + (1 + c) * x * x - x ** 3) / (1 - c)
    else:
        fx = ((1 + c) * x * x - x ** 3) / c
    assert np.abs(Q.T @ D1 @ Q - np.diag(fx)).max() < 1e-13
    assert abs(t1 - x.sum()) < 1e-13 and abs(t2 - (x ** 2).sum()) < 1e-13
    assert abs(t3 - (x ** 3).sum()) < 1e-13
    assert abs(c_own - ((x ** 2).sum() - (x ** 3).sum()) / (x.sum() - (x ** 2).sum())) < 1e-13
    if method == "hpcp":
        assert abs(np.trace(D1) - t1 - (2 * (t2 - t3) - 2 * c * (t1 - t2))) < 1e-12
    # c = NaN applies the recursion's own coefficient: one step of purify_from
    D1n, _ = oracle.update_at(D, float("nan"), method=method)
    r = oracle.purify_from(D, int(round(x.sum())), tol_ddbar=-np.inf, tol_idem=-np.inf,
                           max_iter=1, method=method)
    assert np.abs(D1n - r.D).max() < 1e-14


def test_power_traces_are_power_sums_of_the_spectrum():
    M = 30
    x = np.random.default_rng(22).uniform(-0.1, 1.1, M)
    D, _ = rand_sym_spectrum(M, x, 10)
    t1, t2, t3, c = oracle.power_traces(D)
    s1, s2, s3 = x.sum(), (x ** 2).sum(), (x ** 3).sum()
    assert abs(t1 - s1) < 1e-12 and abs(t2 - s2) < 1e-12 and abs(t3 - s3) < 1e-12
    assert abs(c - (s2 - s3) / (s1 - s2)) < 1e-12


# ----------------------------------------------------------------- invariants

def test_trace_conserved_every_step():
    """Tr D_{n+1} = Tr D_n = N for all n, with no correction (text after eq. hpcp1a)."""
    w = workloads.config(1)
    r = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=0.0, tol_idem=1e-10)
    assert r.status == oracle.OK
    assert np.abs(r.col("t1") - w.N).max() < 1e-11
    assert abs(np.trace(r.D) - w.N) < 1e-11


def test_initial_guess_constraints():
    """eq. (pmcpguess): lambda(D0) in [0,1], Tr D0 = N, and eqs. (pmcpcons2-3):
    T1 > T2 > T3, T3 > 2 T2 - T1, equivalently c_0 in [0, 1]."""
    w = workloads.spectral(96, 35, 0.1, seed=9)
    D0, mu, beta = oracle.initial_guess(w.H, w.N, w.emin, w.emax)
    ev = np.linalg.eigvalsh(D0)
    assert ev.min() >= -1e-12 and ev.max() <= 1 + 1e-12
    assert abs(np.trace(D0) - w.N) < 1e-11
    t1, t2, t3 = np.trace(D0), np.trace(D0 @ D0), np.trace(D0 @ D0 @ D0)
    assert t1 > t2 > t3 and t3 > 2 * t2 - t1
    # closed form of the guess's eigenvalues
    theta = w.N / w.M
    assert abs(mu - w.lam.mean()) < 1e-12
    assert np.allclose(np.sort(ev), np.sort(theta + beta * (mu - w.lam)), atol=1e-12)
    assert abs(beta - min(theta / (w.emax - mu), (1 - theta) / (mu - w.emin))) < 1e-15


def test_projector_is_fixed_point():
    """An idempotent trace-N input has Tr(D Dbar) = 0: zero updates, unchanged."""
    M, N = 20, 7
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    P = Q[:, :N] @ Q[:, :N].T
    r = oracle.purify_from(P, N, tol_ddbar=1e-12, max_iter=5)
    assert r.status == oracle.OK and r.iters == 0
    assert np.array_equal(r.D, P)


def test_quadratic_convergence_and_c_to_half():
    """Late phase: ||D^2-D||^2 contracts quadratically and c_n -> 1/2."""
    w = workloads.spectral(128, 48, 0.2, seed=21)
    r = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=0.0, tol_idem=1e-12)
    om = r.col("omega")
    late = np.where(om < 1e-3)[0]
    for a, b in zip(late[:-1], late[1:]):
        if om[b] > 1e-26:
            assert om[b] <= 10.0 * om[a] ** 2 + 1e-28
    c = r.col("c")[:-1]
    assert abs(c[-1] - 0.5) < 1e-3


def test_energy_non_increasing():
    """Tr(H D_n) decreases monotonically (variational in gamma; Fig. 3b)."""
    w = workloads.spectral(64, 20, 0.3, seed=5)
    D0, _, _ = oracle.initial_guess(w.H, w.N, w.emin, w.emax)
    energies = []
    for n in range(12):
        r = oracle.purify_from(D0, w.N, tol_ddbar=-np.inf, tol_idem=-np.inf, max_iter=n)
        energies.append(np.sum(w.H * r.D))
    assert np.all(np.diff(energies) <= 1e-12)


# ----------------------------------------------------- definition of the result

def test_two_by_two_closed_form():
    """M = 2, N = 1: the lower eigenprojector is (I - (H - Tr(H)/2 I)/r)/2,
    r = sqrt(((a-d)/2)^2 + b^2)."""
    for a, b, d in [(0.3, -0.7, -0.2), (1.0, 0.25, 1.5), (-2.0, 1e-3, 2.0)]:
        H = np.array([[a, b], [b, d]])
        r = np.hypot((a - d) / 2, b)
        P = 0.5 * (np.eye(2) - (H - 0.5 * (a + d) * np.eye(2)) / r)
        res = oracle.purify(H, 1, tol_ddbar=0.0, tol_idem=1e-13, max_iter=200)
        assert res.status == oracle.OK
        assert np.abs(res.D - P).max() < 1e-12
        Pj, _ = oracle.ground_state_jacobi(H, 1)
        assert np.abs(Pj - P).max() < 1e-14


def test_diagonal_hamiltonian_gives_indicator():
    """H diagonal: D = diag(1 on the N lowest entries, 0 elsewhere)."""
    w = workloads.paper_diagonal(100, 30, 0.2, seed=4)
    r = oracle.purify(w.H, w.N, tol_ddbar=0.0, tol_idem=1e-12)
    assert r.status == oracle.OK
    ref = np.zeros(100)
    ref[np.argsort(w.lam)[: w.N]] = 1.0
    assert np.abs(r.D - np.diag(ref)).max() < 1e-12


def test_jacobi_matches_known_spectrum():
    w = workloads.spectral(64, 24, 0.2, seed=8)
    ev, V, sweeps = oracle.jacobi_eigh(w.H)
    assert sweeps < 60
    assert np.abs(ev - np.sort(w.lam)).max() < 1e-13
    P = oracle.projector(V, w.N)
    assert np.abs(P - oracle.projector_from_spectrum(w.Q, w.lam, w.N)).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(64)).max() < 1e-13


def test_jacobi_matches_library_eigvalsh():
    A = workloads.sym_gaussian(80, seed=3)
    ev, V, _ = oracle.jacobi_eigh(A)
    assert np.abs(ev - np.linalg.eigvalsh(A)).max() < 1e-12
    assert np.abs(A @ V - V * ev).max() < 1e-11


def test_ground_state_energy_ky_fan():
    """min over rank-N projectors of Tr(P H) is the sum of the N lowest
    eigenvalues (Ky Fan); brute force over random projectors at M = 6."""
    rng = np.random.default_rng(0)
    H = workloads.sym_gaussian(6, seed=12)
    N = 3
    r = oracle.purify(H, N, tol_ddbar=0.0, tol_idem=1e-13, max_iter=200)
    assert r.status == oracle.OK
    e_min = np.linalg.eigvalsh(H)[:N].sum()
    assert abs(np.sum(r.D * H) - e_min) < 1e-12
    for _ in range(2000):
        Q, _ = np.linalg.qr(rng.standard_normal((6, N)))
        assert np.trace(Q.T @ H @ Q) >= e_min - 1e-12


def test_chain_matches_definition_and_paper_tests():
    """1D chain, M = 256, N = 100 to ||D^2-D||_F < 1e-10: equals the Jacobi
    projector; [H, D] = 0; Tr(DH) = sum of the N lowest eigenvalues; and the
    converged-state tests of eqs. (testa)-(testc) (readings: ||D||_F^2 = N and
    the ascending eigenbasis diagonal equals diag(I_N, 0))."""
    w = workloads.config(1)
    r = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=0.0, tol_idem=1e-10)
    assert r.status == oracle.OK
    P, ev = oracle.ground_state_jacobi(w.H, w.N)
    M = w.M
    assert np.linalg.norm(r.D - P) / np.sqrt(M) < 1e-10
    assert np.linalg.norm(w.H @ r.D - r.D @ w.H) < 1e-9
    assert abs(np.sum(r.D * w.H) - ev[: w.N].sum()) < 1e-9
    fro = np.linalg.norm(r.D)
    assert abs(fro - np.sqrt(np.trace(r.D))) < 1e-6           # eq. (testa)
    assert abs(fro ** 2 - w.N) < 1e-6                          # eq. (testb), reading
    _, V, _ = oracle.jacobi_eigh(w.H)
    diag = np.diag(V.T @ r.D @ V)
    target = np.r_[np.ones(w.N), np.zeros(M - w.N)]
    assert np.linalg.norm(diag - target) < 1e-6                # eq. (testc), reading


def test_scalar_map_reproduces_matrix_recursion():
    """On H = Q diag(eps) Q^T the matrix recursion and the eigenvalue map give
    the same c_n sequence, iteration count and final D."""
    w = workloads.spectral(128, 47, 0.1, seed=6)
    r = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=1e-9)
    s = oracle.scalar_map(w.lam, w.N, w.emin, w.emax, mu=np.trace(w.H) / w.M, tol_ddbar=1e-9)
    assert r.status == s["status"] == oracle.OK
    assert r.iters == s["iters"]
    # c = Tr(D^2 Dbar)/Tr(D Dbar) loses accuracy as Tr(D Dbar) -> 0 (the reason
    # the paper stops on it): allow rounding of the traces over that denominator
    ddbar = (r.col("t1") - r.col("t2"))[:-1]
    assert np.all(np.abs(r.col("c")[:-1] - s["c"]) <= 1e-10 + 1e-13 / ddbar)
    Dmap = (w.Q * s["x"]) @ w.Q.T
    assert np.abs(r.D - Dmap).max() < 1e-10


def test_scalar_map_with_given_c():
    """c_given: the map's own c sequence gives the map itself, bitwise.  Any
    other sequence moves T1 at every update by the trace of the correction of
    eq. (hpcp3), 2[(T2 - T3) - c (T1 - T2)], which vanishes only for the
    iterate's own c: the given c is the one applied."""
    w = workloads.spectral(300, 100, 0.1, seed=8)
    mu = np.trace(w.H) / w.M
    s = oracle.scalar_map(w.lam, w.N, w.emin, w.emax, mu=mu, tol_ddbar=1e-9)
    f = oracle.scalar_map(w.lam, w.N, w.emin, w.emax, mu=mu, tol_ddbar=1e-9, c_given=s["c"])
    assert f["iters"] == s["iters"] and f["status"] == s["status"]
    for k in ("t1", "t2", "t3", "c"):
        assert np.array_equal(f[k], s[k])
    cg = s["c"] + 1e-3
    g = oracle.scalar_map(w.lam, w.N, w.emin, w.emax, mu=mu, tol_ddbar=0.0,
                          max_iter=len(cg), c_given=cg)
    n = g["iters"]
    assert n >= 5
    t1, t2, t3 = g["t1"][:n], g["t2"][:n], g["t3"][:n]
    step = np.diff(g["t1"][:n + 1])
    assert np.allclose(step, 2.0 * ((t2 - t3) - cg[:n] * (t1 - t2)), rtol=0, atol=1e-10)
    assert np.abs(step).max() > 1e-4
    # the recorded c is still the iterate's own
    assert np.allclose(g["c"][:n], (t2 - t3) / (t1 - t2), rtol=0, atol=1e-12)


# ------------------------------------------------------------- failure paths

def test_degenerate_sizes():
    H = workloads.sym_gaussian(8, seed=1)
    r0 = oracle.purify(H, 0, -10, 10)
    assert r0.status == oracle.OK and r0.iters == 0 and np.all(r0.D == 0)
    rM = oracle.purify(H, 8, -10, 10)
    assert rM.status == oracle.OK and rM.iters == 0 and np.array_equal(rM.D, np.eye(8))


def test_invalid_and_breakdown_paths():
    w = workloads.config(1)
    with pytest.raises(ValueError):
        oracle.purify(w.H, w.M + 1, w.emin, w.emax)
    with pytest.raises(ValueError):        # bounds that do not bracket mu
        oracle.purify(w.H, w.N, 0.5, 2.5)
    r = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=0.0, tol_idem=1e-10, max_iter=1)
    assert r.status == oracle.NOT_CONVERGED and r.iters == 1
    # bounds far inside the spectrum: lambda(D0) leaves [0,1] and the run breaks down
    r = oracle.purify(w.H, w.N, -0.2, 0.2, tol_ddbar=0.0, tol_idem=1e-10)
    assert r.status == oracle.BREAKDOWN
    # NaN input is a breakdown, not a result
    Hn = w.H.copy()
    Hn[3, 4] = Hn[4, 3] = np.nan
    r = oracle.purify(Hn, w.N, w.emin, w.emax, tol_ddbar=0.0, tol_idem=1e-10)
    assert r.status == oracle.BREAKDOWN


def test_gershgorin_bounds():
    w = workloads.config(1)
    lo, hi = oracle.gershgorin(w.H)
    ev = np.linalg.eigvalsh(w.H)
    assert lo <= ev[0] and ev[-1] <= hi
    d = workloads.paper_diagonal(50, 10, 0.5, seed=2)
    lo, hi = oracle.gershgorin(d.H)
    assert lo == d.lam.min() and hi == d.lam.max()
    r = oracle.purify(w.H, w.N, tol_ddbar=0.0, tol_idem=1e-10)   # NaN bounds -> Gershgorin
    assert r.status == oracle.OK and (r.emin, r.emax) == oracle.gershgorin(w.H)


# ------------------------------------------------------ the paper's iteration counts

def test_iteration_counts_against_figure3():
    """Fig. 3 / its discussion: p grows linearly in ln(1/gap), and the wide-gap
    count at theta = 0.5 is about 10 (values and tolerance in the golden file)."""
    g = json.load(open(os.path.join(GOLDEN, "fig3_iteration_counts.json")))
    M = g["M"]

    def pbar(theta, gap):
        ps = []
        for s in range(g["hamiltonians_per_point"]):
            w = workloads.paper_diagonal(M, int(round(theta * M)), gap, seed=g["seed0"] + s)
            res = oracle.scalar_map(w.lam, w.N, w.lam.min(), w.lam.max(), tol_ddbar=g["tol_ddbar"])
            assert res["status"] == oracle.OK
            ps.append(res["iters"])
        return float(np.mean(ps))

    wide = g["theta_half_wide_gap"]
    assert abs(pbar(0.5, 1.0) - wide["paper"]) <= wide["abs_tol"]
    p = [pbar(0.5, gap) for gap in g["linearity_gaps"]]
    slopes = np.diff(p) / np.diff(np.log(1.0 / np.array(g["linearity_gaps"])))
    assert slopes.min() > 0
    assert slopes.max() / slopes.min() < g["linearity_slope_ratio_max"]
    lo, hi = g["color_map_range"]
    assert all(lo - wide["abs_tol"] <= x <= hi for x in p)


# ---------------------------------------------------------- acceptance checks

def test_verify_quantities_closed_forms(oracle_lib):
    """Tr D, ||D||_F^2, ||D^2 - D||_F, Tr(DH), ||HD - DH||_F by hand: a diagonal
    pair, a 2x2 pair with a known commutator, and the ground-state projector of
    a known spectrum (trace = ||D||_F^2 = N, energy = sum of the N lowest
    eigenvalues, idempotent, commuting with H)."""
    d = np.array([0.25, 1.0, -0.5, 2.0])
    h = np.array([1.0, -2.0, 3.0, 0.5])
    q = oracle.verify_quantities(np.diag(d), np.diag(h))
    assert q["trace"] == pytest.approx(2.75) and q["fro2"] == pytest.approx(5.3125)
    assert q["idem"] == pytest.approx(np.sqrt(np.sum((d * d - d) ** 2)))
    assert q["energy"] == pytest.approx(0.25 - 2.0 - 1.5 + 1.0) and q["comm"] == 0.0
    q = oracle.verify_quantities(np.array([[1.0, 0.0], [0.0, 0.0]]), np.array([[0.0, 1.0], [1.0, 0.0]]))
    assert q["comm"] == pytest.approx(np.sqrt(2.0)) and q["idem"] == 0.0 and q["energy"] == 0.0
    w = workloads.spectral(64, 20, 0.2, 5)
    P = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    q = oracle.verify_quantities(P, w.H)
    assert q["trace"] == pytest.approx(20, abs=1e-12) and q["fro2"] == pytest.approx(20, abs=1e-12)
    assert q["idem"] < 1e-13 and q["comm"] < 1e-13
    assert q["energy"] == pytest.approx(np.sort(w.lam)[:20].sum(), abs=1e-12)


# ------------------------------------- PM recursion and hole-particle guesses

def test_pmcp_step_conserves_trace_and_reduces_to_mcweeny(oracle_lib):
    """eqs. (pm1a)/(pm1b): Tr D' = Tr D in both branches of c; a spectrum
    symmetric about 1/2 (c = 1/2) gives McWeeny's 3D^2 - 2D^3 in both
    recursions; and PMCP converges to the ground-state projector."""
    M = 10
    for lam, low in ((np.linspace(0.02, 0.6, M), True), (np.linspace(0.4, 0.98, M), False)):
        D, _ = rand_sym_spectrum(M, lam, 5)
        N = int(round(np.trace(D)))
        r = oracle.purify_from(D, N, tol_ddbar=0.0, max_iter=1, method="pmcp")
        assert (r.col("c")[0] <= 0.5) == low
        assert abs(np.trace(r.D) - np.trace(D)) < 1e-12
    lam = np.linspace(0.1, 0.9, M)
    D, _ = rand_sym_spectrum(M, lam, 6)
    mcw = 3 * D @ D - 2 * D @ D @ D
    for method in ("pmcp", "hpcp"):
        r = oracle.purify_from(D, 5, tol_ddbar=0.0, max_iter=1, method=method)
        assert r.col("c")[0] == pytest.approx(0.5, abs=1e-14)
        assert np.abs(r.D - mcw).max() < 1e-12
    w = workloads.spectral(64, 20, 0.2, 11)
    r = oracle.purify_ex(w.H, w.N, w.emin, w.emax, method="pmcp", tol_ddbar=0.0, tol_idem=1e-10)
    assert r.status == oracle.OK
    assert np.abs(r.D - oracle.projector_from_spectrum(w.Q, w.lam, w.N)).max() < 1e-9


def test_hp_guess_is_a_slope_change_with_closed_form_moments(oracle_lib):
    """eq. (hpcpguess) built from the particle and hole matrices equals
    theta I + beta_a (mu I - H) with beta_a = a beta_min + (1-a) beta_max; its
    trace is N for every alpha and Tr(D0+^2) = N theta + beta_a^2 ||H - mu I||_F^2."""
    w = workloads.spectral(40, 12, 0.3, 9)
    M, N = w.M, w.N
    theta, mu = N / M, np.trace(w.H) / M
    bt, bb = theta / (w.emax - mu), (1 - theta) / (mu - w.emin)
    bmin, bmax = min(bt, bb), max(bt, bb)
    S = np.sum((w.H - mu * np.eye(M)) ** 2)
    for a in (0.0, 0.3, 0.5, 1.0):
        D0, mu_o, slope, a_used = oracle.initial_guess_hp(w.H, N, w.emin, w.emax, "hp", alpha=a)
        ba = a * bmin + (1 - a) * bmax
        assert a_used == a and slope == pytest.approx(ba, rel=1e-14)
        assert np.abs(D0 - (theta * np.eye(M) + ba * (mu * np.eye(M) - w.H))).max() < 1e-14
        assert np.trace(D0) == pytest.approx(N, abs=1e-12)
        assert np.sum(D0 * D0) == pytest.approx(N * theta + ba ** 2 * S, rel=1e-12)


@pytest.mark.parametrize("N", [2, 6, 34, 38])
def test_alpha_search_hits_its_target(oracle_lib, N):
    """eq. (hpcpguessalpha): Tr(D0+^2) = N - delta N (theta < 1 - delta) or
    N - delta (M - N) (theta > delta) at the searched alpha."""
    M, delta = 40, 2.0 / 3.0
    w = workloads.spectral(M, N, 0.3, 10)
    D0, _, _, a = oracle.initial_guess_hp(w.H, N, w.emin, w.emax, "search", delta=delta)
    target = N - delta * N if N / M < 1 - delta else N - delta * (M - N)
    assert 0.0 < a < 1.0
    assert np.sum(D0 * D0) == pytest.approx(target, rel=1e-10)


def test_matrix_and_eigenvalue_routes_agree_for_every_method_and_guess(oracle_lib):
    for theta in (0.01, 0.05, 0.3, 0.5, 0.95):
        w = workloads.paper_diagonal(100, int(round(theta * 100)), 1.0, 3000)
        for method in ("hpcp", "pmcp"):
            for init in ("pmcp", "hp", "search"):
                r = oracle.purify_ex(w.H, w.N, method=method, init=init)
                s = oracle.scalar_map(w.lam, w.N, w.lam.min(), w.lam.max(), method=method,
                                      init=init)
                assert r.status == s["status"] == oracle.OK
                assert r.iters == s["iters"] and abs(r.alpha - s["alpha"]) < 1e-12
                # c_n is a ratio of trace differences, each accurate to ~1e-14 M
                ddbar = np.abs(r.col("t1") - r.col("t2"))[:-1]
                assert np.all(np.abs(r.col("c")[:-1] - s["c"]) <= 1e-12 + 1e-14 * 100 / ddbar)


def test_fig3_hole_particle_claims(oracle_lib):
    """The Fig. 3 discussion (values and readings in the golden file)."""
    g = json.load(open(os.path.join(GOLDEN, "fig3_hole_particle.json")))
    M = g["M"]

    def counts(theta, method, init, fallback=True):
        ps = []
        for s in range(g["hamiltonians_per_point"]):
            w = workloads.paper_diagonal(M, int(round(theta * M)), g["gap"], g["seed0"] + s)
            if fallback:
                r = oracle.scalar_map(w.lam, w.N, w.lam.min(), w.lam.max(), tol_ddbar=g["tol_ddbar"],
                                      method=method, init=init)
                ps.append(r["iters"] if r["status"] == oracle.OK else None)
            else:   # the raw alpha = 1/2 guess, no fall-back
                D0, _, _, _ = oracle.initial_guess_hp(w.H, w.N, w.lam.min(), w.lam.max(), "hp")
                r = oracle.purify_from(D0, w.N, tol_ddbar=g["tol_ddbar"])
                ps.append(r.iters if r.status == oracle.OK else None)
        return ps

    def mean(ps):
        assert all(p is not None for p in ps)
        return float(np.mean(ps))

    r05 = mean(counts(0.05, "pmcp", "pmcp")) / mean(counts(0.05, "hpcp", "pmcp"))
    lo, hi = g["theta_0.05"]["ratio_range"]
    assert lo <= r05 <= hi, r05
    h01 = mean(counts(0.01, "hpcp", "search"))
    p01 = mean(counts(0.01, "pmcp", "search"))
    t = g["theta_0.01_search"]
    assert abs(h01 - t["hpcp"]) <= t["hpcp_abs_tol"], h01
    assert t["ratio_range"][0] <= p01 / h01 <= t["ratio_range"][1], p01 / h01
    flat = [mean(counts(th, "hpcp", "hp")) for th in g["alpha_half_flat_thetas"]]
    assert max(flat) - min(flat) <= g["alpha_half_flat_spread_max"], flat
    for th in g["alpha_half_runaway_thetas"]:
        raw = counts(th, "hpcp", "hp", fallback=False)
        assert sum(p is None for p in raw) > len(raw) // 2
    for th in g["search_pole_thetas"]:
        extra = mean(counts(th, "hpcp", "search")) - mean(counts(th, "hpcp", "hp"))
        assert g["search_pole_extra_range"][0] <= extra <= g["search_pole_extra_range"][1], extra
    # the search fixes the extreme fillings for both recursions
    for th in (0.01, 0.05, 0.95):
        for m in ("hpcp", "pmcp"):
            assert mean(counts(th, m, "search")) < mean(counts(th, m, "pmcp"))


@pytest.mark.parametrize("method", ["hpcp", "pmcp"])
def test_hole_purification_is_particle_purification_of_minus_h(oracle_lib, method):
    """Purifying Dbar = I - D0 for (H, N) is purifying D for (-H, M - N) with
    the bounds reflected (the PMCP guess of -H is I - D0), then D = I - Dbar:
    the same projector.  HPCP is moreover hole-particle symmetric, so its hole
    run reproduces the particle run itself."""
    w = workloads.spectral(48, 15, 0.2, 12)
    M, N = w.M, w.N
    r = oracle.purify_ex(w.H, N, w.emin, w.emax, method=method, hole=True, tol_ddbar=1e-10)
    m = oracle.purify_ex(-w.H, M - N, -w.emax, -w.emin, method=method, tol_ddbar=1e-10)
    assert r.status == m.status == oracle.OK and r.iters == m.iters
    assert np.abs(r.D - (np.eye(M) - m.D)).max() < 1e-12
    ref = oracle.projector_from_spectrum(w.Q, w.lam, N)
    assert np.abs(r.D - ref).max() < 1e-8
    if method == "hpcp":
        p = oracle.purify_ex(w.H, N, w.emin, w.emax, tol_ddbar=1e-10)
        assert p.iters == r.iters and np.abs(p.D - r.D).max() < 1e-12
