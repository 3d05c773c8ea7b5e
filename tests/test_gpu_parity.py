"""GPU parity: the HIP purification (through the C ABI) against the CPU oracle.

Small and medium sizes compare element by element with the oracle's
step-by-step recursion (same seeded input bytes); large sizes compare with
the definition of the result (the projector onto the N lowest eigenvectors,
in closed form for H = Q diag(lam) Q^T) and with the oracle's eigenvalue map,
which predicts every c_n and the iteration count exactly.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1512_07236_amd as gcp  # noqa: E402

# Error bound of each precision in ||D - D_ref||_F / sqrt(M) at M <= 1024 for
# well-gapped spectra.  FP64 is held to the oracle's own accuracy; the split
# encodings to the accumulated rounding of their operands (bounds derived
# from the unit roundoff of each encoding, see the design notes).
ERR_TOL = {"fp64": 1e-11, "fp32": 2e-6, "fp16x3": 1e-6, "bf16x6": 1e-6, "bf16x3": 1e-4,
           "fp16": 3e-3, "bf16": 3e-2}


TOL_DDBAR = {"fp64": 1e-9, "fp32": 1e-6, "fp16x3": 1e-6, "bf16x6": 1e-6, "bf16x3": 2e-5,
             "fp16": 2e-3, "bf16": 5e-2}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_gpu(H):
    return torch.from_numpy(np.ascontiguousarray(H)).cuda()


def rel_err(D, ref):
    return float(np.linalg.norm(D - ref) / math.sqrt(D.shape[0]))


def run_gpu(w, precision, **opts):
    log(f"[gpu] {w.name} precision={precision} opts={opts}")
    D, res = gcp.purify(to_gpu(w.H), w.N, w.emin, w.emax, precision=precision, **opts)
    torch.cuda.synchronize()
    return D.cpu().numpy(), res


@pytest.fixture(scope="module", autouse=True)
def _oracle(oracle_lib):
    return oracle_lib


# ------------------------------------------------------------ FP64 vs oracle

def test_fp64_chain_matches_oracle_step_by_step():
    """1D chain, M = 256, N = 100, stop at ||D^2 - D||_F < 1e-10: same
    iteration count, same c_n, same iterates' traces, same D as the oracle."""
    w = workloads.config(1)
    ref = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=0.0, tol_idem=1e-10)
    D, res = run_gpu(w, "fp64", tol_ddbar=0.0, tol_idem=1e-10)
    assert res.status == gcp.OK and ref.status == oracle.OK
    assert res.iters == ref.iters
    h = res.history
    assert h.shape[0] == ref.iters + 1
    # c_n = (T2 - T3)/(T1 - T2): the traces agree to FP64 rounding of sums of
    # size ~N, so c_n agrees to that over Tr(D Dbar)
    ddbar = ref.col("t1")[:-1] - ref.col("t2")[:-1]
    ctol = 1e-12 + 1e-14 * w.N / np.abs(ddbar)
    assert np.all(np.abs(res.col("c")[:-1] - ref.col("c")[:-1]) <= ctol)
    assert np.abs(res.col("t1") - w.N).max() < 1e-10
    assert np.abs(res.col("t2") - ref.col("t2")).max() < 1e-10
    assert np.abs(D - ref.D).max() < 1e-12
    P, ev = oracle.ground_state_jacobi(w.H, w.N)
    assert rel_err(D, P) < 1e-10
    assert abs(np.sum(D * w.H) - ev[: w.N].sum()) < 1e-9


@pytest.mark.parametrize("M,N", [(200, 71), (384, 190), (520, 100)])
def test_fp64_ragged_and_multi_tile_match_oracle(M, N):
    """Sizes that are not multiples of the 128 tile (internal zero padding)
    and span several tiles: element-wise equal to the oracle recursion."""
    w = workloads.spectral(M, N, gap=0.1, seed=M)
    ref = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=1e-9)
    D, res = run_gpu(w, "fp64", tol_ddbar=1e-9)
    assert res.status == gcp.OK and res.iters == ref.iters
    assert np.abs(D - ref.D).max() < 1e-12
    assert np.abs(res.col("t1") - N).max() < 1e-10
    assert rel_err(D, oracle.projector_from_spectrum(w.Q, w.lam, N)) < 1e-9


def test_fp64_lagrangian_history_matches_oracle():
    w = workloads.spectral(256, 100, gap=0.2, seed=17)
    ref = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=1e-8)
    _, res = run_gpu(w, "fp64", tol_ddbar=1e-8)
    assert res.iters == ref.iters
    ddbar = np.abs(ref.col("t1") - ref.col("t2"))[:-1]
    ctol = 1e-12 + 1e-14 * w.N / ddbar
    for name in ("c", "gamma"):
        assert np.all(np.abs(res.col(name)[:-1] - ref.col(name)[:-1]) <= ctol), name
    for name in ("t3", "omega", "lagrangian", "step"):
        a, b = res.col(name)[:-1], ref.col(name)[:-1]
        assert np.allclose(a, b, rtol=1e-9, atol=1e-11 + 1e-14 * w.N), name


# --------------------------------------------------------- every precision

@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16x3", "bf16x6", "bf16x3", "fp16", "bf16"])
def test_precisions_trace_exact_and_error_bounded(precision):
    """Every precision: Tr D_n = N to 1e-10 at every step (no correction),
    the result within the precision's error bound of the definition, and the
    same iteration count as the eigenvalue map (high-precision modes)."""
    w = workloads.spectral(640, 234, gap=0.1, seed=33)
    # stop above each encoding's noise floor of Tr(D Dbar): below it c_n is
    # rounding noise and leaves [0, 1] (reported as a breakdown)
    tol = TOL_DDBAR[precision]
    D, res = run_gpu(w, precision, tol_ddbar=tol)
    assert res.status in gcp.SUCCESS, res
    assert np.abs(res.col("t1") - w.N).max() < 1e-10
    assert abs(np.trace(D) - w.N) < 1e-10
    err = rel_err(D, oracle.projector_from_spectrum(w.Q, w.lam, w.N))
    log(f"  {precision}: iters={res.iters} err={err:.3e}")
    assert err < ERR_TOL[precision]
    if precision in ("fp64", "fp32", "fp16x3", "bf16x6"):
        s = oracle.scalar_map(w.lam, w.N, w.emin, w.emax, mu=np.trace(w.H) / w.M, tol_ddbar=tol)
        assert abs(res.iters - s["iters"]) <= (0 if precision == "fp64" else 1)


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x6"])
@pytest.mark.parametrize("fold", [1, 3, 1000])
def test_fold_period_changes_only_rounding(precision, fold):
    """Any fold period (1 = every step, 1000 = never at this size) gives the
    same result to the encoding's accuracy, with the trace exact."""
    w = workloads.spectral(512, 200, gap=0.1, seed=5)
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    D, r = run_gpu(w, precision, tol_ddbar=TOL_DDBAR[precision], fold_every=fold)
    assert r.status in gcp.SUCCESS
    e = rel_err(D, ref)
    log(f"  {precision} fold={fold}: err {e:.3e}")
    assert e < 2 * ERR_TOL[precision] and abs(np.trace(D) - w.N) < 1e-10


def test_determinism_bitwise():
    w = workloads.spectral(384, 150, gap=0.1, seed=8)
    H = to_gpu(w.H)
    outs = []
    for _ in range(2):
        D, res = gcp.purify(H, w.N, w.emin, w.emax, precision="fp16x3")
        outs.append((D.cpu().numpy(), res.history))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1], equal_nan=True)


# ----------------------------------------------------------- edge cases

def test_n_zero_and_full():
    w = workloads.spectral(130, 0, gap=0.1, seed=1)
    D, res = run_gpu(w, "fp64")
    assert res.status == gcp.OK and res.iters == 0 and np.all(D == 0)
    w = workloads.spectral(130, 130, gap=0.1, seed=1)
    D, res = run_gpu(w, "fp16x3")
    assert res.status == gcp.OK and res.iters == 0 and np.array_equal(D, np.eye(130))


def test_tiny_and_diagonal():
    H = np.array([[0.3, -0.7], [-0.7, -0.2]])
    w = workloads.Workload("2x2", H, 1, float("nan"), float("nan"))
    D, res = run_gpu(w, "fp64", tol_ddbar=0.0, tol_idem=1e-13, max_iter=200)
    r = np.hypot(0.25, 0.7)
    P = 0.5 * (np.eye(2) - (H - 0.05 * np.eye(2)) / r)
    assert res.status == gcp.OK and np.abs(D - P).max() < 1e-12
    d = workloads.paper_diagonal(100, 30, 0.2, seed=4)
    D, res = run_gpu(d, "fp32", tol_ddbar=1e-7)
    ref = np.zeros(100)
    ref[np.argsort(d.lam)[:30]] = 1.0
    assert np.abs(D - np.diag(ref)).max() < 1e-6


def test_gershgorin_bounds_and_scalars_match_oracle():
    w = workloads.config(1)
    H = to_gpu(w.H)
    with gcp.Context(w.M, precision="fp64", tol_ddbar=0.0, tol_idem=1e-10) as ctx:
        ctx.init(H, w.N)   # NaN bounds -> Gershgorin
        s = ctx.init_scalars()
        lo, hi = oracle.gershgorin(w.H)
        assert s["emin"] == lo and s["emax"] == hi
        D, res = ctx.purify()
        ref = oracle.purify(w.H, w.N, tol_ddbar=0.0, tol_idem=1e-10)
        assert abs(s["mu"] - ref.mu) < 1e-15 and abs(s["beta"] - ref.beta) < 1e-15
        assert res.iters == ref.iters
        assert np.abs(D.cpu().numpy() - ref.D).max() < 1e-12


def test_status_paths():
    w = workloads.config(1)
    H = to_gpu(w.H)
    with gcp.Context(w.M, precision="fp64", tol_ddbar=0.0, tol_idem=1e-10, max_iter=1) as ctx:
        ctx.init(H, w.N, w.emin, w.emax)
        D, res = ctx.purify()
        assert res.status == gcp.ERR_NOT_CONVERGED and res.iters == 1
        ref = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=0.0, tol_idem=1e-10, max_iter=1)
        assert np.abs(D.cpu().numpy() - ref.D).max() < 1e-13
    with gcp.Context(w.M, precision="fp64", tol_ddbar=0.0, tol_idem=1e-10) as ctx:
        ctx.init(H, w.N, -0.2, 0.2)
        _, res = ctx.purify()
        ref = oracle.purify(w.H, w.N, -0.2, 0.2, tol_ddbar=0.0, tol_idem=1e-10)
        assert res.status == gcp.ERR_BREAKDOWN and ref.status == oracle.BREAKDOWN
        with pytest.raises(gcp.GCPError):
            ctx.init(H, w.N, 0.5, 2.5)          # mu outside (emin, emax)
        with pytest.raises(gcp.GCPError):
            ctx.init(H, w.M + 1, -3, 3)
    Hn = w.H.copy()
    Hn[3, 4] = Hn[4, 3] = np.nan
    wn = workloads.Workload("nan", Hn, w.N, w.emin, w.emax)
    _, res = run_gpu(wn, "fp64", tol_ddbar=0.0, tol_idem=1e-10)
    assert res.status == gcp.ERR_BREAKDOWN


def test_output_leading_dimension_and_fp32_output():
    w = workloads.spectral(160, 60, gap=0.2, seed=2)
    H = to_gpu(w.H)
    big = torch.zeros((160, 200), dtype=torch.float64, device="cuda")
    with gcp.Context(160, precision="fp64", tol_ddbar=1e-10) as ctx:
        ctx.init(H, w.N, w.emin, w.emax)
        D, res = ctx.purify(out=big[:, :160])
        D32, _ = ctx.purify(dtype=torch.float32)
    b = big.cpu().numpy()
    assert np.all(b[:, 160:] == 0)
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    assert rel_err(b[:, :160], ref) < 1e-9
    assert np.abs(D32.cpu().numpy() - b[:, :160]).max() < 1e-6


# ------------------------------------------------------------ full sizes

@pytest.fixture(scope="module")
def config3():
    log("[gpu] generating workload 3 (M = 8192, N = 3000, gap 0.05)")
    w = workloads.config(3)
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    s = oracle.scalar_map(w.lam, w.N, w.emin, w.emax, mu=np.trace(w.H) / w.M, tol_ddbar=1e-7)
    return w, ref, s


@pytest.mark.parametrize("precision,tol_ddbar,err_tol", [("fp64", 1e-7, 1e-9),
                                                          ("fp16x3", 1e-5, 1e-6),
                                                          ("bf16x6", 1e-5, 1e-6)])
def test_full_size_spectral_8192(config3, precision, tol_ddbar, err_tol):
    """M = 8192, N = 3000, gap 0.05: the bench workload.  Error against the
    closed-form projector, trace at every step, and the c_n sequence against
    the eigenvalue map."""
    w, ref, s = config3
    s = oracle.scalar_map(w.lam, w.N, w.emin, w.emax, mu=np.trace(w.H) / w.M, tol_ddbar=tol_ddbar)
    D, res = run_gpu(w, precision, tol_ddbar=tol_ddbar)
    err = rel_err(D, ref)
    log(f"  {precision}: iters={res.iters} (map {s['iters']}) err={err:.3e} "
        f"trace err={abs(np.trace(D) - w.N):.2e} ms={res.ms_total:.1f}")
    assert res.status in gcp.SUCCESS
    assert np.abs(res.col("t1") - w.N).max() < 1e-10
    assert err < err_tol
    assert abs(res.iters - s["iters"]) <= (0 if precision == "fp64" else 1)
    if precision != "fp64":
        # the split encodings' c_n and T3 are checked one update at a time
        # against the oracle's traces of the GPU's own iterate
        # (tests/test_gpu_elementwise.py); along the whole trajectory their
        # iterates drift from the exact ones by the accumulated rounding.
        return
    # FP64: the eigenvalue map driven by the GPU's own c_n follows the GPU's
    # iterates to FP64 rounding of their elements, which moves the traces by
    # far less than their summation does.  (The free-running map applies its
    # own c_n, which near convergence differs by e/(T1 - T2) and moves the
    # next T3 by about 6 dc Tr(D^3 Dbar), as large as e itself.)
    # c_n = (T2 - T3)/(T1 - T2) moves by e/(T1 - T2) for an absolute error e
    # of the traces.  The traces (~N = 3000) are tree sums over 8192 rows;
    # the top levels dominate, each adding ~2^-53 x 3000 x 2^(-k/2) at depth
    # k: ~1.1e-12 RMS per trace and ~1.5e-12 for the difference, so e = 4e-12
    # (3 sigma).
    n = res.iters
    sf = oracle.scalar_map(w.lam, w.N, w.emin, w.emax, mu=np.trace(w.H) / w.M,
                           tol_ddbar=0.0, max_iter=n, c_given=res.col("c")[:n])
    assert sf["iters"] == n
    ddbar = (res.col("t1") - res.col("t2"))[:n]
    ctol, cnum = 1e-11, 4e-12
    dc = np.abs(res.col("c")[:n] - sf["c"][:n])
    ratio = dc / (ctol + cnum / np.abs(ddbar))
    k = int(np.argmax(ratio))
    log(f"  c_n: worst n={k} dc={dc[k]:.3e} ddbar={ddbar[k]:.3e} ratio={ratio[k]:.3f}")
    assert np.all(ratio <= 1.0)
    # T3 of every iterate against the driven map's power sum: one trace's
    # 3 sigma (3.3e-12) is below e
    dt3 = np.abs(res.col("t3")[:n] - sf["t3"][:n])
    log(f"  T3: max |dT3| = {dt3.max():.3e}")
    assert np.all(dt3 <= cnum)



def test_full_size_fold_against_one_accumulator(config3):
    """M = 8192, FP16X3: the chunked accumulation is what brings the error
    down.  Per output element the product runs 256 K stages of 3 MFMA
    products; one accumulator rounds each term about 3 x 256 = 768 times, the
    default fold (every sqrt(256 / 3) = 9 stages) about 3 x 9 + 256 / 9 = 56
    times, a factor sqrt(768 / 56) = 3.7 in the accumulated rounding.  The
    error of the whole solve must shrink by at least half that."""
    w, ref, _ = config3
    errs = {}
    for fold in (0, 1000):
        D, res = run_gpu(w, "fp16x3", tol_ddbar=1e-5, fold_every=fold)
        assert res.status in gcp.SUCCESS
        errs[fold] = rel_err(D, ref)
        log(f"  fp16x3 fold={fold}: iters={res.iters} err={errs[fold]:.3e}")
    assert errs[0] < errs[1000] / (3.7 / 2)


def test_full_size_ksplit_combines_in_fp64(config3):
    """M = 8192, FP16X3 with every pair split along K over 8 blocks whose
    FP32 totals are added in FP64: each block folds its 32 of the 256 K
    stages every 3 (sqrt(32 / 3)), about 3 x 3 + 32 / 3 = 20 roundings per
    term against 3 x 9 + 256 / 9 = 56 for the whole-K fold, a factor
    sqrt(56 / 20) = 1.7 in the accumulated rounding; with the encoding's own
    share unchanged the error must still drop by at least 1.2."""
    w, ref, _ = config3
    D0, r0 = run_gpu(w, "fp16x3", tol_ddbar=1e-6)
    D8, r8 = run_gpu(w, "fp16x3", tol_ddbar=1e-6, ksplit=8)
    e0, e8 = rel_err(D0, ref), rel_err(D8, ref)
    log(f"  fp16x3: err {e0:.3e} (whole K), {e8:.3e} (ksplit 8); iters {r0.iters}, {r8.iters}")
    assert r8.status in gcp.SUCCESS and abs(r8.iters - r0.iters) <= 1
    assert np.abs(r8.col("t1") - w.N).max() < 1e-10
    assert e8 < e0 / 1.2

# ------------------------------------------------------- precision schedule

def _ctx_run(w, **opts):
    with gcp.Context(w.M, **opts) as ctx:
        ctx.init(to_gpu(w.H), w.N, w.emin, w.emax)
        D, res = ctx.purify()
        torch.cuda.synchronize()
        return D.cpu().numpy(), res


def test_schedule_never_triggered_is_bitwise_the_single_precision_run():
    w = workloads.spectral(384, 150, 0.1, 50)
    D1, r1 = _ctx_run(w, precision="fp16x3", tol_ddbar=1e-6)
    D2, r2 = _ctx_run(w, precision="fp16x3", late_precision="fp64", switch_ddbar=0.0,
                      tol_ddbar=1e-6)
    assert r1.iters == r2.iters and np.array_equal(D1, D2)


def test_schedule_from_the_start_matches_the_late_precision_run():
    """FP64 -> FP16X3 at n = 0: only the first D^2 is FP64, so the run is the
    FP16X3 run up to FP16X3 rounding."""
    w = workloads.spectral(384, 150, 0.1, 51)
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    D1, r1 = _ctx_run(w, precision="fp16x3", tol_ddbar=1e-6)
    D2, r2 = _ctx_run(w, precision="fp64", late_precision="fp16x3", switch_ddbar=1e30,
                      tol_ddbar=1e-6)
    assert abs(r1.iters - r2.iters) <= 1
    assert rel_err(D2, ref) < ERR_TOL["fp16x3"]
    assert np.abs(r2.col("t1") - w.N).max() < 1e-10


@pytest.mark.parametrize("early,late,switch,err_lo,err_hi", [("fp16x3", "fp64", 1e-3, 0.0, 1e-6),
                                                             ("bf16x6", "fp64", 1e-3, 0.0, 1e-6),
                                                             ("bf16", "fp16x3", 1e-1, 1e-4, 3e-2)])
def test_schedule_switch(early, late, switch, err_lo, err_hi):
    """Trace exact through the switch, convergence below the early encoding's
    rounding floor when the late one is FP64, and the early phase's error kept
    (rounding in the occupied-virtual block is not undone later).  The switch
    point lies above the early encoding's floor of Tr(D Dbar) (TOL_DDBAR)."""
    M, N = 520, 200
    w = workloads.spectral(M, N, 0.1, 52)
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    tol = 1e-11 if late == "fp64" else 1e-5
    D, res = _ctx_run(w, precision=early, late_precision=late, switch_ddbar=switch,
                      tol_ddbar=tol, max_iter=60)
    err = rel_err(D, ref)
    idem = float(np.linalg.norm(D @ D - D))
    log(f"  {early}->{late}: iters={res.iters} err={err:.3e} idem={idem:.2e}")
    assert res.status in gcp.SUCCESS
    assert np.abs(res.col("t1") - w.N).max() < 1e-10
    assert err_lo <= err < err_hi
    if late == "fp64":
        assert idem < 1e-9


def test_three_phase_schedule_never_entering_the_last_is_the_two_phase_run():
    w = workloads.spectral(384, 150, 0.1, 53)
    D2, r2 = _ctx_run(w, precision="fp16x3", late_precision="bf16x6", switch_ddbar=1e-2,
                      tol_ddbar=1e-6)
    D3, r3 = _ctx_run(w, precision="fp16x3", late_precision="bf16x6", switch_ddbar=1e-2,
                      final_precision="fp64", final_ddbar=0.0, tol_ddbar=1e-6)
    assert r3.iters == r2.iters and np.array_equal(D3, D2)
    assert np.array_equal(r3.history, r2.history, equal_nan=True)
    assert r3.mfma_flops == r2.mfma_flops


@pytest.mark.parametrize("phases,err_lo,err_hi", [
    (("bf16", 1e-1, "fp16x3", 1e-3, "fp64"), 1e-4, 3e-2),
    (("fp16x3", 1e-1, "bf16x6", 1e-3, "fp64"), 0.0, 1e-6),
    (("bf16x6", 1e-1, "fp32", 1e-3, "fp64"), 0.0, 1e-6),
])
def test_three_phase_schedule(phases, err_lo, err_hi):
    """Three encodings entered at two thresholds of Tr(D Dbar): the trace
    stays exact through both switches, the final FP64 phase makes D
    idempotent to FP64 level and reaches a tolerance far below the earlier
    encodings' floors, and the error is the earliest phase's (rounding in
    the occupied-virtual block is not undone).  The issued MFMA flops count
    each phase's launches with its own number of products.  At each switch
    D^2 is formed again in the new encoding, so that the first update of a
    precise phase carries none of the earlier encoding's rounding of D^2
    (BF16X6 -> FP64 at 1e-3 broke down without it: the first FP64 update's
    Tr(D Dbar) came out at -5e-8, BF16X6 noise far above FP64's floor)."""
    early, sw1, late, sw2, final = phases
    M, N = 520, 200
    w = workloads.spectral(M, N, 0.1, 52)
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    D, res = _ctx_run(w, precision=early, late_precision=late, switch_ddbar=sw1,
                      final_precision=final, final_ddbar=sw2, tol_ddbar=1e-11, max_iter=60)
    err = rel_err(D, ref)
    idem = float(np.linalg.norm(D @ D - D))
    ddbar = res.col("t1") - res.col("t2")
    # updates in each phase: the switch follows the D^2 whose Tr(D Dbar) is
    # within the threshold, so update n runs its K2 in the new encoding
    n1 = int(np.argmax(np.abs(ddbar) <= sw1))
    n2 = int(np.argmax(np.abs(ddbar) <= sw2))
    log(f"  {early}->{late}->{final}: iters={res.iters} switches at {n1}, {n2} err={err:.3e} "
        f"idem={idem:.2e}")
    assert res.status in gcp.SUCCESS
    assert 0 < n1 <= n2 < res.iters
    assert np.abs(res.col("t1") - w.N).max() < 1e-10
    assert err_lo <= err < err_hi
    assert idem < 1e-9
    # first phase: K1 of updates 0..n1 and K2 of 0..n1-1; at a switch D^2 is
    # formed again in the new encoding (a second K1 of the same update), so
    # the second phase has K1 (again) and K2 of n1..n2-1 and K1 of n2
    tile = (w.M + 255) // 256 * 256
    nt = tile // 128
    tile_fl = nt * (nt + 1) / 2 * 2.0 * 128 * 128 * tile
    prods = {"bf16": 1, "fp16x3": 3, "bf16x6": 6, "fp64": 1, "fp32": 1}
    launches = res.gemm_launches
    a = 2 * n1 + 1
    b = 2 * (n2 - n1) + 1 if n2 > n1 else 0
    assert launches == 2 * res.iters + (2 if n2 > n1 else 1)
    expect = tile_fl * (a * prods[early] + b * prods[late] + (launches - a - b) * prods[final])
    assert res.mfma_flops == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("precision,tol_ddbar,err_tol", [("fp64", 1e-9, 1e-10),
                                                          ("fp32", 1e-6, 2.5e-6)])
def test_full_size_spectral_4096_fp64_vs_fp32(precision, tol_ddbar, err_tol):
    """M = 4096, N = 2048, gap 0.1, stopping at the paper's Tr(D Dbar) bound
    (FP64: 1e-9): FP64 to the oracle's accuracy, FP32 to its rounding.  The
    FP32 product runs 128 K stages of 8 MFMA steps; the default fold (every
    4 stages, sqrt(128 / 8)) rounds each term about 8*4 + 128/4 = 64 times,
    2^-24 sqrt(64) = 4.8e-7 relative per product, about 0.25x that times an
    amplification of 1-4 in the metric, over ~2p = 24 products adding in
    quadrature: 6e-7 to 2.5e-6.  One accumulator over K (fold never) rounds
    each term 1024 times, sqrt(1024 / 64) = 4x more."""
    w = workloads.config(2)
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    D, res = run_gpu(w, precision, tol_ddbar=tol_ddbar)
    err = rel_err(D, ref)
    log(f"  {precision}: iters={res.iters} err={err:.3e} ms={res.ms_total:.1f}")
    assert res.status in gcp.SUCCESS
    assert np.abs(res.col("t1") - w.N).max() < 1e-10
    assert err < err_tol
    if precision == "fp32":
        D1, r1 = run_gpu(w, precision, tol_ddbar=tol_ddbar, fold_every=1000)
        err1 = rel_err(D1, ref)
        log(f"  fp32 one accumulator: iters={r1.iters} err={err1:.3e}")
        assert err < err1 / 2
