"""The iteration loop: device-side stop decisions with batched host checks,
and the stop at the encoding's rounding floor.

The decision to stop (the paper's test on Tr(D Dbar), made before c_n is
formed) is taken on the device; the host enqueues sync_every updates between
checks and launches past the stop do nothing, so the iterates and the
history must not depend on sync_every.
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


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solve(w, **opts):
    log(f"[gpu] {w.name} {opts}")
    H = torch.from_numpy(np.ascontiguousarray(w.H)).cuda()
    with gcp.Context(w.M, **opts) as ctx:
        ctx.init(H, w.N, w.emin, w.emax)
        D, res = ctx.purify()
        torch.cuda.synchronize()
        return D.cpu().numpy(), res


# (workload, options, whether the stop needs the square of the last iterate:
# the idempotency test and max_iter are decided after it, a stop on
# Tr(D Dbar) from the last update's traces; switches of encoding, each of
# which forms D^2 once more)
@pytest.mark.parametrize("case", [
    ("chain", {"precision": "fp64", "tol_ddbar": 0.0, "tol_idem": 1e-10}, True, 0),
    ("spectral", {"precision": "fp16x3", "tol_ddbar": 1e-6}, False, 0),
    ("spectral", {"precision": "fp32", "tol_ddbar": 1e-6, "max_iter": 7}, True, 0),
    ("spectral", {"precision": "fp16x3", "late_precision": "fp64", "switch_ddbar": 1e-2,
                  "tol_ddbar": 1e-10}, False, 1),
])
def test_sync_every_changes_nothing_but_the_host_syncs(case):
    kind, opts, last_square, switches = case
    w = workloads.config(1) if kind == "chain" else workloads.spectral(520, 200, 0.1, 61)
    D1, r1 = solve(w, sync_every=1, profile=True, **opts)
    p = r1.iters
    launches = 2 * p + (1 if last_square else 0) + switches
    assert r1.gemm_launches == launches
    assert math.isnan(r1.idem) != last_square
    for k in (2, 3, 4, 7, 50):
        Dk, rk = solve(w, sync_every=k, profile=True, **opts)
        assert rk.status == r1.status and rk.iters == p
        assert np.array_equal(Dk, D1)
        assert np.array_equal(rk.history, r1.history, equal_nan=True)
        assert rk.gemm_launches == launches   # void launches past the stop not counted
        if "late_precision" not in opts:
            assert rk.host_syncs <= math.ceil((p + 1) / k), (k, rk.host_syncs, p)
        log(f"  sync_every={k}: p={p} host syncs {rk.host_syncs} (every update: {r1.host_syncs})")


@pytest.mark.parametrize("precision,M,N", [("fp16x3", 8192, 3000), ("bf16x3", 640, 234)])
def test_stop_at_the_rounding_floor(precision, M, N):
    """A tolerance far below the encoding's rounding floor: the solve stops
    with STOPPED_AT_FLOOR (not a breakdown), the result keeps its accuracy
    and its trace; without a floor the old rule reports a breakdown or runs
    out of iterations."""
    w = workloads.config(3) if M == 8192 else workloads.spectral(M, N, 0.1, 62)
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    D, res = solve(w, precision=precision, tol_ddbar=1e-11, max_iter=60)
    err = float(np.linalg.norm(D - ref) / math.sqrt(w.M))
    last = res.history[-1]
    log(f"  {precision}: status {res.status} p={res.iters} err={err:.3e} "
        f"last Tr(D Dbar)={last[1] - last[2]:.3e}")
    assert res.status == gcp.STOPPED_AT_FLOOR
    assert abs(np.trace(D) - w.N) < 1e-10
    assert err <= (1e-6 if precision == "fp16x3" else 1e-4)
    D0, r0 = solve(w, precision=precision, tol_ddbar=1e-11, max_iter=60, floor_ddbar=0.0)
    assert r0.status in (gcp.ERR_BREAKDOWN, gcp.ERR_NOT_CONVERGED)


@pytest.mark.parametrize("precision,tol", [("fp16x3", 1e-6), ("fp64", 1e-9), ("bf16x3", 1e-11)])
def test_stop_on_the_last_traces_skips_only_the_last_square(precision, tol):
    """A stop on Tr(D Dbar) (the tolerance, or the rounding floor while
    Tr(D Dbar) stops decreasing) is decided from the traces of the last
    update.  Forcing the square of the last iterate (an idempotency test that
    never fires, tol_idem = 1e-300) must give the same status, p, D and
    history except the last row's T3 and Omega, with one launch more."""
    w = workloads.spectral(640, 234, 0.1, 63)
    Da, ra = solve(w, precision=precision, tol_ddbar=tol, max_iter=60)
    Db, rb = solve(w, precision=precision, tol_ddbar=tol, max_iter=60, tol_idem=1e-300)
    log(f"  {precision}: status {ra.status} p={ra.iters} launches {ra.gemm_launches} / "
        f"{rb.gemm_launches} idem {ra.idem} / {rb.idem:.2e}")
    assert ra.status in gcp.SUCCESS
    assert ra.status == rb.status and ra.iters == rb.iters
    assert np.array_equal(Da, Db)
    p = ra.iters
    assert np.array_equal(ra.history[:p], rb.history[:p], equal_nan=True)
    assert np.array_equal(ra.history[p, :3], rb.history[p, :3])
    assert ra.gemm_launches == 2 * p and rb.gemm_launches == 2 * p + 1
    assert math.isnan(ra.idem) and rb.idem >= 0.0
