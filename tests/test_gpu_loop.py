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


@pytest.mark.parametrize("case", [
    ("chain", {"precision": "fp64", "tol_ddbar": 0.0, "tol_idem": 1e-10}),
    ("spectral", {"precision": "fp16x3", "tol_ddbar": 1e-6}),
    ("spectral", {"precision": "fp32", "tol_ddbar": 1e-6, "max_iter": 7}),
    ("spectral", {"precision": "fp16x3", "late_precision": "fp64", "switch_ddbar": 1e-2,
                  "tol_ddbar": 1e-10}),
])
def test_sync_every_changes_nothing_but_the_host_syncs(case):
    kind, opts = case
    w = workloads.config(1) if kind == "chain" else workloads.spectral(520, 200, 0.1, 61)
    D1, r1 = solve(w, sync_every=1, profile=True, **opts)
    p = r1.iters
    assert r1.gemm_launches == 2 * p + 1
    for k in (2, 3, 4, 7, 50):
        Dk, rk = solve(w, sync_every=k, profile=True, **opts)
        assert rk.status == r1.status and rk.iters == p
        assert np.array_equal(Dk, D1)
        assert np.array_equal(rk.history, r1.history, equal_nan=True)
        assert rk.gemm_launches == 2 * p + 1   # void launches past the stop not counted
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
