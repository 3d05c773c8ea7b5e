"""gcp_purify_static: the solve without allocation, through the C ABI.

Two calls in a row, the second with a smaller input, each compared with the
context entry points (gcp_create + gcp_init + gcp_purify) on the same input:
the same kernels and launch configuration run on the static workspace, so
the results are bitwise equal.  A size above the maximum is refused with a
clear error.
"""
import ctypes
import sys

import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1512_07236_amd as gcp  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def static_call(L, H, w, out, opts):
    r = gcp.CResult()
    st = L.gcp_purify_static(ctypes.c_void_p(H.data_ptr()), H.stride(0), w.M, w.N, w.emin,
                             w.emax, ctypes.byref(opts), ctypes.c_void_p(out.data_ptr()),
                             gcp.DTYPE_F64, out.stride(0),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                             ctypes.byref(r))
    torch.cuda.synchronize()
    return st, r


@pytest.mark.parametrize("cases", [
    [(1000, 377, "fp16x3", {}), (520, 200, "fp16x3", {})],
    [(777, 300, "fp64", {"tol_ddbar": 0.0, "tol_idem": 1e-10}),
     (256, 100, "bf16x6", {"late_precision": int(gcp.Precision.FP64), "switch_ddbar": 1e-2,
                           "tol_ddbar": 1e-9})],
])
def test_static_solve_equals_the_context_solve(cases):
    L = gcp.load_library()
    for M, N, prec, extra in cases:
        w = workloads.spectral(M, N, 0.1, M + 3)
        H = torch.from_numpy(w.H).cuda()
        o = gcp.default_options()
        o.precision = int(gcp.Precision.parse(prec))
        for k, v in extra.items():
            setattr(o, k, v)
        kw = {k: v for k, v in extra.items()}
        if "late_precision" in kw:
            kw["late_precision"] = gcp.Precision(kw["late_precision"])
        D_ref, r_ref = gcp.purify(H, N, w.emin, w.emax, precision=prec, **kw)
        D = torch.full((M, M), float("nan"), dtype=torch.float64, device="cuda")
        st, r = static_call(L, H, w, D, o)
        log(f"  M={M} {prec}: static status {st} p={r.iters}; context status {r_ref.status} "
            f"p={r_ref.iters}")
        assert st == r_ref.status and r.iters == r_ref.iters
        assert r.t1 == r_ref.t1 and r.t2 == r_ref.t2
        assert r.idem == r_ref.idem or (math.isnan(r.idem) and math.isnan(r_ref.idem))
        assert torch.equal(D, D_ref)


def test_static_solve_refuses_sizes_and_options_it_cannot_serve():
    L = gcp.load_library()
    w = workloads.spectral(1100, 400, 0.1, 9)
    H = torch.from_numpy(w.H).cuda()
    D = torch.empty((1100, 1100), dtype=torch.float64, device="cuda")
    st, _ = static_call(L, H, w, D, gcp.default_options())
    assert st == gcp.ERR_INVALID_ARG and b"GCP_STATIC_MAX_M" in L.gcp_last_error(None)
    w = workloads.spectral(300, 100, 0.1, 9)
    H = torch.from_numpy(w.H).cuda()
    D = torch.empty((300, 300), dtype=torch.float64, device="cuda")
    o = gcp.default_options()
    o.keep_iterates = 1
    st, _ = static_call(L, H, w, D, o)
    assert st == gcp.ERR_INVALID_ARG and b"keep_iterates" in L.gcp_last_error(None)
