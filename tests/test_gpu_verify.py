"""GPU parity of gcp_verify (the FP64 acceptance checks of a density matrix)
with their definitions in the oracle (oracle.verify_quantities), on the same
D and H bytes, and with the closed forms of the ground state.

Tolerances: the GPU forms Tr D, ||D||_F^2 and Tr(DH) as fixed-order FP64 sums
of M^2 terms (relative rounding ~1e-15 * sqrt(M^2)); ||D^2 - D||_F and
||HD - DH||_F come from FP64 MFMA products whose rounding, ~1e-16 * M * |D|^2
per element, sets an absolute floor near 1e-13 * M."""
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


@pytest.fixture(scope="module", autouse=True)
def _oracle(oracle_lib):
    return oracle_lib


def to_gpu(A, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(A)).to(dtype).cuda()


def check(q, ref, M):
    for k in ("trace", "fro2", "energy"):
        assert abs(q[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), (k, q[k], ref[k])
    for k in ("idem", "comm"):
        assert abs(q[k] - ref[k]) <= 1e-13 * M + 1e-12 * ref[k], (k, q[k], ref[k])


@pytest.mark.parametrize("M,N", [(200, 71), (384, 190)])
def test_verify_converged_matches_oracle_and_ground_state(M, N):
    w = workloads.spectral(M, N, 0.1, 40 + M)
    log(f"[gpu] verify {w.name}")
    with gcp.Context(M, tol_ddbar=1e-10) as ctx:
        H = to_gpu(w.H)
        ctx.init(H, w.N, w.emin, w.emax)
        D, res = ctx.purify(raise_on_failure=True)
        q = ctx.verify(D, H)
        torch.cuda.synchronize()
    Dh = D.cpu().numpy()
    ref = oracle.verify_quantities(Dh, w.H)
    check(q, ref, M)
    assert abs(q["trace"] - N) < 1e-10 and abs(q["fro2"] - N) < 1e-8
    assert abs(q["energy"] - np.sort(w.lam)[:N].sum()) < 1e-8
    assert q["idem"] < 1e-8 and q["comm"] < 1e-8


def test_verify_general_matrices_fp32_and_leading_dimensions():
    """A non-projector D (FP32, padded leading dimension) and a non-symmetric
    H: both are read as their symmetric parts."""
    M = 300
    rng = np.random.default_rng(7)
    D = (0.1 * rng.standard_normal((M, M))).astype(np.float32)
    H = rng.standard_normal((M, M))
    Dg = torch.zeros((M, M + 20), dtype=torch.float32, device="cuda")
    Dg[:, :M] = to_gpu(D, torch.float32)
    Hg = torch.zeros((M, M + 8), dtype=torch.float64, device="cuda")
    Hg[:, :M] = to_gpu(H)
    with gcp.Context(M) as ctx:
        q = ctx.verify(Dg[:, :M], Hg[:, :M])
    ref = oracle.verify_quantities(D.astype(np.float64), H)
    check(q, ref, M)


def test_verify_full_size_mixed_result():
    """M = 8192, N = 3000: the FP16X3 solve checked in FP64 against the same
    definitions and against the ground state (sum of the N lowest eigenvalues)."""
    w = workloads.config(3)
    log(f"[gpu] verify {w.name} fp16x3")
    with gcp.Context(w.M, precision="fp16x3", tol_ddbar=1e-5) as ctx:
        H = to_gpu(w.H)
        ctx.init(H, w.N, w.emin, w.emax)
        D, res = ctx.purify(raise_on_failure=True)
        q = ctx.verify(D, H)
        torch.cuda.synchronize()
    log(f"  {q}")
    ref = oracle.verify_quantities(D.cpu().numpy(), w.H)
    check(q, ref, w.M)
    e0 = np.sort(w.lam)[: w.N].sum()
    # error 6e-7 in ||D - D_ref||_F / sqrt(M) moves Tr(DH) to second order only
    assert abs(q["energy"] - e0) < 1e-6 * w.N
    assert abs(q["trace"] - w.N) < 1e-10
