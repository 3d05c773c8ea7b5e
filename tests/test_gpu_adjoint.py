"""GPU parity of the adjoint (gcp_backward through the C ABI) with the oracle.

The reference is the hand-written FP64 adjoint of ``oracle.grad`` evaluated
at the oracle's own FP64 iterates for the same number of updates p that the
GPU forward applied (the loss gradients and inputs are the same seeded
arrays).  At the bench size the reference is the Daleckii-Krein derivative
of the exact projector, computed row by row from the known eigenbasis, which
the converged recursion's gradient reaches.

Tolerances (max-norm, relative to the reference's largest entry):
  * FP64 adjoint: the two forwards' c_n differ by the FP64 rounding of the
    traces over Tr(D Dbar) (about 1e-14 N / Tr(D Dbar)), and the gradient
    moves by about that times |Gbar|, plus FP64 rounding of the products;
  * FP32 adjoint: FP32 storage and accumulation, about 1e-6 relative per
    update, compounding over p updates;
  * split-encoding forward: its iterates carry ~2^-22 relative rounding, which
    the adjoint sees as a perturbed D_n.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import grad
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


def gpu_grad(w, Gp, precision="fp64", bwd_precision="fp64", dtype=torch.float64, **opts):
    log(f"[gpu] adjoint {w.name} fwd={precision} bwd={bwd_precision} {opts}")
    with gcp.Context(w.M, precision=precision, keep_iterates=True, bwd_precision=bwd_precision,
                     **opts) as ctx:
        ctx.init(to_gpu(w.H), w.N, w.emin, w.emax)
        D, res = ctx.purify()
        dH, bres = ctx.backward(to_gpu(Gp, dtype))
        torch.cuda.synchronize()
        return dH.cpu().numpy().astype(np.float64), res, bres


def rel_max(a, ref):
    return float(np.abs(a - ref).max() / np.abs(ref).max())


def fp64_tol(w, p):
    """1e-14 N / min Tr(D Dbar) over the differentiated updates (oracle traces)."""
    if p == 0:
        return 1e-12
    _, _, t12, _, _ = grad.forward_iterates(w.H, w.N, w.emin, w.emax, p)
    return 1e-12 + 1e-14 * w.N / np.abs(t12).min()


CASES = [(200, 71, 0.1, 21), (384, 190, 0.1, 22), (520, 100, 0.2, 23)]


@pytest.mark.parametrize("M,N,gap,seed", CASES)
def test_fp64_adjoint_matches_oracle(M, N, gap, seed):
    """Ragged sizes (several 128-tiles and a padded tail); a non-symmetric
    dL/dD, of which only the symmetric part counts."""
    w = workloads.spectral(M, N, gap, seed)
    Gp = np.random.default_rng(seed + 100).standard_normal((M, M))
    dH, res, bres = gpu_grad(w, Gp, tol_ddbar=1e-6)
    assert res.status in gcp.SUCCESS and bres.iters == res.iters
    ref = grad.adjoint(w.H, w.N, w.emin, w.emax, res.iters, Gp)
    err, tol = rel_max(dH, ref), fp64_tol(w, res.iters)
    log(f"  p={res.iters} err={err:.3e} tol={tol:.3e}")
    assert np.array_equal(dH, dH.T)
    assert err <= tol


@pytest.mark.parametrize("M,N,gap,seed", CASES[1:])
def test_fp32_adjoint_matches_oracle(M, N, gap, seed):
    w = workloads.spectral(M, N, gap, seed)
    Gp = workloads.sym_gaussian(M, seed + 200)
    dH, res, bres = gpu_grad(w, Gp, bwd_precision="fp32", dtype=torch.float32, tol_ddbar=1e-6)
    ref = grad.adjoint(w.H, w.N, w.emin, w.emax, res.iters, Gp)
    err = rel_max(dH, ref)
    log(f"  p={res.iters} err={err:.3e}")
    assert err <= 2e-5 * max(res.iters, 1)


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x6"])
def test_split_forward_fp32_adjoint(precision):
    w = workloads.spectral(384, 150, 0.1, 24)
    Gp = workloads.sym_gaussian(384, 224)
    dH, res, bres = gpu_grad(w, Gp, precision=precision, bwd_precision="fp32", tol_ddbar=1e-6)
    ref = grad.adjoint(w.H, w.N, w.emin, w.emax, res.iters, Gp)
    err = rel_max(dH, ref)
    log(f"  {precision}: p={res.iters} err={err:.3e}")
    assert err <= 1e-3


def test_zero_updates_is_the_initial_guess_adjoint():
    """max_iter = 0: only D_0 = theta I + beta (mu I - H) is differentiated."""
    w = workloads.spectral(200, 60, 0.1, 25)
    Gp = workloads.sym_gaussian(200, 225)
    dH, res, _ = gpu_grad(w, Gp, max_iter=0)
    assert res.iters == 0 and res.status == gcp.ERR_NOT_CONVERGED
    ref = grad.adjoint(w.H, w.N, w.emin, w.emax, 0, Gp)
    assert rel_max(dH, ref) <= 1e-13


def test_not_converged_run_is_differentiated_as_applied():
    w = workloads.spectral(256, 100, 0.1, 26)
    Gp = workloads.sym_gaussian(256, 226)
    dH, res, _ = gpu_grad(w, Gp, max_iter=4)
    assert res.iters == 4 and res.status == gcp.ERR_NOT_CONVERGED
    ref = grad.adjoint(w.H, w.N, w.emin, w.emax, 4, Gp)
    assert rel_max(dH, ref) <= fp64_tol(w, 4)


@pytest.mark.parametrize("N", [0, 128])
def test_degenerate_filling_gives_zero(N):
    w = workloads.spectral(128, 64, 0.1, 27)
    w.N = N
    dH, res, _ = gpu_grad(w, workloads.sym_gaussian(128, 227))
    assert res.iters == 0
    assert np.all(dH == 0.0)


def test_repeated_backward_is_linear_and_deterministic():
    w = workloads.spectral(320, 120, 0.1, 28)
    G1 = workloads.sym_gaussian(320, 228)
    G2 = workloads.sym_gaussian(320, 229)
    with gcp.Context(w.M, keep_iterates=True) as ctx:
        ctx.init(to_gpu(w.H), w.N, w.emin, w.emax)
        ctx.purify()
        a, _ = ctx.backward(to_gpu(G1))
        b, _ = ctx.backward(to_gpu(G2))
        s, _ = ctx.backward(to_gpu(G1 + 2.0 * G2))
        a2, _ = ctx.backward(to_gpu(G1))
        torch.cuda.synchronize()
    a, b, s, a2 = (x.cpu().numpy() for x in (a, b, s, a2))
    assert np.array_equal(a, a2)
    assert rel_max(a + 2.0 * b, s) <= 1e-12


def test_leading_dimensions_and_fp32_buffers():
    M = 200
    w = workloads.spectral(M, 80, 0.1, 29)
    Gp = workloads.sym_gaussian(M, 230)
    with gcp.Context(M, keep_iterates=True) as ctx:
        ctx.init(to_gpu(w.H), w.N, w.emin, w.emax)
        ctx.purify()
        ref, _ = ctx.backward(to_gpu(Gp))
        big = torch.zeros((M, M + 40), dtype=torch.float64, device="cuda")
        big[:, :M] = to_gpu(Gp)
        out = torch.full((M, M + 24), 7.0, dtype=torch.float64, device="cuda")
        L = gcp.load_library()
        r = gcp.CResult()
        import ctypes
        st = L.gcp_backward(ctx._h, ctypes.c_void_p(big.data_ptr()), M + 40,
                            ctypes.c_void_p(out.data_ptr()), M + 24, gcp.DTYPE_F64,
                            ctypes.byref(r))
        assert st == gcp.OK
        f32, _ = ctx.backward(to_gpu(Gp, torch.float32))
        torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    o = out.cpu().numpy()
    assert np.array_equal(o[:, :M], ref)
    assert np.all(o[:, M:] == 7.0)            # padding columns untouched
    # FP32 input/output buffers, FP64 adjoint arithmetic
    assert rel_max(f32.cpu().numpy().astype(np.float64), ref) <= 1e-6


def test_state_errors():
    w = workloads.spectral(128, 50, 0.1, 30)
    g = to_gpu(np.eye(128))
    with gcp.Context(128) as ctx:                       # keep_iterates off
        ctx.init(to_gpu(w.H), w.N, w.emin, w.emax)
        ctx.purify()
        with pytest.raises(gcp.GCPError) as e:
            ctx.backward(g)
        assert e.value.status == gcp.ERR_STATE
    with gcp.Context(128, keep_iterates=True) as ctx:
        ctx.init(to_gpu(w.H), w.N, w.emin, w.emax)
        with pytest.raises(gcp.GCPError) as e:           # no purify yet
            ctx.backward(g)
        assert e.value.status == gcp.ERR_STATE
        ctx.purify()
        ctx.backward(g)
        ctx.init(to_gpu(w.H), w.N, w.emin, w.emax)      # a new init invalidates
        with pytest.raises(gcp.GCPError) as e:
            ctx.backward(g)
        assert e.value.status == gcp.ERR_STATE


def test_autograd_function_matches_oracle():
    w = workloads.spectral(256, 90, 0.1, 31)
    P = workloads.sym_gaussian(256, 231)
    H = to_gpu(w.H).requires_grad_(True)
    D = gcp.purify_autograd(H, w.N, w.emin, w.emax, tol_ddbar=1e-6)
    loss = (D * to_gpu(P)).sum()
    loss.backward()
    torch.cuda.synchronize()
    r = oracle.purify(w.H, w.N, w.emin, w.emax, tol_ddbar=1e-6)
    ref = grad.adjoint(w.H, w.N, w.emin, w.emax, r.iters, P)
    assert rel_max(H.grad.cpu().numpy(), ref) <= fp64_tol(w, r.iters)


def test_autograd_repeated_backward_and_side_stream():
    """retain_iterates=True keeps the stored iterates for a second backward
    through a retained graph (the same gradient, bitwise); without it the
    second backward raises a clear error.  A solve started while a side
    stream is current waits for that stream's work on H."""
    w = workloads.spectral(256, 90, 0.1, 32)
    P = to_gpu(workloads.sym_gaussian(256, 232))
    H = to_gpu(w.H).requires_grad_(True)
    D = gcp.purify_autograd(H, w.N, w.emin, w.emax, tol_ddbar=1e-6, retain_iterates=True)
    loss = (D * P).sum()
    g1, = torch.autograd.grad(loss, H, retain_graph=True)
    g2, = torch.autograd.grad(loss, H)
    assert torch.equal(g1, g2)
    D = gcp.purify_autograd(H, w.N, w.emin, w.emax, tol_ddbar=1e-6)
    loss = (D * P).sum()
    torch.autograd.grad(loss, H, retain_graph=True)
    with pytest.raises(RuntimeError, match="retain_iterates"):
        torch.autograd.grad(loss, H)
    side = torch.cuda.Stream()
    Hd = to_gpu(w.H)
    with gcp.Context(256, tol_ddbar=1e-6) as ctx:
        ctx.init(Hd, w.N, w.emin, w.emax)
        ref, _ = ctx.purify()
        with torch.cuda.stream(side):
            H2 = Hd * 1.0          # written on the side stream
            ctx.init(H2, w.N, w.emin, w.emax)
            D2, _ = ctx.purify()
        side.synchronize()
        assert torch.equal(D2, ref)


def test_full_size_cubic_lattice_adjoint():
    """The 16 x 16 x 8 periodic lattice (M = 2048, N = 682) with
    L = Tr(D P), P symmetric Gaussian: FP64 and FP32 adjoints against the
    oracle's FP64 adjoint at the same p."""
    w = workloads.config(4)
    P = workloads.sym_gaussian(w.M, 40)
    dH64, res, bres = gpu_grad(w, P, tol_ddbar=1e-8, max_iter=200)
    assert res.status == gcp.OK
    log(f"  p={res.iters} backward {bres.ms_total:.1f} ms ({bres.gemm_launches} products)")
    ref = grad.adjoint(w.H, w.N, w.emin, w.emax, res.iters, P)
    err64 = rel_max(dH64, ref)
    dH32, res32, _ = gpu_grad(w, P, bwd_precision="fp32", tol_ddbar=1e-8, max_iter=200)
    assert res32.iters == res.iters
    err32 = rel_max(dH32, ref)
    log(f"  fp64 err={err64:.3e} (tol {fp64_tol(w, res.iters):.3e})  fp32 err={err32:.3e}")
    assert err64 <= fp64_tol(w, res.iters)
    assert err32 <= 2e-5 * res.iters


def _dk_rows(w, u, rows):
    """Rows of the Daleckii-Krein gradient of L = u^T P u (P the projector
    onto the N lowest eigenvectors of H = Q diag(lam) Q^T)."""
    order = np.argsort(w.lam, kind="stable")
    occ, vir = order[: w.N], order[w.N:]
    V = w.Q
    wv = V.T @ u
    F = 1.0 / (w.lam[occ][:, None] - w.lam[vir][None, :])      # occ x vir
    out = []
    for i in rows:
        a = V[i] * wv
        y = np.zeros(w.M)
        y[vir] = a[occ] @ F
        y[occ] = F @ a[vir]
        out.append(V @ (wv * y))
    return np.array(out)


# FP64: the recursion's gradient one update past tol 1e-9 equals the projector
# derivative to rounding.  Split forward stopped at 1e-5 + FP32 adjoint: up to
# ~1e-6 from the unfinished last update plus the FP32 adjoint's 2e-5 per update.
@pytest.mark.parametrize("precision,bwd,tol_ddbar,err_tol", [("fp64", "fp64", 1e-9, 1e-7),
                                                             ("fp16x3", "fp32", 1e-5, 1e-3)])
def test_full_size_spectral_8192_against_daleckii_krein(precision, bwd, tol_ddbar, err_tol):
    """M = 8192, N = 3000, gap 0.05 with L = u^T D u: sampled rows of dL/dH
    against the exact projector derivative (known eigenbasis)."""
    w = workloads.config(3)
    u = np.random.default_rng(33).standard_normal(w.M)
    dH, res, bres = gpu_grad(w, np.outer(u, u), precision=precision, bwd_precision=bwd,
                             tol_ddbar=tol_ddbar)
    assert res.status in gcp.SUCCESS
    rows = [0, 1, 777, 4095, 6000, 8191]
    ref = _dk_rows(w, u, rows)
    err = float(np.abs(dH[rows] - ref).max() / np.abs(ref).max())
    log(f"  {precision}/{bwd}: p={res.iters} DK err={err:.3e} backward {bres.ms_total:.1f} ms "
        f"({bres.gemm_flops / bres.ms_total / 1e9:.1f} TFLOP/s algorithmic)")
    assert np.array_equal(dH, dH.T)
    assert err <= err_tol


def test_adjoint_through_a_precision_switch():
    """FP16X3 then FP64 (switch below Tr(D Dbar) = 1e-3): the kept iterates
    change encoding mid-run; the FP64 adjoint still matches the oracle's."""
    w = workloads.spectral(384, 150, 0.1, 34)
    Gp = workloads.sym_gaussian(384, 234)
    dH, res, _ = gpu_grad(w, Gp, precision="fp16x3", late_precision="fp64", switch_ddbar=1e-3,
                          tol_ddbar=1e-9)
    assert res.status in gcp.SUCCESS
    ref = grad.adjoint(w.H, w.N, w.emin, w.emax, res.iters, Gp)
    err = rel_max(dH, ref)
    log(f"  p={res.iters} err={err:.3e}")
    assert err <= 1e-3


@pytest.mark.parametrize("opts", [{}, {"bwd_precision": "fp32"},
                                  {"precision": "fp16x3", "late_precision": "fp64",
                                   "switch_ddbar": 1e-2, "tol_ddbar": 1e-9},
                                  {"precision": "fp64", "late_precision": "fp16x3",
                                   "switch_ddbar": 1e30, "tol_ddbar": 1e-6},
                                  {"precision": "fp16x3", "late_precision": "bf16x6",
                                   "switch_ddbar": 1e-1, "final_precision": "fp64",
                                   "final_ddbar": 1e-3, "tol_ddbar": 1e-9},
                                  {"hole": True}, {"max_iter": 0}])
def test_checkpointed_backward_is_bitwise_the_kept_one(opts):
    """checkpoint_every = 3 and 5: every segment is recomputed from its
    checkpoint with the forward's kernels, so the gradient is bitwise the one
    from kept iterates (including a precision switch inside a segment, one at
    the first update, where the kept D_0 must be the re-encoded one that K2
    reads, a three-phase schedule, the hole recursion and a run with no
    update)."""
    w = workloads.spectral(384, 150, 0.1, 35)
    Gp = workloads.sym_gaussian(384, 235)
    o = {"tol_ddbar": 1e-6}
    o.update(opts)
    bw = o.pop("bwd_precision", "fp64")
    dt = torch.float32 if bw == "fp32" else torch.float64
    ref, r0, _ = gpu_grad(w, Gp, bwd_precision=bw, dtype=dt, **o)
    for ck in (3, 5):
        dH, r, _ = gpu_grad(w, Gp, bwd_precision=bw, dtype=dt, checkpoint_every=ck, **o)
        assert r.iters == r0.iters
        assert np.array_equal(dH, ref), (ck, float(np.abs(dH - ref).max()))


def test_full_size_16384_bf16x6_checkpointed_adjoint():
    """M = 16384, N = 8192, gap 0.02: BF16 MFMA forward (BF16X6, FP32
    accumulation), iterates checkpointed every 8 updates and recomputed in the
    FP32 backward; D against the closed form and sampled rows of dL/dH for
    L = u^T D u against the Daleckii-Krein derivative."""
    w = workloads.config(5)
    log(f"[gpu] {w.name}")
    u = np.random.default_rng(55).standard_normal(w.M)
    with gcp.Context(w.M, precision="bf16x6", tol_ddbar=1e-5, keep_iterates=True,
                     checkpoint_every=8, bwd_precision="fp32") as ctx:
        ctx.init(to_gpu(w.H), w.N, w.emin, w.emax)
        D, res = ctx.purify(raise_on_failure=True)
        ug = to_gpu(u)
        dH, bres = ctx.backward(torch.outer(ug, ug))
        torch.cuda.synchronize()
        D = D.cpu().numpy()
        dH = dH.cpu().numpy()
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    err = float(np.linalg.norm(D - ref) / np.sqrt(w.M))
    rows = [0, 5000, 16383]
    dk = _dk_rows(w, u, rows)
    gerr = float(np.abs(dH[rows] - dk).max() / np.abs(dk).max())
    log(f"  p={res.iters} err={err:.2e} forward {res.ms_total:.0f} ms, backward "
        f"{bres.ms_total:.0f} ms, DK err={gerr:.2e}")
    assert abs(np.trace(D) - w.N) < 1e-9
    assert err < 1e-5
    assert gerr < 1e-3
