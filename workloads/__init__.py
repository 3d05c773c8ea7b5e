"""Seeded synthetic Hamiltonians for the purification workloads.

This module only draws random numbers and assembles matrices; it holds none of
the purification arithmetic, so both the CPU oracle and the GPU path consume
exactly the bytes produced here.

All generators use numpy's PCG64 (``default_rng(seed)``) and return float64
arrays in C order.  The paper's own test matrices (dense, symmetric, with a
chosen spectrum and gap, Section "efficiency and limitations") are mirrored by
:func:`spectral` (dense, eigenvectors from a random orthogonal matrix) and
:func:`paper_diagonal` (the paper's "vanishing off-diagonal elements" reading);
the tight-binding lattices give sparse-pattern, physically structured H.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Workload:
    """One purification problem: H (M x M, symmetric), N occupied states and
    spectral bounds [emin, emax] passed to the solver.

    ``Q``/``lam`` are set when the spectrum is known by construction
    (H = Q diag(lam) Q^T); ``name`` describes the recipe.
    """

    name: str
    H: np.ndarray
    N: int
    emin: float
    emax: float
    Q: Optional[np.ndarray] = None
    lam: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.H.shape[0])


def chain_1d(M: int, N: int, seed: int, onsite: float = 0.5, hop: float = -1.0,
             emin: float = -2.5, emax: float = 2.5) -> Workload:
    """Open 1D tight-binding chain: H_ii ~ U[-onsite, onsite], H_{i,i+1} = hop."""
    rng = np.random.default_rng(seed)
    H = np.zeros((M, M))
    H[np.diag_indices(M)] = rng.uniform(-onsite, onsite, M)
    i = np.arange(M - 1)
    H[i, i + 1] = hop
    H[i + 1, i] = hop
    return Workload(f"chain1d_M{M}_N{N}_s{seed}", H, N, emin, emax)


def cubic_3d(Lx: int, Ly: int, Lz: int, N: int, seed: int, onsite: float = 1.0,
             hop: float = -1.0, emin: float = -7.0, emax: float = 7.0) -> Workload:
    """Periodic simple-cubic tight-binding lattice; site index x + Lx*(y + Ly*z)."""
    rng = np.random.default_rng(seed)
    M = Lx * Ly * Lz
    H = np.zeros((M, M))
    H[np.diag_indices(M)] = rng.uniform(-onsite, onsite, M)
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    site = x + Lx * (y + Ly * z)
    for dx, dy, dz in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        nb = (x + dx) % Lx + Lx * (((y + dy) % Ly) + Ly * ((z + dz) % Lz))
        # accumulate so that a dimension of length 2 (both neighbours equal) stays consistent
        np.add.at(H, (site, nb), hop)
        np.add.at(H, (nb, site), hop)
    return Workload(f"cubic3d_{Lx}x{Ly}x{Lz}_N{N}_s{seed}", H, N, emin, emax)


def random_orthogonal(M: int, rng: np.random.Generator) -> np.ndarray:
    """Q factor of the QR decomposition of an iid standard-normal matrix."""
    G = rng.standard_normal((M, M))
    Q, _ = np.linalg.qr(G)
    return np.ascontiguousarray(Q)


def spectral(M: int, N: int, gap: float, seed: int, emin: float = -1.0,
             emax: float = 1.0) -> Workload:
    """Dense H = Q diag(lam) Q^T with N eigenvalues uniform in [-1, -gap/2] and
    M-N uniform in [gap/2, 1]; Q from the QR of a seeded Gaussian matrix.

    The eigenvalues are drawn first (occupied block, then the rest), then Q.
    """
    rng = np.random.default_rng(seed)
    lam = np.concatenate([rng.uniform(-1.0, -gap / 2, N), rng.uniform(gap / 2, 1.0, M - N)])
    Q = random_orthogonal(M, rng)
    H = (Q * lam) @ Q.T
    H = 0.5 * (H + H.T)
    return Workload(f"spectral_M{M}_N{N}_gap{gap:g}_s{seed}", np.ascontiguousarray(H), N,
                    emin, emax, Q=Q, lam=lam, meta={"gap": gap})


def paper_diagonal(M: int, N: int, gap: float, seed: int, lo: float = -2.5,
                   hi: float = 2.5) -> Workload:
    """Diagonal H with eigenvalues random in [lo, e_N] U [e_N + gap, hi].

    The gap-free width (hi - lo - gap) is split in the ratio N : M-N, so
    e_N = lo + (N/M)(hi - lo - gap) and e_{N+1} = e_N + gap; both are placed
    exactly and the others are uniform in their intervals, in a random order
    along the diagonal.  Bounds are reported as [lo, hi].
    """
    rng = np.random.default_rng(seed)
    homo = lo + (N / M) * (hi - lo - gap)
    lumo = homo + gap
    parts = []
    if N > 0:
        parts.append(np.append(rng.uniform(lo, homo, N - 1), homo))
    if M - N > 0:
        parts.append(np.append(rng.uniform(lumo, hi, M - N - 1), lumo))
    lam = np.concatenate(parts)
    lam = lam[rng.permutation(M)]
    H = np.diag(lam)
    return Workload(f"paperdiag_M{M}_N{N}_gap{gap:g}_s{seed}", H, N, lo, hi,
                    Q=np.eye(M), lam=lam, meta={"gap": gap, "homo": homo, "lumo": lumo})


def sym_gaussian(M: int, seed: int) -> np.ndarray:
    """P = (G + G^T)/2 with G iid N(0, 1)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((M, M))
    return np.ascontiguousarray(0.5 * (G + G.T))


def config(k: int, scale: int = 1) -> Workload:
    """The five standard workloads (``scale`` divides M for quick runs where the
    recipe allows it; scale=1 is the full size)."""
    if k == 1:
        return chain_1d(256 // scale, 100 // scale, seed=1)
    if k == 2:
        M = 4096 // scale
        return spectral(M, M // 2, gap=0.1, seed=2)
    if k == 3:
        M = 8192 // scale
        return spectral(M, (3000 * M) // 8192, gap=0.05, seed=3)
    if k == 4:
        if scale != 1:
            raise ValueError("the 16x16x8 lattice has no reduced form")
        return cubic_3d(16, 16, 8, 682, seed=4)
    if k == 5:
        M = 16384 // scale
        return spectral(M, M // 2, gap=0.02, seed=5)
    raise ValueError(f"unknown workload {k}")
