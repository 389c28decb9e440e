"""Seeded synthetic inputs (gauge fields and proposals).

This module generates inputs only; it holds none of the method's
arithmetic and is shared by the tests, the benchmark and the smoke check.
Both the HIP library and the CPU oracle receive the same arrays from here.

Links are U = exp(i c H) with H = sum_a h_a lambda_a / 2, h_a ~ N(0, 1)
(Gell-Mann matrices, tr(T_a T_b) = delta_ab / 2), one independent H per
link.  A proposal U' redraws a chosen set of links with fresh H.  Random
streams: numpy Philox with key (seed, tag); tag 0 draws the H of U, tag 1
the link selection, tag 2 the H of redrawn links.

Canonical layout: U[site, mu, row, col] complex128, site = x0 + L0*(x1 +
L1*(x2 + L2*x3)), U[x, mu] is the link from x to x + mu.
"""
from __future__ import annotations

import numpy as np


def gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return lam


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed) & (2**64 - 1), tag]))


def su3_from_h(h: np.ndarray, scale: float) -> np.ndarray:
    """exp(i * scale * H) for H = sum_a h[..., a] lambda_a / 2 (via eigh)."""
    H = np.einsum("...a,aij->...ij", h, gell_mann()) / 2
    w, v = np.linalg.eigh(H)
    return (v * np.exp(1j * scale * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def gauge_field(L, scale: float, seed: int) -> np.ndarray:
    V = int(np.prod(L))
    h = _rng(seed, 0).standard_normal((V, 4, 8))
    return np.ascontiguousarray(su3_from_h(h, scale))


def unit_gauge(L) -> np.ndarray:
    V = int(np.prod(L))
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1
    return U


def bernoulli_links(L, p: float, seed: int) -> np.ndarray:
    """mask[site, mu]: each link chosen independently with probability p."""
    V = int(np.prod(L))
    return _rng(seed, 1).random((V, 4)) < p


def redraw(U: np.ndarray, mask: np.ndarray, scale: float, seed: int) -> np.ndarray:
    """U' = U with the links where mask is true replaced by fresh exp(i c H')."""
    Up = U.copy()
    idx = np.nonzero(mask)
    h = _rng(seed, 2).standard_normal((len(idx[0]), 8))
    Up[idx] = su3_from_h(h, scale)
    return np.ascontiguousarray(Up)


def spinor(L, seed: int, tag: int = 7) -> np.ndarray:
    """A generic complex Gaussian test field psi[site, 4, 3]."""
    V = int(np.prod(L))
    r = _rng(seed, tag)
    return (r.standard_normal((V, 4, 3)) + 1j * r.standard_normal((V, 4, 3))) / np.sqrt(2)


# Solver settings (fields of wdr_solver_params, by name) of the mixed-precision
# form of the large-lattice workloads: CG on the normal equations (their kappa
# lies above the free-field critical value, where the Schwarz-preconditioned
# GCR stalls) with FP16 inner iterations, an FP32 middle level and FP64 outer
# reliable updates; FP16 block solves.
LARGE_MIXED = dict(solver=1, inner=2, middle=1, max_iter=20000)

# Workloads: lattice, blocks, kappa, link scale, noise and solver settings of
# the standard cases.  "seed" keys the Philox streams above.
WORKLOADS = {
    "wilson4_full_z2": dict(L=(4, 4, 4, 4), B=(2, 2, 2, 2), kappa=0.12, scale=0.3, op="full", noise="z2",
                            n_noise=12, proposal="bernoulli", p=0.10, seed=1112124300),
    "wilson8_dd16": dict(L=(8, 8, 8, 8), B=(4, 4, 4, 4), kappa=0.135, scale=0.5, op="schur", noise="gauss",
                         n_noise=8, proposal="active", seed=1112124301),
    "wilson16_dd256": dict(L=(16, 16, 16, 16), B=(4, 4, 4, 4), kappa=0.150, scale=0.25, op="schur",
                           noise="gauss", n_noise=16, proposal="black_blocks", seed=1112124302,
                           mixed=LARGE_MIXED),
    "wilson32_dd4096": dict(L=(32, 32, 32, 32), B=(4, 4, 4, 4), kappa=0.155, scale=0.2, op="schur",
                            noise="gauss", n_noise=32, proposal="active", seed=1112124303,
                            mixed=LARGE_MIXED),
    # recursive DD in the block geometry of the paper's realistic run: 8^4
    # blocks with 4^4 sub-blocks, links of a 6^4 core redrawn in every block
    "recursive16_dd8": dict(L=(16, 16, 16, 16), B=(8, 8, 8, 8), Bsub=(4, 4, 4, 4), kappa=0.150, scale=0.25,
                            op="schur", noise="gauss", n_noise=8, proposal="core6", seed=1112124304),
}

# batched proposals of uneven sizes: (lattice, count); 4^4 blocks (12^4 has 3
# blocks per direction: fine for the full operator, which needs no colouring)
BATCH_SIZES = (((8, 8, 8, 8), 24), ((12, 12, 12, 12), 24), ((16, 16, 16, 16), 16))
BATCH_SEED = 1112124400


def batch_proposals(sizes=BATCH_SIZES, seed0: int = BATCH_SEED, kappa_lo: float = 0.12, kappa_hi: float = 0.15):
    """Seeds and hopping parameters of the batched-proposal workload: proposal
    j has seed seed0 + j and kappa uniform in [kappa_lo, kappa_hi] (tag 4)."""
    out, j = [], 0
    for L, count in sizes:
        for _ in range(count):
            u = _rng(seed0 + j, 4).random()
            out.append(dict(L=L, seed=seed0 + j, kappa=kappa_lo + (kappa_hi - kappa_lo) * u))
            j += 1
    return out
