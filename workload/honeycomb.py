"""Honeycomb lattice inputs and the named workloads.

Section 2 of the paper fixes the problem: a V x V hopping matrix K, N_t time
slices of width delta = beta / N_t, and an auxiliary field phi with one real
value per (time slice, site).  The slice matrix is B_t = exp(delta*kappa*K) *
diag(exp(i*phi_t)).  The paper names no lattice; the workloads here use the
L x L periodic honeycomb lattice (N = 2 L^2 sites) with unit nearest-neighbour
hopping, and Gaussian fields of variance delta*U (the Hubbard-Stratonovich
weight exp(-phi^2 / (2 delta U))).

Nothing in this file computes a determinant, a product of slices or a Green's
function: it only produces inputs.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def honeycomb_site(i: int, j: int, sub: int, L: int) -> int:
    """Site index of sublattice `sub` (0 = A, 1 = B) in unit cell (i, j)."""
    return 2 * ((i % L) * L + (j % L)) + sub


def honeycomb_hopping(L: int) -> np.ndarray:
    """Real symmetric N x N adjacency of the periodic L x L honeycomb lattice.

    A(i, j) bonds to B(i, j), B(i-1, j) and B(i, j-1) (indices mod L), one
    unit entry per bond.  L >= 2 (L = 1 would create multi-edges).
    """
    if L < 2:
        raise ValueError("honeycomb lattice needs L >= 2")
    n = 2 * L * L
    K = np.zeros((n, n), dtype=np.float64)
    for i in range(L):
        for j in range(L):
            a = honeycomb_site(i, j, 0, L)
            for (bi, bj) in ((i, j), (i - 1, j), (i, j - 1)):
                b = honeycomb_site(bi, bj, 1, L)
                K[a, b] = 1.0
                K[b, a] = 1.0
    return K


def sample_phi(seed: int, Nt: int, N: int, delta: float, U: float) -> np.ndarray:
    """phi[t-1, x] ~ N(0, delta*U) (variance delta*U), drawn row-major in (t, x).

    Row t-1 holds the field of slice B_t; B_1 (row 0) acts first.
    """
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, math.sqrt(delta * U), size=(Nt, N)).astype(np.float64)


def uniform_phi(c: np.ndarray, N: int) -> np.ndarray:
    """Field that is constant in space on every slice: phi[t, x] = c[t]."""
    c = np.asarray(c, dtype=np.float64)
    return np.repeat(c[:, None], N, axis=1)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One field configuration of the honeycomb model."""

    L: int
    Nt: int
    beta: float
    U: float
    seed: int
    kappa: float = 1.0
    s: int = 8          # stabilisation interval (QR every s slices)
    c: int = 16         # checkpoint interval of the force sweep

    @property
    def N(self) -> int:
        return 2 * self.L * self.L

    @property
    def delta(self) -> float:
        return self.beta / self.Nt

    @property
    def dk(self) -> float:
        return self.delta * self.kappa

    def K(self) -> np.ndarray:
        return honeycomb_hopping(self.L)

    def phi(self) -> np.ndarray:
        return sample_phi(self.seed, self.Nt, self.N, self.delta, self.U)


def batched_mix(count: int = 256, base_seed: int = 3000) -> list[Workload]:
    """Mixed-size batch: L cycles through {3,5,6,7,8}, N_t through {32..512}.

    delta = 0.125 everywhere (beta = N_t / 8), U = 3, seed base_seed + i.
    """
    Ls = [3, 5, 6, 7, 8]
    Nts = [32, 64, 128, 256, 512]
    out = []
    for i in range(count):
        L = Ls[i % 5]
        Nt = Nts[(i // 5) % 5]
        out.append(Workload(L=L, Nt=Nt, beta=Nt * 0.125, U=3.0, seed=base_seed + i))
    return out


def hmc_batch(count: int = 32, base_seed: int = 5000) -> list[Workload]:
    """Large dense batch: L = 16 (N = 512), N_t = 512, beta = 64, U = 3."""
    return [Workload(L=16, Nt=512, beta=64.0, U=3.0, seed=base_seed + j, s=16)
            for j in range(count)]


WORKLOADS = {
    # plain stabilised determinant, L=3 (N=18), N_t=16, beta=2, U=2, s=4
    "plain_det_L3": Workload(L=3, Nt=16, beta=2.0, U=2.0, seed=1, s=4),
    # low temperature single configuration, L=6 (N=72), N_t=256, beta=32, s=8
    "lowT_L6": Workload(L=6, Nt=256, beta=32.0, U=3.0, seed=2, s=8),
    # adjoint force, L=8 (N=128), N_t=256, beta=32, checkpoints every 16
    "force_L8": Workload(L=8, Nt=256, beta=32.0, U=3.0, seed=4, s=8, c=16),
}
