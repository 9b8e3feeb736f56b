"""Seeded synthetic inputs: jittered cubic lattices in reduced units.

This module only draws random inputs; it holds none of the method's
arithmetic, so both the GPU path and the oracle may be fed from it.

Recipe (the paper's setup of Sec. 4 restated in reduced units m = a = kB = 1):
  * n_side^3 particles, site (i + 1/2) a of a simple cubic lattice, ids in
    x-fastest lattice order, plus a uniform jitter U(-jitter, jitter) per
    component;
  * momenta Maxwell-Boltzmann at temperature T: N(0, m kB T) per component,
    minus the mean so that the total momentum is zero;
  * internal energies eps_i = Cv T (so that T_i = T for the ideal gas).
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n_side: int
    Cv: float
    T: float
    steps: int
    spacing: float = 1.0
    jitter: float = 0.05
    m: float = 1.0
    kB: float = 1.0
    h: float = 2.5
    eta: float = 1.0
    zeta: float = 0.0
    dt: float = 0.005
    seed: int = 0          # Philox key
    init_seed: int = 0     # numpy generator seed of the initial state

    @property
    def n(self) -> int:
        return self.n_side ** 3

    @property
    def box(self) -> float:
        return self.n_side * self.spacing


# The five synthetic workloads (sizes of the paper's setting scaled up).
WORKLOADS = {
    "lattice10_cv10": Workload("lattice10_cv10", 10, Cv=10.0, T=1.0, steps=100),
    "lattice128_cv1.5_T0.1": Workload("lattice128_cv1.5_T0.1", 128, Cv=1.5, T=0.1, steps=1000),
    "lattice256_cv10": Workload("lattice256_cv10", 256, Cv=10.0, T=1.0, steps=200),
    "lattice64_cv10": Workload("lattice64_cv10", 64, Cv=10.0, T=1.0, steps=50),
}


def lattice_state(n_side: int, spacing: float = 1.0, jitter: float = 0.05, m: float = 1.0,
                  kB: float = 1.0, T: float = 1.0, Cv: float = 10.0, seed: int = 0):
    """Returns q (3, N), p (3, N), eps (N,), id (N,) as numpy arrays."""
    n = n_side ** 3
    rng = np.random.default_rng(seed)
    k = np.arange(n)
    site = np.stack([k % n_side, (k // n_side) % n_side, k // (n_side * n_side)]).astype(np.float64)
    q = (site + 0.5) * spacing + rng.uniform(-jitter, jitter, size=(3, n))
    L = n_side * spacing
    q = np.where(q >= L, q - L, np.where(q < 0.0, q + L, q))
    p = rng.normal(0.0, np.sqrt(m * kB * T), size=(3, n))
    p -= p.mean(axis=1, keepdims=True)
    eps = np.full(n, Cv * T)
    ids = k.astype(np.uint32)
    return np.ascontiguousarray(q), np.ascontiguousarray(p), eps, ids


def workload_state(w: Workload):
    return lattice_state(w.n_side, w.spacing, w.jitter, w.m, w.kB, w.T, w.Cv, w.init_seed)


def shuffled(q, p, eps, ids, seed: int = 1):
    """The same particles in a random storage order (for order-independence checks)."""
    perm = np.random.default_rng(seed).permutation(eps.shape[0])
    return (np.ascontiguousarray(q[:, perm]), np.ascontiguousarray(p[:, perm]),
            eps[perm].copy(), ids[perm].copy())
