"""Seeded synthetic inputs: jittered simple-cubic lattices in reduced units.

This module only draws random inputs; it holds none of the method's
arithmetic, so both the GPU path and the oracle may be fed from it.

Recipe (the setup of Sec. 4 of the paper restated in reduced units
m = a = kB = 1):
  * nx * ny * nz particles on the sites (i + 1/2) a of a simple cubic
    lattice, ids in x-fastest lattice order, plus a uniform jitter
    U(-jitter, jitter) per component; box = (nx, ny, nz) a;
  * momenta Maxwell-Boltzmann at temperature T: N(0, m kB T) per component,
    minus the mean so that the total momentum is zero;
  * internal energies eps_i = Cv T (so that T_i = T for the ideal gas).
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    dims: tuple
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
        return int(np.prod(self.dims))

    @property
    def box(self) -> tuple:
        return tuple(float(d * self.spacing) for d in self.dims)


# Synthetic workloads.  The 1M and 8M boxes hold N = 2^20 and 2^23 particles
# on 128 x 128 x 64 and 256 x 256 x 128 lattices.
WORKLOADS = {
    "lattice10_cv10": Workload("lattice10_cv10", (10, 10, 10), Cv=10.0, T=1.0, steps=100),
    "lattice128x128x64_cv1.5_T0.1": Workload("lattice128x128x64_cv1.5_T0.1", (128, 128, 64),
                                             Cv=1.5, T=0.1, steps=1000),
    "lattice256x256x128_cv10": Workload("lattice256x256x128_cv10", (256, 256, 128),
                                        Cv=10.0, T=1.0, steps=200),
    "lattice64_cv10": Workload("lattice64_cv10", (64, 64, 64), Cv=10.0, T=1.0, steps=50),
}


def lattice_state(dims, spacing: float = 1.0, jitter: float = 0.05, m: float = 1.0,
                  kB: float = 1.0, T: float = 1.0, Cv: float = 10.0, seed: int = 0):
    """Returns q (3, N), p (3, N), eps (N,), id (N,) as numpy arrays.
    dims: an int (cube) or (nx, ny, nz)."""
    nx, ny, nz = (dims,) * 3 if np.ndim(dims) == 0 else tuple(dims)
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    k = np.arange(n)
    site = np.stack([k % nx, (k // nx) % ny, k // (nx * ny)]).astype(np.float64)
    q = (site + 0.5) * spacing + rng.uniform(-jitter, jitter, size=(3, n))
    L = np.array([nx, ny, nz], np.float64)[:, None] * spacing
    q = np.where(q >= L, q - L, np.where(q < 0.0, q + L, q))
    p = rng.normal(0.0, np.sqrt(m * kB * T), size=(3, n))
    p -= p.mean(axis=1, keepdims=True)
    eps = np.full(n, Cv * T)
    ids = k.astype(np.uint32)
    return np.ascontiguousarray(q), np.ascontiguousarray(p), eps, ids


def workload_state(w: Workload):
    return lattice_state(w.dims, w.spacing, w.jitter, w.m, w.kB, w.T, w.Cv, w.init_seed)


def uniform_state(n: int, box, T: float = 1.0, Cv: float = 10.0, m: float = 1.0,
                  kB: float = 1.0, seed: int = 0):
    """n particles uniformly at random in a (possibly non-cubic) box."""
    rng = np.random.default_rng(seed)
    L = np.asarray(box, np.float64).reshape(3, 1)
    q = rng.uniform(0.0, 1.0, size=(3, n)) * L
    p = rng.normal(0.0, np.sqrt(m * kB * T), size=(3, n))
    if n:
        p -= p.mean(axis=1, keepdims=True)
    return np.ascontiguousarray(q), np.ascontiguousarray(p), np.full(n, Cv * T), \
        np.arange(n, dtype=np.uint32)


def shuffled(q, p, eps, ids, seed: int = 1):
    """The same particles in a random storage order."""
    perm = np.random.default_rng(seed).permutation(eps.shape[0])
    return (np.ascontiguousarray(q[:, perm]), np.ascontiguousarray(p[:, perm]),
            eps[perm].copy(), ids[perm].copy())


def replica_set(nbox: int = 256, seed: int = 0):
    """A batch of independent boxes of uneven size and state: n_b =
    round(exp(U[ln 2048, ln 65536])^(1/3)) lattice sites per side (13..40),
    T_b ~ U[0.1, 2], C_v,b ~ U[1.5, 50] (k_B = 1), replica index b.  Returns
    a list of (side, T, Cv)."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(np.log(2048.0), np.log(65536.0), nbox)) ** (1.0 / 3.0))
    T = rng.uniform(0.1, 2.0, nbox)
    Cv = rng.uniform(1.5, 50.0, nbox)
    return [(int(s), float(t), float(c)) for s, t, c in zip(sides, T, Cv)]
