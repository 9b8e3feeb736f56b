"""The oracle's parallel step variant (density, energy update and forces per
particle on several threads; the F/D sweep phase by phase over the phase's
disjoint tasks, reading A12) gives the single-threaded so_step bit for bit:
with the plain build on one thread (the task decomposition itself) and with
the OpenMP build on four threads."""
import numpy as np
import pytest

import oracle as O
from paper_1707_04232_amd.workload import lattice_state, shuffled, uniform_state

CASES = {
    "ems_cv1.5": (lambda: lattice_state(14, Cv=1.5, T=0.1), 14.0,
                  dict(Cv=1.5, dt=0.05)),
    "ems_theta2_seedhi_rep3": (lambda: lattice_state(12, Cv=10.0, T=1.0), 12.0,
                               dict(Cv=10.0, dt=0.5, fd_every=2, seed=0x123456789ABCDEF0,
                                    replica=3)),
    "ams_cubic_ragged": (lambda: shuffled(*uniform_state(2500, (12.0, 14.0, 16.0), T=0.5,
                                                        Cv=3.0, seed=4)),
                         (12.0, 14.0, 16.0), dict(Cv=3.0, dt=0.2, fd_mode=O.FD_AMS,
                                                  kernel=O.KERNEL_CUBIC, zeta=0.4)),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("omp", [False, True])
def test_parallel_step_equals_serial(name, omp):
    make, box, kw = CASES[name]
    q, p, eps, ids = make()
    P = O.OracleParams(n=len(eps), box=box, **kw)
    A = O.State.from_arrays(q, p, eps, ids)
    O.prepare(P, A)
    B = A.copy()
    rc, sa = O.step(P, A, 0, 5)
    rc2, sb, used = O.step_parallel(P, B, 0, 5, threads=4, omp=omp)
    assert rc == rc2 == 0
    assert used == (4 if omp else 1)
    assert sum(s["proposed"] for s in sa) > 0
    for x, y in zip(sa, sb):
        for k in ("proposed", "rej_energy", "rej_ratio", "marginal", "negeps", "E", "KE"):
            assert x[k] == y[k], k
    for k in ("q", "p", "eps", "rho", "f", "id", "cell_start"):
        assert np.array_equal(getattr(A, k), getattr(B, k)), k
