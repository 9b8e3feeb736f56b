"""Pins of the oracle's cells, density, forces, pair schedule and
Velocity-Verlet against brute force, -grad H and symmetry (Sec. 2-3.1)."""
import numpy as np
import pytest

import oracle as O
from paper_1707_04232_amd.workload import lattice_state, shuffled


def small(n_side=10, jitter=0.05, Cv=10.0, T=1.0, seed=0, **kw):
    q, p, eps, ids = lattice_state(n_side, jitter=jitter, Cv=Cv, T=T, seed=seed)
    P = O.OracleParams(n=n_side**3, box=float(n_side), Cv=Cv, **kw)
    return P, O.State.from_arrays(q, p, eps, ids)


def lattice_sum_numpy(kernel_fn, h):
    """sum over all lattice vectors n in Z^3 with |n| < h of kernel_fn(|n|)."""
    k = int(np.ceil(h))
    g = np.arange(-k, k + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    r = np.sqrt(X**2 + Y**2 + Z**2).ravel()
    r = r[r < h]
    return sum(kernel_fn(x) for x in r), len(r)


@pytest.mark.parametrize("kernel,expected", [(O.KERNEL_LUCY, 1.0006029911),
                                             (O.KERNEL_CUBIC, 0.9985173935)])
def test_perfect_lattice_density(kernel, expected):
    # eq. (sdpd-rho-v) including j = i (A3): on a perfect unit lattice every
    # particle sees the same 81 sites (shells |n|^2 = 0..6)
    s, cnt = lattice_sum_numpy(lambda r: O.kernel_w(kernel, 2.5, r), 2.5)
    assert cnt == 81
    assert s == pytest.approx(expected, abs=1e-9)
    P, S = small(jitter=0.0, kernel=kernel)
    O.build_cells(P, S)
    rho = O.density(P, S)
    assert np.abs(rho - s).max() < 1e-13


@pytest.mark.parametrize("kernel", [O.KERNEL_LUCY, O.KERNEL_CUBIC])
def test_density_cells_equal_bruteforce(kernel):
    P, S = small(n_side=10, jitter=0.4, kernel=kernel)
    q0 = S.q.copy()
    O.build_cells(P, S)
    rho_c = O.density(P, S)
    rho_b = O.density_bruteforce(P, S.q)
    assert np.abs(rho_c - rho_b).max() < 1e-14
    # the numpy brute force over the unsorted input agrees, matched by id
    d = q0[:, :, None] - q0[:, None, :]
    d -= 10.0 * np.round(d / 10.0)
    r = np.sqrt((d**2).sum(0))
    W = np.vectorize(lambda x: O.kernel_w(kernel, 2.5, x))(np.where(r < 2.5, r, 2.5))
    rho_np = W.sum(1)
    assert np.abs(rho_np[S.id] - rho_c).max() < 1e-13


def test_build_cells_sorted_and_order_independent():
    P, S = small(n_side=12, jitter=0.45)
    q, p, eps, ids = shuffled(S.q, S.p, S.eps, S.id, seed=3)
    S2 = O.State.from_arrays(q, p, eps, ids)
    O.build_cells(P, S)
    O.build_cells(P, S2)
    assert np.array_equal(S.id, S2.id) and np.array_equal(S.q, S2.q)
    assert np.array_equal(S.cell_start, S2.cell_start)
    nc = O.grid(P)
    assert nc == (4, 4, 4)
    cs = S.cell_start.astype(np.int64)
    for c in range(len(cs) - 1):
        sl = slice(cs[c], cs[c + 1])
        assert np.all(np.diff(S.id[sl].astype(np.int64)) > 0)
        cx = np.floor(S.q[0, sl] * (nc[0] / 12.0)).astype(int)
        cy = np.floor(S.q[1, sl] * (nc[1] / 12.0)).astype(int)
        cz = np.floor(S.q[2, sl] * (nc[2] / 12.0)).astype(int)
        assert np.all(cx + nc[0] * (cy + nc[1] * cz) == c)


def test_grid_rules():
    assert O.grid(O.OracleParams(n=1, box=128.0)) == (50, 50, 50)
    assert O.grid(O.OracleParams(n=1, box=10.0)) == (4, 4, 4)
    assert O.grid(O.OracleParams(n=1, box=256.0)) == (102, 102, 102)
    with pytest.raises(O.OracleError):
        O.grid(O.OracleParams(n=1, box=9.0))          # fewer than 4 cells
    with pytest.raises(O.OracleError):
        O.grid(O.OracleParams(n=1, box=10.0, ncell=(6, 4, 4)))   # cell < h


def test_cell_cap_overflow_is_reported():
    P, S = small(n_side=10, cell_cap=8)
    with pytest.raises(O.OracleError) as e:
        O.build_cells(P, S)
    assert e.value.rc == O.ECELLCAP


def _hamiltonian_terms(P, q, S_ent):
    rho = O.density_bruteforce(P, q)
    return np.array([O.eps_at_entropy(P, s, r) for s, r in zip(S_ent, rho)])


@pytest.mark.parametrize("kernel", [O.KERNEL_LUCY, O.KERNEL_CUBIC])
def test_force_is_minus_grad_H(kernel):
    # Sec. 3.1: dp_i = -grad_{q_i} H(q, p, S) = sum_j F_cons,ij with
    # H_pot = sum_i E(S_i, rho_i(q)); pins eq. (cons-forces) against the
    # density code and the closure by central differences
    P, S = small(n_side=10, jitter=0.3, kernel=kernel, Cv=1.5, T=0.1)
    O.prepare(P, S)
    S_ent = np.array([O.entropy(P, e, r) for e, r in zip(S.eps, S.rho)])
    f_b = O.forces_bruteforce(P, S.q, S.rho, S.eps)
    assert np.abs(f_b - S.f).max() < 1e-14
    rng = np.random.default_rng(1)
    d = 1e-6
    for _ in range(10):
        c, i = rng.integers(3), rng.integers(P.n)
        qp, qm = S.q.copy(), S.q.copy()
        qp[c, i] += d
        qm[c, i] -= d
        dH = (_hamiltonian_terms(P, qp, S_ent) - _hamiltonian_terms(P, qm, S_ent)).sum()
        assert -dH / (2 * d) == pytest.approx(S.f[c, i], abs=2e-7 * max(1.0, abs(S.f[c, i])))


def test_force_sums_to_zero_and_vanishes_on_lattice():
    P, S = small(n_side=10, jitter=0.3)
    O.prepare(P, S)
    assert np.abs(S.f.sum(axis=1)).max() < 1e-13
    P, S = small(n_side=10, jitter=0.0)
    O.prepare(P, S)
    assert np.abs(S.f).max() < 1e-14


def _by_id(S):
    o = np.argsort(S.id)
    return S.q[:, o], S.p[:, o], S.eps[o]


def test_velocity_verlet_is_reversible():
    # eq. (sdpd-verlet) with the F/D part off: forward K steps, flip momenta,
    # K steps, flip again returns to the start (up to rounding)
    P, S = small(n_side=10, jitter=0.05, fd_mode=O.FD_NONE)
    O.prepare(P, S)
    q0, p0, e0 = _by_id(S)
    rc, _ = O.step(P, S, 0, 20)
    assert rc == 0
    S.p *= -1
    S.f[:] = O.forces(P, S)
    rc, _ = O.step(P, S, 20, 20)
    assert rc == 0
    S.p *= -1
    q1, p1, e1 = _by_id(S)
    dq = q1 - q0
    dq -= 10.0 * np.round(dq / 10.0)
    assert np.abs(dq).max() < 1e-11
    assert np.abs(p1 - p0).max() < 1e-11
    assert np.abs(e1 - e0).max() < 1e-11


def test_velocity_verlet_energy_error_scales_as_dt_squared():
    errs = []
    for dt in (0.01, 0.005):
        P, S = small(n_side=10, jitter=0.05, fd_mode=O.FD_NONE, dt=dt)
        O.prepare(P, S)
        rc, st = O.step(P, S, 0, int(round(0.4 / dt)))
        E = np.array([s["E"] for s in st])
        errs.append(np.abs(E - E[0]).max())
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.5


def test_pair_schedule_is_exact_cover_by_matchings():
    # every pair with r < h appears once; each (phase, round) class is a
    # matching; keys ascend (reading A12)
    P, S = small(n_side=10, jitter=0.45)
    O.build_cells(P, S)
    pl = O.fd_pair_list(P, S)
    d = S.q[:, :, None] - S.q[:, None, :]
    d -= 10.0 * np.round(d / 10.0)
    r2 = (d**2).sum(0)
    iu, ju = np.nonzero(np.triu(r2 < 6.25, k=1))
    brute = set(zip(iu.tolist(), ju.tolist()))
    mine = [(min(a, b), max(a, b)) for a, b in zip(pl["i"].tolist(), pl["j"].tolist())]
    assert len(mine) == len(set(mine)) == len(brute)
    assert set(mine) == brute
    key = pl["phase"].astype(np.int64) * 64 + pl["round"]
    assert np.all(np.diff(key) >= 0)
    assert pl["phase"].min() >= 0 and pl["phase"].max() <= 104 and pl["round"].max() < 64
    for k in np.unique(key):
        sel = key == k
        parts = np.concatenate([pl["i"][sel], pl["j"][sel]])
        assert len(np.unique(parts)) == len(parts)
    # phase 0 holds exactly the pairs that share a cell
    cs = S.cell_start.astype(np.int64)
    cell = np.searchsorted(cs, np.arange(P.n), side="right") - 1
    same = cell[pl["i"]] == cell[pl["j"]]
    assert np.array_equal(same, pl["phase"] == 0)
