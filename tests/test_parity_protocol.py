"""The comparison protocol of the GPU parity tests, checked on the CPU with the
oracle alone: the stage-by-stage oracle step equals so_step bit for bit, and
the taint rule covers every particle a divergent decision can reach (planted
divergences leave every untainted particle bitwise unchanged, and a rule that
propagates along only one side of a pair would miss some)."""
import numpy as np
import pytest

import oracle as O
import parity_util as PU
from paper_1707_04232_amd.workload import lattice_state


def _state(dims=10, Cv=1.5, T=0.1, **kw):
    q, p, eps, ids = lattice_state(dims, Cv=Cv, T=T)
    box = tuple(float(d) for d in ((dims,) * 3 if np.ndim(dims) == 0 else dims))
    P = O.OracleParams(n=len(eps), box=box, Cv=Cv, **kw)
    R = O.State.from_arrays(q, p, eps, ids)
    O.prepare(P, R)
    return P, R


SEED_HI = 0x1234_5678_9ABC_DEF0


@pytest.mark.parametrize("kw", [dict(), dict(fd_every=2, seed=SEED_HI),
                                dict(fd_mode=O.FD_AMS, kernel=O.KERNEL_CUBIC, replica=5)])
def test_logged_step_equals_so_step(kw):
    P, R = _state(dt=0.05, **kw)
    A = R.copy()
    rc, ref = O.step(P, A, 0, 5)
    assert rc == 0
    for k in range(5):
        rc, st, log = PU.oracle_step_logged(P, R, k)
        assert rc == 0
        for key in ("proposed", "rej_energy", "rej_ratio", "marginal", "E", "KE"):
            assert st[key] == ref[k][key], (k, key)
        swept = k % P.fd_every == 0
        assert (log is not None) == swept
        if swept:
            assert len(log) == st["proposed"]
    for key in ("q", "p", "eps", "rho", "f", "id", "cell_start"):
        assert np.array_equal(getattr(R, key), getattr(A, key)), key


def _planted(P, R, victims, factor=1.3, step=3):
    """Sweep R as it is (reference) and a copy whose victims' energies were
    changed before the sweep (a divergence planted at those particles)."""
    A, B = R.copy(), R.copy()
    B.eps[victims] *= factor
    rc, _, log = O.fd_sweep(P, A, step, log=True)
    assert rc == 0
    rc, _, logb = O.fd_sweep(P, B, step, log=True)
    assert rc == 0
    assert np.array_equal(log[["i", "j", "phase", "round"]], logb[["i", "j", "phase", "round"]])
    return A, B, log


def test_taint_covers_planted_divergence():
    # an elongated box: one sweep carries a divergence across ~10 cells, so
    # the taint of two particles covers part of the box only
    P, R = _state(dims=(12, 12, 60), dt=0.5)
    n = len(R.eps)
    victims = np.array([5, 100])
    A, B, log = _planted(P, R, victims)
    pre = np.zeros(n, bool)
    pre[victims] = True
    t, npairs = PU.taint(log, n, np.zeros(len(log), bool), pre=pre)
    assert t[victims].all() and npairs > 0
    keep = ~t
    assert 0.05 < keep.mean() < 0.999        # the taint spreads, but not everywhere
    for k in ("p", "eps"):
        assert np.array_equal(getattr(A, k)[..., keep], getattr(B, k)[..., keep]), k
    diff = (np.abs(A.p - B.p).max(axis=0) > 0) | (A.eps != B.eps)
    assert diff[t].any()
    # a rule that lets only the second particle of a pair taint the first
    # misses particles the divergence reached
    half = pre.copy()
    for rec in log:
        if half[rec["j"]]:
            half[rec["i"]] = True
    assert (diff & ~half).any()
    # forces read the energies: differences stay within the pair neighbourhood
    A.f[:] = O.forces(P, A)
    B.f[:] = O.forces(P, B)
    nb = PU.neighbours(log, t)
    fdiff = np.abs(A.f - B.f).max(axis=0) > 0
    assert not (fdiff & ~nb).any()
    assert (nb & ~t).any()


def test_seed_windows():
    log = np.zeros(6, O.PAIRREC_DTYPE)
    log["decision"] = [0, 2, 1, 0, 0, 1]
    log["a_minus_lnU"] = [1e-9, -1.5e-9, 0.0, 0.3, -3e-9, 0.0]
    log["bound_gap"] = [0.1, 0.1, 0.1, 0.1, 0.1, 2e-13]
    s = PU.seeds(log, O.FD_EMS, eps_scale=0.15)
    # ratio window 2e-9; an energy-bound rejection has no ratio; bound window
    # 2e-12 of the largest energy
    assert s.tolist() == [True, True, False, False, False, True]
    s = PU.seeds(log, O.FD_AMS, eps_scale=0.15)
    assert s.tolist() == [False] * 5 + [True]
    assert not PU.seeds(log, O.FD_SSA, eps_scale=0.15).any()


def _closest_ratio_pair(log, lo=0.0):
    """Position of the ratio decision closest to its threshold among the
    last (1 - lo) of the sweep."""
    amlu = np.where(log["decision"] != 1, np.abs(log["a_minus_lnU"]), np.inf)
    amlu[: int(lo * len(log))] = np.inf
    return int(np.argmin(amlu))


def _as_gpu(R, st, marginal):
    g = {k: getattr(R, k).copy() for k in ("q", "p", "eps", "rho", "f", "id")}
    return g, dict(st, marginal=marginal)


def test_sweep_resync_by_inverted_outcome(monkeypatch):
    """A planted "other side" that decided one pair the other way: with that
    pair in the window the protocol finds the inversion and compares every
    particle; an other side that differs at a pair outside the window fails."""
    P, R = _state(dims=(12, 12, 60), dt=0.5)
    A = R.copy()
    rc, ost, log = O.fd_sweep(P, A, 3, log=True)
    assert rc == 0
    k = _closest_ratio_pair(log)
    monkeypatch.setattr(PU, "RATIO_WINDOW", abs(log["a_minus_lnU"][k]) * 1.0001)
    monkeypatch.setattr(PU, "BOUND_WINDOW", 0.0)
    assert PU.seeds(log, O.FD_EMS, 1.0).sum() == 1
    say = lambda *a: None
    B = R.copy()
    rc, stb, logb = O.fd_sweep(P, B, 3, flip={k: 2}, log=True)
    assert rc == 0
    assert (log["decision"][k] == 0) == (logb["decision"][k] == 2)   # that pair inverted
    assert np.array_equal(log["decision"][:k], logb["decision"][:k])
    assert not np.array_equal(A.p, B.p)
    g, gst = _as_gpu(B, stb, 1)
    Rm, stm = PU.sweep_and_compare(P, R, 3, g, gst, 1e-10, say)
    assert np.array_equal(Rm.p, B.p) and stm["rej_ratio"] == stb["rej_ratio"]
    # the outcome inverted at a pair outside the window
    m = _closest_ratio_pair(log, lo=0.5) if k < len(log) // 2 else _closest_ratio_pair(log[: len(log) // 2])
    assert m != k
    C = R.copy()
    rc, stc, _ = O.fd_sweep(P, C, 3, flip={m: 2})
    g, gst = _as_gpu(C, stc, 1)
    with pytest.raises(AssertionError):
        PU.sweep_and_compare(P, R, 3, g, gst, 1e-10, say)
    # a marginal count with no pair in the window is refused
    monkeypatch.setattr(PU, "RATIO_WINDOW", 0.0)
    g, gst = _as_gpu(A, ost, 1)
    with pytest.raises(AssertionError):
        PU.sweep_and_compare(P, R, 3, g, gst, 1e-10, say)


def test_sweep_taint_fallback(monkeypatch):
    """With more seeds than the re-sync tries, the taint rule: the planted
    inversion is excused inside the taint, a difference outside it is not."""
    P, R = _state(dims=(12, 12, 60), dt=0.5)
    A = R.copy()
    rc, ost, log = O.fd_sweep(P, A, 3, log=True)
    k = _closest_ratio_pair(log, lo=0.8)
    monkeypatch.setattr(PU, "RATIO_WINDOW", abs(log["a_minus_lnU"][k]) * 1.0001)
    monkeypatch.setattr(PU, "BOUND_WINDOW", 0.0)
    monkeypatch.setattr(PU, "MAX_FLIP_SEEDS", 0)
    sm = PU.seeds(log, O.FD_EMS, 1.0)
    t, _ = PU.taint(log, len(R.eps), sm)
    assert 0.0 < t.mean() < 0.9
    say = lambda *a: None
    B = R.copy()
    rc, stb, _ = O.fd_sweep(P, B, 3, flip={pos: 2 for pos in np.flatnonzero(sm)})
    g, gst = _as_gpu(B, stb, 1)
    PU.sweep_and_compare(P, R, 3, g, gst, 1e-10, say, min_left=0.1)
    other = int(np.flatnonzero(~t)[0])
    g["eps"][other] *= 1.0 + 1e-6
    with pytest.raises(AssertionError):
        PU.sweep_and_compare(P, R, 3, g, gst, 1e-10, say, min_left=0.1)
    g["eps"][other] = B.eps[other]
    with pytest.raises(AssertionError):   # too little left
        PU.sweep_and_compare(P, R, 3, g, gst, 1e-10, say, min_left=1.0)


def test_step_resync_by_inverted_outcome(monkeypatch):
    """The same at the level of a full step (sweep inside order B)."""
    P, R = _state(dims=10, dt=0.5)
    A = R.copy()
    rc, ost, log = PU.oracle_step_logged(P, A, 2)
    k = _closest_ratio_pair(log)
    monkeypatch.setattr(PU, "RATIO_WINDOW", abs(log["a_minus_lnU"][k]) * 1.0001)
    monkeypatch.setattr(PU, "BOUND_WINDOW", 0.0)
    B = R.copy()
    rc, stb, _ = PU.oracle_step_logged(P, B, 2, flip={k: 2})
    g, gst = _as_gpu(B, stb, 1)
    Rm, _, resync = PU.step_and_compare(P, R, 2, g, gst, 1e-10, lambda *a: None)
    assert not resync and np.array_equal(Rm.p, B.p) and np.array_equal(Rm.f, B.f)
    # unknown GPU count (replayed batch): the oracle's seed decides
    g, gst = _as_gpu(B, stb, None)
    Rm, _, resync = PU.step_and_compare(P, R, 2, g, gst, 1e-10, lambda *a: None)
    assert np.array_equal(Rm.p, B.p)


def test_flip_control():
    """Inversion kind 0 is the plain sweep; a non-ascending position list or
    a kind outside 0..3 is refused."""
    import ctypes as C
    P, R = _state(dims=10, dt=0.5)
    A, B = R.copy(), R.copy()
    O.fd_sweep(P, A, 3)
    O.fd_sweep(P, B, 3, flip={5: 0, 9: 0})
    assert np.array_equal(A.p, B.p) and np.array_equal(A.eps, B.eps)
    st = O._Stats()
    for pos, kind in (([9, 5], [1, 1]), ([5, 5], [1, 2]), ([5], [4])):
        fl = np.ascontiguousarray(pos, np.int64)
        kd = np.ascontiguousarray(kind, np.int32)
        D = R.copy()
        rc = O.lib().so_fd_sweep_flip(C.byref(P.c()), O._d(D.q), O._d(D.p), O._d(D.eps),
                                      O._d(D.rho), O._u(D.id), O._u(D.cell_start), 3, P.dt,
                                      C.byref(st), None, 0,
                                      fl.ctypes.data_as(C.POINTER(C.c_int64)),
                                      kd.ctypes.data_as(C.POINTER(C.c_int32)), len(fl))
        assert rc == O.EINVAL
        assert np.array_equal(D.p, R.p)
