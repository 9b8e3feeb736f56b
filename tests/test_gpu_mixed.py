"""Mixed precision (FP32 density and forces from cell-relative positions,
FP32 geometry and proposal coefficients in the F/D update, everything else
FP64) against the FP64 oracle on a 64^3 jittered lattice
with C_v = 10, T = 1 (the small box of the 8M-particle mixed-precision
workload), and against the FP64 GPU path over a short trajectory.

Tolerances follow from the FP32 arithmetic.  A cell-relative coordinate
(|x| < 2.7) is rounded to 2^-23 relative, ~2.4e-7 absolute; a separation
carries ~1e-6 absolute error, a kernel value W(r) an error of at most
max|W'| * 1e-6 ~ 1e-7 plus its own rounding (~1e-7 relative).  Over ~80
partners rho (~1) is off by at most ~1e-5; the test asks for 2e-5 relative.
A force term m^2 (Pi_i + Pi_j) F r carries ~2e-6 relative error, so f is off
by at most 2e-6 times the sum of |terms| (~80 terms): the test bounds the
error by 2e-4 times the largest possible single term."""
import numpy as np
import pytest

import oracle as O
import parity_util as PU
from paper_1707_04232_amd.workload import lattice_state

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def sd():
    from paper_1707_04232_amd import sdpd
    return sdpd


def _setup(dims, prec, Cv=10.0, T=1.0, **kw):
    sdpd = sd()
    q, p, eps, ids = lattice_state(dims, Cv=Cv, T=T)
    box = tuple(float(d) for d in dims)
    g = sdpd.SdpdParams(n=len(eps), box=box, Cv=Cv, prec=prec, **kw)
    S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
    return g, S, (q, p, eps, ids, box)


def test_mixed_density_forces_vs_oracle():
    sdpd = sd()
    dims = (64, 64, 64)
    say("mixed density/forces vs oracle", dims)
    g, S, (q, p, eps, ids, box) = _setup(dims, sdpd.MIXED)
    with sdpd.Context(g) as ctx:
        ctx.prepare(S)
        ctx.sync()
        G = S.to_numpy()
    P = O.OracleParams(n=len(eps), box=box, Cv=10.0)
    R = O.State.from_arrays(q, p, eps, ids)
    O.prepare(P, R)
    assert np.array_equal(G["id"], R.id)
    erho = np.abs(G["rho"] - R.rho).max() / R.rho.max()
    # largest possible |m^2 (Pi_i + Pi_j) F(r) r|: Lucy F(r) r <= cF h 4/27
    A = P.A if P.A is not None else P.Cv / (3 * P.kB)
    pi_max = A * P.kB * R.eps.max() / (P.m * P.Cv * R.rho.min())
    cF = 315.0 / (4 * np.pi * P.h ** 5)
    term_max = P.m ** 2 * 2 * pi_max * cF * P.h * 4.0 / 27.0
    ef = np.abs(G["f"] - R.f).max() / term_max
    say(f"rho rel err {erho:.2e}, f err {ef:.2e} of the largest pair term")
    assert erho <= 2e-5
    assert ef <= 2e-4
    assert np.abs(G["f"].sum(axis=1)).max() < 1e-6 * term_max * len(eps)


MIXED_FD_CASES = [((16, 12, 12), 9), ((10, 10, 10), 10)]


@pytest.mark.parametrize("dims,step", MIXED_FD_CASES, ids=["16x12x12", "10"])
def test_mixed_fd_sweep_vs_oracle(dims, step):
    """The mixed path's F/D sweep computes the geometry and the proposal
    coefficients (alpha, b of eq. (proposal)) in FP32 and everything else in
    FP64, with the Metropolis ratio of eq. (metropolis-ratio) evaluated for
    exactly those coefficients; the oracle is FP64 throughout.

    Pair set: on a lattice with jitter 0.01 every pair distance is at least
    0.016 away from h (the sixth neighbour shell lies at sqrt(6) = 2.449,
    the seventh at 2.83), far beyond the ~1e-6 FP32 error of r, so both sides
    hold the same pairs; the oracle is given the GPU's densities.

    Decisions: the FP32 coefficients carry a few ulp (~3e-7) of relative
    error, which moves log-ratio a (a sum of O(1) terms) by ~1e-6 and the
    energy bound by ~1e-7 of the energies.  The cases (box, step) are chosen
    so that no decision of the oracle lies within 2e-5 of its boundary
    (checked below on the oracle's log), so every decision must agree.

    State: a pair update moves v by (alpha - 1) v + b G; the FP32 error of
    the coefficients puts ~3e-7 of that on it.  A particle takes part in
    ~65 pairs, so p is off by at most ~2e-5 of the momentum scale and eps
    by less; the test asks 2e-5 of the largest value for both."""
    sdpd = sd()
    say("mixed F/D sweep vs oracle", dims, "step", step)
    q, p, eps, ids = lattice_state(dims, Cv=1.5, T=0.1, jitter=0.01)
    box = tuple(float(d) for d in dims)
    g = sdpd.SdpdParams(n=len(eps), box=box, Cv=1.5, prec=sdpd.MIXED, dt=0.05)
    S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
    with sdpd.Context(g) as ctx:
        ctx.prepare(S)
        rho_gpu = S.rho.cpu().numpy().copy()
        st = ctx.fd_metropolis(S, step=step)
        G = S.to_numpy()
    P = O.OracleParams(n=len(eps), box=box, Cv=1.5, dt=0.05)
    R = O.State.from_arrays(q, p, eps, ids)
    O.prepare(P, R)
    assert np.array_equal(G["id"], R.id)
    # the pair set is fixed far from the cutoff
    log = O.fd_pair_list(P, R)
    x = R.q[:, log["i"]] - R.q[:, log["j"]]
    L = np.array(box)[:, None]
    x -= L * np.rint(x / L)
    r = np.sqrt((x * x).sum(axis=0))
    assert r.max() < P.h - 0.01
    say(f"rho: mixed vs FP64 {np.abs(rho_gpu - R.rho).max():.2e}")
    R.rho[:] = rho_gpu
    R0 = R.copy()
    rc, ost, olog = O.fd_sweep(P, R, step, log=True)
    assert rc == 0
    evaluated = olog["decision"] != 1
    margin = np.abs(olog["a_minus_lnU"][evaluated]).min()
    gap = np.abs(olog["bound_gap"]).min() / np.abs(R0.eps).max()
    say(f"closest decision: |a - ln U| {margin:.2e}, energy bound {gap:.2e}")
    assert margin > 2e-5 and gap > 1e-4, "case no longer clear of the decision boundaries"
    for k in ("proposed", "rej_energy", "rej_ratio"):
        assert st[k] == ost[k], (k, st[k], ost[k])
    ep = PU.rel_masked(G["p"], R.p, np.ones(len(eps), bool))
    ee = PU.rel_masked(G["eps"], R.eps, np.ones(len(eps), bool))
    say(f"p rel err {ep:.2e}, eps rel err {ee:.2e}, rejections {st['rej_ratio']}")
    assert ep <= 2e-5 and ee <= 2e-5


def test_mixed_trajectory_vs_oracle():
    """50 steps of the mixed path against the FP64 oracle (16^3, C_v = 10,
    T = 1): per-step energies within the FP32 error of the forces, counters
    within the decisions that FP32 forces can move, and the kinetic
    temperature."""
    sdpd = sd()
    dims = (16, 16, 16)
    say("mixed trajectory vs oracle", dims)
    g, S, (q, p, eps, ids, box) = _setup(dims, sdpd.MIXED, Cv=10.0, T=1.0)
    with sdpd.Context(g) as ctx:
        ctx.prepare(S)
        gst = ctx.step(S, 0, 50)
    P = O.OracleParams(n=len(eps), box=box, Cv=10.0)
    R = O.State.from_arrays(q, p, eps, ids)
    O.prepare(P, R)
    rc, ost = O.step(P, R, 0, 50)
    assert rc == 0
    Eg = np.array([s["E"] for s in gst])
    Eo = np.array([s["E"] for s in ost])
    dE = np.abs(Eg - Eo).max() / np.abs(Eo).max()
    n = len(eps)
    Tg, To = 2 * gst[-1]["KE"] / (3 * n), 2 * ost[-1]["KE"] / (3 * n)
    rg = sum(s["rej_energy"] + s["rej_ratio"] for s in gst)
    ro = sum(s["rej_energy"] + s["rej_ratio"] for s in ost)
    pg = sum(s["proposed"] for s in gst)
    po = sum(s["proposed"] for s in ost)
    say(f"E rel diff {dE:.2e}, T {Tg:.6f} vs {To:.6f}, rejections {rg} vs {ro}, "
        f"pairs {pg} vs {po}")
    assert dE <= 1e-5
    assert abs(Tg - To) <= 1e-3 * To
    assert abs(pg - po) <= 1e-5 * po
    assert abs(rg - ro) <= max(5, 0.05 * ro)


def test_mixed_trajectory_statistics_match_fp64():
    # 100 steps of the 64^3 box: energy drift, kinetic temperature and the
    # rejection rate agree with the FP64 path (which is pinned to the oracle)
    sdpd = sd()
    dims = (32, 32, 32)
    out = {}
    for prec in (sdpd.FP64, sdpd.MIXED):
        say("trajectory", "mixed" if prec else "fp64")
        g, S, _ = _setup(dims, prec, Cv=10.0, T=1.0)
        with sdpd.Context(g) as ctx:
            ctx.prepare(S)
            st = ctx.step(S, 0, 100)
        E = np.array([s["E"] for s in st])
        KE = np.array([s["KE"] for s in st])
        prop = sum(s["proposed"] for s in st)
        rej = sum(s["rej_energy"] + s["rej_ratio"] for s in st)
        out[prec] = (E, KE, rej / prop)
    E64, KE64, r64 = out[sdpd.FP64]
    E32, KE32, r32 = out[sdpd.MIXED]
    n = 32 ** 3
    assert np.abs(E32 - E64).max() <= 1e-4 * np.abs(E64).max()
    T64, T32 = 2 * KE64[-20:].mean() / (3 * n), 2 * KE32[-20:].mean() / (3 * n)
    assert abs(T32 - T64) <= 1e-3 * T64
    assert abs(r32 - r64) <= 0.02 * r64
