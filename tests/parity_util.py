"""Comparison protocol of the GPU parity tests (test infrastructure).

Every decision of the Metropolized F/D sweep compares two FP64 numbers: the
log ratio a of eq. (metropolis-ratio) with ln U (Sec. 3.3.2, step 4), and
min(eps_i, eps_j) with the energy change Delta of eq. (energy-bound).  The
GPU and the oracle compute them with different rounding, so a decision whose
two numbers lie within the rounding margin (|a - ln U| <= 1e-9, or the bound
within 1e-12 relative; reading A16) may go either way on the two sides.  When
either side reports such a decision the states are still compared element by
element:

  * seeds: the pairs of the oracle's sweep log whose tests lie within a
    window wider than the GPU's margin (the GPU's marginal pairs are among
    them, since the two sides' values differ by rounding only);
  * re-sync: with at most MAX_FLIP_SEEDS seeds, the oracle sweep is re-run
    with every combination of inverted outcomes of the seeds' tests (a test
    control of the oracle, so_fd_sweep_flip); one combination must then
    match the GPU in every particle and every counter;
  * taint (more seeds than that): in sweep order, a pair is tainted when it
    is a seed or touches a tainted particle, and then both of its particles
    are tainted (pairs of one (phase, round) class are disjoint, so a class
    is processed at once); every untainted particle must agree element by
    element, at least `min_left` of them must remain, and the rejection
    counters may differ by at most the number of tainted pairs.  In a full
    step the forces and the second half kick read the energies of the
    tainted particles, so momenta and forces may differ on the tainted
    particles and on every particle sharing an active pair with one.

`oracle_step_logged` is one step of the oracle's `so_step`, composed from its
exported stages in the same order (a CPU test pins it to `so_step` bit for
bit), that also returns the sweep's pair log and takes the test inversions.
"""
import itertools

import numpy as np

import oracle as O

RATIO_WINDOW = 2e-9        # |a - ln U| of a seed (the GPU's margin is 1e-9)
BOUND_WINDOW = 2e-12       # |min eps - Delta| of a seed, relative to the largest energy
MAX_FLIP_SEEDS = 3         # up to 4^3 oracle re-runs; beyond, the taint rule


def oracle_step_logged(P, R, step, flip=()):
    """One step of order B on the oracle state R (in place), stage by stage
    as so_step runs them.  Returns (rc, stats, sweep log or None)."""
    theta = max(int(P.fd_every), 1)
    O.kick(P, R, 0.5 * P.dt)
    O.drift(P, R, P.dt)
    O.build_cells(P, R)
    rho_new = O.density(P, R)
    O.update_eps_const_entropy(P, R.eps, R.rho, rho_new)
    R.rho[:] = rho_new
    rc, log = 0, None
    st = {"proposed": 0, "rej_energy": 0, "rej_ratio": 0, "marginal": 0, "negeps": 0}
    if step % theta == 0 and P.fd_mode != O.FD_NONE:
        rc, sw, log = O.fd_sweep(P, R, step, log=True, flip=flip)
        st.update({k: sw[k] for k in st})
    R.f[:] = O.forces(P, R)
    O.kick(P, R, 0.5 * P.dt)
    obs = O.observe(P, R)
    st.update({k: obs[k] for k in ("E", "Eint", "KE", "P", "min_eps")})
    return rc, st, log


def seeds(log, fd_mode, eps_scale):
    """Pairs of the log whose decision lies within the (widened) margin."""
    if fd_mode in (O.FD_SSA, O.FD_NONE) or log is None or len(log) == 0:
        return np.zeros(0 if log is None else len(log), bool)
    s = np.abs(log["bound_gap"]) <= BOUND_WINDOW * eps_scale
    if fd_mode == O.FD_EMS:   # the ratio was evaluated unless the bound rejected
        s |= (log["decision"] != 1) & (np.abs(log["a_minus_lnU"]) <= RATIO_WINDOW)
    return s


def seed_choices(log, fd_mode, eps_scale):
    """For each seed pair, its position and the test inversions to try: 0
    (none), the bound (1) when the bound lies in its window, the Metropolis
    test (2) when the ratio lies in its window, and both (3) when both do."""
    out = []
    if fd_mode in (O.FD_SSA, O.FD_NONE) or log is None:
        return out
    for k in np.flatnonzero(seeds(log, fd_mode, eps_scale)):
        b = abs(log["bound_gap"][k]) <= BOUND_WINDOW * eps_scale
        r = fd_mode == O.FD_EMS and log["decision"][k] != 1 and \
            abs(log["a_minus_lnU"][k]) <= RATIO_WINDOW
        kinds = [0] + ([1] if b else []) + ([2] if r else []) + ([3] if b and r else [])
        if b and fd_mode == O.FD_EMS and log["decision"][k] == 1:
            kinds += [3]   # an inverted bound rejection goes on to the ratio
        out.append((int(k), sorted(set(kinds))))
    return out


def flip_combinations(choices):
    """Every assignment of one inversion per seed, the no-inversion one first
    skipped (the caller has tried it)."""
    pos = [k for k, _ in choices]
    for combo in itertools.product(*[kinds for _, kinds in choices]):
        flip = {p: c for p, c in zip(pos, combo) if c}
        if flip:
            yield flip


def taint(log, n, seed_mask, pre=None):
    """Propagate the taint through the sweep in its order.  Returns (particle
    mask, number of tainted pairs)."""
    t = np.zeros(n, bool) if pre is None else pre.copy()
    if log is None or len(log) == 0:
        return t, 0
    i = log["i"].astype(np.int64)
    j = log["j"].astype(np.int64)
    key = log["phase"].astype(np.int64) * 4096 + log["round"].astype(np.int64)
    first = np.flatnonzero(seed_mask)
    start = int(first[0]) if first.size else len(log)
    if t.any():
        start = 0
    if start == len(log):
        return t, 0
    bounds = np.flatnonzero(np.diff(key)) + 1
    edges = np.concatenate([[0], bounds, [len(log)]])
    npairs = 0
    for a, b in zip(edges[:-1], edges[1:]):
        if b <= start:
            continue
        ii, jj = i[a:b], j[a:b]
        hit = seed_mask[a:b] | t[ii] | t[jj]
        if hit.any():
            npairs += int(hit.sum())
            t[ii[hit]] = True
            t[jj[hit]] = True
    return t, npairs


def neighbours(log, mask):
    """mask plus every particle sharing a logged (active) pair with it."""
    out = mask.copy()
    if log is None or len(log) == 0 or not mask.any():
        return out
    i = log["i"].astype(np.int64)
    j = log["j"].astype(np.int64)
    m = mask[i] | mask[j]
    out[i[m]] = True
    out[j[m]] = True
    return out


def rel_masked(a, b, keep):
    """max |a - b| over the kept particles, relative to max |b| over all."""
    scale = max(np.abs(b).max(), 1e-300) if b.size else 1.0
    if not keep.any():
        return 0.0
    return np.abs(a[..., keep] - b[..., keep]).max() / scale


def _state_error(g, R, keys, keep=None):
    n = len(R.eps)
    keep = np.ones(n, bool) if keep is None else keep
    return {k: rel_masked(g[k], getattr(R, k), keep) for k in keys}


def _counters(st):
    return (st["proposed"], st["rej_energy"], st["rej_ratio"])


def sweep_and_compare(P, R0, step, g, gst, tol, say, dt_fd=None, keys=("p", "eps"),
                      min_left=0.5):
    """Run the oracle's F/D sweep from R0 (not modified) and compare the
    GPU's state g and counters gst with it (protocol above).  Returns the
    oracle state the GPU was matched with and the oracle's stats."""
    n = len(R0.eps)
    R = R0.copy()
    rc, ost, log = O.fd_sweep(P, R, step, dt_fd, log=True)
    assert rc == 0 or P.fd_mode == O.FD_SSA
    assert np.array_equal(g["id"], R.id), "particle order differs"
    assert gst["proposed"] == ost["proposed"]
    say(f"marginal decisions: gpu {gst['marginal']}, oracle {ost['marginal']}")
    if gst["marginal"] + ost["marginal"] == 0:
        assert _counters(gst) == _counters(ost)
        for k, e in _state_error(g, R, keys).items():
            assert e <= tol, f"{k}: relative error {e:.3e} > {tol:.0e}"
        return R, ost
    eps_scale = float(np.abs(R0.eps).max())
    choices = seed_choices(log, P.fd_mode, eps_scale)
    assert choices, "a side reports a marginal decision but no pair lies in the window"
    if len(choices) <= MAX_FLIP_SEEDS:
        tried = [(None, R, ost)]
        for flip in flip_combinations(choices):
            Rf = R0.copy()
            rc, stf, _ = O.fd_sweep(P, Rf, step, dt_fd, flip=flip)
            tried.append((flip, Rf, stf))
        for flip, Rf, stf in tried:
            err = _state_error(g, Rf, keys)
            if max(err.values()) <= tol and _counters(gst) == _counters(stf):
                say(f"re-synced: {len(choices)} seed pairs, oracle outcomes inverted {flip}")
                return Rf, stf
        raise AssertionError(f"no inversion of the {len(choices)} seed pairs matches the GPU")
    t, npairs = taint(log, n, seeds(log, P.fd_mode, eps_scale))
    keep = ~t
    say(f"taint: {len(choices)} seed pairs, {npairs} tainted pairs, "
        f"{int(t.sum())} of {n} particles excluded")
    d = abs(gst["rej_energy"] + gst["rej_ratio"] - ost["rej_energy"] - ost["rej_ratio"])
    assert d <= npairs
    assert keep.mean() >= min_left, f"only {keep.mean():.2%} of the particles left to compare"
    for k, e in _state_error(g, R, keys, keep).items():
        assert e <= tol, f"{k}: relative error {e:.3e} > {tol:.0e}"
    return R, ost


def _sweep_eps_scale(P, R0):
    """Largest energy entering the sweep of a step from R0 (after the
    constant-entropy update): the scale of the bound window."""
    Rd = R0.copy()
    O.kick(P, Rd, 0.5 * P.dt)
    O.drift(P, Rd, P.dt)
    O.build_cells(P, Rd)
    rho_new = O.density(P, Rd)
    O.update_eps_const_entropy(P, Rd.eps, Rd.rho, rho_new)
    return float(np.abs(Rd.eps).max())


def step_and_compare(P, R0, step, g, gst, tol, say, min_left=0.5, ost=None, R=None):
    """Run one oracle step from R0 (not modified; so_step's result R and
    stats ost may be passed in) and compare the GPU's state g and per-step
    stats gst with it.  gst["marginal"] = None means the GPU's count is not
    known (a replayed batch): then the protocol runs whenever the oracle's
    log holds a seed.  Returns (oracle state, stats, resync) where resync says
    the GPU state must be replaced by the oracle's before going on."""
    n = len(R0.eps)
    log = None
    if R is None or gst["marginal"] is None:
        R = R0.copy()
        rc, ost, log = oracle_step_logged(P, R, step)
        assert rc == 0
    assert np.array_equal(g["id"], R.id), "particle order differs"
    assert gst["proposed"] == ost["proposed"]
    for k, e in _state_error(g, R, ("q", "rho")).items():
        assert e <= tol, f"{k}: relative error {e:.3e} > {tol:.0e}"
    if gst["marginal"] is None:
        gst = dict(gst, marginal=int(seeds(log, P.fd_mode, _sweep_eps_scale(P, R0)).sum()))
    say(f"step {step}: marginal decisions: gpu {gst['marginal']}, oracle {ost['marginal']}")
    if gst["marginal"] + ost["marginal"] == 0:
        assert _counters(gst) == _counters(ost)
        assert abs(gst["E"] - ost["E"]) <= tol * abs(ost["E"])
        for k, e in _state_error(g, R, ("p", "eps", "f")).items():
            assert e <= tol, f"{k}: relative error {e:.3e} > {tol:.0e}"
        return R, ost, False
    if log is None:
        R = R0.copy()
        rc, ost, log = oracle_step_logged(P, R, step)
        assert rc == 0
    eps_scale = _sweep_eps_scale(P, R0)
    choices = seed_choices(log, P.fd_mode, eps_scale)
    assert choices, "a side reports a marginal decision but no pair lies in the window"
    if len(choices) <= MAX_FLIP_SEEDS:
        tried = [(None, R, ost)]
        for flip in flip_combinations(choices):
            Rf = R0.copy()
            rc, stf, _ = oracle_step_logged(P, Rf, step, flip=flip)
            tried.append((flip, Rf, stf))
        for flip, Rf, stf in tried:
            err = _state_error(g, Rf, ("p", "eps", "f"))
            if max(err.values()) <= tol and _counters(gst) == _counters(stf) and \
                    abs(gst["E"] - stf["E"]) <= tol * abs(stf["E"]):
                say(f"re-synced: {len(choices)} seed pairs, oracle outcomes inverted {flip}")
                return Rf, stf, False
        raise AssertionError(f"no inversion of the {len(choices)} seed pairs matches the GPU")
    t, npairs = taint(log, n, seeds(log, P.fd_mode, eps_scale))
    tp = neighbours(log, t)
    say(f"taint: {len(choices)} seed pairs, {npairs} tainted pairs, {int(t.sum())} energies "
        f"and {int(tp.sum())} momenta/forces of {n} excluded")
    d = abs(gst["rej_energy"] + gst["rej_ratio"] - ost["rej_energy"] - ost["rej_ratio"])
    assert d <= npairs
    assert (~tp).mean() >= min_left, f"only {(~tp).mean():.2%} of the particles left"
    for k, e in _state_error(g, R, ("eps",), ~t).items():
        assert e <= tol, f"{k}: relative error {e:.3e} > {tol:.0e}"
    for k, e in _state_error(g, R, ("p", "f"), ~tp).items():
        assert e <= tol, f"{k}: relative error {e:.3e} > {tol:.0e}"
    return R, ost, True


def load_state(S, R):
    """Copy the oracle state R into the device state S (a re-sync)."""
    import torch
    for k in ("q", "p", "eps", "rho", "f"):
        getattr(S, k).copy_(torch.as_tensor(np.ascontiguousarray(getattr(R, k))))
    S.id.copy_(torch.as_tensor(R.id.astype(np.int32)))
    torch.cuda.synchronize()


def stepwise_trajectory(ctx, S, op, R, step0, nsteps, tol, say):
    """Step both sides one step at a time from equal states, comparing after
    every step; the GPU state is replaced by the oracle's after a step that
    needed the taint rule.  Returns the oracle state and the number of
    re-synced steps."""
    resyncs = 0
    for k in range(step0, step0 + nsteps):
        gst = ctx.step(S, k, 1)[0]
        R, _, resync = step_and_compare(op, R, k, S.to_numpy(), gst, tol, say)
        if resync:
            load_state(S, R)
            resyncs += 1
    return R, resyncs
