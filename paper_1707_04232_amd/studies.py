"""Scheme studies of Sec. 4 redone on the GPU path, in reduced units.

    python -m paper_1707_04232_amd.studies [--out FILE]

* F/D only (positions fixed, Sec. 4.1): for EMS and AMS and a range of time
  steps, the relative L2 distance of eq. (error-dist) between the histogram
  of the internal energies (150 bins on [0.1, 20] k_B T) and the Gamma law
  of eq. (dist-analytic) at the temperature fixed by the total energy, and
  the rejection rate with its log-log slope against dt.
* Full steps with multiple time steps (Sec. 4.2): the F/D sweep every theta
  steps with theta dt, theta = 1, 5, 10: throughput and energy drift.

Prints one JSON object per measurement.
"""
import argparse
import json
import sys
import time

import numpy as np
from scipy import stats

from . import sdpd
from .workload import WORKLOADS, lattice_state, workload_state


def energy_distribution_error(samples, T, Cv, kB=1.0, nbins=150):
    """eq. (error-dist) with the Gamma law of eq. (dist-analytic)."""
    lo, hi = 0.1 * kB * T, 20.0 * kB * T
    hist, edges = np.histogram(samples, bins=nbins, range=(lo, hi))
    width = edges[1] - edges[0]
    dens = hist / (len(samples) * width)
    mid = 0.5 * (edges[1:] + edges[:-1])
    mu = stats.gamma.pdf(mid, a=Cv / kB, scale=kB * T)
    return float(np.sqrt(((dens - mu) ** 2).sum() / (mu ** 2).sum()))


def fd_only(mode, dt, n_side=32, Cv=1.5, T=1.0, sweeps=240, burn=40, every=4, seed=0):
    """F/D sweeps at fixed positions; returns the distribution error, the
    rejection rate and the measured temperature."""
    q, p, eps, ids = lattice_state(n_side, jitter=0.2, Cv=Cv, T=T, seed=seed)
    n = len(eps)
    prm = sdpd.SdpdParams(n=n, box=float(n_side), Cv=Cv, dt=dt, fd=mode)
    S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
    samples, prop, rej = [], 0, 0
    with sdpd.Context(prm) as ctx:
        ctx.prepare(S)
        o = ctx.observe(S)
        # temperature fixed by the total energy: n Cv T + (3/2)(n - 1) kB T = E
        Tt = o["E"] / (n * Cv + 1.5 * (n - 1) * prm.kB)
        for k in range(sweeps):
            st = ctx.fd_metropolis(S, step=k)
            prop += st["proposed"]
            rej += st["rej_energy"] + st["rej_ratio"]
            if k >= burn and (k - burn) % every == 0:
                samples.append(S.eps.cpu().numpy().copy())
    samples = np.concatenate(samples)
    return {"mode": {sdpd.FD_EMS: "EMS", sdpd.FD_AMS: "AMS"}[mode], "dt": dt, "n": n, "Cv": Cv,
            "T_target": Tt, "error_dist": energy_distribution_error(samples, Tt, Cv),
            "mean_eps_over_CvT": float(samples.mean() / (Cv * Tt)),
            "rejection_rate": rej / max(prop, 1), "samples": int(samples.size)}


def mts(theta, workload="lattice64_cv10", steps=400, warmup=10):
    """Full steps with the F/D sweep every theta steps (theta dt)."""
    w = WORKLOADS[workload]
    q, p, eps, ids = workload_state(w)
    prm = sdpd.SdpdParams(n=w.n, box=w.box, Cv=w.Cv, dt=w.dt, fd_every=theta)
    S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
    import torch
    with sdpd.Context(prm) as ctx:
        ctx.prepare(S)
        ctx.step(S, 0, warmup, stats=False)
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.step(S, warmup, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    E = np.array([s["E"] for s in st])
    x = np.arange(len(E), dtype=np.float64) - (len(E) - 1) / 2.0
    slope = float((x * (E - E.mean())).sum() / (x * x).sum())
    prop = sum(s["proposed"] for s in st)
    rej = sum(s["rej_energy"] + s["rej_ratio"] for s in st)
    return {"theta": theta, "workload": workload, "n": w.n, "steps": steps,
            "particle_steps_per_s": w.n * steps / el, "ms_per_step": 1e3 * el / steps,
            "drift_per_1e3_steps_per_particle_kBT": slope * 1e3 / (w.n * w.kB * w.T),
            "rejection_rate": rej / max(prop, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="also write the JSON lines to this file")
    ap.add_argument("--dts", default="0.01,0.05,0.2,1,2,5")
    args = ap.parse_args()
    out = open(args.out, "w") if args.out else None

    def emit(d):
        line = json.dumps(d)
        print(line, flush=True)
        if out:
            out.write(line + "\n")
            out.flush()

    dts = [float(x) for x in args.dts.split(",")]
    rates = {}
    for mode in (sdpd.FD_EMS, sdpd.FD_AMS):
        for dt in dts:
            r = fd_only(mode, dt)
            emit({"study": "fd_only", **r})
            if mode == sdpd.FD_EMS:
                rates[dt] = r["rejection_rate"]
    pts = [(np.log10(d), np.log10(r)) for d, r in rates.items() if r > 0]
    if len(pts) >= 2:
        x, y = np.array(pts).T
        emit({"study": "rejection_scaling", "mode": "EMS",
              "loglog_slope": float(np.polyfit(x, y, 1)[0]),
              "dts": list(rates), "rates": list(rates.values())})
    for theta in (1, 5, 10):
        emit({"study": "mts", **mts(theta)})
    if out:
        out.close()


if __name__ == "__main__":
    sys.exit(main())
