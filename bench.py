"""Throughput benchmark: full SDPD steps (Velocity-Verlet with density and
pressure forces + one Metropolized F/D sweep) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line: particle-steps/s over the K timed steps, the energy
drift per 1000 steps, the roofline of the dominant kernel (the F/D phase
kernel, timed with HIP events on the library's stream during the timed
steps) and the oracle's single-core rate on a bounded sample.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "lattice128x128x64_cv1.5_T0.1"

# FP64 VALU peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP64_VALU_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# Algorithmic FP64 work of one EMS pair update, in flops (FMA = 2): 209
# basic operations of the formulas plus 4 log, 1 log1p, 2 expm1, 4 sqrt,
# 9 reciprocals, 1 reciprocal square root and 2 sin/cos(pi t), each weighted
# by the FP64 operations of its gfx950 implementation (46, 63, 38, 16, 9, 10
# and 43 flops): 209 + 564 = 773.
FLOPS_PER_EMS_PAIR = 773.0
# What a pair executes: the bracketed Metropolis test replaces the two
# logarithms and the log1p of the comparison (2 x 46 + 63 = 155 flops) by
# cubic bounds (33 flops), so a pair that the bounds decide executes
# 773 - 155 + 33 = 651 flops and a pair whose logarithms are evaluated
# 773 + 33 = 806.
# 1.1 % of the pairs of this workload's relaxed state reach the evaluated
# comparison (0.06 % in the first steps from the lattice), counted with a
# build of the sweep whose marginal counter counts every evaluation.
FLOPS_PER_PAIR_BRACKETED = 651.0
FLOPS_PER_PAIR_EVALUATED = 806.0
EVALUATED_SHARE = 0.011
FLOPS_PER_PAIR_EXECUTED = (FLOPS_PER_PAIR_BRACKETED * (1.0 - EVALUATED_SHARE)
                           + FLOPS_PER_PAIR_EVALUATED * EVALUATED_SHARE)
# Whole-step floor.  Compulsory HBM bytes per particle-step of the method in
# FP64 (one pass over the state per stage): cells re-sorted every step (keys
# and ids 32 B, gather of q, p, eps, rho, id 136 B), density and energy update
# (q, eps, rho in; rho, eps out: 56 B), F/D sweep (q, rho, eps, p, id in;
# p, eps out: 100 B), kicks, drift and force (236 B).
HBM_BYTES_PER_PARTICLE_STEP = {"cells": 170.0, "density": 56.0, "fd": 100.0,
                               "kick_drift_force": 236.0}
# FP64 flops (FMA = 2) per pair term of the particle passes, with the
# square root at its 16 flops: a density term 12 + 16, a force term 25 + 16,
# a candidate distance test 9 (both passes gather over all 27 cells)
FLOPS_DENSITY_TERM = 28.0
FLOPS_FORCE_TERM = 41.0
FLOPS_CANDIDATE = 9.0
# compulsory HBM bytes of the F/D phase kernel: per staged particle entry its
# list entry (4), p and eps read and written (64), q, rho, id read (36); per
# pair its schedule entry (8)
BYTES_PER_STAGED = 104.0
BYTES_PER_PAIR_ENTRY = 8.0
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "fd_sweep_traffic.json")
FD_SOURCES = ["fd.hip", "fd_math.hpp", "fd_elem.hpp", "tasks.hpp", "schedule.hip",
              "sdpd_internal.hpp", "fastdiv.hpp"]


def fd_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in FD_SOURCES:
        with open(os.path.join(ROOT, "paper_1707_04232_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record():
    """The committed PMC record of the F/D sweep kernel (calibrated
    FETCH_SIZE + WRITE_SIZE bytes of one launch, with the algorithmic bytes of
    the same step), or None when the kernel sources changed since the
    counters were taken."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != fd_source_hash():
        return None
    return rec


def measured_traffic():
    """HBM bytes per F/D sweep launch from the committed record, or None."""
    rec = traffic_record()
    return None if rec is None else rec.get("bytes_per_launch")


def step_floor(w, pairs_per_step, ms_per_step):
    """Floor of the whole step from the two roofs: compulsory HBM bytes at
    8 TB/s and algorithmic FP64 flops at 78.6 TFLOP/s, each as a fraction of
    the measured step time; the larger floor is the one that binds."""
    n = w.n
    nc = [max(4, int(b / w.h) // 2 * 2) for b in w.box]
    cand = 27.0 * n / (nc[0] * nc[1] * nc[2])         # candidates per particle
    act = 2.0 * pairs_per_step / n                     # neighbours within h
    ppp = pairs_per_step / n                           # F/D pairs per particle
    flops = {"fd": ppp * FLOPS_PER_EMS_PAIR,
             "density": act * FLOPS_DENSITY_TERM + cand * FLOPS_CANDIDATE,
             "forces": act * FLOPS_FORCE_TERM + cand * FLOPS_CANDIDATE}
    bytes_ = sum(HBM_BYTES_PER_PARTICLE_STEP.values())
    f_tot = sum(flops.values())
    hbm_ms = n * bytes_ / (HBM_PEAK_GBS * 1e9) * 1e3
    valu_ms = n * f_tot / (FP64_VALU_PEAK_TFLOPS * 1e12) * 1e3
    return {"hbm_bytes_per_particle_step": bytes_,
            "hbm_bytes_by_stage": HBM_BYTES_PER_PARTICLE_STEP,
            "fp64_flops_per_particle_step": f_tot,
            "fp64_flops_by_stage": flops,
            "candidates_per_particle": cand, "neighbours_per_particle": act,
            "hbm_floor_ms": hbm_ms, "valu_floor_ms": valu_ms,
            "hbm_frac": hbm_ms / ms_per_step, "valu_frac": valu_ms / ms_per_step,
            "binds": "valu" if valu_ms >= hbm_ms else "hbm",
            "t_floor_ms": max(hbm_ms, valu_ms),
            "frac": max(hbm_ms, valu_ms) / ms_per_step}


def linear_slope(y):
    x = np.arange(len(y), dtype=np.float64)
    x -= x.mean()
    return float((x * (y - y.mean())).sum() / (x * x).sum())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(w, sample_dims=(64, 64, 64), nsteps=2, par_steps=3):
    """The oracle as it stands, on the host of the GPU: its parallel step
    variant (OpenMP, bit for bit the serial result) on the host's threads over
    par_steps full steps of the workload itself, its single-threaded step on
    nsteps steps of a sub-lattice of sample_dims (same density, heat
    capacity, temperature, time step), and the small 10^3 case in full
    (100 steps, one thread)."""
    import oracle as O
    from paper_1707_04232_amd.workload import WORKLOADS, lattice_state, workload_state

    def params(dims, ww):
        return O.OracleParams(n=int(np.prod(dims)), box=tuple(float(d) for d in dims), Cv=ww.Cv,
                              dt=ww.dt, eta=ww.eta, zeta=ww.zeta, h=ww.h, m=ww.m, kB=ww.kB,
                              seed=ww.seed)

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    # parallel variant on the workload itself
    q, p, eps, ids = workload_state(w)
    P = params(w.dims, w)
    S = O.State.from_arrays(q, p, eps, ids)
    O.prepare(P, S)
    t0 = time.perf_counter()
    rc_par, _, used = O.step_parallel(P, S, 0, par_steps, threads=threads)
    t_par = time.perf_counter() - t0
    del S
    # single thread on a sub-lattice
    q, p, eps, ids = lattice_state(sample_dims, Cv=w.Cv, T=w.T, seed=w.init_seed)
    P = params(sample_dims, w)
    S = O.State.from_arrays(q, p, eps, ids)
    O.prepare(P, S)
    t0 = time.perf_counter()
    rc, _ = O.step(P, S, 0, nsteps)
    t_one = time.perf_counter() - t0
    n_one = int(np.prod(sample_dims))
    # the small case in full
    c1 = WORKLOADS["lattice10_cv10"]
    q, p, eps, ids = workload_state(c1)
    P = params(c1.dims, c1)
    S = O.State.from_arrays(q, p, eps, ids)
    O.prepare(P, S)
    t0 = time.perf_counter()
    rc1, _ = O.step(P, S, 0, c1.steps)
    t_c1 = time.perf_counter() - t0
    return {"value": w.n * par_steps / t_par, "unit": "particle-steps/s", "cores": used,
            "kind": "oracle",
            "sample": f"{par_steps} full steps (cells, density, EMS sweep, forces) of the workload "
                      f"itself ({w.n} particles) with the oracle's parallel step variant (OpenMP, "
                      f"bit-identical to the single-threaded step) on {used} threads, "
                      f"{t_par:.1f} s, rc={rc_par}",
            "cpu": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": n_one * nsteps / t_one, "cores": 1,
                              "sample": f"{nsteps} full steps of a {sample_dims[0]}x"
                                        f"{sample_dims[1]}x{sample_dims[2]} sub-lattice "
                                        f"({n_one} particles), {t_one:.1f} s, rc={rc}"},
            "small_case_in_full": {"value": c1.n * c1.steps / t_c1, "cores": 1,
                                   "sample": f"{c1.name}: {c1.n} particles, {c1.steps} steps, "
                                             f"{t_c1:.1f} s, rc={rc1}"}}


def replicas_bench(args):
    """Batched replicas: 256 boxes of uneven size and state, each a context of
    its own, advanced together by the library's batch: by default every stage
    of a step is one launch for all boxes (--batch-layout fused); with
    --batch-layout graphs each box's launches are captured into a graph per
    stream (args.streams streams, a hardware queue per stream).  Compared
    with launching every box's step from the host in turn.  --prec mixed
    runs the density and force passes in FP32 (the F/D update stays FP64)."""
    import torch
    from paper_1707_04232_amd import sdpd
    from paper_1707_04232_amd.workload import lattice_state, replica_set
    nbox = 256
    boxes = replica_set(nbox, seed=0)
    streams = [torch.cuda.Stream() for _ in range(args.streams)]
    ctxs, states, n_tot = [], [], 0
    for b, (side, T, Cv) in enumerate(boxes):
        q, p, eps, ids = lattice_state(side, Cv=Cv, T=T, seed=b)
        prm = sdpd.SdpdParams(n=len(eps), box=float(side), Cv=Cv, replica=b,
                              prec=sdpd.MIXED if args.prec == "mixed" else sdpd.FP64)
        S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
        with torch.cuda.stream(streams[b % len(streams)]):
            ctx = sdpd.Context(prm)
        ctx.prepare(S)
        ctxs.append(ctx)
        states.append(S)
        n_tot += len(eps)
    torch.cuda.synchronize()
    print(f"# replicas: {nbox} boxes, {n_tot} particles, sides {min(b[0] for b in boxes)}.."
          f"{max(b[0] for b in boxes)}", file=sys.stderr, flush=True)
    tuned = None
    if args.tasks:
        tt = tuple(int(x) for x in args.tasks.split(","))
        for ctx in ctxs:   # LDS capacities as the defaults give these task counts
            ctx.tune(tt, (-1,) * 4, (-1,) * 4)
            if args.lds_scale != 1.0:
                t = ctx.get_tuning()
                ctx.tune(tt, [max(128, int(x * args.lds_scale) // 16 * 16)
                              for x in t["lds_particles"]],
                         [max(64, int(x * args.lds_scale) // 64 * 64) for x in t["lds_pairs"]])
        tuned = {"fd_tasks": {"all": tt}, "seconds": 0.0}
    elif args.autotune:
        # the library's autotuner on the largest box of each size class (sides
        # in bands of 7 sites); its tuning is then given to every box of the class
        t0 = time.perf_counter()
        classes = {}
        for b, (side, _, _) in enumerate(boxes):
            classes.setdefault((side - 13) // 7, []).append(b)
        tuned = {}
        for cl, members in sorted(classes.items()):
            lead = max(members, key=lambda b: boxes[b][0])
            t = ctxs[lead].autotune(states[lead], trials=3)
            for b in members:
                ctxs[b].tune(t["fd_tasks"], t["lds_particles"], t["lds_pairs"])
            tuned[f"sides {13 + 7 * cl}..{19 + 7 * cl}"] = t["fd_tasks"]
        torch.cuda.synchronize()
        tuned = {"fd_tasks": tuned, "seconds": time.perf_counter() - t0}
        print(f"# autotuned {tuned}", file=sys.stderr, flush=True)
    if args.lds_budget:
        # every box's LDS capacities scaled down (per phase class, keeping the
        # proportion of particles to pair entries) to fit the budget, so that
        # one persistent sweep launch keeps its workgroups per CU
        budget = int(args.lds_budget * 1024)
        for ctx in ctxs:
            t = ctx.get_tuning()
            cps, ces = list(t["lds_particles"]), list(t["lds_pairs"])
            for k in range(4):
                f = min(1.0, (budget - 1320) / (36.0 * cps[k] + 4.0 * ces[k]))
                cps[k] = max(128, int(cps[k] * f) // 16 * 16)
                ces[k] = max(64, int(ces[k] * f) // 64 * 64)
            ctx.tune(t["fd_tasks"], cps, ces)
        tuned = dict(tuned or {}, lds_budget_kib=args.lds_budget)
    t0 = time.perf_counter()
    B = sdpd.Batch(ctxs, states, layout={"fused": sdpd.BATCH_FUSED, "flow": sdpd.BATCH_FUSED_FLOW,
                                         "graphs": sdpd.BATCH_GRAPHS}[args.batch_layout],
                   parts=args.batch_parts)
    t_capture = time.perf_counter() - t0
    B.run(0, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.run(args.warmup, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for c in ctxs:
        c.sync()
    E = [c.observe(S)["E"] for c, S in zip(ctxs, states)]
    # energy drift of the batch over the timed steps: each box's E observed
    # once more after a short further run (no per-step records in a batch)
    B.run(args.warmup + args.steps, 10)
    torch.cuda.synchronize()
    E10 = [c.observe(S)["E"] for c, S in zip(ctxs, states)]
    # the same boxes stepped eagerly, box after box, from the host
    k0 = args.warmup + args.steps
    neager = max(2, min(20, args.steps // 10))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(neager):
        for c, S in zip(ctxs, states):
            c.step(S, k0 + k, 1, stats=False)
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - t0
    B.close()
    for c in ctxs:
        c.close()
    value = n_tot * args.steps / el
    out = {
        "metric": "particle-steps/s (full SDPD step), 256 replica boxes in one batch",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "replicas256", "boxes": nbox, "n_total": n_tot,
                   "sides": [min(b[0] for b in boxes), max(b[0] for b in boxes)],
                   "T_range": [0.1, 2.0], "Cv_range": [1.5, 50.0], "streams": len(streams),
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "dt": 0.005, "fd": "EMS", "prec": args.prec,
                   "batch_layout": args.batch_layout, "batch_parts": args.batch_parts},
        "eager_sequential": {"value": n_tot * neager / el_eager, "steps": neager,
                             "ms_per_step": 1e3 * el_eager / neager},
        "graph_speedup": (n_tot * args.steps / el) / (n_tot * neager / el_eager),
        "capture_s": t_capture,
        "autotune": tuned,
        "sum_E_final": float(np.sum(E)),
        "sum_E_after_10_more_steps": float(np.sum(E10)),
        "relative_energy_change_10_steps": float(abs(np.sum(E10) - np.sum(E)) / abs(np.sum(E))),
    }
    print(json.dumps(out), flush=True)


def adjoint_bench(args):
    """Adjoint of the conservative dynamics on a 64^3 lattice (C_v = 10,
    T = 1, F/D off): K = 50 steps forward with checkpoints every 10, then the
    reverse pass for each of the two observables, the final kinetic energy
    and the mean pressure A kB rho eps / (m Cv); their q0 gradients are
    checked against central differences of the forward along one random
    direction, and the gradients with respect to A, Cv (at fixed A) and rho0
    are reported (the explicit dependence of the mean pressure on A and Cv
    included)."""
    import torch
    from paper_1707_04232_amd import sdpd
    from paper_1707_04232_amd.workload import WORKLOADS, workload_state
    w = WORKLOADS["lattice64_cv10"]
    K, every = 50, 10
    q, p, eps, ids = workload_state(w)
    A = w.Cv / (3.0 * w.kB)
    prm = sdpd.SdpdParams(n=w.n, box=w.box, Cv=w.Cv, dt=w.dt, fd=sdpd.FD_NONE, A=A)
    rng = np.random.default_rng(1)

    def prepared(qq):
        S = sdpd.DeviceState.from_numpy(qq, p, eps, ids)
        ctx = sdpd.Context(prm)
        ctx.prepare(S)
        return ctx, S

    def by_id(S):
        order = S.id.long()
        out = [torch.empty_like(x) for x in (S.q, S.p, S.eps, S.rho)]
        out[0][:, order], out[1][:, order], out[2][order], out[3][order] = S.q, S.p, S.eps, S.rho
        return out

    def observables(qK, pK, eK, rK):
        return (float((pK * pK).sum() / (2.0 * w.m)),
                float((A * w.kB * rK * eK / (w.m * w.Cv)).sum() / w.n))

    def gradients(ctx, S):
        qK, pK, eK, rK = by_id(S)
        J = observables(qK, pK, eK, rK)
        z = torch.zeros_like(qK)
        gk = ctx.adjoint_vjp(z, pK / w.m)
        c = A * w.kB / (w.m * w.Cv * w.n)
        gp = ctx.adjoint_vjp(z, torch.zeros_like(pK), c * rK, c * eK)
        gp = dict(gp, dA=gp["dA"] + J[1] / A, dCv=gp["dCv"] - J[1] / w.Cv)
        return J, gk, gp

    for _ in range(2):   # warm up the code paths
        c2, S2 = prepared(q)
        c2.adjoint_forward(S2, K, every)
        gradients(c2, S2)
        c2.sync()
        c2.close()
    torch.cuda.synchronize()
    ctx, S = prepared(q)
    t0 = time.perf_counter()
    ctx.adjoint_forward(S, K, every)
    ctx.sync()
    t1 = time.perf_counter()
    J, gk, gp = gradients(ctx, S)
    ctx.sync()
    t2 = time.perf_counter()
    ctx.close()
    d = rng.normal(size=q.shape)
    delta = 1e-6
    Js = []
    for sgn in (1, -1):
        c, Sx = prepared(q + sgn * delta * d)
        c.step(Sx, 0, K, stats=False)
        c.sync()
        Js.append(observables(*by_id(Sx)))
        c.close()
    checks = {}
    for k, (name, g) in enumerate((("kinetic_energy", gk), ("mean_pressure", gp))):
        fd = (Js[0][k] - Js[1][k]) / (2 * delta)
        ad = float((g["dq0"].cpu().numpy()[:, ids] * d).sum())
        checks[name] = {"J": J[k], "dq0_dot_d": {"adjoint": ad, "central_differences": fd,
                                                  "rel_diff": abs(ad - fd) / abs(fd)},
                        "dJ_dA": g["dA"], "dJ_dCv_fixed_A": g["dCv"], "dJ_drho0": g["drho0"]}
    out = {
        "metric": "particle-steps/s of the adjoint (forward with checkpoints + two reverse "
                  "passes), 64^3",
        "value": w.n * K / (t2 - t0), "unit": "particle-steps/s", "n_gpus": 1, "steps": K,
        "warmup": 2, "ms_per_step": 1e3 * (t2 - t0) / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "adjoint64", "n": w.n, "lattice": list(w.dims), "Cv": w.Cv,
                   "T": w.T, "dt": w.dt, "steps": K, "checkpoint_every": every, "fd": "none"},
        "forward_s": t1 - t0, "backward_s_two_observables": t2 - t1,
        "observables": checks,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=WORKLOAD,
                    help="workload name (the default is the headline 1M-particle case)")
    ap.add_argument("--prec", choices=("fp64", "mixed"), default="fp64",
                    help="arithmetic of the density and force passes")
    ap.add_argument("--fd-every", type=int, default=1,
                    help="F/D sweep every this many steps, with theta * dt (multiple time steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--streams", type=int, default=32,
                    help="streams of the replicas workload (at most 32)")
    ap.add_argument("--autotune", action="store_true",
                    help="replicas workload: run the library's autotuner per box size class "
                         "(it times single-box sweeps; the default tuning serves the batch "
                         "better)")
    ap.add_argument("--batch-layout", choices=("fused", "flow", "graphs"), default="fused",
                    help="replicas workload: one launch per stage for all boxes (fused), the "
                         "same with one persistent F/D sweep launch for all boxes (flow), or "
                         "each box's launches captured into graphs per stream (graphs)")
    ap.add_argument("--tasks", default="",
                    help="replicas workload: tasks per workgroup of the four F/D phase classes "
                         "for every box, e.g. 4,4,8,12 (instead of the autotuner)")
    ap.add_argument("--lds-scale", type=float, default=1.0,
                    help="replicas workload with --tasks: scale of the LDS capacities")
    ap.add_argument("--lds-budget", type=float, default=0.0,
                    help="replicas workload: scale every box's F/D LDS capacities down to at "
                         "most this many KiB per workgroup (after any autotuning)")
    ap.add_argument("--batch-parts", type=int, default=0,
                    help="replicas workload, fused layout: parts of the batch, each on its own "
                         "stream (0 = the library's choice)")
    ap.add_argument("--no-timing", action="store_true",
                    help="do not bracket kernels with HIP events")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (a known-traffic "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is described in the design notes, not built)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "replicas256":
        if not 1 <= args.streams <= 32:
            ap.error("--streams must be in 1..32")
        # one hardware queue per stream, set before HIP starts (HIP's default is 4)
        os.environ["GPU_MAX_HW_QUEUES"] = str(max(4, args.streams))
    import torch
    from paper_1707_04232_amd import sdpd
    from paper_1707_04232_amd.workload import WORKLOADS, workload_state

    if args.workload == "replicas256":
        torch.cuda.set_device(0)
        replicas_bench(args)
        return
    if args.workload == "adjoint64":
        torch.cuda.set_device(0)
        adjoint_bench(args)
        return
    w = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)   # reads and writes nbytes once (elementwise kernel)
        torch.cuda.synchronize()
        print(f"# copy calibration: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr,
              flush=True)
        del src, dst
    q, p, eps, ids = workload_state(w)
    S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
    prec = sdpd.MIXED if args.prec == "mixed" else sdpd.FP64
    prm = sdpd.SdpdParams(n=w.n, box=w.box, m=w.m, h=w.h, kB=w.kB, Cv=w.Cv, eta=w.eta,
                          zeta=w.zeta, dt=w.dt, fd=sdpd.FD_EMS, seed=w.seed, prec=prec,
                          fd_every=args.fd_every)
    ctx = sdpd.Context(prm)
    ctx.prepare(S)
    print(f"# {w.name}: n={w.n}, {args.prec}, warmup {args.warmup}, timed {args.steps}",
          file=sys.stderr, flush=True)
    if args.warmup:
        ctx.step(S, 0, args.warmup, stats=False)
    ctx.sync()
    # timed region: events around the F/D sweep only (the roofline's kernel);
    # the other kernels run without events
    if not args.no_timing:
        ctx.set_timing_classes(["fd"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.step(S, args.warmup, args.steps, stats=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.timing()
    ctx.set_timing(False)
    ctx.sync()
    last_pairs, last_staged = ctx.fd_schedule_size()
    # per-kernel breakdown: a short run after the timed region, every class timed
    breakdown = None
    if not args.no_timing:
        nb = max(1, min(50, args.steps))
        ctx.set_timing(True)
        ctx.step(S, args.warmup + args.steps, nb, stats=False)
        tb = ctx.timing()
        ctx.set_timing(False)
        ctx.sync()
        breakdown = {k: {"ms_per_step": v[0] / nb, "launches": v[1]} for k, v in tb.items()}
    elapsed = t1 - t0
    value = w.n * args.steps / elapsed

    E = np.array([s["E"] for s in st])
    proposed = sum(s["proposed"] for s in st)
    rej_e = sum(s["rej_energy"] for s in st)
    rej_r = sum(s["rej_ratio"] for s in st)
    slope = linear_slope(E) if len(E) > 1 else 0.0
    drift = {"per_1e3_steps_per_particle_kBT": slope * 1000.0 / (w.n * w.kB * w.T),
             "per_1e3_steps_relative": slope * 1000.0 / abs(E[0]),
             "E0": float(E[0]), "E_last": float(E[-1])}

    roof = None
    fd_ms, fd_launches = tm["fd"]
    if fd_launches:
        avg_ms = fd_ms / fd_launches
        flops_per_launch = FLOPS_PER_EMS_PAIR * proposed / fd_launches
        achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
        nsweeps = sum(1 for k in range(args.warmup, args.warmup + args.steps)
                      if k % args.fd_every == 0)
        launches_per_sweep = fd_launches / max(nsweeps, 1)
        alg_bytes = (last_staged * BYTES_PER_STAGED + last_pairs * BYTES_PER_PAIR_ENTRY) \
            / launches_per_sweep
        roof = {"bound": "alu", "kernel": "k_fd_sweep", "achieved": achieved,
                "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VALU_PEAK_TFLOPS, "traffic": measured_traffic(),
                "algorithmic_bytes_per_launch": alg_bytes,
                "avg_launch_ms": avg_ms, "launches": fd_launches,
                "pairs_per_launch": proposed / fd_launches,
                "flops_per_pair": FLOPS_PER_EMS_PAIR,
                "traffic_record": traffic_record(),
                "flops_per_pair_executed": FLOPS_PER_PAIR_EXECUTED,
                "frac_executed": achieved * FLOPS_PER_PAIR_EXECUTED / FLOPS_PER_EMS_PAIR
                / FP64_VALU_PEAK_TFLOPS}

    cpu = None
    if not args.no_cpu_baseline and args.workload == WORKLOAD:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w)

    out = {
        "metric": ("particle-steps/s (full SDPD step) at 1M particles; energy drift per 1e3 steps"
                   if args.workload == WORKLOAD else
                   f"particle-steps/s (full SDPD step) at {w.n} particles; energy drift per 1e3 steps"),
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "lattice": list(w.dims), "box": list(w.box),
                   "Cv": w.Cv, "T": w.T, "dt": w.dt, "h": w.h, "kernel": "lucy",
                   "fd": "EMS", "fd_every": args.fd_every, "prec": args.prec,
                   "steps": args.steps},
        "energy_drift": drift,
        "fd": {"pairs_per_step": proposed / args.steps,
               "staged_per_step_last": last_staged,
               "pairs_per_step_last": last_pairs,
               "rejection_rate": (rej_e + rej_r) / max(proposed, 1),
               "rej_energy": rej_e, "rej_ratio": rej_r},
        "kernel_ms_per_step": breakdown,
        "roofline": roof,
        "step_floor": step_floor(w, proposed / args.steps, 1e3 * elapsed / args.steps),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
