"""Batched replicas: boxes of uneven size, temperature and heat capacity
(replica index = box index in the Philox counter), each its own context,
spread over three streams and advanced by one captured HIP graph.  Every
replay must give exactly (bit for bit) what the eager sdpd_step gives on a
second, independent set of contexts; the replays are interleaved with eager
work on the same contexts (observables, synchronisation) and each replay is
checked."""
import numpy as np
import pytest

from paper_1707_04232_amd.workload import lattice_state, replica_set

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _boxes(nbox, fd_every, streams):
    import torch
    from paper_1707_04232_amd import sdpd
    out = []
    for b, (side, T, Cv) in enumerate(replica_set(nbox, seed=1)):
        side = min(side, 20)   # keep the eager reference quick
        q, p, eps, ids = lattice_state(side, Cv=Cv, T=T, seed=10 + b)
        prm = sdpd.SdpdParams(n=len(eps), box=float(side), Cv=Cv, replica=b, fd_every=fd_every,
                              seed=7)
        S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
        st = streams[b % len(streams)] if streams else torch.cuda.current_stream()
        with torch.cuda.stream(st):
            ctx = sdpd.Context(prm)
        ctx.prepare(S)
        out.append((ctx, S))
    return out


@pytest.mark.parametrize("fd_every", [1, 2])
def test_batch_graph_matches_eager_steps(fd_every):
    import torch
    from paper_1707_04232_amd import sdpd
    say("batch graph vs eager, fd_every", fd_every)
    streams = [torch.cuda.Stream() for _ in range(3)]
    ref = _boxes(6, fd_every, None)
    bat = _boxes(6, fd_every, streams)
    torch.cuda.synchronize()
    with sdpd.Batch([c for c, _ in bat], [s for _, s in bat]) as B:
        with pytest.raises(sdpd.SdpdError):
            if fd_every > 1:
                B.run(1, fd_every)         # blocks must start at a multiple of fd_every
            else:
                raise sdpd.SdpdError(sdpd.EINVAL, "n/a")
        step = 0
        for rep in range(3):
            nsteps = 2 * fd_every
            B.run(step, nsteps)
            for c, S in ref:
                c.step(S, step, nsteps, stats=False)
            step += nsteps
            for (cb, Sb), (cr, Sr) in zip(bat, ref):
                cb.sync()
                cr.sync()
                gb, gr = Sb.to_numpy(), Sr.to_numpy()
                for k in ("q", "p", "eps", "rho", "f", "id"):
                    assert np.array_equal(gb[k], gr[k]), f"replay {rep}: {k} differs"
                ob, orf = cb.observe(Sb), cr.observe(Sr)   # eager work between replays
                assert ob["E"] == orf["E"]
    for c, _ in ref + bat:
        c.close()


_PER_STREAM_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
from paper_1707_04232_amd import sdpd
from tests.test_gpu_batch import _boxes
print("[case] per-stream graphs, GPU_MAX_HW_QUEUES =", __import__("os").environ["GPU_MAX_HW_QUEUES"], flush=True)
streams = [torch.cuda.Stream() for _ in range(3)]
ref = _boxes(6, 1, None)
bat = _boxes(6, 1, streams)
torch.cuda.synchronize()
with sdpd.Batch([c for c, _ in bat], [s for _, s in bat]) as B:
    step = 0
    for rep in range(3):
        B.run(step, 2)
        for c, S in ref:
            c.step(S, step, 2, stats=False)
        step += 2
        for (cb, Sb), (cr, Sr) in zip(bat, ref):
            cb.sync()
            cr.sync()
            gb, gr = Sb.to_numpy(), Sr.to_numpy()
            for k in ("q", "p", "eps", "rho", "f", "id"):
                assert np.array_equal(gb[k], gr[k]), f"replay {rep}: {k} differs"
            assert cb.observe(Sb)["E"] == cr.observe(Sr)["E"]
for c, _ in ref + bat:
    c.close()
print("ok", flush=True)
"""


def test_batch_per_stream_graphs_match_eager_steps():
    """With a hardware queue per stream the batch keeps one graph per stream;
    the queue count is fixed when HIP starts, so this runs in a child process
    (started, not exec'd, from this one) with GPU_MAX_HW_QUEUES = 8."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, GPU_MAX_HW_QUEUES="8")
    say("batch per-stream graphs (child process)")
    r = subprocess.run([sys.executable, "-c", _PER_STREAM_CHILD, root], env=env, cwd=root,
                       capture_output=True, text=True, timeout=150)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-2000:]


def test_batch_refuses_a_retuned_context():
    import torch
    from paper_1707_04232_amd import sdpd
    say("batch after sdpd_tune")
    streams = [torch.cuda.Stream() for _ in range(2)]
    bat = _boxes(2, 1, streams)
    torch.cuda.synchronize()
    with sdpd.Batch([c for c, _ in bat], [s for _, s in bat]) as B:
        B.run(0, 1)
        t = bat[0][0].get_tuning()
        bat[0][0].tune(t["fd_tasks"], t["lds_particles"], t["lds_pairs"])
        with pytest.raises(sdpd.SdpdError):
            B.run(1, 1)
    for c, _ in bat:
        c.sync()
        c.close()
