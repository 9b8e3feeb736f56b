"""sdpd_observe_noalloc, the entry point that allocates nothing, against the
existing sdpd_observe on the same states: two calls in a row, the second
with a smaller input (its partial sums must not mix with what the first left
in the library's fixed scratch array), bit for bit; replays of a captured
HIP graph holding the call; the host-side refusals."""
import ctypes as C

import numpy as np
import pytest

from paper_1707_04232_amd.workload import lattice_state, uniform_state

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _record(st):
    return np.array([st["E"], st["Eint"], st["KE"], *st["P"], st["min_eps"]])


def test_observe_noalloc_matches_observe():
    import torch
    from paper_1707_04232_amd import sdpd
    cases = [
        # 343,000 particles: more than 1024 blocks of 256, the grid-stride path
        ("lattice70", lattice_state(70, Cv=1.5, T=0.1), 70.0),
        ("uniform700", uniform_state(700, (10.0, 10.0, 10.0), seed=3), 10.0),
    ]
    out = torch.full((7,), float("nan"), dtype=torch.float64, device="cuda")
    for name, (q, p, eps, ids), box in cases:
        say("observe_noalloc", name, len(eps))
        eps = eps * np.linspace(0.5, 1.5, len(eps))   # a non-trivial minimum
        prm = sdpd.SdpdParams(n=len(eps), box=box, Cv=1.5)
        S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
        with sdpd.Context(prm) as ctx:
            want = _record(ctx.observe(S))
        sdpd.observe_noalloc(prm, S, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, want), (got, want)


def test_observe_noalloc_in_a_captured_graph():
    import torch
    from paper_1707_04232_amd import sdpd
    say("observe_noalloc in a captured graph")
    q, p, eps, ids = lattice_state(16, Cv=1.5, T=0.1)
    prm = sdpd.SdpdParams(n=len(eps), box=16.0, Cv=1.5)
    S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
    out = torch.zeros(7, dtype=torch.float64, device="cuda")
    sdpd.observe_noalloc(prm, S, out)          # first call on the device: eager
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sdpd.observe_noalloc(prm, S, out)
    ctx = sdpd.Context(prm)
    try:
        for rep in range(3):
            S.p.mul_(1.0 + 0.25 * (rep + 1))       # eager work between replays
            S.eps.add_(0.01 * rep)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            want = _record(ctx.observe(S))
            assert np.array_equal(out.cpu().numpy(), want), f"replay {rep}"
    finally:
        ctx.close()


def test_observe_noalloc_refusals():
    import torch
    from paper_1707_04232_amd import sdpd
    L = sdpd.lib()
    q, p, eps, ids = lattice_state(10)
    S = sdpd.DeviceState.from_numpy(q, p, eps, ids)
    out = torch.zeros(7, dtype=torch.float64, device="cuda")
    good = sdpd.SdpdParams(n=len(eps), box=10.0)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    dst = C.c_void_p(out.data_ptr())
    assert L.sdpd_observe_noalloc(C.byref(good.c()), C.byref(S.c()), stream, dst) == sdpd.OK
    for bad in (dict(Cv=0.4), dict(box=9.0), dict(n=-1), dict(n=1 << 31)):
        kw = dict(n=len(eps), box=10.0)
        kw.update(bad)
        prm = sdpd.SdpdParams(**kw)
        assert L.sdpd_observe_noalloc(C.byref(prm.c()), C.byref(S.c()), stream, dst) == \
            sdpd.EINVAL, bad
    assert L.sdpd_observe_noalloc(C.byref(good.c()), C.byref(S.c()), stream, None) == sdpd.EINVAL
    assert L.sdpd_observe_noalloc(C.byref(good.c()), None, stream, dst) == sdpd.EINVAL
    torch.cuda.synchronize()
