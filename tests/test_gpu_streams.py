"""Stream semantics of the boundary: a plan bound to a caller's stream gives
the same bits as one on the default stream, and evolve is stream-ordered (work
enqueued after it on the plan's stream, with no host synchronisation in
between, sees the evolved state), also in graph mode on the default stream,
where the plan runs on a blocking stream of its own."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_1007_3470_amd as p
    p.load()
    return p


def evolve_on(pkg, w, dtype, stream, **kw):
    """Pack on the current stream, evolve on `stream`, unpack after the
    current stream has waited for it."""
    import torch
    cur = torch.cuda.current_stream()
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, stream=stream, **kw)
    buf = plan.pack(w.psi0)
    if stream is not None:
        stream.wait_stream(cur)
    plan.evolve(buf, w.t0, w.nsteps)
    if stream is not None:
        cur.wait_stream(stream)
        buf.record_stream(stream)
    out = plan.unpack(buf)
    assert plan.device_status() == 0
    return out


@pytest.mark.parametrize("make", [lambda: W.batch_1d(n_inst=64, nsteps=50, seed=3),
                                  lambda: W.gpe_2d(n=64, n_inst=3, nsteps=20)],
                         ids=["batch_1d", "gpe_2d"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_caller_stream_matches_default_stream(pkg, make, use_graph):
    import torch
    w = make()
    ref = evolve_on(pkg, w, "c128", None, use_graph=use_graph)
    s = torch.cuda.Stream()  # default priority
    got = evolve_on(pkg, w, "c128", s, use_graph=use_graph)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("make", [lambda: W.batch_1d(n_inst=64, nsteps=50, seed=4),
                                  lambda: W.gpe_2d(n=64, n_inst=3, nsteps=40)],
                         ids=["batch_1d", "gpe_2d"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_evolve_is_stream_ordered(pkg, make, use_graph):
    """A device copy taken right after evolve on the same (default) stream,
    before any host synchronisation, holds the evolved state."""
    import torch
    w = make()
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt, use_graph=use_graph)
    buf = plan.pack(w.psi0)
    torch.cuda.synchronize()
    plan.evolve(buf, w.t0, w.nsteps)
    snap = buf.clone()  # enqueued behind the evolve, no synchronisation
    torch.cuda.synchronize()
    final = buf.to("cpu")
    assert torch.equal(snap.to("cpu"), final)
    start = torch.from_numpy(np.concatenate([np.asarray(p).ravel() for p in w.psi0]))
    assert not torch.equal(final, start)
