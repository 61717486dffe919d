"""The oracle's thread count changes nothing: its threaded loops (pencils of
an axis transform, points of a pointwise flow) compute every element exactly
as one thread does, so results must be bitwise equal for any count.  CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W


CASES = [
    ("gpe_1d", lambda: W.gpe_1d(n=256, nsteps=40)),
    ("gpe_2d", lambda: W.gpe_2d(n=64, n_inst=1, nsteps=12)),
    ("gpe_3d", lambda: W.gpe_3d(n=32, nsteps=3)),
    ("coupled_2d", lambda: W.coupled_2d(n=32, n_inst=1, nsteps=8)),
    ("coupled_3d", lambda: W.coupled_3d(n=16, nsteps=2)),
    ("fsplit_2d", lambda: W.gpe_2d(n=32, n_inst=1, nsteps=8, rule="fsplit")),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("threads", [2, 3, 8])
def test_threaded_evolve_is_bitwise_single_thread(name, make, threads):
    w = make()
    inst = w.instances[0]
    one = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps, threads=1)
    many = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps, threads=threads)
    assert np.array_equal(one.view(np.float64), many.view(np.float64))
    e1 = oracle.energy(inst, one, 0.37, threads=1)
    e2 = oracle.energy(inst, one, 0.37, threads=threads)
    assert np.array_equal(e1, e2)


def test_threaded_evolve_with_potential_array():
    w = W.gpe_2d(n=64, n_inst=1, nsteps=5)
    inst = w.instances[0]
    x, y = inst.mesh()
    vi = 0.2 * (x + 0.5 * y ** 2) * np.ones(inst.shape)
    one = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps, vi=vi, threads=1)
    many = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps, vi=vi, threads=5)
    assert np.array_equal(one.view(np.float64), many.view(np.float64))


def test_bad_thread_count_rejected():
    w = W.gpe_1d(n=64, nsteps=1)
    with pytest.raises(RuntimeError):
        oracle.evolve(w.instances[0], w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, 1, threads=0)
