"""Graph replay of step runs on small grids (host logic of gpf_step): the
replayed steps must give bit for bit the state of steps launched one by one,
also after a parameter change between runs (the graph is captured again)."""
import numpy as np
import pytest

from paper_2608_26908_amd.workloads import workload, scaled

pytestmark = pytest.mark.gpu


def _sim(cfg):
    from paper_2608_26908_amd.gpf import Sim
    return Sim(cfg, precision="fp32")


def _state(sim):
    return {f: sim.read(f) for f in ("phi", "mu", "u", "fpost")}


@pytest.mark.parametrize("name,n", [("dendrite2d", None), ("adjoint2d", [128, 96])])
def test_graph_replay_is_bitwise(name, n):
    cfg = workload(name) if n is None else scaled(name, n)
    a, b = _sim(cfg), _sim(cfg)
    try:
        a.step(300)            # 4 graph replays of 64 steps and 44 single steps
        for _ in range(300):   # one step per call: never a graph
            b.step(1)
        assert a.step_index == b.step_index == 300
        sa, sb = _state(a), _state(b)
        for f in sa:
            assert np.array_equal(sa[f], sb[f]), f
        # a changed parameter invalidates the captured graph
        a.set_param("tau_pf", 1.2)
        b.set_param("tau_pf", 1.2)
        a.step(200)
        for _ in range(200):
            b.step(1)
        sa, sb = _state(a), _state(b)
        for f in sa:
            assert np.array_equal(sa[f], sb[f]), f
    finally:
        a.close()
        b.close()
