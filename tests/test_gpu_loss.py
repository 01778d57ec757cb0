"""The FP64 totals of the library against the oracle: solute and mass on
every built instance, and the loss of the adjoint inversion, GPF_LOSS (1/2
sum (phi - target)^2 against a device target) with its seed dL/dphi = phi -
target."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import gpu_from, oracle_from
from inputs import KINDS, KINDS4, busy_config, random_state
from paper_2608_26908_amd.workloads import scaled

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", KINDS + KINDS4)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_totals_match_oracle_every_instance(oracle, kind, precision):
    """Solute (nc values) and mass totals of a random state on every built
    instance (one and two solutes, 2D and 3D, three and four phases), FP64
    sums of the stored values: within 1e-13 of the oracle's totals of the
    same state (FP32: the stored state is the FP32 rounding of the oracle's,
    so within 1e-6)."""
    n = [33, 29] if "2d" in kind else [17, 13, 11]
    cfg = busy_config(kind, n)
    st = random_state(cfg, 12)
    g = gpu_from(cfg, st, precision)
    o = oracle_from(cfg, st)
    tol = 1e-13 if precision == "fp64" else 1e-6
    assert np.allclose(g.reduce("solute"), o.total("solute"), rtol=tol, atol=0)
    assert g.reduce("mass") == pytest.approx(o.total("mass"), rel=tol)
    g.close()


@pytest.mark.parametrize("kind,n,precision", [("binary2d", [37, 29], "fp64"), ("binary2d", [37, 29], "fp32"),
                                              ("ternary3d_nc2", [19, 13, 11], "fp64"),
                                              ("ternary3d_nc2", [19, 13, 11], "fp32")])
def test_loss_matches_oracle_side_loss(oracle, kind, n, precision):
    """After 10 steps from a random state: GPF_LOSS equals 1/2 sum (phi -
    target)^2 summed in FP64 over the library's own phi within 1e-14, and
    (FP64) the same sum over the oracle's phi within 1e-13; the seed is phi -
    target exactly."""
    import torch
    cfg = busy_config(kind, n)
    st = random_state(cfg, 5)
    g = gpu_from(cfg, st, precision)
    g.step(10)
    rng = np.random.default_rng(9)
    target = rng.uniform(0.0, 1.0, (cfg["N"],) + g.shape)
    g.set_target(target)
    L = g.reduce("loss")
    phi = g.read("phi")
    assert L == pytest.approx(0.5 * float(((phi - target) ** 2).sum()), rel=1e-14)
    if precision == "fp64":
        o = oracle_from(cfg, st)
        o.step(10)
        assert L == pytest.approx(0.5 * float(((o.get("phi") - target) ** 2).sum()), rel=1e-13)
    seed = g.loss_seed()
    torch.cuda.synchronize()
    assert np.array_equal(seed.cpu().numpy(), phi - target)
    g.close()


def test_loss_needs_a_target_of_the_right_size():
    import torch
    from paper_2608_26908_amd.gpf import GPFError, lib
    cfg = busy_config("binary2d", [16, 12])
    g = gpu_from(cfg, random_state(cfg, 1), "fp64")
    with pytest.raises(GPFError) as e:
        g.reduce("loss")
    assert e.value.code == -6
    t = torch.zeros(3, device="cuda", dtype=torch.float64)
    assert lib().gpf_set_target(g._h, ctypes.c_void_p(t.data_ptr()), 3) == -1
    g.set_target(np.zeros((2, 12, 16)))
    assert g.reduce("loss") > 0
    g.set_target(None)
    with pytest.raises(GPFError):
        g.loss_seed()
    g.close()


def test_loss_autograd_equals_the_adjoint_and_guards_the_run(oracle):
    """gpf_loss (loss and seed inside the library) as a torch.autograd
    function: its value is GPF_LOSS and its gradient the adjoint seeded with
    phi - target; a backward after the simulation was stepped again raises."""
    import torch
    from paper_2608_26908_amd.gpf import Sim, gpf_loss
    cfg = scaled("adjoint2d", [40, 40], init_radius=5.0)
    steps, K = 60, 20
    t = dict(cfg, delta=[[0, 0.025], [0.025, 0]], tau_pf=1.2)
    o = oracle.OracleSim(t)
    o.step(steps)
    sim = Sim(cfg, precision="fp64")
    sim.set_target(o.get("phi"))
    init = sim.checkpoint()
    names = ["delta", "tau_pf", "D"]
    p = torch.tensor([0.02, 1.0, 1.0], dtype=torch.float64, requires_grad=True)
    loss = gpf_loss(p, sim, init, names, steps, K)
    phi = sim.read("phi")
    assert float(loss) == pytest.approx(0.5 * float(((phi - o.get("phi")) ** 2).sum()), rel=1e-14)
    loss.backward()
    ref = sim.adjoint(phi - o.get("phi"), names)
    assert np.allclose(p.grad.numpy(), ref, rtol=1e-12, atol=0)
    q = p.detach().clone().requires_grad_(True)
    loss = gpf_loss(q, sim, init, names, steps, K)
    sim.step(1)
    with pytest.raises(RuntimeError, match="stepped"):
        loss.backward()
    sim.close()


@pytest.mark.parametrize("pattern", ["copy19", "pull19", "pull19_zmarch"])
def test_bandwidth_probe_moves_the_right_values(pattern):
    """The probe kernels copy or pull exactly: out_k = in_k shifted by the
    D3Q19 velocity c_k (periodic), whatever launch shape times them."""
    import torch
    from paper_2608_26908_amd.gpf import bandwidth_probe
    n = (128, 12, 8)
    gbps, a, b = bandwidth_probe(pattern, n, reps=2)
    assert gbps > 0
    c = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
                  [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
    fin = a.cpu().numpy().reshape(19, n[2], n[1], n[0])
    fout = b.cpu().numpy().reshape(19, n[2], n[1], n[0])
    for k in range(19):
        want = fin[k] if pattern == "copy19" else np.roll(fin[k], shift=(c[k, 2], c[k, 1], c[k, 0]), axis=(0, 1, 2))
        assert np.array_equal(fout[k], want), k
