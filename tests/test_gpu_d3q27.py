"""GPU parity on the paper's own 3D lattice, D3Q27 (Table LBM_Schemes),
against the FP64 oracle: the same bars as the D3Q19 path."""
import numpy as np
import pytest

from gpu_helpers import STATE, field_floor, gpu_from, oracle_from, read_state, rel_err, window_step
from inputs import busy_config, random_state
from paper_2608_26908_amd.workloads import scaled, workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
KINDS3 = ["binary3d", "ternary3d_nc2"]


def _cmp(gpu, ora, tol=TOL64):
    ref = {k: ora.get(k) for k in STATE}
    for k in STATE:
        e = rel_err(gpu.read(k), ref[k], field_floor(k, ref))
        assert e <= tol, (k, e)


@pytest.mark.parametrize("kind", KINDS3)
def test_one_step_random_state_fp64(oracle, kind):
    cfg = busy_config(kind, [70, 9, 11], lattice="D3Q27")
    st = random_state(cfg, 8)
    g = gpu_from(cfg, st, "fp64")
    assert g.Q == 27
    o = oracle_from(cfg, st)
    g.step(1)
    o.step(1)
    _cmp(g, o)
    assert rel_err(g.read("rho"), o.get("rho")) <= TOL64


@pytest.mark.parametrize("name,n", [("dendrite3d", [40, 36, 44]), ("eutectic3d", [48, 30, 64])])
def test_workload_100_steps_fp64(oracle, name, n):
    cfg = scaled(name, n, lattice="D3Q27", gbeta=[1e-3] if name == "dendrite3d" else [2e-3, -1e-3])
    from paper_2608_26908_amd.gpf import Sim
    g = Sim(cfg, precision="fp64")
    o = oracle.OracleSim(cfg)
    g.step(100)
    o.step(100)
    _cmp(g, o)


def test_fp32_within_tolerance_after_100_steps(oracle):
    from paper_2608_26908_amd.gpf import Sim
    cfg = scaled("dendrite3d", [64, 64, 64], lattice="D3Q27", gbeta=[1e-3])
    g, o = Sim(cfg, precision="fp32"), oracle.OracleSim(cfg)
    g.step(100)
    o.step(100)
    dphi = np.abs(g.read("phi") - o.get("phi")).max()
    ug, uo = g.read("u"), o.get("u")
    rl2 = np.sqrt(((ug - uo) ** 2).sum() / (uo ** 2).sum())
    print(f"FP32 vs FP64 oracle, D3Q27 dendrite3d [64, 64, 64], 100 steps: "
          f"max|dphi| {dphi:.2e}, rel-L2(U) {rl2:.2e}")
    assert dphi <= 1e-5, dphi
    assert rl2 <= 1e-4, rl2


def test_full_size_sampled_step_fp32(oracle):
    from paper_2608_26908_amd.gpf import Sim
    cfg = workload("dendrite3d", lattice="D3Q27")
    g = Sim(cfg, precision="fp32")
    g.step(20)
    st = read_state(g)
    g.step(1)
    after = read_state(g)
    c = [int(v) for v in cfg["init_center"]]
    r = int(cfg["init_radius"])
    pts = [tuple(c), (c[0] + r, c[1], c[2]), (c[0], c[1] + r, c[2] - 1), (0, 0, 0), (255, 128, 255)]
    tol = dict(phi=1e-5, mu=1e-5, f=1e-5, u=1e-3)
    for pt in pts:
        ref = window_step(cfg, st, 20, pt)
        sl = (slice(None),) + tuple(reversed(pt))
        for k in STATE:
            got = after[k][sl]
            scale = max(np.abs(after[k]).max(), field_floor(k, after), 1e-30)
            assert np.abs(got - ref[k]).max() <= tol[k] * scale, (pt, k, got, ref[k])


@pytest.mark.parametrize("kind", KINDS3)
def test_adjoint_dot_product_fp64(oracle, kind):
    """<w, J v> (oracle complex-step tangent) = <J^T w, v> (library adjoint)
    for perturbations of every state field, over checkpoint segments."""
    cfg = busy_config(kind, [12, 10, 11], lattice="D3Q27")
    st = random_state(cfg, 22)
    steps, K = 5, 2
    g = gpu_from(cfg, st, "fp64")
    g.record(K)
    g.step(steps)
    rng = np.random.default_rng(5)
    w = rng.standard_normal((cfg["N"],) + g.shape)
    g.adjoint(w, [])
    o = oracle_from(cfg, st)
    for field in ("phi", "mu", "u", "f"):
        lam = g.adjoint_state(field)
        v = rng.standard_normal(lam.shape)
        t = o.tangent_cs(steps, field, v, "phi")
        lhs, rhs = float((w * t).sum()), float((lam * v).sum())
        assert abs(lhs - rhs) <= 1e-9 * max(abs(lhs), abs(rhs), 1e-30), (field, lhs, rhs)
