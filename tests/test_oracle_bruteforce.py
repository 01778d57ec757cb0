"""Brute force: the oracle against a literal pure-Python evaluator of the
same discrete step (tests/bruteforce.py) on 8x8 and 4x4x4 random states."""
import numpy as np
import pytest

from bruteforce import Step
from inputs import KINDS, KINDS4, busy_config, random_state


def _compare(oracle, cfg, st, steps):
    sim = oracle.OracleSim(cfg)
    for k in ("phi", "mu", "f", "u"):
        sim.set(k, st[k])
    bf = Step(cfg)
    s = dict(st, step=0)
    for _ in range(steps):
        s = bf.step(s)
    sim.step(steps)
    for k in ("phi", "mu", "f", "u"):
        a, b = sim.get(k), s[k]
        # U is a small moment of O(0.1) populations: its round-off scales with f
        scale = max(np.abs(b).max(), np.abs(s["f"]).max() if k == "u" else 0.0, 1e-300)
        assert np.abs(a - b).max() <= 1e-13 * scale, (k, np.abs(a - b).max(), scale)


@pytest.mark.parametrize("kind", KINDS)
def test_one_step_vs_literal_evaluator(oracle, kind):
    n = [8, 8] if "2d" in kind else [4, 4, 4]
    cfg = busy_config(kind, n)
    _compare(oracle, cfg, random_state(cfg, 11), 1)


@pytest.mark.parametrize("kind", ["binary2d", "ternary2d"])
def test_ten_steps_vs_literal_evaluator(oracle, kind):
    cfg = busy_config(kind, [8, 8])
    _compare(oracle, cfg, random_state(cfg, 12), 10)


def test_lid_and_well_vs_literal_evaluator(oracle):
    cfg = busy_config("binary2d", [8, 8], periodic=[0, 0], lid_u=0.05, potential="well")
    _compare(oracle, cfg, random_state(cfg, 13), 3)


@pytest.mark.parametrize("kind", ["binary2d", "ternary2d", "binary3d"])
def test_shrinkage_vs_literal_evaluator(oracle, kind):
    """The shrinkage force (Eq. shrinkage) switched on with the paper's
    density ratio rho_s / rho_l = 1.2 (eta = 0.2 for every solid)."""
    n = [8, 8] if "2d" in kind else [4, 4, 4]
    cfg = busy_config(kind, n)
    cfg["eta"] = [0.2, 0.2, 0.0] if cfg["N"] == 3 else [0.2, 0.0, 0.0]
    _compare(oracle, cfg, random_state(cfg, 14), 3)


@pytest.mark.parametrize("kind", ["binary3d", "ternary3d_nc2"])
def test_d3q27_vs_literal_evaluator(oracle, kind):
    """The paper's own 3D lattice, D3Q27 (Table LBM_Schemes); the evaluator
    builds it from {-1, 0, 1}^3 and orders it differently (the oracle's
    numbering is compared through the populations' velocities)."""
    from bruteforce import lattice
    cfg = busy_config(kind, [4, 4, 4], lattice="D3Q27")
    st = random_state(cfg, 16)
    sim = oracle.OracleSim(cfg)
    # map the evaluator's velocity order to the oracle's
    c_bf, _ = lattice(3, "D3Q27")
    c_or, _, _ = oracle.lattice(3, 27)
    perm = [c_bf.index(tuple(int(v) for v in c_or[k])) for k in range(27)]
    f_bf = st["f"]
    for k in ("phi", "mu", "u"):
        sim.set(k, st[k])
    sim.set("f", f_bf[perm])
    bf = Step(cfg)
    s = dict(st, step=0)
    for _ in range(3):
        s = bf.step(s)
    sim.step(3)
    for k in ("phi", "mu", "f", "u"):
        a, b = sim.get(k), (s[k][perm] if k == "f" else s[k])
        scale = max(np.abs(b).max(), np.abs(s["f"]).max() if k == "u" else 0.0, 1e-300)
        assert np.abs(a - b).max() <= 1e-13 * scale, (k, np.abs(a - b).max(), scale)


@pytest.mark.parametrize("kind", KINDS4)
def test_four_phases_vs_literal_evaluator(oracle, kind):
    """Three solids and the liquid (the paper's Case 3 system), every term on,
    two solutes."""
    n = [8, 8] if "2d" in kind else [4, 4, 4]
    cfg = busy_config(kind, n)
    _compare(oracle, cfg, random_state(cfg, 17), 3)
