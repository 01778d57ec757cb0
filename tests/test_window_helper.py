"""The windowed one-step oracle used by the full-size sampled GPU checks
reproduces the full-grid oracle step at the window centre."""
import numpy as np
import pytest

from gpu_helpers import STATE, window_step
from inputs import busy_config, random_state
from paper_2608_26908_amd.workloads import scaled


@pytest.mark.parametrize("cfg", [
    busy_config("binary3d", [14, 12, 13]),
    busy_config("ternary2d", [21, 18], periodic=[1, 0]),
    busy_config("ternary3d_nc2", [12, 11, 14], periodic=[1, 0, 0]),
    scaled("eutectic2d", [40, 30]),
])
def test_window_equals_full_step(oracle, cfg):
    st = random_state(cfg, 9)
    full = oracle.OracleSim(cfg)
    for k in STATE:
        full.set(k, st[k])
    full.step(3)
    st3 = {k: full.get(k) for k in STATE}
    full.step(1)
    rng = np.random.default_rng(1)
    n = cfg["n"][: cfg["dim"]]
    pts = [tuple(int(rng.integers(0, m)) for m in n) for _ in range(6)]
    pts += [tuple(0 for _ in n), tuple(m - 1 for m in n)]
    for pt in pts:
        ref = window_step(cfg, st3, 3, pt)
        sl = (slice(None),) + tuple(reversed(pt))
        for k in STATE:
            assert np.abs(full.get(k)[sl] - ref[k]).max() <= 1e-15 * max(1.0, np.abs(ref[k]).max()), (pt, k)
