"""Seeded synthetic inputs shared by the oracle tests and the GPU parity
tests.  Random numbers only: nothing here computes any part of the method."""
import numpy as np

from paper_2608_26908_amd.workloads import workload

D2Q9_W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
D3Q19_W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
D3Q27_W = np.array([8 / 27] + [2 / 27] * 6 + [1 / 54] * 12 + [1 / 216] * 8)


def random_state(cfg, seed):
    """A random valid state: phi on the Gibbs simplex with pure-phase cells
    (about half of them) and mixed cells, mu uniform in [-0.3, 0.3], f near
    rest equilibrium (w_k (1 + 0.01 z)), U^{n-1} = 0.01 z."""
    rng = np.random.default_rng(seed)
    dim, N, nc = cfg["dim"], cfg["N"], cfg["nc"]
    shape = tuple(reversed(cfg["n"][:dim]))
    w = D2Q9_W if dim == 2 else (D3Q27_W if cfg.get("lattice") == "D3Q27" else D3Q19_W)
    kind = rng.uniform(size=shape)
    mixed = rng.dirichlet(np.ones(N), size=shape)  # (..., N)
    phi = np.moveaxis(mixed, -1, 0).copy()
    for a in range(N):
        pure = (kind >= 0.5 + 0.5 * a / N) & (kind < 0.5 + 0.5 * (a + 1) / N)
        for b in range(N):
            phi[b][pure] = 1.0 if a == b else 0.0
    mu = rng.uniform(-0.3, 0.3, size=(nc,) + shape)
    f = w.reshape((-1,) + (1,) * dim) * (1 + 0.01 * rng.standard_normal((len(w),) + shape))
    u = 0.01 * rng.standard_normal((dim,) + shape)
    return dict(phi=phi, mu=mu, f=f, u=u)


def busy_config(kind, n, **kw):
    """Small configurations that switch every term of the step on:
    anisotropy, driving force from both mu and a pulled temperature
    gradient, strong buoyancy, drag, walls on one axis and periodicity on
    another."""
    if kind == "binary2d":
        cfg = workload("dendrite2d", n=list(n), periodic=[1, 0], gbeta=[2e-3],
                       delta=[[0, 0.05], [0.05, 0]], dS=[0.3, 0.0], G=0.02, V=0.5, y0=3.0,
                       T_iso=1.0)
    elif kind == "ternary2d":
        cfg = workload("eutectic2d", n=list(n), periodic=[0, 1], gbeta=[2e-3],
                       delta=[[0, 0.0, 0.04], [0.0, 0, 0.03], [0.04, 0.03, 0]],
                       gamma=[[0, 1.3, 1], [1.3, 0, 0.8], [1, 0.8, 0]])
    elif kind == "ternary2d_nc2":
        cfg = workload("eutectic3d", dim=2, n=list(n), periodic=[1, 0], gbeta=[2e-3, -1e-3],
                       chi=[[1.0, 0.2], [0.2, 0.8]], D=[[0.1, 0.0], [0.0, 0.05], [1.0, 0.7]],
                       pull_axis=1, grav_axis=1, y0=3.0, G=0.01)
    elif kind == "binary3d":
        cfg = workload("dendrite3d", n=list(n), periodic=[0, 1, 0], gbeta=[2e-3],
                       delta=[[0, 0.05], [0.05, 0]], dS=[0.3, 0.0], G=0.02, V=0.5, y0=2.0)
    elif kind == "ternary3d_nc2":
        cfg = workload("eutectic3d", n=list(n), periodic=[1, 0, 1], gbeta=[2e-3, -1e-3],
                       delta=[[0, 0.0, 0.04], [0.0, 0, 0.03], [0.04, 0.03, 0]],
                       chi=[[1.0, 0.2], [0.2, 0.8]], D=[[0.1, 0.0], [0.0, 0.05], [1.0, 0.7]],
                       y0=2.0, G=0.01)
    elif kind == "quaternary2d":
        cfg = workload("eutectic4", n=list(n), periodic=[1, 0], gbeta=[2e-3, -1e-3],
                       delta=[[0, 0, 0, 0.04], [0, 0, 0, 0.03], [0, 0, 0, 0.02], [0.04, 0.03, 0.02, 0]],
                       gamma=[[0, 1.3, 1.1, 1], [1.3, 0, 0.9, 0.8], [1.1, 0.9, 0, 1.2], [1, 0.8, 1.2, 0]],
                       chi=[[1.0, 0.2], [0.2, 0.8]], D=[[0.1, 0.0], [0.0, 0.05], [0.02, 0.03], [1.0, 0.7]],
                       y0=3.0, G=0.01)
    elif kind == "quaternary3d":
        cfg = workload("eutectic4_3d", n=list(n), periodic=[1, 0, 1], gbeta=[2e-3, -1e-3],
                       delta=[[0, 0, 0, 0.04], [0, 0, 0, 0.03], [0, 0, 0, 0.02], [0.04, 0.03, 0.02, 0]],
                       chi=[[1.0, 0.2], [0.2, 0.8]], D=[[0.1, 0.0], [0.0, 0.05], [0.02, 0.03], [1.0, 0.7]],
                       y0=2.0, G=0.01)
    else:
        raise KeyError(kind)
    cfg.update(kw)
    return cfg


KINDS = ["binary2d", "ternary2d", "ternary2d_nc2", "binary3d", "ternary3d_nc2"]
KINDS4 = ["quaternary2d", "quaternary3d"]
