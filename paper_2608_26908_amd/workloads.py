"""Synthetic workloads of the coupled phase-field / lattice-Boltzmann step.

Parameter values only: this module holds none of the method's arithmetic and
is the one place that both the HIP library's tests and the CPU oracle's tests
take their inputs from.  Each workload is a plain dict; sizes, phase counts,
lattices and physical constants follow the paper's Case 1-3 settings
(App. B: gamma = 1, D_solid = 0, D_liquid = 1, eps / dx = 4, T_eq = 1) scaled
to synthetic grids.  Where the paper is silent the value is a stated reading:
  * thermodynamics: parabolic grand potentials with susceptibility chi = 1,
    C^a(mu) = c0[a] + chi mu; a binary dendrite has c0 = (k, 1) so that the
    equilibrium chemical potential is 0, and a far-field supersaturation
    Delta ("undercooling") gives mu_inf = -Delta (1 - k) / chi;
  * eutectics with the App. B data (three components): equilibrium
    compositions c^eq; the coexistence-line slopes m^eq read as dc/dT (their
    zero entries rule out dT/dc).  The solid-state slopes m^eq_{a-a} move each
    solid's parabola centre, c0_a(T) = c^eq_a + m^eq_{a-a} (T - T_E) (key mT,
    liquid 0); the solid-liquid slopes fix the entropy offsets through the
    liquid composition at a-l coexistence, which moves by m^eq_{a-l} (T - T_E)
    when dS_a = m^eq_{a-l} . chi^{-1} (c^eq_a - c^eq_l): 0.32 for all three
    solids (chi = I);
  * the binary eutectic (no slopes in the paper): a symmetric binary (0.2,
    0.8, liquid 0.5) with dS = 0.25 and compositions independent of T;
  * drag constant h = 2.757 and interface thickness W0 = eps / dx;
  * noise: sigma = 1e-3 on mu in every cell, drawn from the seed.
"""
import copy

# D2Q9 / D3Q19 follow from dim.  Phase order: solids first, liquid last.

_COMMON = dict(
    potential="obstacle", dx=1.0, dt=0.1, eps=4.0, tau_pf=1.0,
    chi=[[1.0, 0.0], [0.0, 1.0]], T_E=1.0, T_iso=1.0,
    G=0.0, V=0.0, y0=0.0, rho0=1.0, h_drag=2.757, W0=4.0, lid_u=0.0,
    noise_sigma=1e-3, seed=1, lam_width=0.0, lam_height=0.0,
    init_center=[0.0, 0.0, 0.0], init_radius=0.0,
    eta=[0.0, 0.0, 0.0],  # shrinkage (rho_a - rho_liq) / rho_liq per phase; the paper's 1.2 / 1.0 gives 0.2
    mT=[[0.0, 0.0]] * 4,  # d c0_a / dT per phase and solute (0: compositions independent of T)
)

WORKLOADS = {
    # 2D binary-alloy single dendrite, FP64 (Case 1 shape)
    "dendrite2d": dict(
        _COMMON, dim=2, n=[128, 128], periodic=[0, 0], N=2, nc=1,
        gamma=[[0, 1], [1, 0]], delta=[[0, 0.02], [0.02, 0]],
        c0=[[0.15], [1.0]], dS=[0.0, 0.0], D=[[0.0], [1.0]],
        tau_lb=0.8, gbeta=[1e-5], c_ref=[0.5325], grav_axis=1, grav_sign=-1,
        pull_axis=1, init="seed", init_center=[63.5, 63.5, 0.0], init_radius=8.0,
        mu_inf=[-0.4675], steps=1000, precision="fp64"),
    # 2D eutectic directional solidification (Case 3 shape, binary eutectic)
    "eutectic2d": dict(
        _COMMON, dim=2, n=[1024, 512], periodic=[1, 0], N=3, nc=1,
        gamma=[[0, 1, 1], [1, 0, 1], [1, 1, 0]], delta=[[0] * 3] * 3,
        c0=[[0.2], [0.8], [0.5]], dS=[0.25, 0.25, 0.0], D=[[0.0], [0.0], [1.0]],
        G=1e-4, V=1e-3, y0=20.0, pull_axis=1,
        tau_lb=0.7, gbeta=[5e-6], c_ref=[0.5], grav_axis=1, grav_sign=-1,
        init="lamellae", lam_width=16.0, lam_height=20.0,
        mu_inf=[0.0], steps=20000, precision="fp32"),
    # 3D binary-alloy dendrite with natural convection, FP32 storage
    "dendrite3d": dict(
        _COMMON, dim=3, n=[256, 256, 256], periodic=[0, 0, 0], N=2, nc=1,
        gamma=[[0, 1], [1, 0]], delta=[[0, 0.03], [0.03, 0]],
        c0=[[0.15], [1.0]], dS=[0.0, 0.0], D=[[0.0], [1.0]],
        tau_lb=0.75, gbeta=[1e-5], c_ref=[0.575], grav_axis=2, grav_sign=-1,
        pull_axis=2, init="seed", init_center=[128.0, 128.0, 64.0], init_radius=6.0,
        mu_inf=[-0.425], steps=5000, precision="fp32"),
    # adjoint parameter inversion on a 2D dendrite (forward FP32, FP64 grads)
    "adjoint2d": dict(
        _COMMON, dim=2, n=[256, 256], periodic=[0, 0], N=2, nc=1,
        gamma=[[0, 1], [1, 0]], delta=[[0, 0.02], [0.02, 0]],
        c0=[[0.15], [1.0]], dS=[0.0, 0.0], D=[[0.0], [1.0]],
        tau_lb=0.8, gbeta=[1e-5], c_ref=[0.5325], grav_axis=1, grav_sign=-1,
        pull_axis=1, init="seed", init_center=[127.5, 127.5, 0.0], init_radius=8.0,
        mu_inf=[-0.4675], steps=2000, checkpoint_every=100, precision="fp32",
        target=dict(delta=0.025, tau_pf=1.2, gbeta=2e-5)),
    # 3D ternary eutectic with convection, FP32
    "eutectic3d": dict(
        _COMMON, dim=3, n=[192, 192, 384], periodic=[1, 1, 0], N=3, nc=2,
        gamma=[[0, 1, 1], [1, 0, 1], [1, 1, 0]], delta=[[0] * 3] * 3,
        c0=[[0.6, 0.2], [0.2, 0.6], [1.0 / 3.0, 1.0 / 3.0]],
        mT=[[1.6, 0.0], [0.0, 1.6], [0.0, 0.0]],
        dS=[0.32, 0.32, 0.0],
        D=[[0.0, 0.0], [0.0, 0.0], [1.0, 1.0]],
        G=5e-5, V=5e-4, y0=30.0, pull_axis=2,
        tau_lb=0.75, gbeta=[5e-6, -2.5e-6], c_ref=[1.0 / 3.0, 1.0 / 3.0],
        grav_axis=2, grav_sign=-1,
        init="lamellae", lam_width=12.0, lam_height=30.0,
        mu_inf=[0.0, 0.0], steps=10000, precision="fp32"),
    # Case 3: three solids (alpha, beta, gamma) and the liquid, three
    # components; App. B equilibrium compositions and coexistence slopes;
    # the regular alpha-beta-gamma pattern, four periods across (4 lambda x 700)
    "eutectic4": dict(
        _COMMON, dim=2, n=[144, 700], periodic=[1, 0], N=4, nc=2,
        gamma=[[0, 1, 1, 1], [1, 0, 1, 1], [1, 1, 0, 1], [1, 1, 1, 0]], delta=[[0] * 4] * 4,
        c0=[[0.6, 0.2], [0.2, 0.6], [0.2, 0.2], [1.0 / 3.0, 1.0 / 3.0]],
        mT=[[1.6, 0.0], [0.0, 1.6], [-1.6, -1.6], [0.0, 0.0]],
        dS=[0.32, 0.32, 0.32, 0.0],
        D=[[0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [1.0, 1.0]],
        G=1e-4, V=1e-3, y0=30.0, pull_axis=1,
        tau_lb=0.7, gbeta=[5e-6, -2.5e-6], c_ref=[1.0 / 3.0, 1.0 / 3.0],
        grav_axis=1, grav_sign=-1,
        init="lamellae", lam_width=12.0, lam_height=30.0,
        mu_inf=[0.0, 0.0], steps=20000, precision="fp32"),
    # the same four-phase system in 3D (lamellae extruded along y), FP32
    "eutectic4_3d": dict(
        _COMMON, dim=3, n=[192, 192, 384], periodic=[1, 1, 0], N=4, nc=2,
        gamma=[[0, 1, 1, 1], [1, 0, 1, 1], [1, 1, 0, 1], [1, 1, 1, 0]], delta=[[0] * 4] * 4,
        c0=[[0.6, 0.2], [0.2, 0.6], [0.2, 0.2], [1.0 / 3.0, 1.0 / 3.0]],
        mT=[[1.6, 0.0], [0.0, 1.6], [-1.6, -1.6], [0.0, 0.0]],
        dS=[0.32, 0.32, 0.32, 0.0],
        D=[[0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [1.0, 1.0]],
        G=5e-5, V=5e-4, y0=30.0, pull_axis=2,
        tau_lb=0.75, gbeta=[5e-6, -2.5e-6], c_ref=[1.0 / 3.0, 1.0 / 3.0],
        grav_axis=2, grav_sign=-1,
        init="lamellae", lam_width=16.0, lam_height=30.0,
        mu_inf=[0.0, 0.0], steps=10000, precision="fp32"),
}


def workload(name, **overrides):
    """A deep copy of a named workload with keys overridden."""
    cfg = copy.deepcopy(WORKLOADS[name])
    cfg["name"] = name
    cfg.update(copy.deepcopy(overrides))
    return cfg


def scaled(name, n, **overrides):
    """The named workload on a smaller grid `n`; seed centres and lamella
    heights keep their relative position, so the structure of the full-size
    input (seed in the melt, lamellae at the bottom) is preserved."""
    cfg = workload(name, **overrides)
    full = cfg["n"]
    cfg["n"] = list(n)
    if cfg.get("init") == "seed" and "init_center" not in overrides:
        c = list(cfg["init_center"])
        for a in range(cfg["dim"]):
            c[a] = (c[a] + 0.5) * n[a] / full[a] - 0.5
        cfg["init_center"] = c
    return cfg


def cells(cfg):
    c = 1
    for a in range(cfg["dim"]):
        c *= cfg["n"][a]
    return c
