"""ctypes wrapper of the FP64 CPU oracle (oracle/gpfo.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product package never imports this module
and shares no code with it.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

FIELDS = {"phi": 0, "mu": 1, "f": 2, "rho": 3, "u": 4, "c": 5, "T": 6, "active": 7}
PARAMS = {"delta": 0, "tau_pf": 1, "D": 2, "gbeta": 3, "D1": 4, "gbeta1": 5}


def build(verbose=False):
    """Compile liboracle.so with g++ (no fast-math; OpenMP over cells)."""
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", LIB_PATH, os.path.join(HERE, "gpfo.cpp")]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("periodic", ctypes.c_int32 * 3),
        ("N", ctypes.c_int32), ("nc", ctypes.c_int32), ("potential", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("eps", ctypes.c_double),
        ("tau_pf", ctypes.c_double),
        ("gamma", (ctypes.c_double * 4) * 4), ("delta", (ctypes.c_double * 4) * 4),
        ("chi", (ctypes.c_double * 2) * 2), ("c0", (ctypes.c_double * 2) * 4),
        ("dS", ctypes.c_double * 4), ("T_E", ctypes.c_double), ("T_iso", ctypes.c_double),
        ("D", (ctypes.c_double * 2) * 4),
        ("G", ctypes.c_double), ("V", ctypes.c_double), ("y0", ctypes.c_double),
        ("pull_axis", ctypes.c_int32),
        ("tau_lb", ctypes.c_double), ("rho0", ctypes.c_double),
        ("gbeta", ctypes.c_double * 2), ("c_ref", ctypes.c_double * 2),
        ("grav_axis", ctypes.c_int32), ("grav_sign", ctypes.c_int32),
        ("h_drag", ctypes.c_double), ("W0", ctypes.c_double), ("lid_u", ctypes.c_double),
        ("init_kind", ctypes.c_int32), ("init_center", ctypes.c_double * 3),
        ("init_radius", ctypes.c_double), ("lam_width", ctypes.c_double),
        ("lam_height", ctypes.c_double), ("mu_inf", ctypes.c_double * 2),
        ("noise_sigma", ctypes.c_double), ("eta", ctypes.c_double * 4),
        ("lattice_q", ctypes.c_int32), ("frame_every", ctypes.c_int64),
        ("frame_front", ctypes.c_int64), ("mT", (ctypes.c_double * 2) * 4),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        d, i32, i64, u64, vp = (ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_uint64, ctypes.c_void_p)
        dp = P(d)
        L.gpfo_create.restype = vp
        L.gpfo_create.argtypes = [P(_Params), u64]
        L.gpfo_destroy.argtypes = [vp]
        L.gpfo_set_threads.argtypes = [ctypes.c_int]
        L.gpfo_step.argtypes = [vp, i64]
        L.gpfo_step_index.restype = i64
        L.gpfo_step_index.argtypes = [vp]
        L.gpfo_frame_offset.restype = i64
        L.gpfo_frame_offset.argtypes = [vp]
        L.gpfo_cells.restype = i64
        L.gpfo_cells.argtypes = [vp]
        L.gpfo_Q.restype = i32
        L.gpfo_Q.argtypes = [vp]
        L.gpfo_field_count.restype = i64
        L.gpfo_field_count.argtypes = [vp, i32]
        L.gpfo_get.argtypes = [vp, i32, dp]
        L.gpfo_set.argtypes = [vp, i32, dp]
        L.gpfo_total.argtypes = [vp, i32, dp]
        L.gpfo_lattice.restype = i32
        L.gpfo_lattice.argtypes = [i32, P(i32), dp, P(i32)]
        L.gpfo_aniso_ac.restype = d
        L.gpfo_aniso_ac.argtypes = [i32, dp, d]
        L.gpfo_aniso_A.restype = d
        L.gpfo_aniso_A.argtypes = [i32, dp, d, d]
        L.gpfo_aniso_dAdq.argtypes = [i32, dp, d, d, dp]
        L.gpfo_aniso_dAdq_cs.argtypes = [i32, dp, d, d, d, dp]
        L.gpfo_project.restype = i32
        L.gpfo_project.argtypes = [i32, dp, dp]
        L.gpfo_interp_h.argtypes = [i32, dp, dp, dp]
        L.gpfo_feq.argtypes = [i32, d, dp, dp]
        L.gpfo_guo.argtypes = [i32, d, dp, dp, dp]
        L.gpfo_normal.restype = d
        L.gpfo_normal.argtypes = [u64, u64]
        L.gpfo_grand_potential.restype = i32
        L.gpfo_grand_potential.argtypes = [P(_Params), i32, dp, d, d, dp, dp, dp, dp]
        L.gpfo_loss_grad_cs.argtypes = [vp, i64, dp, i32, d, dp, dp]
        L.gpfo_tangent_cs.argtypes = [vp, i64, i32, dp, d, i32, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fill(dst, src, shape):
    a = np.zeros(shape)
    s = np.asarray(src, dtype=float)
    a[tuple(slice(0, k) for k in s.shape)] = s
    if len(shape) == 1:
        for i in range(shape[0]):
            dst[i] = a[i]
    else:
        for i in range(shape[0]):
            for j in range(shape[1]):
                dst[i][j] = a[i, j]


def make_params(cfg):
    """Translate a workload dict (paper_2608_26908_amd.workloads) into the
    oracle's own parameter struct."""
    p = _Params()
    p.dim = cfg["dim"]
    for a in range(3):
        p.n[a] = cfg["n"][a] if a < len(cfg["n"]) else 1
        p.periodic[a] = int(cfg["periodic"][a]) if a < len(cfg["periodic"]) else 1
    p.N, p.nc = cfg["N"], cfg["nc"]
    p.potential = {"obstacle": 0, "well": 1}[cfg.get("potential", "obstacle")]
    for k in ("dx", "dt", "eps", "tau_pf", "T_E", "T_iso", "G", "V", "y0", "tau_lb", "rho0",
              "h_drag", "W0", "lid_u", "init_radius", "lam_width", "lam_height", "noise_sigma"):
        setattr(p, k, float(cfg.get(k, 0.0)))
    p.pull_axis = cfg.get("pull_axis", 1)
    p.grav_axis = cfg.get("grav_axis", 1)
    p.grav_sign = cfg.get("grav_sign", -1)
    p.init_kind = {"seed": 0, "lamellae": 1, "liquid": 2}[cfg.get("init", "seed")]
    _fill(p.gamma, cfg["gamma"], (4, 4))
    _fill(p.delta, cfg["delta"], (4, 4))
    _fill(p.chi, cfg["chi"], (2, 2))
    _fill(p.c0, cfg["c0"], (4, 2))
    _fill(p.dS, cfg["dS"], (4,))
    _fill(p.D, cfg["D"], (4, 2))
    _fill(p.gbeta, cfg["gbeta"], (2,))
    _fill(p.c_ref, cfg["c_ref"], (2,))
    _fill(p.init_center, cfg.get("init_center", [0, 0, 0]), (3,))
    _fill(p.mu_inf, cfg["mu_inf"], (2,))
    _fill(p.eta, cfg.get("eta", [0.0, 0.0, 0.0]), (4,))
    _fill(p.mT, cfg.get("mT", [[0.0, 0.0]] * 4), (4, 2))
    p.lattice_q = 27 if cfg.get("lattice") == "D3Q27" else 0
    p.frame_every = int(cfg.get("frame_every", 0))
    p.frame_front = int(cfg.get("frame_front", 0))
    return p


class OracleSim:
    """One oracle simulation (FP64 state on the host)."""

    def __init__(self, cfg, seed=None, threads=None):
        self.cfg = dict(cfg)
        self._p = make_params(cfg)
        L = lib()
        if threads is not None:
            L.gpfo_set_threads(int(threads))
        s = cfg.get("seed", 1) if seed is None else seed
        self._h = L.gpfo_create(ctypes.byref(self._p), ctypes.c_uint64(s))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self.dim, self.N, self.nc = cfg["dim"], cfg["N"], cfg["nc"]
        self.n = tuple(cfg["n"][:self.dim])
        self.Q = L.gpfo_Q(self._h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().gpfo_destroy(self._h)
            self._h = None

    @property
    def step_index(self):
        return lib().gpfo_step_index(self._h)

    @property
    def frame_offset(self):
        return lib().gpfo_frame_offset(self._h)

    @property
    def shape(self):
        return tuple(reversed(self.n))

    def step(self, n=1):
        lib().gpfo_step(self._h, int(n))

    def get(self, field):
        fid = FIELDS[field]
        cnt = lib().gpfo_field_count(self._h, fid)
        out = np.empty(cnt)
        if lib().gpfo_get(self._h, fid, _dp(out)) != 0:
            raise ValueError(field)
        return out.reshape((-1,) + self.shape)

    def set(self, field, arr):
        fid = FIELDS[field]
        a = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        if a.size != lib().gpfo_field_count(self._h, fid):
            raise ValueError("size mismatch for " + field)
        if lib().gpfo_set(self._h, fid, _dp(a)) != 0:
            raise ValueError(field)

    def total(self, which):
        out = np.zeros(2)
        lib().gpfo_total(self._h, {"solute": 0, "mass": 1}[which], _dp(out))
        return out[: self.nc] if which == "solute" else out[0]

    def loss_grad_cs(self, nsteps, target, param, h=1e-30):
        t = np.ascontiguousarray(target, dtype=np.float64).ravel()
        loss, grad = ctypes.c_double(), ctypes.c_double()
        rc = lib().gpfo_loss_grad_cs(self._h, int(nsteps), _dp(t), PARAMS[param], h,
                                     ctypes.byref(loss), ctypes.byref(grad))
        if rc != 0:
            raise ValueError(param)
        return loss.value, grad.value

    def tangent_cs(self, nsteps, field, direction, out_field, h=1e-30):
        d = np.ascontiguousarray(direction, dtype=np.float64).ravel()
        cnt = lib().gpfo_field_count(self._h, FIELDS[out_field])
        out = np.empty(cnt)
        rc = lib().gpfo_tangent_cs(self._h, int(nsteps), FIELDS[field], _dp(d), h,
                                   FIELDS[out_field], _dp(out))
        if rc != 0:
            raise ValueError(field)
        return out.reshape((-1,) + self.shape)


# ----- pointwise functions --------------------------------------------------

def _q(dim, Q):
    return Q if Q else (9 if dim == 2 else 19)


def lattice(dim, Q=None):
    """(c, w, opp) of D2Q9 (dim 2), D3Q19 (dim 3) or D3Q27 (dim 3, Q = 27)."""
    c = np.zeros((27, 3), dtype=np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, dtype=np.int32)
    Q = lib().gpfo_lattice(_q(dim, Q), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w),
                           opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return c[:Q, :dim].copy(), w[:Q].copy(), opp[:Q].copy()


def aniso_ac(q, delta):
    q = np.ascontiguousarray(q, dtype=float)
    return lib().gpfo_aniso_ac(len(q), _dp(q), delta)


def aniso_A(q, gamma, delta):
    q = np.ascontiguousarray(q, dtype=float)
    return lib().gpfo_aniso_A(len(q), _dp(q), gamma, delta)


def aniso_dAdq(q, gamma, delta):
    q = np.ascontiguousarray(q, dtype=float)
    out = np.zeros(len(q))
    lib().gpfo_aniso_dAdq(len(q), _dp(q), gamma, delta, _dp(out))
    return out


def aniso_dAdq_cs(q, gamma, delta, h=1e-30):
    q = np.ascontiguousarray(q, dtype=float)
    out = np.zeros(len(q))
    lib().gpfo_aniso_dAdq_cs(len(q), _dp(q), gamma, delta, h, _dp(out))
    return out


def project(v):
    v = np.ascontiguousarray(v, dtype=float)
    out = np.zeros(len(v))
    lib().gpfo_project(len(v), _dp(v), _dp(out))
    return out


def interp_h(phi):
    phi = np.ascontiguousarray(phi, dtype=float)
    N = len(phi)
    h, dh = np.zeros(N), np.zeros(N * N)
    lib().gpfo_interp_h(N, _dp(phi), _dp(h), _dp(dh))
    return h, dh.reshape(N, N)


def feq(dim, rho, u, Q=None):
    u = np.ascontiguousarray(u, dtype=float)
    out = np.zeros(27)
    lib().gpfo_feq(_q(dim, Q), rho, _dp(u), _dp(out))
    return out[: _q(dim, Q)]


def guo(dim, tau, u, F, Q=None):
    u = np.ascontiguousarray(u, dtype=float)
    F = np.ascontiguousarray(F, dtype=float)
    out = np.zeros(27)
    lib().gpfo_guo(_q(dim, Q), tau, _dp(u), _dp(F), _dp(out))
    return out[: _q(dim, Q)]


def normal(seed, j):
    return lib().gpfo_normal(seed, j)


def grand_potential(cfg, a, mu, T, h=1e-30):
    """(psi^a, d psi^a/d mu by complex step, d psi^a/d T by complex step,
    C^a(mu)) at chemical potential mu (nc values) and temperature T."""
    prm = make_params(cfg)
    nc = cfg["nc"]
    mu = np.ascontiguousarray(mu, dtype=float)
    psi, dT = ctypes.c_double(), ctypes.c_double()
    dmu, conc = np.zeros(nc), np.zeros(nc)
    rc = lib().gpfo_grand_potential(ctypes.byref(prm), a, _dp(mu), float(T), h, ctypes.byref(psi),
                                    _dp(dmu), ctypes.byref(dT), _dp(conc))
    if rc != 0:
        raise ValueError("gpfo_grand_potential: invalid arguments")
    return psi.value, dmu, dT.value, conc
