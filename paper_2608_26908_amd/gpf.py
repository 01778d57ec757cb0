"""Python binding of libgpf.so (include/gpf.h): argument marshalling only.

Every step of the method runs in the HIP kernels of the library.  PyTorch
supplies device memory (its caching allocator, through the library's
allocation callbacks) and the stream the kernels run on.  There is no
fallback: if libgpf.so is missing or no GPU is present, calls raise.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpf.so")

GPF_OK = 0
STATUS = {0: "GPF_OK", -1: "GPF_ERR_ARG", -2: "GPF_ERR_PARAM", -3: "GPF_ERR_NOMEM",
          -4: "GPF_ERR_DEVICE", -5: "GPF_ERR_NONFINITE", -6: "GPF_ERR_STATE",
          -7: "GPF_ERR_UNSUPPORTED"}
FIELDS = {"phi": 0, "mu": 1, "f": 2, "rho": 3, "u": 4, "c": 5, "T": 6, "flags": 7, "fpost": 8}
REDUCTIONS = {"solute": 0, "mass": 1, "loss": 2}
PRECISION = {"fp64": 0, "fp32": 1}


class GPFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class GridC(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("dx", ctypes.c_double),
                ("periodic_mask", ctypes.c_uint32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class ParamsC(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("precision", ctypes.c_int32), ("potential", ctypes.c_int32),
        ("dt", ctypes.c_double), ("eps", ctypes.c_double), ("tau_pf", ctypes.c_double),
        ("gamma", (ctypes.c_double * 4) * 4), ("delta", (ctypes.c_double * 4) * 4),
        ("chi", (ctypes.c_double * 2) * 2), ("c0", (ctypes.c_double * 2) * 4),
        ("dS", ctypes.c_double * 4), ("mT", (ctypes.c_double * 2) * 4),
        ("T_E", ctypes.c_double), ("T_iso", ctypes.c_double),
        ("D", (ctypes.c_double * 2) * 4),
        ("G", ctypes.c_double), ("V", ctypes.c_double), ("y0", ctypes.c_double),
        ("pull_axis", ctypes.c_int32),
        ("tau_lb", ctypes.c_double), ("rho0", ctypes.c_double),
        ("gbeta", ctypes.c_double * 2), ("c_ref", ctypes.c_double * 2),
        ("grav_axis", ctypes.c_int32), ("grav_sign", ctypes.c_int32),
        ("h_drag", ctypes.c_double), ("W0", ctypes.c_double), ("eta", ctypes.c_double * 4),
        ("lid_u", ctypes.c_double),
        ("init_kind", ctypes.c_int32), ("init_center", ctypes.c_double * 3),
        ("init_radius", ctypes.c_double), ("lam_width", ctypes.c_double),
        ("lam_height", ctypes.c_double), ("mu_inf", ctypes.c_double * 2),
        ("noise_sigma", ctypes.c_double), ("frame_every", ctypes.c_int64),
        ("frame_front", ctypes.c_int64), ("health_every", ctypes.c_int64),
        ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_user", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2608_26908_amd/build.py` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        L.gpf_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(GridC), i32, i32,
                               ctypes.POINTER(ParamsC), ctypes.c_uint64]
        L.gpf_set_stream.argtypes = [vp, vp]
        L.gpf_step.argtypes = [vp, i64]
        L.gpf_step_timed.argtypes = [vp, i64, dp, i32]
        L.gpf_read.argtypes = [vp, i32, dp, ctypes.c_size_t]
        L.gpf_read_device.argtypes = [vp, i32, vp, ctypes.c_size_t]
        L.gpf_write.argtypes = [vp, i32, dp, ctypes.c_size_t]
        L.gpf_reduce.argtypes = [vp, i32, dp]
        L.gpf_set_target.argtypes = [vp, vp, ctypes.c_size_t]
        L.gpf_reduce_noalloc.argtypes = [vp, i32, vp]
        L.gpf_bandwidth_probe.argtypes = [i32, vp, vp, ctypes.POINTER(i64), i32, vp, dp]
        L.gpf_loss_seed_device.argtypes = [vp, vp, ctypes.c_size_t]
        L.gpf_set_param.argtypes = [vp, ctypes.c_char_p, ctypes.c_double]
        L.gpf_set_step_index.argtypes = [vp, i64]
        L.gpf_step_index.restype = i64
        L.gpf_step_index.argtypes = [vp]
        L.gpf_frame_offset.restype = i64
        L.gpf_frame_offset.argtypes = [vp]
        L.gpf_set_frame_offset.argtypes = [vp, i64]
        L.gpf_last_error.restype = ctypes.c_char_p
        L.gpf_last_error.argtypes = [vp]
        L.gpf_status_string.restype = ctypes.c_char_p
        L.gpf_status_string.argtypes = [ctypes.c_int]
        L.gpf_destroy.argtypes = [vp]
        L.gpf_record.argtypes = [vp, i64]
        L.gpf_adjoint.argtypes = [vp, dp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_char_p), i32, dp]
        L.gpf_adjoint_device.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_char_p), i32, dp]
        L.gpf_adjoint_state.argtypes = [vp, i32, dp, ctypes.c_size_t]
        _lib = L
    return _lib


def _fill(dst, src):
    a = np.asarray(src, dtype=float)
    if a.ndim == 1:
        for i, v in enumerate(a):
            dst[i] = float(v)
    else:
        for i in range(a.shape[0]):
            for j in range(a.shape[1]):
                dst[i][j] = float(a[i, j])


def make_grid(cfg):
    g = GridC()
    g.dim = cfg["dim"]
    for a in range(3):
        g.n[a] = int(cfg["n"][a]) if a < cfg["dim"] else 1
    g.dx = float(cfg["dx"])
    g.periodic_mask = sum(1 << a for a in range(cfg["dim"]) if cfg["periodic"][a])
    return g


def make_params(cfg, precision):
    p = ParamsC()
    p.lattice = 0 if cfg["dim"] == 2 else (2 if cfg.get("lattice") == "D3Q27" else 1)
    p.precision = PRECISION[precision]
    p.potential = {"obstacle": 0, "well": 1}[cfg.get("potential", "obstacle")]
    for k in ("dt", "eps", "tau_pf", "T_E", "T_iso", "G", "V", "y0", "tau_lb", "rho0",
              "h_drag", "W0", "lid_u", "init_radius", "lam_width", "lam_height", "noise_sigma"):
        setattr(p, k, float(cfg.get(k, 0.0)))
    p.pull_axis = int(cfg.get("pull_axis", 1))
    p.grav_axis = int(cfg.get("grav_axis", 1))
    p.grav_sign = int(cfg.get("grav_sign", -1))
    p.init_kind = {"seed": 0, "lamellae": 1, "liquid": 2}[cfg.get("init", "seed")]
    for name in ("gamma", "delta", "chi", "c0", "dS", "D", "gbeta", "c_ref", "mu_inf"):
        _fill(getattr(p, name), cfg[name])
    _fill(p.mT, cfg.get("mT", [[0.0, 0.0]] * 4))
    _fill(p.init_center, cfg.get("init_center", [0.0, 0.0, 0.0]))
    _fill(p.eta, cfg.get("eta", [0.0, 0.0, 0.0]))
    p.health_every = int(cfg.get("health_every", 0))
    p.frame_every = int(cfg.get("frame_every", 0))
    p.frame_front = int(cfg.get("frame_front", 0))
    return p


_LIVE = weakref.WeakSet()


@atexit.register
def _close_live():
    # contexts still open at exit give their memory back while torch's
    # allocator is still there
    for s in list(_LIVE):
        s.close()


class Sim:
    """One simulation context of the HIP library.

    cfg: a workload dict (paper_2608_26908_amd.workloads); precision 'fp64'
    or 'fp32' (default: cfg['precision']).  Device memory comes from torch's
    caching allocator unless torch_alloc=False (then hipMalloc); kernels run
    on torch's current stream.  memory_limit (bytes, torch allocator only):
    allocations beyond it fail as if the device were full."""

    def __init__(self, cfg, precision=None, seed=None, torch_alloc=True, health_every=None,
                 memory_limit=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the library runs only on the device")
        L = lib()
        self.cfg = dict(cfg)
        if health_every is not None:
            self.cfg["health_every"] = health_every
        self.precision = precision or cfg.get("precision", "fp64")
        self.dim, self.N, self.nc = cfg["dim"], cfg["N"], cfg["nc"]
        self.n = tuple(int(v) for v in cfg["n"][: self.dim])
        self.Q = 9 if self.dim == 2 else (27 if self.cfg.get("lattice") == "D3Q27" else 19)
        self.cells = int(np.prod(self.n))
        self._grid = make_grid(self.cfg)
        self._params = make_params(self.cfg, self.precision)
        if torch_alloc:
            torch.cuda.init()

            held = self._held = {}

            def _alloc(nbytes, user):
                if memory_limit is not None and self.device_bytes + int(nbytes) > memory_limit:
                    return None
                try:
                    ptr = torch.cuda.caching_allocator_alloc(int(nbytes))
                except torch.cuda.OutOfMemoryError:
                    return None
                held[ptr] = int(nbytes)
                return ptr

            def _free(ptr, user):
                held.pop(ptr, None)
                torch.cuda.caching_allocator_delete(ptr)
            self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
            self._params.dev_alloc, self._params.dev_free = self._cb
        h = ctypes.c_void_p()
        s = cfg.get("seed", 1) if seed is None else seed
        rc = L.gpf_init(ctypes.byref(h), ctypes.byref(self._grid), self.N, self.nc + 1,
                        ctypes.byref(self._params), ctypes.c_uint64(s))
        if rc != GPF_OK:
            raise GPFError(rc, L.gpf_last_error(None).decode())
        self._h = h
        _LIVE.add(self)
        self._check(L.gpf_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    @property
    def device_bytes(self):
        """device memory the context holds through torch's allocator"""
        return sum(getattr(self, "_held", {}).values())

    # -- plumbing ----------------------------------------------------------
    def _check(self, rc):
        if rc != GPF_OK:
            raise GPFError(rc, lib().gpf_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().gpf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return tuple(reversed(self.n))

    def components(self, field):
        return {"phi": self.N, "mu": self.nc, "f": self.Q, "rho": 1, "u": self.dim,
                "c": self.nc, "T": 1, "flags": 1, "fpost": self.Q}[field]

    # -- the C ABI ---------------------------------------------------------
    @property
    def step_index(self):
        return lib().gpf_step_index(self._h)

    @step_index.setter
    def step_index(self, n):
        self._check(lib().gpf_set_step_index(self._h, int(n)))

    @property
    def frame_offset(self):
        return lib().gpf_frame_offset(self._h)

    @frame_offset.setter
    def frame_offset(self, s):
        self._check(lib().gpf_set_frame_offset(self._h, int(s)))

    def checkpoint(self):
        """exact copy of the state (bitwise resumable): fields, step index,
        moving-frame offset"""
        return {k: self.read(k) for k in ("phi", "mu", "u", "fpost")}, self.step_index, self.frame_offset

    def restore(self, ckpt):
        state, n, off = ckpt
        for k, v in state.items():
            self.write(k, v)
        self.step_index = n
        self.frame_offset = off

    def step(self, n=1):
        self._check(lib().gpf_step(self._h, int(n)))

    def step_timed(self, n=1):
        ms = (ctypes.c_double * 2)()
        self._check(lib().gpf_step_timed(self._h, int(n), ms, 2))
        return float(ms[0]), float(ms[1])

    def read(self, field):
        comps = self.components(field)
        out = np.empty(comps * self.cells, dtype=np.float64)
        self._check(lib().gpf_read(self._h, FIELDS[field],
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
        return out.reshape((comps,) + self.shape)

    def read_device(self, field):
        import torch
        dt = torch.float64 if self.precision == "fp64" else torch.float32
        t = torch.empty((self.components(field),) + self.shape, dtype=dt, device="cuda")
        self._check(lib().gpf_read_device(self._h, FIELDS[field], ctypes.c_void_p(t.data_ptr()),
                                          t.numel() * t.element_size()))
        return t

    def write(self, field, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        self._check(lib().gpf_write(self._h, FIELDS[field],
                                    a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.size))

    def reduce(self, which):
        """FP64 total in a fixed order: 'solute' (nc values), 'mass', or
        'loss' (1/2 sum (phi - target)^2 against set_target's target)."""
        out = (ctypes.c_double * 2)()
        self._check(lib().gpf_reduce(self._h, REDUCTIONS[which], out))
        return np.array(out[: self.nc]) if which == "solute" else float(out[0])

    def reduce_noalloc(self, which, out):
        """The total `which` into the FP64 device tensor `out` (nc values for
        'solute', else one), allocation-free and without synchronising."""
        self._check(lib().gpf_reduce_noalloc(self._h, REDUCTIONS[which], ctypes.c_void_p(out.data_ptr())))

    def set_target(self, target):
        """Loss target phi^target (N x grid): kept on the device as FP64 for
        the context's lifetime or until replaced; None clears it."""
        if target is None:
            self._check(lib().gpf_set_target(self._h, None, 0))
            self._target = None
            return
        import torch
        t = torch.as_tensor(target, dtype=torch.float64, device="cuda").contiguous()
        self._check(lib().gpf_set_target(self._h, ctypes.c_void_p(t.data_ptr()), t.numel()))
        self._target = t

    def loss_seed(self):
        """dL/dphi = phi - target (FP64 tensor on the device) at the current state."""
        import torch
        t = torch.empty((self.N,) + self.shape, dtype=torch.float64, device="cuda")
        self._check(lib().gpf_loss_seed_device(self._h, ctypes.c_void_p(t.data_ptr()), t.numel()))
        return t

    def set_param(self, name, value):
        self._check(lib().gpf_set_param(self._h, name.encode(), float(value)))

    # -- adjoint -------------------------------------------------------------
    def record(self, checkpoint_every):
        self._check(lib().gpf_record(self._h, int(checkpoint_every)))
        self.recording = getattr(self, "recording", 0) + 1

    def adjoint(self, dL_dphi, names):
        """FP64 dL/dp for the named parameters, given dL/dphi at the current
        state (a host array, or a GPU tensor: then gpf_adjoint_device reads
        it in place); the adjoint of the recorded initial state is then
        available from adjoint_state()."""
        arr = (ctypes.c_char_p * len(names))(*[n.encode() for n in names])
        out = (ctypes.c_double * max(1, len(names)))()
        if getattr(dL_dphi, "is_cuda", False):
            import torch
            seed = dL_dphi.detach().to(torch.float64).contiguous()
            self._check(lib().gpf_adjoint_device(self._h, ctypes.c_void_p(seed.data_ptr()), seed.numel(),
                                                 arr, len(names), out))
        else:
            seed = np.ascontiguousarray(dL_dphi, dtype=np.float64).ravel()
            self._check(lib().gpf_adjoint(self._h, seed.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          seed.size, arr, len(names), out))
        return np.array(out[: len(names)])

    def adjoint_state(self, field):
        comps = self.components(field)
        out = np.empty(comps * self.cells, dtype=np.float64)
        self._check(lib().gpf_adjoint_state(self._h, FIELDS[field],
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            out.size))
        return out.reshape((comps,) + self.shape)


def _forward_run(ctx, params, sim, initial, names, n_steps, checkpoint_every):
    sim.restore(initial)
    for name, v in zip(names, params.detach().cpu().tolist()):
        sim.set_param(name, v)
    sim.record(checkpoint_every)
    sim.step(n_steps)
    ctx.sim, ctx.names = sim, list(names)
    # the adjoint reverses whatever the context holds: remember which run this is
    ctx.recording, ctx.step_index = sim.recording, sim.step_index
    ctx.param_device, ctx.param_dtype = params.device, params.dtype


def _check_same_run(ctx):
    if ctx.sim.recording != ctx.recording or ctx.sim.step_index != ctx.step_index:
        raise RuntimeError("the simulation was recorded again or stepped since this forward run: "
                           "its adjoint would be that of another trajectory")


def _autograd_functions():
    import torch

    class GPFRun(torch.autograd.Function):
        """phi after n_steps of the coupled step as a differentiable function
        of scalar parameters.  forward: restore the initial checkpoint, set
        the parameters, record and run; backward: the hand-written adjoint
        (gpf_adjoint_device), FP64 parameter gradients."""

        @staticmethod
        def forward(ctx, params, sim, initial, names, n_steps, checkpoint_every):
            _forward_run(ctx, params, sim, initial, names, n_steps, checkpoint_every)
            return sim.read_device("phi")

        @staticmethod
        def backward(ctx, grad_phi):
            _check_same_run(ctx)
            g = ctx.sim.adjoint(grad_phi, ctx.names)
            return (torch.tensor(g, dtype=ctx.param_dtype, device=ctx.param_device),
                    None, None, None, None, None)

    class GPFLoss(torch.autograd.Function):
        """The loss L = 1/2 sum (phi - target)^2 after n_steps (the target set
        with Sim.set_target), FP64 and computed by the library (GPF_LOSS);
        backward seeds the adjoint with dL/dphi = phi - target computed on the
        device (gpf_loss_seed_device)."""

        @staticmethod
        def forward(ctx, params, sim, initial, names, n_steps, checkpoint_every):
            _forward_run(ctx, params, sim, initial, names, n_steps, checkpoint_every)
            return torch.tensor(sim.reduce("loss"), dtype=torch.float64, device=params.device)

        @staticmethod
        def backward(ctx, grad_loss):
            _check_same_run(ctx)
            g = ctx.sim.adjoint(ctx.sim.loss_seed(), ctx.names)
            g = torch.tensor(g, dtype=ctx.param_dtype, device=ctx.param_device)
            return g * grad_loss.to(g.device, g.dtype), None, None, None, None, None

    return GPFRun, GPFLoss


_FUNCS = None


def gpf_run(params, sim, initial, names, n_steps, checkpoint_every):
    """Differentiable run (torch.autograd): phi after n_steps, see GPFRun."""
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _autograd_functions()
    return _FUNCS[0].apply(params, sim, initial, tuple(names), n_steps, checkpoint_every)


def gpf_loss(params, sim, initial, names, n_steps, checkpoint_every):
    """Differentiable loss (torch.autograd): L = 1/2 sum (phi - target)^2
    after n_steps against sim's target, see GPFLoss."""
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _autograd_functions()
    return _FUNCS[1].apply(params, sim, initial, tuple(names), n_steps, checkpoint_every)


PROBES = {"copy19": 0, "pull19": 1, "pull19_zmarch": 2}


def bandwidth_probe(pattern, n, reps=20, buffers=None):
    """Read + write GB/s of an access pattern of the population update
    without its arithmetic (gpf_bandwidth_probe): 'copy19', 'pull19' (one
    thread per cell) or 'pull19_zmarch' (the dominant kernel's launch shape),
    on an n[0] x n[1] x n[2] FP32 grid; buffers: (in, out) torch tensors of
    19 * cells floats each (allocated when None).  Returns (GB/s, in, out)."""
    import torch
    cells = int(n[0]) * int(n[1]) * int(n[2])
    if buffers is None:
        buffers = (torch.randn(19 * cells, device="cuda"), torch.empty(19 * cells, device="cuda"))
    a, b = buffers
    nn = (ctypes.c_int64 * 3)(*[int(v) for v in n])
    out = ctypes.c_double()
    rc = lib().gpf_bandwidth_probe(PROBES[pattern], ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                   nn, int(reps), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                   ctypes.byref(out))
    if rc != GPF_OK:
        raise GPFError(rc, "gpf_bandwidth_probe")
    return out.value, a, b
