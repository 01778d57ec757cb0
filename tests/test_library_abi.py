"""CPU checks of the C-ABI library: it loads, exports every entry point
include/gpf.h declares, its structs match the ctypes mirror byte for byte,
and parameter validation rejects bad input before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpf.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(gpf_\w+)\s*\(", text,
                                 re.M)))


@pytest.fixture(scope="module")
def gpf():
    from paper_2608_26908_amd import gpf as g
    g.lib()
    return g


def test_every_declared_symbol_is_exported(gpf):
    names = _declared()
    assert len(names) >= 12, names
    for n in names:
        assert hasattr(gpf.lib(), n), n


def test_struct_layout_matches_header(gpf, tmp_path):
    """Compile a probe against include/gpf.h and compare sizeof/offsetof
    with the ctypes mirror used by the binding."""
    fields = [f for f, _ in gpf.ParamsC._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "gpf.h"', "int main(void){",
           'printf("%zu %zu\\n", sizeof(gpf_params), sizeof(gpf_grid));']
    for f in fields:
        src.append(f'printf("%zu\\n", offsetof(gpf_params, {f}));')
    for f in ("dim", "n", "dx", "periodic_mask"):
        src.append(f'printf("%zu\\n", offsetof(gpf_grid, {f}));')
    src.append("return 0;}")
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(gpf.ParamsC)
    assert vals[1] == ctypes.sizeof(gpf.GridC)
    for f, v in zip(fields, vals[2:2 + len(fields)]):
        assert getattr(gpf.ParamsC, f).offset == v, f
    for f, v in zip(("dim", "n", "dx", "periodic_mask"), vals[2 + len(fields):]):
        assert getattr(gpf.GridC, f).offset == v, f


def _try_init(gpf, cfg, N=None, K=None, **pk):
    p = gpf.make_params(cfg, "fp64")
    for k, v in pk.items():
        setattr(p, k, v)
    g = gpf.make_grid(cfg)
    h = ctypes.c_void_p()
    rc = gpf.lib().gpf_init(ctypes.byref(h), ctypes.byref(g), N or cfg["N"], K or cfg["nc"] + 1,
                            ctypes.byref(p), 1)
    return rc, gpf.lib().gpf_last_error(None).decode(), h


@pytest.mark.parametrize("change,code,word", [
    (dict(tau_lb=0.5), -2, "tau_lb"),
    (dict(dt=0.0), -2, "dt"),
    (dict(dt=0.5), -2, "bound"),
    (dict(lattice=1), -2, "lattice"),
    (dict(lattice=2), -2, "lattice"),
    (dict(grav_axis=2), -2, "axis"),
    (dict(grav_sign=0), -2, "grav_sign"),
    (dict(W0=0.0), -2, "W0"),
    (dict(precision=7), -1, "precision"),
    (dict(frame_every=-1), -2, "frame_every"),
    (dict(frame_every=10, frame_front=500), -2, "frame_front"),
])
def test_init_rejects_bad_parameters_without_device(gpf, change, code, word):
    from paper_2608_26908_amd.workloads import workload
    rc, msg, h = _try_init(gpf, workload("dendrite2d"), **change)
    assert rc == code and word in msg and not h.value


def test_init_rejects_unsupported_instances(gpf):
    from paper_2608_26908_amd.workloads import workload
    cfg = workload("dendrite2d")
    assert _try_init(gpf, cfg, N=4)[0] == -7
    assert _try_init(gpf, cfg, K=4)[0] == -7
    h = ctypes.c_void_p()
    assert gpf.lib().gpf_init(ctypes.byref(h), None, 2, 2, None, 1) == -1
    assert gpf.lib().gpf_status_string(-5) == b"non-finite state"


def test_binding_fails_loudly_without_gpu(gpf):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2608_26908_amd.workloads import workload
    with pytest.raises(RuntimeError):
        gpf.Sim(workload("dendrite2d"))


def test_moving_frame_needs_walls_on_the_pull_axis(gpf):
    from paper_2608_26908_amd.workloads import workload
    cfg = workload("eutectic2d", periodic=[1, 1])
    rc, msg, h = _try_init(gpf, cfg, frame_every=10, frame_front=20)
    assert rc == -2 and "walls" in msg and not h.value


def test_null_context_is_an_argument_error(gpf):
    """Every entry point that takes a context answers GPF_ERR_ARG for NULL
    (no device work, so this runs without a GPU)."""
    L = gpf.lib()
    names = (ctypes.c_char_p * 1)(b"D")
    out = (ctypes.c_double * 1)()
    seed = (ctypes.c_double * 4)()
    assert L.gpf_adjoint(None, seed, 4, names, 1, out) == -1
    assert L.gpf_adjoint_device(None, ctypes.c_void_p(1), 4, names, 1, out) == -1
    assert L.gpf_adjoint_state(None, 0, seed, 4) == -1
    assert L.gpf_record(None, 4) == -1
    assert L.gpf_step(None, 1) == -1
    assert L.gpf_reduce(None, 2, out) == -1
    assert L.gpf_set_target(None, None, 0) == -1
    assert L.gpf_loss_seed_device(None, ctypes.c_void_p(1), 4) == -1


def test_reduction_enum_has_the_loss():
    """GPF_LOSS is value 2 of gpf_reduction in the header, as the binding uses it."""
    from paper_2608_26908_amd.gpf import REDUCTIONS
    text = open(HEADER).read()
    m = re.search(r"typedef enum \{([^}]*)\} gpf_reduction;", text)
    vals = dict((k.strip(), int(v)) for k, v in (e.split("=") for e in m.group(1).split(",")))
    assert vals == {"GPF_SUM_SOLUTE": 0, "GPF_SUM_MASS": 1, "GPF_LOSS": 2}
    assert REDUCTIONS == {"solute": 0, "mass": 1, "loss": 2}
