"""gpf_reduce_noalloc (the allocation-free variant of gpf_reduce, partial sums
in the library's static device array) against gpf_reduce, through the C
ABI: two calls in a row, the second on a smaller context, for every total."""
import ctypes

import numpy as np
import pytest

from inputs import busy_config, random_state
from gpu_helpers import gpu_from

pytestmark = pytest.mark.gpu


def test_reduce_noalloc_equals_reduce_twice_second_smaller():
    import torch
    from paper_2608_26908_amd.gpf import lib
    big = busy_config("ternary3d_nc2", [40, 36, 30])
    small = busy_config("binary2d", [21, 17])
    sims = [gpu_from(big, random_state(big, 3), "fp64"), gpu_from(small, random_state(small, 4), "fp32")]
    assert sims[0].cells > sims[1].cells
    for s in sims:
        s.step(3)
        s.set_target(np.random.default_rng(2).uniform(0, 1, (s.N,) + s.shape))
    torch.cuda.synchronize()
    for s in sims:
        for which in ("solute", "mass", "loss"):
            ref = np.atleast_1d(s.reduce(which))
            out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
            assert lib().gpf_reduce_noalloc(s._h, {"solute": 0, "mass": 1, "loss": 2}[which],
                                            ctypes.c_void_p(out.data_ptr())) == 0
            torch.cuda.synchronize()
            got = out.cpu().numpy()[: ref.size]
            assert np.array_equal(got, ref), (which, got, ref)
            if ref.size == 1:
                assert np.isnan(out.cpu().numpy()[1])
    for s in sims:
        s.close()
