"""Argument checks of the Python binding and the batch (CPU).

Every device array is validated on the host before its address reaches the
library: a host tensor, a wrong element type, a non-contiguous view or one
shorter than the call needs raises ValueError, so no kernel ever runs on it.
GPU-resident tensors cannot be made here; a stand-in object that reports
itself as a GPU tensor exercises the type, layout and size checks (each is
rejected before the library is called, so its address is never used).
"""
import os

import numpy as np
import pytest
import torch

import meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2508_17917_amd", "libdgmi.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdgmi.so not built")


class FakeDevice:
    """Looks like a GPU tensor to the binding's checks."""

    is_cuda = True

    def __init__(self, shape, dtype=torch.float64, contiguous=True, strides=None):
        self.shape = tuple(shape)
        self.dtype = dtype
        self._contig = contiguous
        self._strides = strides

    def data_ptr(self):
        return 0

    def numel(self):
        return int(np.prod(self.shape))

    def is_contiguous(self):
        return self._contig

    def dim(self):
        return len(self.shape)

    def stride(self, i):
        if self._strides is not None:
            return self._strides[i]
        return int(np.prod(self.shape[i + 1:]))


@pytest.fixture(scope="module")
def host_ctx():
    from paper_2508_17917_amd import Solver
    s = Solver(3, mg.periodic_square(2, 2, 1.0, 1.0), device=False)
    yield s
    s.close()


def state(s, **kw):
    return FakeDevice((s.K, 4, s.Np), **kw)


def test_state_arguments_are_checked(host_ctx):
    from paper_2508_17917_amd import _lib as L
    s = host_ctx
    good = state(s)
    cases = {
        "host tensor": torch.zeros((s.K, 4, s.Np), dtype=torch.float64),
        "float32": state(s, dtype=torch.float32),
        "non-contiguous": state(s, contiguous=False),
        "too short": FakeDevice((s.K - 1, 4, s.Np)),
        "not a tensor": np.zeros((s.K, 4, s.Np)),
    }
    for name, bad in cases.items():
        with pytest.raises(ValueError):
            L.dg_rhs(s.h, bad, good)
        with pytest.raises(ValueError):
            L.dg_rhs(s.h, good, bad)
        with pytest.raises(ValueError):
            L.dg_rk_step(s.h, good, bad, 1e-3)
        with pytest.raises(ValueError):
            L.dg_rk_steps(s.h, bad, good, 2, 1e-3)
        with pytest.raises(ValueError):
            L.dg_rk_stage(s.h, good, bad, good, 0.0, 1.0, 1e-3)
        with pytest.raises(ValueError):
            L.dg_force(s.h, bad)
        with pytest.raises(ValueError):
            L.dg_cfl_time_step(s.h, bad)
        with pytest.raises(ValueError):
            L.dg_autotune(s.h, bad)


def test_force_buffers_are_sized(host_ctx):
    from paper_2508_17917_amd import _lib as L
    s = host_ctx
    good = state(s)
    with pytest.raises(ValueError, match="needs 15"):
        L.dg_rk_steps(s.h, good, state(s), 5, 1e-3, force=FakeDevice((14,)))
    with pytest.raises(ValueError):
        L.dg_force_device(s.h, good, FakeDevice((2,)))
    with pytest.raises(ValueError):
        L.dg_force_device(s.h, good, FakeDevice((3,), dtype=torch.float32))


def test_valid_arguments_reach_the_library(host_ctx):
    """Arguments that pass the checks reach the library, which refuses the
    call on a context without device set-up (no kernel runs)."""
    from paper_2508_17917_amd import _lib as L
    s = host_ctx
    with pytest.raises(L.DGError) as e:
        L.dg_rhs(s.h, state(s), state(s), stream=0)
    assert e.value.code == L.DG_ESTATE


def test_row_arrays_are_checked():
    from paper_2508_17917_amd import _lib as L
    good = FakeDevice((100, 28), dtype=torch.float32)
    assert L._rows(good, 100, 28, "X")[1] == 28
    with pytest.raises(ValueError):
        L._rows(FakeDevice((99, 28), dtype=torch.float32), 100, 28, "X")
    with pytest.raises(ValueError):
        L._rows(FakeDevice((100, 27), dtype=torch.float32), 100, 28, "X")
    with pytest.raises(ValueError):
        L._rows(FakeDevice((100, 28)), 100, 28, "X")                       # float64
    with pytest.raises(ValueError):
        L._rows(FakeDevice((100, 28), dtype=torch.float32, strides=(28, 2)), 100, 28, "X")
    with pytest.raises(ValueError):
        L._rows(torch.zeros((100, 28), dtype=torch.float32), 100, 28, "X")  # host
    with pytest.raises(ValueError):
        L.dg_mlp_forward(None, good, good)                                  # unknown network


def test_batch_rejects_a_repeated_context(host_ctx):
    from paper_2508_17917_amd import _lib as L
    with pytest.raises(L.DGError) as e:
        L.dg_batch_create([host_ctx.h, host_ctx.h])
    assert e.value.code == L.DG_EINVAL
    assert "twice" in str(e.value)
