"""Input checks of the differentiable stencil (CPU): a host tensor, another
dtype or another shape is refused with ValueError before any call reaches
the runtime (the library takes raw device pointers to dense fp32)."""
import pytest
import torch

from paper_1809_05657_amd import autograd as ag


class _NoCalls:
    """Stands in for the runtime: any call is a test failure."""

    def __getattr__(self, name):
        raise AssertionError(f"runtime call {name} reached before the input check")


def _solver(shape=(4, 5, 6)):
    s = ag.Stencil3D.__new__(ag.Stencil3D)
    s.rt, s.shape, s.T, s.ckpt, s.part, s.coef = _NoCalls(), shape, 8, 8, 0, None
    return s


@pytest.mark.parametrize("t,msg", [
    (torch.zeros(4, 5, 6, dtype=torch.float64), "float32"),
    (torch.zeros(4, 5, 7), "shape"),
    (torch.zeros(4, 5, 6), "GPU tensor"),
])
def test_forward_and_backward_refuse_bad_fields(t, msg):
    s = _solver()
    with pytest.raises(ValueError, match=msg):
        s.forward(t, [0.1] * 7)
    with pytest.raises(ValueError, match=msg):
        s.backward(t)


def test_check_field_refuses_non_tensors():
    with pytest.raises(ValueError, match="torch.Tensor"):
        ag.check_field([[1.0]], (1, 1), "x")
