"""Host logic of the differentiable Born wrapper, with a stand-in for the
library context (no GPU): the backward pass refuses a context whose window
changed after the forward pass."""
import pytest
import torch

from paper_1801_00819_amd.autograd import BornFn


class _Stub:
    """Linear map y = 2 x with the context's generation counter."""

    device = True

    def __init__(self):
        self.generation = 0

    def apply_born(self, m):
        return 2.0 * m

    def apply_adjoint(self, d):
        return 2.0 * d

    def update(self):
        self.generation += 1


def test_backward_uses_the_forward_window():
    ctx = _Stub()
    m = torch.ones(3, requires_grad=True)
    BornFn.apply(m, ctx).sum().backward()
    assert torch.equal(m.grad, torch.full((3,), 2.0))


def test_backward_refuses_a_changed_window():
    ctx = _Stub()
    m = torch.ones(3, requires_grad=True)
    d = BornFn.apply(m, ctx)
    ctx.update()
    with pytest.raises(RuntimeError, match="window changed"):
        d.sum().backward()
