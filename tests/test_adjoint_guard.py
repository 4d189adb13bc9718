"""The autograd function over the adjoint refuses a backward whose tape (the
network's recording) was overwritten by a later forward or by new weights or
g_scale.  Host logic only: a stand-in network records the calls."""
import torch

from paper_1412_0595_amd.adjoint import vbar


class FakeNet:
    """The Network methods the autograd function calls, without a GPU."""

    def __init__(self):
        self.tape_generation = 0
        self.weight_count = 3
        self.n_instances = 2

    def set_weights_device(self, w):
        self.tape_generation += 1

    def set_gscale(self, s):
        self.tape_generation += 1

    def forward_record(self, pop, n_steps, ckpt_every):
        self.tape_generation += 1
        return torch.full((4,), float(self.tape_generation), dtype=torch.float64)

    def backward(self, dv):
        return torch.ones(self.weight_count), torch.ones(self.n_instances, dtype=torch.float64), None


def test_backward_of_the_latest_forward_runs():
    net = FakeNet()
    w = torch.zeros(3, requires_grad=True)
    s = torch.ones(2, dtype=torch.float64, requires_grad=True)
    vbar(net, w, s, 2, 10, 5).sum().backward()
    assert torch.equal(w.grad, torch.ones(3)) and torch.equal(s.grad, torch.ones(2, dtype=torch.float64))


def test_backward_after_another_forward_raises():
    net = FakeNet()
    w = torch.zeros(3, requires_grad=True)
    s = torch.ones(2, dtype=torch.float64, requires_grad=True)
    first = vbar(net, w, s, 2, 10, 5)
    vbar(net, w, s, 2, 10, 5)
    try:
        first.sum().backward()
    except RuntimeError as e:
        assert "another forward" in str(e)
    else:
        raise AssertionError("expected the stale backward to raise")


def test_backward_after_new_weights_raises():
    net = FakeNet()
    w = torch.zeros(3, requires_grad=True)
    s = torch.ones(2, dtype=torch.float64, requires_grad=True)
    out = vbar(net, w, s, 2, 10, 5)
    net.set_weights_device(torch.zeros(3))
    try:
        out.sum().backward()
    except RuntimeError:
        pass
    else:
        raise AssertionError("expected the stale backward to raise")
