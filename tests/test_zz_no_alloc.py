"""snn_backward_noalloc, the backward pass with its scratch in the library's
fixed device array (for callers that cannot allocate), against snn_backward
on the same recording, through the C ABI: two calls in a row, the second on
a smaller recording, each against the existing entry point's output; and the
size limit."""
import numpy as np
import pytest

from paper_1412_0595_amd import netgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_0595_amd import snn as S
    S.load()
    return S


def say(*a):
    print(*a, flush=True)


def _loss_grad(vbar, spec):
    """dL/dVbar of L = sum_b mean_j (Vbar_bj - y_bj)^2."""
    y = np.concatenate(spec["target"])
    sizes = [inst["pops"][2]["n"] for inst in spec["instances"]]
    w = np.concatenate([np.full(n, 1.0 / n) for n in sizes])
    return 2 * w * (vbar - y)


def _recorded(snn, n_inst, scale, T, K):
    import torch
    spec = netgen.make_config(5, n_instances=n_inst, scale=scale)
    net = snn.Network(spec, record_vbar=("C",))
    vbar = net.forward_record(2, T, K)
    dv = torch.tensor(_loss_grad(vbar.cpu().numpy(), spec), dtype=torch.float64, device=net.device)
    return net, dv


def _check_against_backward(snn, net, dv, label):
    """The no-alloc call into outputs pre-filled with NaN (so that a missed
    clear shows) against snn_backward: dL/dg bit for bit (each synapse is
    accumulated by one lane in a fixed order), dL/dg_scale within 1e-12
    relative (its partial sums meet in double atomics, whose order varies)."""
    import torch
    dg0, ds0, mism = net.backward(dv, check=True)
    assert mism == 0
    dg1 = torch.full((net.weight_count,), float("nan"), dtype=torch.float32, device=net.device)
    ds1 = torch.full((net.n_instances,), float("nan"), dtype=torch.float64, device=net.device)
    net.backward_noalloc(dv, dg1, ds1)
    torch.cuda.synchronize()
    a, b = dg0.cpu().numpy(), dg1.cpu().numpy()
    s0, s1 = ds0.cpu().numpy(), ds1.cpu().numpy()
    rel = np.max(np.abs(s1 - s0) / np.abs(s0))
    say(f"  {label}: {a.size} weights, dL/dg identical {np.array_equal(a, b)} "
        f"(nonzero {int(np.count_nonzero(a))}); dL/dg_scale max relative difference {rel:.1e}")
    assert np.array_equal(a, b)
    assert np.all(np.isfinite(s1)) and rel <= 1e-12


def test_noalloc_backward_matches_backward_twice(snn):
    say("case: no-alloc backward, 4 instances at scale 0.3 (T 300, K 60), then 2 at scale 0.15 (T 200, K 40)")
    net1, dv1 = _recorded(snn, 4, 0.3, 300, 60)
    _check_against_backward(snn, net1, dv1, "first call")
    net2, dv2 = _recorded(snn, 2, 0.15, 200, 40)
    _check_against_backward(snn, net2, dv2, "second call, smaller recording")
    # the first net again, after the smaller call left its contents behind
    _check_against_backward(snn, net1, dv1, "first net again")
    net1.close()
    net2.close()


def test_noalloc_backward_rejects_oversized_recording(snn):
    """A recording whose tape exceeds the fixed array is refused with
    SNN_ERANGE before any work is enqueued; snn_backward still runs it."""
    import torch
    say("case: no-alloc backward beyond its scratch size (K = 4400 on 240 loss neurons)")
    net, dv = _recorded(snn, 4, 0.3, 4400, 4400)
    n_loss = dv.numel()
    need = 256 + 8 * n_loss * (4400 * (4 + 2 * 2) + 4 + 2)
    assert need > snn.NOALLOC_SCRATCH_BYTES
    dg = torch.zeros(net.weight_count, dtype=torch.float32, device=net.device)
    ds = torch.zeros(net.n_instances, dtype=torch.float64, device=net.device)
    with pytest.raises(snn.SNNError) as e:
        net.backward_noalloc(dv, dg, ds)
    assert e.value.code == snn.SNN_ERANGE
    say(f"  refused: {e.value}")
    net.backward(dv)
    torch.cuda.synchronize()
    net.close()
