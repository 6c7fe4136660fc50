"""asd_solve_static (the allocation-free solve over the library's static
workspace) against asd_solve on a plan with a workspace of its own: two
calls in a row, the second with a smaller batch, bit-identical bounds and
input minimisers; batches beyond the static workspace are refused."""
import numpy as np
import pytest

from paper_2101_05844_amd import workloads as WL
from tests import helpers as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _A():
    from paper_2101_05844_amd import asdual as A
    A.lib()
    return A


def _batch_prefix(batch, n):
    l0, u0, lh, uh, c = batch
    return (l0[:n].contiguous(), u0[:n].contiguous(), [a[:n].contiguous() for a in lh],
            [a[:n].contiguous() for a in uh], c[:n].contiguous())


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_solve_static_matches_plan_solve(prec):
    A = _A()
    w = H.workloads_small()[2]
    ops, lh, uh = H.oracle_bounds(w)
    batch = H.gpu_batch(w, lh, uh)
    net = A.Net(w.layers)
    prm = A.params_from_schedule(w.schedule, A.ASD_PREC_FP64 if prec == "fp64" else A.ASD_PREC_FP32)
    for n in (w.S, 4):  # two calls in a row, the second smaller
        b = _batch_prefix(batch, n)
        ref, x_ref = A.Plan(net, n, prm).solve(*b, want_x0=True)
        got, x_got = A.solve_static(net, prm, *b, want_x0=True)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (n, got, ref)
        assert torch.equal(x_got, x_ref), n
        assert torch.isfinite(got).all()


def test_solve_static_refuses_oversize_batch():
    A = _A()
    w = WL.cifar_conv_config(S=64)
    net = A.Net(w.layers)
    prm = A.params_from_schedule(w.schedule)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")
    sizes = [w.layers[0].n_in] + [L.n_out for L in w.layers]
    lh = [torch.zeros(w.S, n, device="cuda") for n in sizes[1:-1]]
    with pytest.raises(A.AsdError) as ei:
        A.solve_static(net, prm, t(w.l0), t(w.u0), lh, lh, t(w.c))
    assert ei.value.status == 1  # ASD_EINVAL
    assert "static workspace" in str(ei.value)
