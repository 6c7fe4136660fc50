"""GPU parity, through the C ABI, of nets whose output layer is a
convolution (the sub-networks of eq:primal-intermediates end in the layer
they bound) and of the solver-based intermediate bounds (App. E).

Tolerances: as in test_gpu_parity for solves and fixed-dual evaluation.
Intermediate bounds of an FP64 plan are compared with the oracle's
(fp32_bounds=True: the same outward float32 storage of each layer's bounds)
within 1e-6 * (1 + |bound|): the FP64 solves agree to about 1e-8, and their
bounds, rounded outward to float32 on both sides, then feed the next
layer's solves.  FP32 plans: every bound valid (sampled pre-activations inside), at
least as tight as interval propagation, and within a tenth of the interval
width of the oracle's (a run parts from the FP64 run at near-ties)."""
import numpy as np
import pytest

from oracle import asd_oracle as O
from paper_2101_05844_amd import workloads as WL
from tests import helpers as H
from tests.test_gpu_parity import _A, _eval_all_alternatives, _setup

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# 16 channels into the output convolution: the matrix-core transposed
# convolution; 5 channels: the column kernel
CONV_OUT_MFMA = [WL.ConvSpec(2, 8, 8, 16, 3, 1, 1), WL.ConvSpec(16, 8, 8, 6, 4, 2, 1)]
CONV_OUT_COL = [WL.ConvSpec(2, 7, 9, 5, 3, 1, 1), WL.ConvSpec(5, 7, 9, 6, 4, 2, 1)]
IB_CONV = [WL.ConvSpec(2, 4, 4, 16, 3, 1, 1), WL.ConvSpec(16, 4, 4, 4, 4, 2, 1), WL.DenseSpec(4 * 2 * 2, 9),
           WL.DenseSpec(9, 3)]
IB_DENSE = [WL.DenseSpec(11, 17), WL.DenseSpec(17, 13), WL.DenseSpec(13, 7), WL.DenseSpec(7, 2)]


def conv_out_workloads():
    sched = WL.Schedule(bigm_iters=12, as_iters=14, add_every=5, add_count=2, max_masks=4)
    return [WL.custom_config(CONV_OUT_MFMA, S=7, seed=61, eps=0.05, schedule=sched, max_fixed=4,
                             name="convout-16"),
            WL.custom_config(CONV_OUT_COL, S=9, seed=62, eps=0.05, schedule=sched, max_fixed=3,
                             name="convout-5")]


def ib_workloads():
    sched = WL.Schedule(bigm_iters=30, as_iters=20, add_every=8, add_count=2, max_masks=3)
    return [WL.custom_config(IB_CONV, S=2, seed=63, eps=0.05, schedule=sched, name="ib-conv"),
            WL.custom_config(IB_DENSE, S=2, seed=64, eps=0.2, centre_range=(-1.0, 1.0), schedule=sched,
                             name="ib-dense")]


@pytest.mark.parametrize("wi", [0, 1])
def test_conv_output_layer_fp64_end_to_end(wi):
    """Whole FP64 runs on a net ending in a convolution agree with the
    oracle within 1e-8 (eq:dual-active-set with alpha_n = c over the
    convolution's outputs, b_n^T c over its per-channel bias)."""
    w = conv_out_workloads()[wi]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp64")
    lb = plan.solve(*batch).cpu().numpy()
    prm = O.params_from_schedule(w.schedule)
    for s, p in enumerate(probs):
        r = O.solve(p, prm)
        assert abs(lb[s] - r.bound) <= 1e-8 * max(1.0, abs(r.bound)), (s, lb[s], r.bound)


@pytest.mark.parametrize("wi", [0, 1])
@pytest.mark.parametrize("n_masks", [0, 3])
def test_conv_output_layer_iteration_kernels(wi, n_masks):
    """The FP32 iteration kernels with a convolutional output layer (the
    transposed convolution into the last ReLU layer takes -c as its
    operand), evaluated at imported duals under every kernel choice: f, g,
    x*, z* and the supergradient match the oracle within 1e-5 of their row
    scales."""
    w = conv_out_workloads()[wi]
    A, ops, probs, net, plan, _ = _setup(w)
    rng = np.random.default_rng(700 + 10 * wi + n_masks)
    states = [H.random_integral_state(p, rng, n_masks, scale=0.5) for p in probs]
    H.import_states(plan, probs, states)
    _eval_all_alternatives(A, plan, probs, states, n_masks)


def test_bound_gradient_refuses_a_convolutional_output_layer():
    w = conv_out_workloads()[1]
    A, ops, probs, net, plan, batch = _setup(w)
    plan.solve(*batch)
    with pytest.raises(A.AsdError, match="dense output layer"):
        plan.bound_grad(torch.ones(w.S, dtype=torch.float64, device="cuda"))


def _preacts(ops, xs):
    out, x = [], np.asarray(xs, np.float64).T
    for op in ops:
        x = op.W @ x + op.b[:, None]
        out.append(x.T)
        x = np.maximum(x, 0.0)
    return out


def _gpu_ib(A, w, prec):
    net = A.Net(w.layers)
    prm = A.params_from_schedule(w.schedule, prec)
    t = lambda a: torch.as_tensor(H.f32(a), device="cuda").contiguous()
    lh, uh = net.intermediate_bounds(t(w.l0), t(w.u0), prm)
    return [a.cpu().numpy() for a in lh], [a.cpu().numpy() for a in uh]


@pytest.mark.parametrize("wi", [0, 1])
def test_intermediate_bounds_fp64_match_oracle(wi):
    """asd_intermediate_bounds with FP64 inner solves equals the oracle's
    intermediate_bounds (eq:primal-intermediates per neuron and sign, on the
    sub-network of layers 1..k, combined with interval propagation) for
    every box, layer and neuron."""
    w = ib_workloads()[wi]
    A = _A()
    lh, uh = _gpu_ib(A, w, A.ASD_PREC_FP64)
    ops = O.ops_from_workload_layers(w.layers)
    prm = O.params_from_schedule(w.schedule)
    for d in range(w.S):
        l0, u0 = w.l0[d].astype(np.float64), w.u0[d].astype(np.float64)
        ol, ou = O.intermediate_bounds(ops, l0, u0, prm, fp32_bounds=True)
        ibl, ibu = O.interval_bounds(ops, l0, u0)
        tight = 0
        for k in range(len(ol)):
            assert np.all(np.abs(lh[k][d] - ol[k]) <= 1e-6 * (1 + np.abs(ol[k]))), (d, k, lh[k][d], ol[k])
            assert np.all(np.abs(uh[k][d] - ou[k]) <= 1e-6 * (1 + np.abs(ou[k]))), (d, k, uh[k][d], ou[k])
            tight += int(np.sum(lh[k][d] > ibl[k] + 1e-6) + np.sum(uh[k][d] < ibu[k] - 1e-6))
        assert tight > 0, d


@pytest.mark.parametrize("wi", [0, 1])
def test_intermediate_bounds_fp32_valid(wi):
    """FP32 inner solves: every bound contains the pre-activations of
    sampled inputs, is at least as tight as interval propagation from the
    box, and lies within a tenth of the interval width of the oracle's."""
    w = ib_workloads()[wi]
    A = _A()
    lh, uh = _gpu_ib(A, w, A.ASD_PREC_FP32)
    ops = O.ops_from_workload_layers(w.layers)
    prm = O.params_from_schedule(w.schedule)
    rng = np.random.default_rng(3)
    for d in range(w.S):
        l0, u0 = w.l0[d].astype(np.float64), w.u0[d].astype(np.float64)
        ibl, ibu = O.interval_bounds(ops, l0, u0)
        ol, ou = O.intermediate_bounds(ops, l0, u0, prm)
        xs = l0 + rng.uniform(0, 1, (3000, l0.size)) * (u0 - l0)
        pre = _preacts(ops, np.concatenate([xs, l0[None], u0[None]]))
        for k in range(len(lh)):
            assert np.all(pre[k] >= lh[k][d] - 1e-6) and np.all(pre[k] <= uh[k][d] + 1e-6), (d, k)
            assert np.all(lh[k][d] >= ibl[k] - 1e-6 * (1 + np.abs(ibl[k]))), (d, k)
            assert np.all(uh[k][d] <= ibu[k] + 1e-6 * (1 + np.abs(ibu[k]))), (d, k)
            width = ibu[k] - ibl[k]
            assert np.all(np.abs(lh[k][d] - ol[k]) <= 0.1 * width + 1e-6), (d, k)
            assert np.all(np.abs(uh[k][d] - ou[k]) <= 0.1 * width + 1e-6), (d, k)


def test_intermediate_bounds_two_layer_net_is_interval_propagation():
    """A net with one ReLU layer needs no workspace: its bounds are exactly
    interval propagation (the box-constrained LP)."""
    w = WL.custom_config([WL.DenseSpec(6, 5), WL.DenseSpec(5, 2)], S=3, seed=65)
    A = _A()
    lh, uh = _gpu_ib(A, w, A.ASD_PREC_FP32)
    net = A.Net(w.layers)
    t = lambda a: torch.as_tensor(H.f32(a), device="cuda").contiguous()
    il, iu = net.interval_bounds(t(w.l0), t(w.u0))
    assert len(lh) == 1 and np.array_equal(lh[0], il[0].cpu().numpy()) and np.array_equal(uh[0], iu[0].cpu().numpy())
