"""Sign-class kernels (the bound gradient, and the FP64 final bound of FP32
plans) on nets with exact zero weights and boxes with points, against the
FP64 oracle, through the C ABI.

Those kernels split every (output, input) pair of a layer by the sign of its
weight (w > 0, w < 0, w = 0: a mask always contains the pair) and by the
input's point-box bit (likewise).  Random weights never hit w = 0 and random
boxes are never points, so here a quarter of the weights are exactly zero
and a fifth of the boxes (input coordinates and pre-activation bounds) are
points away from zero.  At fixed duals and masks both sides evaluate the
same function of the given boxes, valid or not.  Shapes: the dense net, the
small conv net and the net with the matrix-core shapes (together every
lane/tap configuration of the weight-gradient kernel, both the tap walk and
the vector-load form of the final sums).
  final bound at imported duals: within 1e-10 of the sum of the magnitudes
      of the terms of d_B (FP64 sums on both sides, different order);
  bound gradient: weight and bias gradients summed over the subproblems
      with mixed-sign factors, box gradients per subproblem, within 1e-9 of
      the summed magnitudes (as the general gradient test).
"""
import dataclasses

import numpy as np
import pytest

from oracle import asd_oracle as O
from tests import helpers as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _A():
    from paper_2101_05844_amd import asdual as A
    A.lib()
    return A


def _workload(wi, seed):
    """Workload wi of the small set with zero weights and point boxes; returns
    the workload, oracle ops and the pre-activation bounds both sides use."""
    w = H.workloads_small()[wi]
    rng = np.random.default_rng(seed)
    layers = []
    for L in w.layers:
        W = L.W.copy()
        W[rng.random(W.shape) < 0.25] = 0.0
        layers.append(dataclasses.replace(L, W=W.astype(np.float32)))
    w = dataclasses.replace(w, layers=layers)
    ops, lh, uh = H.oracle_bounds(w)
    l0, u0 = w.l0.copy(), w.u0.copy()
    pick = rng.random(l0.shape) < 0.2
    mid = H.f32(np.clip((l0 + u0) / 2, 0.05, None))
    w.l0 = np.where(pick, mid, l0).astype(np.float32)
    w.u0 = np.where(pick, mid, u0).astype(np.float32)
    lh2, uh2 = [], []
    for a, b in zip(lh, uh):
        pk = rng.random(a.shape) < 0.2
        val = H.f32(np.abs(b) * 0.5 + 0.01)
        lh2.append(np.where(pk, val, a).astype(np.float32))
        uh2.append(np.where(pk, val, b).astype(np.float32))
    assert any((L.W == 0).any() for L in layers)
    return w, ops, lh2, uh2


def _plan(A, w, ops, lh, uh, prec, max_masks=4):
    probs = H.oracle_problems(w, ops, lh, uh)
    net = A.Net(w.layers)
    prm = A.params_from_schedule(w.schedule, A.ASD_PREC_FP64 if prec == "fp64" else A.ASD_PREC_FP32)
    prm.max_masks = max(prm.max_masks, max_masks)
    plan = A.Plan(net, w.S, prm)
    plan.init(*H.gpu_batch(w, lh, uh))
    return net, plan, probs


@pytest.mark.parametrize("wi", [0, 1, 2])
@pytest.mark.parametrize("n_masks", [0, 3, 8])
def test_final_bound_with_zero_weights_and_points(wi, n_masks):
    """FP32 plan: asd_bound's FP64 final bound at imported float32 duals and
    masks (up to the largest mask count, 8) equals the oracle's d_B at the
    same duals."""
    A = _A()
    w, ops, lh, uh = _workload(wi, 500 + wi)
    net, plan, probs = _plan(A, w, ops, lh, uh, "fp32", max_masks=n_masks)
    rng = np.random.default_rng(510 + 10 * wi + n_masks)
    states = [H.random_integral_state(p, rng, n_masks, scale=0.5) for p in probs]
    H.import_states(plan, probs, states)
    lb = plan.bound().cpu().numpy()
    worst = 0.0
    for s, (p, st) in enumerate(zip(probs, states)):
        d = O.evaluate(p, st)[0]
        sc = H.objective_scale(p, st)
        worst = max(worst, abs(lb[s] - d) / sc)
        assert abs(lb[s] - d) <= 1e-10 * sc, (s, lb[s], d, sc)
    print(w.name, n_masks, "max |lb - d| / sum |terms|:", worst, flush=True)


def _check(got, ref, mag, tol, what):
    bad = np.abs(got - ref) > tol * (1 + mag)
    assert not bad.any(), (what, np.flatnonzero(bad)[:5], got[bad][:5], ref[bad][:5])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("wi", [0, 1, 2])
@pytest.mark.parametrize("n_masks", [3, 8])
def test_bound_gradient_with_zero_weights_and_points(wi, prec, n_masks):
    """asd_bound_grad at imported duals and masks (three, or the largest
    count, 8) against the oracle's Danskin gradient."""
    A = _A()
    w, ops, lh, uh = _workload(wi, 520 + wi)
    net, plan, probs = _plan(A, w, ops, lh, uh, prec, max_masks=n_masks)
    rng = np.random.default_rng(530 + wi + n_masks)
    states = [H.random_integral_state(p, rng, n_masks, scale=0.5) for p in probs]
    H.import_states(plan, probs, states)
    gs = rng.uniform(-1.0, 2.0, w.S)
    dW, db, dl0, du0 = plan.bound_grad(torch.as_tensor(gs))
    torch.cuda.synchronize()
    ora = [O.bound_gradient(p, st) for p, st in zip(probs, states)]
    for k in range(len(ops)):
        for i, got in ((0, dW[k]), (1, db[k])):
            ref = sum(gs[s] * ora[s][i][k] for s in range(w.S))
            mag = sum(abs(gs[s]) * np.abs(ora[s][i][k]) for s in range(w.S))
            _check(got.cpu().numpy().reshape(-1), np.ravel(ref), np.ravel(mag), 1e-9,
                   ("dW" if i == 0 else "db", k))
    for i, got in ((2, dl0), (3, du0)):
        g = got.cpu().numpy()
        for s in range(w.S):
            ref = gs[s] * ora[s][i]
            _check(g[s], ref, np.abs(ref), 1e-9, ("dl0" if i == 2 else "du0", s))
