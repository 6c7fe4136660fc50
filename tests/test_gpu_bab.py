"""GPU branch and bound (Sec. 6.2 stratified bounding, Sec. 7.3 warm starts)
against the FP64 branch-and-bound oracle, through the C ABI.

Instances: the 5-8-8-1 net on boxes of half-width 0.3 (5-12 ambiguous
neurons), its output shifted so that the exact minimum (activation-pattern
enumeration) sits at a fraction of the root's relaxation gap above or below
zero, so that deciding the property takes splits.  Weights, boxes and root
bounds are float32 values, the same on both sides.
  FP64 plans: the same tree as the oracle: verdict, batch and node counts,
              and per batch every child's split, algorithm (stratification)
              and lower bound (within 1e-7 relative); upper bounds within
              1e-5 (the library takes x*_0 as float32 and bounds the
              output by interval propagation at the point, rounded outward);
  FP32 plans: the verdict the exact minimum fixes.
"""
import dataclasses

import numpy as np
import pytest

from oracle import asd_bab as B
from oracle import asd_oracle as O
from paper_2101_05844_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _A():
    from paper_2101_05844_amd import asdual as A
    A.lib()
    return A


def f32v(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def instance(seed, frac, eps=0.3):
    """Workload layers, oracle ops, box, c and float32 root bounds of the
    shifted property."""
    w = WL.tiny_config(seed)
    ops = O.ops_from_workload_layers(w.layers)
    centre = (w.l0[0].astype(np.float64) + w.u0[0].astype(np.float64)) / 2
    l0, u0 = f32v(centre - eps), f32v(centre + eps)
    c = w.c[0].astype(np.float64)
    lh, uh = O.interval_bounds(ops, l0, u0)
    m, _ = B.exact_minimum(ops, l0, u0, c, lh[:-1], uh[:-1])
    root = O.solve(O.make_problem(ops, l0, u0, lh[:-1], uh[:-1], c), O.params_from_schedule(w.schedule)).bound
    gap = m - root
    last = w.layers[-1]
    b_new = (last.b.astype(np.float64) + (frac * gap - m) / float(c.sum())).astype(np.float32)
    layers = list(w.layers[:-1]) + [dataclasses.replace(last, b=b_new)]
    ops = O.ops_from_workload_layers(layers)
    lh, uh = O.interval_bounds(ops, l0, u0)
    lo = [np.nextafter(a.astype(np.float32), np.float32(-np.inf)).astype(np.float64) for a in lh[:-1]]
    hi = [np.nextafter(a.astype(np.float32), np.float32(np.inf)).astype(np.float64) for a in uh[:-1]]
    m2, _ = B.exact_minimum(ops, l0, u0, c, lo, hi)
    return w, layers, ops, l0, u0, c, lo, hi, m2


def oracle_params(w, batch):
    tight = O.params_from_schedule(w.schedule)
    loose = O.params_from_schedule(w.schedule)
    loose.as_iters = 0
    return B.BaBParams(loose=loose, tight=tight, batch=batch, max_batches=40)


CASES = [(1000, 0.3), (1002, 0.3), (1005, 0.3), (1002, -0.1), (1005, -0.1), (1009, -0.1)]


@pytest.mark.parametrize("seed,frac", CASES)
def test_fp64_tree_matches_oracle(seed, frac):
    A = _A()
    from paper_2101_05844_amd import bab
    w, layers, ops, l0, u0, c, lo, hi, m = instance(seed, frac)
    ref = B.bab(ops, l0, u0, c, lo, hi, oracle_params(w, 2))
    net = A.Net(layers)
    drv = bab.BranchAndBound(net, A.params_from_schedule(w.schedule, A.ASD_PREC_FP64), batch=2, max_batches=40)
    got = drv.run(l0, u0, c, lo, hi)
    assert got["verdict"] == ref.verdict, (got["verdict"], ref.verdict, m)
    assert (got["verdict"] == "verified") == (m > 0) or got["verdict"] == "unknown"
    assert got["batches"] == ref.batches and got["nodes"] == ref.nodes
    assert abs(got["root"]["lb_tight"] - ref.root["lb_tight"]) <= 1e-7 * (1 + abs(ref.root["lb_tight"]))
    assert len(got["trace"]) == len(ref.trace)
    for gb, rb in zip(got["trace"], ref.trace):
        assert len(gb) == len(rb)
        for (gp, gc, gs, gh, glb, gub), (rp, rc, rs, rh, rlb, rub) in zip(gb, rb):
            assert (gp, gc, gs, gh) == (rp, rc, rs, rh)
            assert abs(glb - rlb) <= 1e-7 * (1 + abs(rlb)), (glb, rlb)
            assert abs(gub - rub) <= 1e-5 * (1 + abs(rub)), (gub, rub)
    if got["verdict"] == "falsified":
        x = got["counterexample"]
        assert float(O.network_output(ops, x) @ c) <= 1e-6


@pytest.mark.parametrize("seed,frac", CASES)
def test_fp32_verdicts(seed, frac):
    A = _A()
    from paper_2101_05844_amd import bab
    w, layers, ops, l0, u0, c, lo, hi, m = instance(seed, frac)
    net = A.Net(layers)
    drv = bab.BranchAndBound(net, A.params_from_schedule(w.schedule, A.ASD_PREC_FP32), batch=2, max_batches=40)
    got = drv.run(l0, u0, c, lo, hi)
    assert got["verdict"] == ("verified" if m > 0 else "falsified"), (got["verdict"], m)
    if got["verdict"] == "falsified":
        assert float(O.network_output(ops, got["counterexample"]) @ c) <= 1e-6


def test_warm_start_and_batches():
    """Cold starts (children from zero duals) follow the oracle's cold tree;
    on this instance the warm starts verify the property where the cold
    ones stop at a subdomain they cannot decide; a wider batch verifies it
    too."""
    A = _A()
    from paper_2101_05844_amd import bab
    w, layers, ops, l0, u0, c, lo, hi, m = instance(1005, 0.3)
    net = A.Net(layers)
    prm = A.params_from_schedule(w.schedule, A.ASD_PREC_FP64)
    warm = bab.BranchAndBound(net, prm, batch=2).run(l0, u0, c, lo, hi)
    cold = bab.BranchAndBound(net, prm, batch=2, warm=False).run(l0, u0, c, lo, hi)
    wide = bab.BranchAndBound(net, prm, batch=8).run(l0, u0, c, lo, hi)
    ref = B.bab(ops, l0, u0, c, lo, hi, dataclasses.replace(oracle_params(w, 2), warm=False))
    assert (cold["verdict"], cold["batches"], cold["nodes"]) == (ref.verdict, ref.batches, ref.nodes)
    assert warm["verdict"] == wide["verdict"] == "verified"
    assert cold["verdict"] in ("verified", "unknown")
    assert warm["trace"][0][0][4] != cold["trace"][0][0][4]
