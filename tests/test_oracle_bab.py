"""Pins of the branch-and-bound oracle (Sec. 6.2) against the exact minimum
of small networks (every activation pattern of the ambiguous neurons, one
linear program each), sampled network outputs and the Anderson LP."""
import numpy as np
import pytest

from oracle import asd_bab as B
from oracle import asd_oracle as O
from oracle import lp
from paper_2101_05844_amd import workloads as WL


def tiny(seed):
    w = WL.tiny_config(seed)
    ops = O.ops_from_workload_layers(w.layers)
    l0, u0 = w.l0[0].astype(np.float64), w.u0[0].astype(np.float64)
    lh, uh = O.interval_bounds(ops, l0, u0)
    return w, ops, l0, u0, w.c[0].astype(np.float64), lh[:-1], uh[:-1]


def bab_params(w):
    tight = O.params_from_schedule(w.schedule)
    loose = O.params_from_schedule(w.schedule)
    loose.as_iters = 0
    return B.BaBParams(loose=loose, tight=tight, batch=2, max_batches=40)


@pytest.mark.parametrize("seed", [1000, 1001, 1002, 1003])
def test_exact_minimum_against_sampling_and_lp(seed):
    w, ops, l0, u0, c, lh, uh = tiny(seed)
    m, x = B.exact_minimum(ops, l0, u0, c, lh, uh)
    # attained: the network at the argmin gives the value
    assert abs(float(O.network_output(ops, x) @ c) - m) <= 1e-7 * (1 + abs(m))
    # a minimum: no sampled point is lower
    pts = WL.random_points_in_box(l0, u0, 20000, seed)
    assert float((O.network_output(ops, pts) @ c).min()) >= m - 1e-9
    # above the relaxation's optimum
    v = lp.lp_value(ops, l0, u0, lh, uh, c, "anderson")
    assert v <= m + 1e-9


def wide(seed, eps=0.3):
    """The tiny net on a box of half-width eps around its centre: 5-10
    ambiguous neurons, a relaxation gap that takes splits to close."""
    w = WL.tiny_config(seed)
    ops = O.ops_from_workload_layers(w.layers)
    centre = (w.l0[0].astype(np.float64) + w.u0[0].astype(np.float64)) / 2
    l0, u0 = centre - eps, centre + eps
    lh, uh = O.interval_bounds(ops, l0, u0)
    return w, ops, l0, u0, w.c[0].astype(np.float64), lh[:-1], uh[:-1]


def shifted(ops, l0, u0, c, target):
    """The net with its output bias moved so that the exact minimum is `target`."""
    lh, uh = O.interval_bounds(ops, l0, u0)
    m, _ = B.exact_minimum(ops, l0, u0, c, lh[:-1], uh[:-1])
    out = list(ops)
    out[-1] = O.dense_op(ops[-1].W.toarray(), ops[-1].b + (target - m) / float(c.sum()))
    lh, uh = O.interval_bounds(out, l0, u0)
    m2, _ = B.exact_minimum(out, l0, u0, c, lh[:-1], uh[:-1])
    assert abs(m2 - target) < 1e-9
    return out, lh[:-1], uh[:-1]


def root_gap(w, ops, l0, u0, c, lh, uh):
    m, _ = B.exact_minimum(ops, l0, u0, c, lh, uh)
    root = O.solve(O.make_problem(ops, l0, u0, lh, uh, c), O.params_from_schedule(w.schedule)).bound
    return m - root


@pytest.mark.parametrize("seed", [1000, 1002, 1004, 1005, 1006, 1008])
def test_verified_trees_cover_the_box_with_true_leaves(seed):
    """Move the exact minimum to 0.3 of the root's relaxation gap: the
    property holds, the root cannot show it, and the tree does.  Its
    discarded leaves cover the box (every sampled input's pre-activations lie
    in some leaf's bounds: no region was dropped by a split) and each has an
    exact minimum > 0 (no leaf was discarded wrongly)."""
    w, ops, l0, u0, c, lh, uh = wide(seed)
    gap = root_gap(w, ops, l0, u0, c, lh, uh)
    assert gap > 0.01
    opsx, lh2, uh2 = shifted(ops, l0, u0, c, 0.3 * gap)
    r = B.bab(opsx, l0, u0, c, lh2, uh2, bab_params(w))
    assert r.verdict == "verified", r
    assert r.batches >= 1
    assert all(st == "pruned" for *_, st in r.leaves)
    for la, ua, lb, st in r.leaves:
        m, _ = B.exact_minimum(opsx, l0, u0, c, la, ua)
        assert m > 0, (m, lb)
    pts = WL.random_points_in_box(l0, u0, 3000, seed)
    pre, x = [], pts.T
    for k, op in enumerate(opsx[:-1]):
        y = op.W @ x + op.b[:, None]
        pre.append(y)
        x = np.maximum(y, 0.0)
    inside = np.zeros(pts.shape[0], dtype=bool)
    for la, ua, lb, st in r.leaves:
        ok = np.ones(pts.shape[0], dtype=bool)
        for y, lo, hi in zip(pre, la, ua):
            ok &= np.all((y >= lo[:, None] - 1e-9) & (y <= hi[:, None] + 1e-9), axis=0)
        inside |= ok
    assert inside.all(), int((~inside).sum())


@pytest.mark.parametrize("seed,frac", [(1002, -0.1), (1005, -0.1), (1009, -0.1), (1004, -0.05)])
def test_false_properties_found_after_splits(seed, frac):
    """Move the exact minimum below zero by a fraction of the root's gap where
    the root's x*_0 does not disprove the property: the tree finds a point of
    output <= 0."""
    w, ops, l0, u0, c, lh, uh = wide(seed)
    gap = root_gap(w, ops, l0, u0, c, lh, uh)
    opsx, lh2, uh2 = shifted(ops, l0, u0, c, frac * gap)
    r = B.bab(opsx, l0, u0, c, lh2, uh2, bab_params(w))
    assert r.verdict == "falsified", r
    assert r.batches >= 1
    assert float(O.network_output(opsx, r.counterexample) @ c) <= 0.0


def test_never_claims_a_false_property():
    """Soundness over random shifts around zero: 'verified' only with a
    positive exact minimum, 'falsified' only with a point of output <= 0."""
    rng = np.random.default_rng(7)
    for seed in (1000, 1002, 1005):
        w, ops, l0, u0, c, lh, uh = wide(seed)
        gap = root_gap(w, ops, l0, u0, c, lh, uh)
        for _ in range(4):
            target = float(rng.uniform(-0.5, 0.5)) * gap
            opsx, lh2, uh2 = shifted(ops, l0, u0, c, target)
            r = B.bab(opsx, l0, u0, c, lh2, uh2, bab_params(w))
            if r.verdict == "verified":
                assert target > 0
            if r.verdict == "falsified":
                assert target <= 0
                assert float(O.network_output(opsx, r.counterexample) @ c) <= 0.0


def test_subtrees_and_stratification():
    # |s| = 2^(-lb/i + 1) - 1: a parent at lb = -2i needs a subtree of 7 nodes
    # with a_l; a gain of i saves one level (3 nodes): ratio 7/3
    assert abs(B.subtree_ratio(-2.0, 1.0, 1.0) - 7.0 / 3.0) < 1e-12
    # a gain that closes the subtree at once
    assert B.subtree_ratio(-0.5, 2.0, 1.0) == float("inf")
    # no gain, no saving
    assert abs(B.subtree_ratio(-3.0, 0.0, 0.5) - 1.0) < 1e-12
