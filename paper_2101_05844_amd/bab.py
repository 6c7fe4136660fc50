"""Branch and bound with stratified bounding (Sec. 6.2) over the GPU solver.

The tree bookkeeping (open subdomains, splits, the stratification estimate)
runs on the host; every bound is a batched solve of the library (Big-M for
the loose algorithm a_l, Big-M then Active Set for the tight one a_t), every
upper bound the library's interval propagation at the solve's x*_0, and the
warm starts (Sec. 7.3) move duals between device arrays.

Rules (the same as the FP64 reference the tests compare against):
  * canonical form: the property holds when min c^T x_hat_n over the input
    box is > 0; a subdomain with lower bound > 0 is discarded; a point whose
    output is <= 0 disproves the property (its output's upper bound from
    interval propagation at the point, rounded outward, is <= 0);
  * a child fixes one ReLU's phase through its pre-activation bounds
    (lhat := max(lhat, 0) or uhat := min(uhat, 0)), the others are the
    parent's;
  * branching picks the unfixed neuron with lhat < 0 < uhat of largest
    -lhat uhat / (uhat - lhat), ties to the lower layer, then index; a
    subdomain without one and with lower bound <= 0 leaves the verdict
    "unknown" unless its x*_0 disproves the property;
  * best first: up to `batch` open subdomains of lowest bound (ties by
    creation order) are split per batch, their children bounded together;
  * a child starts from its parent's final alpha, beta_0, beta_1 (masks,
    moments and step counts empty);
  * stratification: at the root both algorithms run, their difference is
    l_{a_t - a_l}; i is the exponential moving average (weight 0.25 of the
    newest) of lb(child) - lb(parent); a child of an easy parent is hard when
    |s|_{a_l} / |s|_{a_t} > c_{a_t/a_l} with |s| = 2^(-lb/i + 1) - 1 (lb the
    parent's bound, plus l_{a_t - a_l} for a_t), while i is defined and
    positive; hard subtrees stay hard; c_{a_t/a_l} defaults to
    (T_M + 2 T) / T_M.
"""
from __future__ import annotations

import itertools
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import asdual as A


def branch_neuron(lhat: Sequence[np.ndarray], uhat: Sequence[np.ndarray]):
    """(layer k, neuron i) to split, or None."""
    best, arg = -1.0, None
    for k, (lo, hi) in enumerate(zip(lhat, uhat), start=1):
        amb = (lo < 0) & (hi > 0)
        if not amb.any():
            continue
        score = np.where(amb, -lo * hi / np.where(amb, hi - lo, 1.0), -1.0)
        i = int(np.argmax(score))
        if score[i] > best:
            best, arg = float(score[i]), (k, i)
    return arg


def subtree_ratio(l_parent: float, gain: float, i: float) -> float:
    """|s|_{a_l} / |s|_{a_t} (inf when only a_t is predicted to close the subtree)."""
    def size(lb):
        return 2.0 ** min(-lb / i + 1.0, 1000.0) - 1.0
    sl, st = size(l_parent), size(l_parent + gain)
    if st <= 0:
        return math.inf if sl > 0 else 1.0
    return sl / st


class _Domain:
    __slots__ = ("id", "lhat", "uhat", "lb", "duals", "hard", "depth")

    def __init__(self, id, lhat, uhat, lb, duals, hard, depth):
        self.id, self.lhat, self.uhat, self.lb = id, lhat, uhat, lb
        self.duals, self.hard, self.depth = duals, hard, depth


class BranchAndBound:
    """Stratified branch and bound on one net.  `tight` holds the solver
    schedule of a_t (its as_iters > 0); a_l is the same with as_iters = 0."""

    def __init__(self, net: "A.Net", tight: "A.Params", batch: int = 4, max_batches: int = 40,
                 rho: float = 0.25, overhead: Optional[float] = None, warm: bool = True):
        self.net, self.batch, self.max_batches = net, batch, max_batches
        self.rho, self.warm = rho, warm
        self.tight = tight
        self.loose = A.Params.from_buffer_copy(tight)
        self.loose.as_iters = 0
        tm = max(1, tight.bigm_iters)
        self.overhead = overhead if overhead is not None else (tm + 2 * tight.as_iters) / tm
        self.dtype = torch.float64 if tight.precision == A.ASD_PREC_FP64 else torch.float32
        S = 2 * batch
        self.plans = {False: A.Plan(net, S, self.loose), True: A.Plan(net, S, self.tight)}
        self.root_plans = {False: A.Plan(net, 1, self.loose), True: A.Plan(net, 1, self.tight)}
        self.n = net.n

    # -- one batched bound ----------------------------------------------------
    def _bound(self, plan, hard: bool, l0, u0, c, rows):
        """rows: [(lhat list, uhat list, warm duals or None)]; returns per row
        (lb, ub, x0, duals)."""
        S = plan.S
        m = len(rows)
        pad = [rows[-1]] * (S - m)
        dev = "cuda"
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)
        L0 = f32(np.repeat(l0[None], S, 0))
        U0 = f32(np.repeat(u0[None], S, 0))
        Cm = f32(np.repeat(c[None], S, 0))
        LH = [f32(np.stack([r[0][k] for r in rows + pad])) for k in range(self.n - 1)]
        UH = [f32(np.stack([r[1][k] for r in rows + pad])) for k in range(self.n - 1)]
        plan.init(L0, U0, LH, UH, Cm)
        if self.warm and any(r[2] is not None for r in rows):
            for f_idx, field in enumerate((A.ASD_F_ALPHA, A.ASD_F_BETA0, A.ASD_F_BETA1)):
                for k in range(1, self.n):
                    zero = torch.zeros(self.net.sizes[k], dtype=self.dtype, device=dev)
                    src = torch.stack([r[2][f_idx][k - 1] if r[2] is not None else zero for r in rows + pad])
                    plan.set(field, k, src)
            # the derived sums of the iteration kernels follow the imported duals
            plan.set_counts(0, 0, [], recompute=False)
        plan.run(A.ASD_PHASE_BIGM, 0, plan.params.bigm_iters)
        if hard:
            plan.run(A.ASD_PHASE_AS, 0, plan.params.as_iters)
        lb, x0 = plan.bound(want_x0=True)
        duals = [[plan.get(field, k) for k in range(1, self.n)]
                 for field in (A.ASD_F_ALPHA, A.ASD_F_BETA0, A.ASD_F_BETA1)]
        # upper bound: the network at x*_0 by interval propagation at the point
        lh, uh = self.net.interval_bounds(x0, x0)
        lo_out, hi_out = lh[-1].double().cpu().numpy(), uh[-1].double().cpu().numpy()
        ub = np.where(c[None] >= 0, c[None] * hi_out, c[None] * lo_out).sum(axis=1)
        lb = lb.cpu().numpy()
        x0 = x0.cpu().numpy()
        out = []
        for s in range(m):
            out.append((float(lb[s]), float(ub[s]), x0[s].astype(np.float64),
                        [[duals[f][k][s].clone() for k in range(self.n - 1)] for f in range(3)]))
        return out

    def run(self, l0, u0, c, lhat, uhat):
        """Verdict ("verified", "falsified", "unknown") for the property
        c^T x_hat_n > 0 over the box [l0, u0] with root pre-activation bounds
        lhat, uhat (float32 values; lists over the ReLU layers)."""
        l0 = np.asarray(l0, np.float64)
        u0 = np.asarray(u0, np.float64)
        c = np.asarray(c, np.float64)
        lhat = [np.asarray(a, np.float64) for a in lhat]
        uhat = [np.asarray(a, np.float64) for a in uhat]
        ids = itertools.count()
        rid = next(ids)
        (lb_l, ub_l, x_l, _), = self._bound(self.root_plans[False], False, l0, u0, c, [(lhat, uhat, None)])
        (lb_t, ub_t, x_t, du_t), = self._bound(self.root_plans[True], True, l0, u0, c, [(lhat, uhat, None)])
        gain = lb_t - lb_l
        root = {"lb_loose": lb_l, "lb_tight": lb_t, "gain": gain, "ub": min(ub_l, ub_t), "overhead": self.overhead}
        res = lambda v, b, nodes, x, trace: {"verdict": v, "batches": b, "nodes": nodes, "counterexample": x,
                                              "trace": trace, "root": root}
        nodes = 2
        for ub, x in ((ub_l, x_l), (ub_t, x_t)):
            if ub <= 0:
                return res("falsified", 0, nodes, x, [])
        if lb_t > 0:
            return res("verified", 0, nodes, None, [])
        if branch_neuron(lhat, uhat) is None:
            return res("unknown", 0, nodes, None, [])
        open_ = [_Domain(rid, lhat, uhat, lb_t, du_t, False, 0)]  # the rule marks subtrees below the root
        undecided = 0
        ema = None
        trace = []
        for b in range(self.max_batches):
            if not open_:
                return res("verified" if undecided == 0 else "unknown", b, nodes, None, trace)
            open_.sort(key=lambda d: (d.lb, d.id))
            parents = []
            while open_ and len(parents) < self.batch:
                d = open_.pop(0)
                parents.append((d, branch_neuron(d.lhat, d.uhat)))
            children = []
            for d, (k, i) in parents:
                la = [a.copy() for a in d.lhat]
                ua = [a.copy() for a in d.uhat]
                la[k - 1][i] = max(la[k - 1][i], 0.0)
                li = [a.copy() for a in d.lhat]
                ui = [a.copy() for a in d.uhat]
                ui[k - 1][i] = min(ui[k - 1][i], 0.0)
                for side, cl, cu in (("active", la, ua), ("inactive", li, ui)):
                    if d.hard:
                        hard = True
                    elif ema is None or ema <= 0:
                        hard = False
                    else:
                        hard = subtree_ratio(d.lb, gain, ema) > self.overhead
                    children.append([d, next(ids), (k, i, side), hard, cl, cu, None])
            for hard in (True, False):
                idx = [j for j, ch in enumerate(children) if ch[3] == hard]
                if not idx:
                    continue
                outs = self._bound(self.plans[hard], hard, l0, u0, c,
                                   [(children[j][4], children[j][5], children[j][0].duals) for j in idx])
                for j, o in zip(idx, outs):
                    children[j][6] = o
            nodes += len(children)
            for d, cid, sp, hard, cl, cu, (lb, ub, x0, du) in children:
                delta = lb - d.lb
                ema = delta if ema is None else (1.0 - self.rho) * ema + self.rho * delta
            trace.append([(d.id, cid, sp, hard, o[0], o[1]) for d, cid, sp, hard, cl, cu, o in children])
            for d, cid, sp, hard, cl, cu, (lb, ub, x0, du) in children:
                if ub <= 0:
                    return res("falsified", b + 1, nodes, x0, trace)
            for d, cid, sp, hard, cl, cu, (lb, ub, x0, du) in children:
                if lb > 0:
                    continue
                if branch_neuron(cl, cu) is None:
                    undecided += 1
                    continue
                open_.append(_Domain(cid, cl, cu, lb, du, hard, d.depth + 1))
        done = not open_ and undecided == 0
        return res("verified" if done else "unknown", self.max_batches, nodes, None, trace)
