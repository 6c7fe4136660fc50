"""FP64 CPU oracle of branch and bound with stratified bounding (Sec. 6.2).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library and imports nothing from it; it bounds subdomains with the
Active Set / Big-M oracle of asd_oracle.py.

Source: De Palma et al., "Scaling the Convex Barrier with Sparse Dual
Algorithms" (arXiv:2101.05844):

  * branch and bound, pruning, upper bounds ... Sec. 6.2 (sec:stratified) and
                                                its footnote on x*_0
  * stratified bounding ...................... Sec. 6.2 (tree-size estimates
                                                |s|_{a_l}, |s|_{a_t}, overhead
                                                c_{a_t/a_l})
  * batches, parent warm starts .............. Sec. 7.3

The property is the canonical form: it holds when the minimum of c^T x_hat_n
over the input box is > 0; a subdomain is discarded when its lower bound is
> 0, and a point whose network output is <= 0 disproves the property.  The
verdict "verified" needs every subdomain discarded.

Readings (kept with the design notes too):

  B1  Branching is on ReLUs: a child fixes one neuron's phase through its
      pre-activation bounds (active: lhat := max(lhat, 0); inactive:
      uhat := min(uhat, 0)); the other bounds are the parent's (no
      re-propagation).
  B2  The branching rule (the paper uses BaBSR, outside this build) picks
      the unfixed neuron with lhat < 0 < uhat of largest interval score
      -lhat uhat / (uhat - lhat) (the height of the Planet triangle), ties to
      the lower layer, then the lower index.  A subdomain with no such
      neuron and lower bound <= 0 cannot be split: it disproves the property
      if its x*_0 does, and otherwise leaves the verdict "unknown" (the
      iterative bound may be below the exact value the relaxation then has).
  B3  Best first: the open subdomains are ordered by lower bound (ties by
      creation order); each batch splits up to `batch` of them and bounds
      their children together.
  B4  Warm starts: a child's alpha, beta_0, beta_1 start at its parent's
      final values; masks, Adam moments and step counts start empty (the
      split changes the bounds the mask constants are made of).
  B5  Stratification: a_l is the Big-M solver (Algorithm 3) alone, a_t is
      Big-M followed by Active Set.  At the root both run (from zero duals);
      l_{a_t - a_l} is their difference and the root keeps a_t's bound and
      duals, but is not itself marked hard (the rule marks subtrees below
      it).  i(s) is an exponential moving average (weight rho = 0.25 of
      the newest) of lb(child) - lb(parent) over the children in batch order;
      before the first batch, or while i <= 0, a child uses its parent's
      algorithm (a_l below the root).  Otherwise a child s of parent p is
      hard when the estimated subtree sizes satisfy |s|_{a_l} / |s|_{a_t} >
      c_{a_t/a_l} (or |s|_{a_t} = 0 < |s|_{a_l}); a hard subdomain's
      descendants stay hard.  c_{a_t/a_l} defaults to (T_M + 2 T) / T_M
      (an Active Set iteration counted as two Big-M ones).
  B6  The upper bound of a bounded subdomain is the network output at its
      x*_0 (the footnote of Sec. 6.2); it is computed in FP64.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Optional

import numpy as np
from scipy.optimize import linprog

from . import asd_oracle as O


@dataclasses.dataclass
class BaBParams:
    loose: O.SolveParams            # a_l: as_iters = 0
    tight: O.SolveParams            # a_t
    batch: int = 4                  # subdomains split per batch
    max_batches: int = 40
    rho: float = 0.25               # B5
    overhead: Optional[float] = None  # c_{a_t/a_l}; None: B5's default
    warm: bool = True               # B4


@dataclasses.dataclass
class Domain:
    id: int
    lhat: List[np.ndarray]
    uhat: List[np.ndarray]
    lb: float
    state: Optional[O.DualState]
    hard: bool
    depth: int


@dataclasses.dataclass
class BaBResult:
    verdict: str                    # "verified", "falsified" or "unknown"
    batches: int
    nodes: int                      # subdomains bounded (root included)
    counterexample: Optional[np.ndarray]
    trace: list                     # per batch: [(parent id, child id, split, hard, lb, ub)]
    root: dict
    leaves: list = dataclasses.field(default_factory=list)  # (lhat, uhat, lb, "pruned" | "undecided" | "open")


def overhead_default(p: BaBParams) -> float:
    tm = max(1, p.loose.bigm_iters)
    return (tm + 2 * p.tight.as_iters) / tm


def branch_neuron(lhat, uhat):
    """B2: (layer k, neuron i) of the largest interval score, or None."""
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


def split(d: Domain, k: int, i: int, ids):
    """B1: the active and the inactive child."""
    la = [a.copy() for a in d.lhat]
    ua = [a.copy() for a in d.uhat]
    la[k - 1][i] = max(la[k - 1][i], 0.0)
    li = [a.copy() for a in d.lhat]
    ui = [a.copy() for a in d.uhat]
    ui[k - 1][i] = min(ui[k - 1][i], 0.0)
    return (next(ids), la, ua), (next(ids), li, ui)


def warm_state(p: O.Problem, parent: Optional[O.DualState]) -> O.DualState:
    """B4: the parent's alpha, beta_0, beta_1; everything else empty."""
    st = O.zero_state(p)
    if parent is not None:
        for k in range(p.n - 1):
            st.alpha[k] = parent.alpha[k].copy()
            st.beta0[k] = parent.beta0[k].copy()
            st.beta1[k] = parent.beta1[k].copy()
    return st


def bound_domain(ops, l0, u0, c, lhat, uhat, prm: O.SolveParams, start: Optional[O.DualState], warm: bool):
    p = O.make_problem(ops, l0, u0, lhat, uhat, c)
    st = warm_state(p, start if warm else None)
    r = O.solve(p, prm, state=st)
    ub = float(O.network_output(ops, r.x0) @ p.c)
    return r.bound, ub, r.x0, r.state


def subtree_ratio(l_parent: float, gain: float, i: float) -> float:
    """|s|_{a_l} / |s|_{a_t} of Sec. 6.2 (inf when only a_t is predicted to
    close the subtree at once)."""
    def size(lb):
        e = min(-lb / i + 1.0, 1000.0)
        return 2.0 ** e - 1.0
    sl, st = size(l_parent), size(l_parent + gain)
    if st <= 0:
        return math.inf if sl > 0 else 1.0
    return sl / st


def bab(ops, l0, u0, c, lhat, uhat, prm: BaBParams) -> BaBResult:
    """Branch and bound over the input box [l0, u0] with root pre-activation
    bounds lhat, uhat (lists over ReLU layers)."""
    l0 = np.asarray(l0, np.float64)
    u0 = np.asarray(u0, np.float64)
    c = np.asarray(c, np.float64)
    lhat = [np.asarray(a, np.float64) for a in lhat]
    uhat = [np.asarray(a, np.float64) for a in uhat]
    c_over = prm.overhead if prm.overhead is not None else overhead_default(prm)
    ids = itertools.count()
    rid = next(ids)
    lb_l, ub_l, x_l, _ = bound_domain(ops, l0, u0, c, lhat, uhat, prm.loose, None, False)
    lb_t, ub_t, x_t, st_t = bound_domain(ops, l0, u0, c, lhat, uhat, prm.tight, None, False)
    gain = lb_t - lb_l
    root = {"lb_loose": lb_l, "lb_tight": lb_t, "gain": gain, "ub": min(ub_l, ub_t), "overhead": c_over}
    nodes = 2
    for ub, x in ((ub_l, x_l), (ub_t, x_t)):
        if ub <= 0:
            return BaBResult("falsified", 0, nodes, x, [], root)
    if lb_t > 0:
        return BaBResult("verified", 0, nodes, None, [], root, [(lhat, uhat, lb_t, "pruned")])
    if branch_neuron(lhat, uhat) is None:
        return BaBResult("unknown", 0, nodes, None, [], root, [(lhat, uhat, lb_t, "undecided")])
    leaves = []
    open_ = [Domain(rid, lhat, uhat, lb_t, st_t, False, 0)]  # B5: the rule marks subtrees below the root
    undecided = 0
    ema = None
    trace = []
    for b in range(prm.max_batches):
        if not open_:
            return BaBResult("verified" if undecided == 0 else "unknown", b, nodes, None, trace, root, leaves)
        open_.sort(key=lambda d: (d.lb, d.id))
        parents = []
        while open_ and len(parents) < prm.batch:
            d = open_.pop(0)
            parents.append((d, branch_neuron(d.lhat, d.uhat)))
        rows = []
        for d, (k, i) in parents:
            for side, (cid, la, ua) in zip(("active", "inactive"), split(d, k, i, ids)):
                if d.hard:
                    hard = True
                elif ema is None or ema <= 0:
                    hard = False
                else:
                    hard = subtree_ratio(d.lb, gain, ema) > c_over
                rows.append((d, cid, (k, i, side), hard, la, ua))
        out = []
        for d, cid, sp, hard, la, ua in rows:
            lb, ub, x0, st = bound_domain(ops, l0, u0, c, la, ua, prm.tight if hard else prm.loose, d.state, prm.warm)
            nodes += 1
            out.append((d, cid, sp, hard, la, ua, lb, ub, x0, st))
        for d, cid, sp, hard, la, ua, lb, ub, x0, st in out:
            delta = lb - d.lb
            ema = delta if ema is None else (1.0 - prm.rho) * ema + prm.rho * delta
        trace.append([(d.id, cid, sp, hard, lb, ub) for d, cid, sp, hard, la, ua, lb, ub, x0, st in out])
        for d, cid, sp, hard, la, ua, lb, ub, x0, st in out:
            if ub <= 0:
                return BaBResult("falsified", b + 1, nodes, x0, trace, root, leaves)
        for d, cid, sp, hard, la, ua, lb, ub, x0, st in out:
            if lb > 0:
                leaves.append((la, ua, lb, "pruned"))
                continue
            if branch_neuron(la, ua) is None:
                undecided += 1  # B2
                leaves.append((la, ua, lb, "undecided"))
                continue
            open_.append(Domain(cid, la, ua, lb, st, hard, d.depth + 1))
    done = not open_ and undecided == 0
    leaves += [(d.lhat, d.uhat, d.lb, "open") for d in open_]
    return BaBResult("verified" if done else "unknown", prm.max_batches, nodes, None, trace, root, leaves)


# ----------------------------------------------------------------------------
# Exact minimum of small networks (for the pins): every activation pattern of
# the ambiguous neurons, one linear program each
# ----------------------------------------------------------------------------


def exact_minimum(ops, l0, u0, c, lhat, uhat, max_patterns: int = 4096):
    """min of c^T x_hat_n(x_0), x_hat_n the exact network, over the inputs of
    the box whose pre-activations lie within lhat, uhat (the whole box when
    the bounds hold on it; a branch-and-bound subdomain otherwise): for each
    activation pattern of the neurons whose bounds straddle zero (the others
    keep the phase their bounds force), the network is affine on the inputs
    where the pattern holds, so its minimum there is a linear program with a
    sign constraint per such neuron and the bound constraints of every
    neuron.  Returns (value, argmin)."""
    Ws = [op.W.toarray() for op in ops]
    bs = [op.b for op in ops]
    n0 = Ws[0].shape[1]
    amb = [np.flatnonzero((lo < 0) & (hi > 0)) for lo, hi in zip(lhat, uhat)]
    n_amb = sum(len(a) for a in amb)
    if 2 ** n_amb > max_patterns:
        raise ValueError(f"{n_amb} ambiguous neurons: too many patterns")
    best, arg = math.inf, None
    for bits in itertools.product((0, 1), repeat=n_amb):
        it = iter(bits)
        # affine map of x_0 to the pre-activations of each layer under the pattern
        A = np.eye(n0)
        a0 = np.zeros(n0)
        rows_ub, rhs_ub = [], []
        ok = True
        for k in range(len(ops) - 1):
            Z = Ws[k] @ A
            z0 = Ws[k] @ a0 + bs[k]
            act = (lhat[k] >= 0).astype(np.float64)
            for i in amb[k]:
                act[i] = float(next(it))
            for i in range(len(act)):
                if lhat[k][i] < 0 < uhat[k][i]:
                    if act[i]:       # pre-activation >= 0
                        rows_ub.append(-Z[i])
                        rhs_ub.append(z0[i])
                    else:            # pre-activation <= 0
                        rows_ub.append(Z[i])
                        rhs_ub.append(-z0[i])
                # lhat <= pre-activation <= uhat
                rows_ub.append(-Z[i])
                rhs_ub.append(z0[i] - lhat[k][i])
                rows_ub.append(Z[i])
                rhs_ub.append(uhat[k][i] - z0[i])
            A = act[:, None] * Z
            a0 = act * z0
        if not ok:
            continue
        obj = c @ (Ws[-1] @ A)
        const = float(c @ (Ws[-1] @ a0 + bs[-1]))
        res = linprog(obj, A_ub=np.array(rows_ub) if rows_ub else None,
                      b_ub=np.array(rhs_ub) if rhs_ub else None,
                      bounds=list(zip(l0, u0)), method="highs")
        if res.status == 0 and res.fun + const < best:
            best, arg = float(res.fun + const), res.x
    return best, arg
