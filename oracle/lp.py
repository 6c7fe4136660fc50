"""Exact LP values of the relaxations on tiny networks (HiGHS via SciPy).

TEST INFRASTRUCTURE ONLY (see asd_oracle.py).  These are the plain
definitions the dual iterations approach from below:

  * LP_M  - the Big-M relaxation, eq:primal-bigm (Sec. 2.1), equal to Planet
            (App. B, sec:planet-eq);
  * LP_A  - the Anderson-type relaxation with pre-activation bounds kept in
            M_k, eq:primal-anderson (Sec. 2.2), every mask enumerated;
  * LP_A' - the original formulation without them, eq:orig-anderson-set
            (App. F): alpha rows plus all 2^F masks (the all-zero and all-one
            masks included), with the box on x_hat;
  * intermediate bounds by eq:primal-intermediates (App. E).

Variables: x_0, then for k = 1..n-1 the triple (x_hat_k, x_k, z_k), then
x_hat_n.  Only practical for fan-ins of about 10 or less.
"""
from __future__ import annotations

import itertools
from typing import List, Optional, Sequence

import numpy as np
from scipy.optimize import linprog

from .asd_oracle import LinearOp


def _dense(op: LinearOp) -> np.ndarray:
    return op.W.toarray()


def lp_value(ops: Sequence[LinearOp], l0, u0, lhat: Sequence, uhat: Sequence, c,
             relaxation: str = "bigm", n_layers: Optional[int] = None,
             sense: str = "min") -> float:
    """min (or max) c^T x_hat_m over the relaxed network truncated at layer m.

    relaxation in {"bigm", "anderson", "anderson_orig"}; lhat/uhat hold the
    pre-activation bounds of layers 1..m-1 (entries beyond are ignored).
    """
    m = len(ops) if n_layers is None else n_layers
    Ws = [_dense(op) for op in ops[:m]]
    bs = [op.b for op in ops[:m]]
    sizes = [Ws[0].shape[1]] + [W.shape[0] for W in Ws]
    # variable offsets
    off = {}
    pos = 0
    off[("x", 0)] = pos
    pos += sizes[0]
    for k in range(1, m):
        for name in ("xh", "x", "z"):
            off[(name, k)] = pos
            pos += sizes[k]
    off[("xh", m)] = pos
    pos += sizes[m]
    nv = pos

    lb = np.full(nv, -np.inf)
    ub = np.full(nv, np.inf)
    lb[off[("x", 0)]:off[("x", 0)] + sizes[0]] = l0
    ub[off[("x", 0)]:off[("x", 0)] + sizes[0]] = u0
    for k in range(1, m):
        lh, uh = np.asarray(lhat[k - 1], float), np.asarray(uhat[k - 1], float)
        s = sizes[k]
        lb[off[("xh", k)]:off[("xh", k)] + s] = lh
        ub[off[("xh", k)]:off[("xh", k)] + s] = uh
        lb[off[("x", k)]:off[("x", k)] + s] = np.maximum(lh, 0)
        ub[off[("x", k)]:off[("x", k)] + s] = np.maximum(uh, 0)
        lb[off[("z", k)]:off[("z", k)] + s] = 0.0
        ub[off[("z", k)]:off[("z", k)] + s] = 1.0

    A_eq, b_eq = [], []
    for k in range(1, m + 1):
        W, b = Ws[k - 1], bs[k - 1]
        prev = off[("x", k - 1)]
        for i in range(sizes[k]):
            row = np.zeros(nv)
            row[off[("xh", k)] + i] = 1.0
            row[prev:prev + sizes[k - 1]] -= W[i]
            A_eq.append(row)
            b_eq.append(b[i])

    A_ub, b_ub = [], []
    for k in range(1, m):
        W, b = Ws[k - 1], bs[k - 1]
        lh, uh = np.asarray(lhat[k - 1], float), np.asarray(uhat[k - 1], float)
        lp_, up_ = (np.asarray(l0, float), np.asarray(u0, float)) if k == 1 else (
            np.maximum(np.asarray(lhat[k - 2], float), 0), np.maximum(np.asarray(uhat[k - 2], float), 0))
        prev = off[("x", k - 1)]
        for i in range(sizes[k]):
            xi, xhi, zi = off[("x", k)] + i, off[("xh", k)] + i, off[("z", k)] + i
            # alpha: x_hat - x <= 0
            row = np.zeros(nv); row[xhi] = 1; row[xi] = -1
            A_ub.append(row); b_ub.append(0.0)
            if relaxation in ("bigm", "anderson"):
                # beta_0: x - uhat z <= 0
                row = np.zeros(nv); row[xi] = 1; row[zi] = -uh[i]
                A_ub.append(row); b_ub.append(0.0)
                # beta_1: x - x_hat - lhat z <= -lhat
                row = np.zeros(nv); row[xi] = 1; row[xhi] = -1; row[zi] = -lh[i]
                A_ub.append(row); b_ub.append(-lh[i])
            if relaxation in ("anderson", "anderson_orig"):
                w = W[i]
                Lchk = np.where(w >= 0, lp_, up_)
                Uchk = np.where(w >= 0, up_, lp_)
                for bits in itertools.product((0.0, 1.0), repeat=sizes[k - 1]):
                    I = np.asarray(bits)
                    LI = float(np.sum(w * I * Lchk))
                    UI = float(np.sum(w * (1 - I) * Uchk))
                    # x <= (W.I) x_prev + z b - LI (1 - z) + UI z
                    row = np.zeros(nv)
                    row[xi] = 1.0
                    row[prev:prev + sizes[k - 1]] -= w * I
                    row[zi] = -b[i] - LI - UI
                    A_ub.append(row); b_ub.append(-LI)

    cost = np.zeros(nv)
    cost[off[("xh", m)]:off[("xh", m)] + sizes[m]] = np.asarray(c, float)
    if sense == "max":
        cost = -cost
    res = linprog(cost, A_ub=np.array(A_ub) if A_ub else None,
                  b_ub=np.array(b_ub) if b_ub else None,
                  A_eq=np.array(A_eq), b_eq=np.array(b_eq),
                  bounds=list(zip(lb, ub)), method="highs")
    if res.status != 0:
        raise RuntimeError(f"LP failed: {res.message}")
    return float(res.fun) if sense == "min" else float(-res.fun)


def lp_intermediate_bounds(ops: Sequence[LinearOp], l0, u0, relaxation: str = "bigm"):
    """Pre-activation bounds of layers 1..n-1 by eq:primal-intermediates with
    C_k = the given relaxation on the layers before (App. E; layer 1 reduces
    to the box-constrained LP, i.e. interval bounds)."""
    lhat: List[np.ndarray] = []
    uhat: List[np.ndarray] = []
    for i in range(1, len(ops)):
        n_i = ops[i - 1].n_out
        lo, hi = np.zeros(n_i), np.zeros(n_i)
        for j in range(n_i):
            e = np.zeros(n_i); e[j] = 1.0
            lo[j] = lp_value(ops, l0, u0, lhat, uhat, e, relaxation, n_layers=i, sense="min")
            hi[j] = lp_value(ops, l0, u0, lhat, uhat, e, relaxation, n_layers=i, sense="max")
        lhat.append(lo)
        uhat.append(hi)
    return lhat, uhat
