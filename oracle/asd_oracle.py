"""FP64 CPU oracle for the Active Set dual of the Anderson-type relaxation.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library and imports nothing from it.

Source: De Palma, Behl, Bunel, Torr, Kumar, "Scaling the Convex Barrier with
Sparse Dual Algorithms" (JMLR 2024, arXiv:2101.05844).  Every function below
follows one passage of the paper, cited by section and equation label:

  * problem and notation ............ Sec. 2 (eq:noncvx_pb), Sec. 2.2 (L/U check
                                      matrices, eq:primal-anderson)
  * separation oracle ............... Sec. 2.2, eq:oracle
  * dual, f_k and g_k ............... Sec. 3, eq:dual-anderson,
                                      eq:dual-anderson-functions; App. D
                                      (sec:dual-derivation)
  * restricted (Active Set) dual .... Sec. 4.1, eq:dual-active-set
  * inner minimisation .............. Sec. 4.1, eq:as-primalk-min, eq:as-primal0-min
  * supergradient ................... Sec. 4.1, eq:as-supergradient
  * Active Set loop ................. Sec. 4, Algorithm 1 (alg:active-set)
  * Big-M initialisation ............ App. B (sec:dual-init), Algorithm 3
                                      (alg:bigm)
  * Adam ascent, schedule ........... Sec. 7.1 (experimental setting)
  * intermediate bounds ............. App. E (sec:intermediate,
                                      eq:primal-intermediates)

Readings taken where the paper is ambiguous or inconsistent (the same list
is kept with the design notes):

  R1  x*_k lies in the post-activation box [l_k, u_k] (the box of the inner
      problem in eq:dual-active-set), not the pre-activation box printed in
      eq:as-primalk-min.
  R2  x*_0 maximises f_0^T x_0 over the input box (the Lagrangian carries
      -f_0^T x_0), i.e. u_0 where f_0 >= 0 and l_0 elsewhere.
  R3  The U-check term of the beta_{k,I} supergradient enters with a minus
      sign, as in the constraint (eq:primal-anderson) and the Lagrangian of
      App. D; eq:as-supergradient prints a plus.
  R4  The Big-M f_k uses beta_{k+1,1} (as in eq:dual-bigm, App. B).
  R5  The constant term of the Lagrangian includes b_n^T alpha_n (App. D has
      it; eq:dual-anderson's sum stops at n-1).  alpha_n is the objective row
      c (the paper's "alpha_n = I" for a scalar output).
  R6  Tie rules follow the printed ">=": f >= 0 -> u, g >= 0 -> z = 1,
      oracle coefficient >= 0 -> mask bit 1.
  R7  The oracle's sign rule is applied over all 2^F masks; a returned row
      that is all ones or all zeros is kept as an ordinary active-set mask.
  R8  Additions happen at Active Set iterations t with (t mod omega) < V while
      fewer than K_max masks are active (Algorithm 1's "t <= nb_vars_to_add"
      read as V additions per period, matching "2 new variables" in Sec. 7.1).
  R9  Adam: beta1 0.9, beta2 0.999, eps 1e-8; moments and step counters of
      alpha/beta_0/beta_1 reset when the Active Set phase starts (the step size
      "is reset"); each added beta_{k,I} starts with zero moments and its own
      step counter; the step size is not rescaled at additions.
  R10 Learning rates decrease linearly: lr_t = lr0 + (lr1 - lr0) t / (T - 1).
  R11 The returned bound is d at the final duals (Algorithm 1's return).
  R20 l2-ball input domain (Sec. 2 allows any convex C; l2 balls among the
      examples): x*_0 maximises f_0^T x_0 over the ball (the centre moved by
      the radius along f_0); the check matrices of layer 1 use the ball's
      box hull as [l_0, u_0]; no masks are added at layer 1.  At an interior
      x*_0 (every x*_0 but where f_0 has one nonzero entry) eq:oracle gives
      only all-one rows (z = 1) and rows selecting the zero weights
      (z = 0), whose constraints x <= x_hat - (W Lchk)(1 - z) and
      x <= (b + W Uchk) z are implied by the beta_0 and beta_1 constraints
      for pre-activation bounds within the box hull's interval bounds.
"""
from __future__ import annotations

import copy
import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------
# Layers as explicit linear operators (App. G writes convolutions through
# their equivalent linear operator; we store it as a sparse matrix whose
# pattern is each output neuron's receptive field).
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class LinearOp:
    W: sp.csr_matrix      # [n_out, n_in], float64, explicit receptive-field pattern
    b: np.ndarray         # [n_out] float64
    widx: Optional[np.ndarray] = None   # per stored entry: flat index into the layer's weight tensor
    bidx: Optional[np.ndarray] = None   # per output neuron: index into the layer's bias vector

    @property
    def n_out(self) -> int:
        return self.W.shape[0]

    @property
    def n_in(self) -> int:
        return self.W.shape[1]

    @property
    def rows(self) -> np.ndarray:
        """Row index of every stored entry."""
        return np.repeat(np.arange(self.n_out), np.diff(self.W.indptr))

    @property
    def cols(self) -> np.ndarray:
        return self.W.indices

    @property
    def w(self) -> np.ndarray:
        return self.W.data

    def with_data(self, data: np.ndarray) -> sp.csr_matrix:
        """Same pattern, new entries (used for W (.) I)."""
        return sp.csr_matrix((data, self.W.indices, self.W.indptr), shape=self.W.shape)


def dense_op(W: np.ndarray, b: np.ndarray) -> LinearOp:
    W = np.asarray(W, dtype=np.float64)
    n_out, n_in = W.shape
    indptr = np.arange(n_out + 1, dtype=np.int64) * n_in
    indices = np.tile(np.arange(n_in, dtype=np.int64), n_out)
    M = sp.csr_matrix((W.reshape(-1).copy(), indices, indptr), shape=(n_out, n_in))
    return LinearOp(M, np.asarray(b, dtype=np.float64).copy(), widx=np.arange(n_out * n_in, dtype=np.int64),
                    bidx=np.arange(n_out, dtype=np.int64))


def conv_op(weight: np.ndarray, bias: np.ndarray, c_in: int, h_in: int, w_in: int,
            stride: int, pad: int) -> LinearOp:
    """2-D convolution (cross-correlation, zero padding) as a sparse matrix.

    Output neuron (co, oy, ox) reads input (ci, oy*stride - pad + ky,
    ox*stride - pad + kx) with weight weight[co, ci, ky, kx]; taps that fall
    in the padding have no entry.  Neurons are flattened in (c, y, x) order.
    """
    weight = np.asarray(weight, dtype=np.float64)
    c_out, c_in_w, kh, kw = weight.shape
    assert c_in_w == c_in
    h_out = (h_in + 2 * pad - kh) // stride + 1
    w_out = (w_in + 2 * pad - kw) // stride + 1
    rows, cols, vals, widx = [], [], [], []
    for co in range(c_out):
        for oy in range(h_out):
            for ox in range(w_out):
                r = (co * h_out + oy) * w_out + ox
                for ci in range(c_in):
                    for ky in range(kh):
                        iy = oy * stride - pad + ky
                        if iy < 0 or iy >= h_in:
                            continue
                        for kx in range(kw):
                            ix = ox * stride - pad + kx
                            if ix < 0 or ix >= w_in:
                                continue
                            rows.append(r)
                            cols.append((ci * h_in + iy) * w_in + ix)
                            vals.append(weight[co, ci, ky, kx])
                            widx.append(((co * c_in + ci) * kh + ky) * kw + kx)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    n_out = c_out * h_out * w_out
    # rows are generated in increasing order and columns increase within a row
    indptr = np.zeros(n_out + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    M = sp.csr_matrix((vals, cols, indptr), shape=(n_out, c_in * h_in * w_in))
    b = np.repeat(np.asarray(bias, dtype=np.float64), h_out * w_out)
    return LinearOp(M, b, widx=np.asarray(widx, dtype=np.int64),
                    bidx=np.repeat(np.arange(c_out, dtype=np.int64), h_out * w_out))


def ops_from_workload_layers(layers) -> List[LinearOp]:
    """Build LinearOps from workload layers (objects with .kind/.W/.b/.spec)."""
    ops = []
    for L in layers:
        if L.kind == "dense":
            ops.append(dense_op(L.W, L.b))
        else:
            s = L.spec
            ops.append(conv_op(L.W, L.b, s.c_in, s.h_in, s.w_in, s.stride, s.pad))
    return ops


# ----------------------------------------------------------------------------
# Problem data
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Problem:
    """One subproblem: min c^T x_hat_n over the relaxed network (Sec. 2).

    ops[k-1] is layer k (k = 1..n); lhat[k-1], uhat[k-1] are the
    pre-activation bounds of ReLU layer k (k = 1..n-1); c is the objective row
    over layer n's outputs (the paper's alpha_n).
    """
    ops: List[LinearOp]
    l0: np.ndarray
    u0: np.ndarray
    lhat: List[np.ndarray]
    uhat: List[np.ndarray]
    c: np.ndarray
    # input domain C (Sec. 2): None for the box [l0, u0]; (centre, radius)
    # for the l2 ball, whose box hull [l0, u0] then bounds x_0 in the
    # check matrices of layer 1 (R20)
    ball: Optional[tuple] = None

    @property
    def n(self) -> int:
        return len(self.ops)

    def W(self, k: int) -> LinearOp:
        """Layer k, 1-based as in the paper."""
        return self.ops[k - 1]

    def lu(self, k: int):
        """Post-activation bounds of layer k (k = 0 is the input box).

        l_k = max(lhat_k, 0), u_k = max(uhat_k, 0) (App. E, last paragraph).
        """
        if k == 0:
            return self.l0, self.u0
        return np.maximum(self.lhat[k - 1], 0.0), np.maximum(self.uhat[k - 1], 0.0)

    def hat(self, k: int):
        return self.lhat[k - 1], self.uhat[k - 1]


def make_problem(ops, l0, u0, lhat, uhat, c, ball=None) -> Problem:
    f64 = lambda a: np.asarray(a, dtype=np.float64).copy()
    b = None if ball is None else (f64(ball[0]), float(ball[1]))
    return Problem(ops, f64(l0), f64(u0), [f64(a) for a in lhat], [f64(a) for a in uhat], f64(c), b)


# ----------------------------------------------------------------------------
# Interval propagation (App. E: intermediate bounds; the paper takes the
# better of Wong-Kolter and interval propagation, we use the latter)
# ----------------------------------------------------------------------------


def interval_bounds(ops: Sequence[LinearOp], l0: np.ndarray, u0: np.ndarray):
    """Pre-activation bounds of every layer by interval arithmetic.

    x_hat_k in [W_k^+ l_{k-1} + W_k^- u_{k-1} + b_k, W_k^+ u_{k-1} + W_k^- l_{k-1} + b_k],
    l_k = max(lhat_k, 0), u_k = max(uhat_k, 0).  Returns lists over k = 1..n.
    """
    l = np.asarray(l0, np.float64)
    u = np.asarray(u0, np.float64)
    lhat, uhat = [], []
    for op in ops:
        Wp = op.with_data(np.maximum(op.w, 0.0))
        Wm = op.with_data(np.minimum(op.w, 0.0))
        lo = Wp @ l + Wm @ u + op.b
        hi = Wp @ u + Wm @ l + op.b
        lhat.append(lo)
        uhat.append(hi)
        l, u = np.maximum(lo, 0.0), np.maximum(hi, 0.0)
    return lhat, uhat


def network_output(ops: Sequence[LinearOp], x0: np.ndarray) -> np.ndarray:
    """Exact forward pass x_hat_n(x0) (eq:noncvx_pb), x0 of shape [n0] or [m, n0]."""
    x = np.asarray(x0, np.float64)
    batched = x.ndim == 2
    x = x.T if batched else x
    for k, op in enumerate(ops):
        x = op.W @ x + (op.b[:, None] if batched else op.b)
        if k < len(ops) - 1:
            x = np.maximum(x, 0.0)
    return x.T if batched else x


# ----------------------------------------------------------------------------
# Per-layer constants of the Anderson constraints (Sec. 2.2)
# ----------------------------------------------------------------------------


def check_matrices(op: LinearOp, l_prev: np.ndarray, u_prev: np.ndarray):
    """L-check and U-check entries on the stored pattern (Sec. 2.2).

    Lchk[i,j] = l[j] if W[i,j] >= 0 else u[j];  Uchk[i,j] = u[j] if W[i,j] >= 0 else l[j].
    """
    w, j = op.w, op.cols
    Lchk = np.where(w >= 0, l_prev[j], u_prev[j])
    Uchk = np.where(w >= 0, u_prev[j], l_prev[j])
    return Lchk, Uchk


@dataclasses.dataclass
class Mask:
    """One active-set member I in B_k with its multiplier beta_{k,I}."""
    I: np.ndarray          # bool over the stored pattern of W_k
    WI: sp.csr_matrix      # W_k (.) I
    LI: np.ndarray         # (W (.) I (.) Lchk) <> 1   [n_k]
    UI: np.ndarray         # (W (.) (1-I) (.) Uchk) <> 1   [n_k]
    beta: np.ndarray       # beta_{k,I} >= 0   [n_k]
    m: np.ndarray          # Adam first moment
    v: np.ndarray          # Adam second moment
    step: int              # Adam step counter of this multiplier
    x_prev: np.ndarray     # x*_{k-1} the oracle was called at
    z: np.ndarray          # z*_k the oracle was called at


def oracle_mask(op: LinearOp, l_prev, u_prev, x_prev, z):
    """Most violated Anderson constraint per neuron (Sec. 2.2, eq:oracle).

    I[i,j] = 1[ ((1 - z[i]) Lchk[i,j] + z[i] Uchk[i,j] - x_prev[j]) W[i,j] >= 0 ],
    for any x_prev in the box and z in [0,1] (Prop. 1 shows this maximises
    the beta_{k,I} supergradient entry over all masks).
    """
    Lchk, Uchk = check_matrices(op, l_prev, u_prev)
    r, j, w = op.rows, op.cols, op.w
    coeff = ((1.0 - z[r]) * Lchk + z[r] * Uchk - x_prev[j]) * w
    return coeff >= 0.0


def mask_constants(op: LinearOp, I: np.ndarray, l_prev, u_prev):
    """LI = (W (.) I (.) Lchk) <> 1 and UI = (W (.) (1 - I) (.) Uchk) <> 1 (row sums)."""
    Lchk, Uchk = check_matrices(op, l_prev, u_prev)
    If = I.astype(np.float64)
    LI = op.with_data(op.w * If * Lchk) @ np.ones(op.n_in)
    UI = op.with_data(op.w * (1.0 - If) * Uchk) @ np.ones(op.n_in)
    return LI, UI


def new_mask(op: LinearOp, I: np.ndarray, l_prev, u_prev, x_prev, z) -> Mask:
    LI, UI = mask_constants(op, I, l_prev, u_prev)
    n = op.n_out
    WI = op.with_data(op.w * I.astype(np.float64))
    return Mask(I=I.copy(), WI=WI, LI=LI, UI=UI, beta=np.zeros(n), m=np.zeros(n),
                v=np.zeros(n), step=0, x_prev=np.asarray(x_prev, np.float64).copy(),
                z=np.asarray(z, np.float64).copy())


# ----------------------------------------------------------------------------
# Dual state
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class DualState:
    """alpha_k, beta_{k,0}, beta_{k,1} (k = 1..n-1, stored at index k-1) and B_k."""
    alpha: List[np.ndarray]
    beta0: List[np.ndarray]
    beta1: List[np.ndarray]
    masks: List[List[Mask]]
    # Adam state of alpha/beta0/beta1 (shared step counter)
    m: dict
    v: dict
    step: int = 0

    def copy(self) -> "DualState":
        return copy.deepcopy(self)


def zero_state(p: Problem) -> DualState:
    """All duals 0 except alpha_n = c: the interval-propagation start (App. B)."""
    sizes = [p.W(k).n_out for k in range(1, p.n)]
    z = lambda: [np.zeros(s) for s in sizes]
    m = {"alpha": z(), "beta0": z(), "beta1": z()}
    v = {"alpha": z(), "beta0": z(), "beta1": z()}
    return DualState(z(), z(), z(), [[] for _ in sizes], m, v, 0)


# ----------------------------------------------------------------------------
# Dual functions (Sec. 3 eq:dual-anderson-functions restricted to B as in
# Sec. 4.1 eq:dual-active-set)
# ----------------------------------------------------------------------------


def dual_functions(p: Problem, st: DualState):
    """f_k (k = 0..n-1), g_k (k = 1..n-1) and the constant term of L_B.

    f_k = alpha_k - W_{k+1}^T alpha_{k+1} - sum_{I in B_k + {0,1}} beta_{k,I}
          + sum_{I in B_{k+1} + {0,1}} (W_{k+1} (.) I)^T beta_{k+1,I}
        (the I = 0 member is beta_{k,0}, the I = 1 member is beta_{k,1};
         alpha_0 = beta_0 = 0, alpha_n = c, beta_n = 0)
    g_k = sum_{B_k} UI (.) beta_I + beta_{k,0} (.) uhat_k + beta_{k,1} (.) lhat_k
          + sum_{B_k} LI (.) beta_I + sum_{B_k} beta_I (.) b_k
    const = sum_{k=1..n} b_k^T alpha_k + sum_{k=1..n-1} ( sum_{B_k} LI^T beta_I
            + beta_{k,1}^T (lhat_k - b_k) )
    """
    n = p.n
    alpha = lambda k: p.c if k == n else st.alpha[k - 1]
    f = []
    for k in range(0, n):
        op_next = p.W(k + 1)
        fk = -(op_next.W.T @ alpha(k + 1))
        if k + 1 <= n - 1:
            fk = fk + op_next.W.T @ st.beta1[k]
            for M in st.masks[k]:
                fk = fk + M.WI.T @ M.beta
        if k >= 1:
            own = st.alpha[k - 1] - st.beta0[k - 1] - st.beta1[k - 1]
            for M in st.masks[k - 1]:
                own = own - M.beta
            fk = fk + own
        f.append(fk)
    g = []
    const = float(p.W(n).b @ p.c)
    for k in range(1, n):
        lh, uh = p.hat(k)
        b = p.W(k).b
        gk = st.beta0[k - 1] * uh + st.beta1[k - 1] * lh
        const += float(b @ st.alpha[k - 1]) + float(st.beta1[k - 1] @ (lh - b))
        for M in st.masks[k - 1]:
            gk = gk + M.UI * M.beta + M.LI * M.beta + M.beta * b
            const += float(M.LI @ M.beta)
        g.append(gk)
    return f, g, const


def ball_maximiser(f0: np.ndarray, centre: np.ndarray, radius: float) -> np.ndarray:
    """argmax of f0^T x over the l2 ball ||x - centre|| <= radius: the centre
    moved by radius along f0 (the centre itself where f0 = 0)."""
    nrm = float(np.linalg.norm(f0))
    return centre.copy() if nrm == 0.0 else centre + radius * f0 / nrm


def inner_min(p: Problem, f, g):
    """Closed-form minimiser of L_B over the primal box (eq:as-primalk-min,
    eq:as-primal0-min, with readings R1, R2, R6); over an l2 ball input
    domain x*_0 maximises f_0^T x_0 on the ball (R2, R20)."""
    x = []
    for k in range(0, p.n):
        l, u = p.lu(k)
        if k == 0 and p.ball is not None:
            x.append(ball_maximiser(f[0], p.ball[0], p.ball[1]))
            continue
        x.append(np.where(f[k] >= 0, u, l))
    z = [np.where(gk >= 0, 1.0, 0.0) for gk in g]
    return x, z


def dual_value(f, g, const, x, z) -> float:
    """d_B = const - sum_k f_k^T x*_k - sum_k g_k^T z*_k (eq:dual-active-set)."""
    d = const
    for fk, xk in zip(f, x):
        d -= float(fk @ xk)
    for gk, zk in zip(g, z):
        d -= float(gk @ zk)
    return d


def evaluate(p: Problem, st: DualState):
    """d_B at the given duals with its primal minimiser (x*, z*) and f, g."""
    f, g, const = dual_functions(p, st)
    x, z = inner_min(p, f, g)
    return dual_value(f, g, const, x, z), x, z, f, g


def supergradient(p: Problem, st: DualState, x, z):
    """Supergradient of d_B at (x*, z*) (eq:as-supergradient, reading R3).

    grad alpha_k   = W_k x*_{k-1} + b_k - x*_k
    grad beta_k0   = x*_k - z*_k (.) uhat_k
    grad beta_k1   = x*_k - (W_k x*_{k-1} + b_k) + (1 - z*_k) (.) lhat_k
    grad beta_k,I  = x*_k - (W_k (.) I) x*_{k-1} + LI (.) (1 - z*_k)
                     - z*_k (.) b_k - UI (.) z*_k
    Returns dicts of lists over k = 1..n-1 (masks: list of lists).
    """
    ga, gb0, gb1, gI = [], [], [], []
    for k in range(1, p.n):
        op = p.W(k)
        lh, uh = p.hat(k)
        xh = op.W @ x[k - 1] + op.b
        xk, zk = x[k], z[k - 1]
        ga.append(xh - xk)
        gb0.append(xk - zk * uh)
        gb1.append(xk - xh + (1.0 - zk) * lh)
        gI.append([xk - M.WI @ x[k - 1] + M.LI * (1.0 - zk) - zk * op.b - M.UI * zk
                   for M in st.masks[k - 1]])
    return {"alpha": ga, "beta0": gb0, "beta1": gb1, "masks": gI}


# ----------------------------------------------------------------------------
# Updates (Sec. 7.1: Adam on the supergradient, then projection to >= 0)
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class AdamConsts:
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    # "exact": moments kept at full precision; "bf16": moments stored between
    # steps as bfloat16 (each step uses the unrounded update, then stores it
    # rounded); a storage choice of the implementation, not of the paper
    moments: str = "exact"


def round_bf16(a):
    """Nearest bfloat16 value (8 significant bits, float32's exponent range,
    ties to even) of each entry, returned as float64.  Written from the
    format's definition: the spacing of representable values in [2^e, 2^(e+1))
    is 2^(e-7), with e clamped at float32's smallest normal exponent -126."""
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = a != 0
    _, e = np.frexp(a[nz])                  # a = f 2^e with 0.5 <= |f| < 1
    q = np.ldexp(1.0, np.maximum(e - 1, -126) - 7)
    out[nz] = np.rint(a[nz] / q) * q        # rint rounds halves to even
    return out


def adam_ascent(theta, m, v, grad, step, lr, c: AdamConsts):
    """One projected Adam ascent step; returns (theta, m, v).

    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
    theta <- max(0, theta + lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)).
    With c.moments == "bf16" the returned (stored) moments are rounded to
    bfloat16.
    """
    m = c.beta1 * m + (1.0 - c.beta1) * grad
    v = c.beta2 * v + (1.0 - c.beta2) * grad * grad
    mhat = m / (1.0 - c.beta1 ** step)
    vhat = v / (1.0 - c.beta2 ** step)
    theta = np.maximum(theta + lr * mhat / (np.sqrt(vhat) + c.eps), 0.0)
    if c.moments == "bf16":
        m, v = round_bf16(m), round_bf16(v)
    return theta, m, v


def plain_ascent(theta, grad, lr):
    """Projected supergradient ascent step theta <- max(0, theta + lr g)."""
    return np.maximum(theta + lr * grad, 0.0)


def apply_step(st: DualState, grads, lr: float, rule: str, c: AdamConsts):
    if rule == "adam":
        st.step += 1
    for name in ("alpha", "beta0", "beta1"):
        vals = getattr(st, name)
        for i in range(len(vals)):
            if rule == "adam":
                vals[i], st.m[name][i], st.v[name][i] = adam_ascent(
                    vals[i], st.m[name][i], st.v[name][i], grads[name][i], st.step, lr, c)
            else:
                vals[i] = plain_ascent(vals[i], grads[name][i], lr)
    for k, masks in enumerate(st.masks):
        for M, gm in zip(masks, grads["masks"][k]):
            if rule == "adam":
                M.step += 1
                M.beta, M.m, M.v = adam_ascent(M.beta, M.m, M.v, gm, M.step, lr, c)
            else:
                M.beta = plain_ascent(M.beta, gm, lr)


def reset_moments(st: DualState):
    for name in ("alpha", "beta0", "beta1"):
        for i in range(len(st.m[name])):
            st.m[name][i] = np.zeros_like(st.m[name][i])
            st.v[name][i] = np.zeros_like(st.v[name][i])
    st.step = 0


def linear_lr(lr0: float, lr1: float, t: int, T: int) -> float:
    """Reading R10: linear decrease from lr0 (t = 0) to lr1 (t = T - 1)."""
    if T <= 1:
        return lr0
    return lr0 + (lr1 - lr0) * t / (T - 1)


# ----------------------------------------------------------------------------
# The solver (Algorithm 1, initialised by Algorithm 3)
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class SolveParams:
    bigm_iters: int = 180
    as_iters: int = 500
    add_every: int = 450
    add_count: int = 2
    max_masks: int = 7
    bigm_lr: tuple = (1e-2, 1e-4)
    as_lr: tuple = (1e-3, 1e-6)
    rule: str = "adam"
    adam: AdamConsts = dataclasses.field(default_factory=AdamConsts)
    # "exact": the state is kept in FP64; "fp32": after every iteration the
    # duals, moments and mask constants are stored as float32 values (a
    # storage choice of an implementation, not of the paper: it measures how
    # far FP32 rounding of the state alone moves a whole run)
    storage: str = "exact"


def params_from_schedule(s) -> SolveParams:
    return SolveParams(s.bigm_iters, s.as_iters, s.add_every, s.add_count, s.max_masks,
                       tuple(s.bigm_lr), tuple(s.as_lr), "adam",
                       AdamConsts(s.adam_beta1, s.adam_beta2, s.adam_eps))


def add_masks(p: Problem, st: DualState, x, z):
    """Active-set extension (Algorithm 1): for each layer k, append the
    oracle's mask called at the current (x*, z*) with beta_{k,I} = 0."""
    for k in range(1, p.n):
        if k == 1 and p.ball is not None:
            continue  # R20: at an interior x*_0 layer 1's masks repeat beta_0 / beta_1 constraints
        op = p.W(k)
        l_prev, u_prev = p.lu(k - 1)
        I = oracle_mask(op, l_prev, u_prev, x[k - 1], z[k - 1])
        st.masks[k - 1].append(new_mask(op, I, l_prev, u_prev, x[k - 1], z[k - 1]))


def is_addition_iter(t: int, prm: SolveParams, n_active: int) -> bool:
    """Reading R8."""
    return (t % prm.add_every) < prm.add_count and n_active < prm.max_masks


def round_state_fp32(st: DualState):
    """Every stored value of the state rounded to the nearest float32."""
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    for name in ("alpha", "beta0", "beta1"):
        vals = getattr(st, name)
        for i in range(len(vals)):
            vals[i] = r(vals[i])
            st.m[name][i] = r(st.m[name][i])
            st.v[name][i] = r(st.v[name][i])
    for masks in st.masks:
        for M in masks:
            M.beta, M.m, M.v, M.LI, M.UI = r(M.beta), r(M.m), r(M.v), r(M.LI), r(M.UI)


def bigm_iteration(p: Problem, st: DualState, lr: float, prm: SolveParams):
    """One iteration of Algorithm 3 (B empty): inner min, supergradient, step."""
    d, x, z, _, _ = evaluate(p, st)
    apply_step(st, supergradient(p, st, x, z), lr, prm.rule, prm.adam)
    if prm.storage == "fp32":
        round_state_fp32(st)
    return d


def as_iteration(p: Problem, st: DualState, t: int, lr: float, prm: SolveParams):
    """One iteration of Algorithm 1's inner loop."""
    d, x, z, _, _ = evaluate(p, st)
    n_active = max(len(m) for m in st.masks) if st.masks else 0
    if p.n > 1 and is_addition_iter(t, prm, n_active):
        add_masks(p, st, x, z)
    apply_step(st, supergradient(p, st, x, z), lr, prm.rule, prm.adam)
    if prm.storage == "fp32":
        round_state_fp32(st)
    return d


@dataclasses.dataclass
class SolveResult:
    bound: float
    x0: np.ndarray
    state: DualState
    trace: List[float]
    snapshots: dict


def solve(p: Problem, prm: SolveParams, snapshot_at: Sequence = (), trace: bool = False,
          state: Optional[DualState] = None) -> SolveResult:
    """Big-M initialisation (Algorithm 3) then Active Set (Algorithm 1).

    snapshot_at: iterations ("bigm", t) / ("as", t) whose state *before* the
    iteration is recorded (deep copies), plus ("as", T) for the end state.
    """
    st = zero_state(p) if state is None else state
    snaps, tr = {}, []
    want = set(snapshot_at)
    for t in range(prm.bigm_iters):
        if ("bigm", t) in want:
            snaps[("bigm", t)] = st.copy()
        d = bigm_iteration(p, st, linear_lr(*prm.bigm_lr, t, prm.bigm_iters), prm)
        if trace:
            tr.append(d)
    if prm.rule == "adam":
        reset_moments(st)
    for t in range(prm.as_iters):
        if ("as", t) in want:
            snaps[("as", t)] = st.copy()
        d = as_iteration(p, st, t, linear_lr(*prm.as_lr, t, prm.as_iters), prm)
        if trace:
            tr.append(d)
    if ("as", prm.as_iters) in want:
        snaps[("as", prm.as_iters)] = st.copy()
    d, x, _, _, _ = evaluate(p, st)
    return SolveResult(d, x[0], st, tr, snaps)


def solve_batch(problems: Sequence[Problem], prm: SolveParams) -> np.ndarray:
    return np.array([solve(p, prm).bound for p in problems])


# ----------------------------------------------------------------------------
# Intermediate bounds by the solver (App. E, eq:primal-intermediates)
# ----------------------------------------------------------------------------


def interval_step(op: LinearOp, l_prev: np.ndarray, u_prev: np.ndarray):
    """Interval propagation through one layer from the box [l_prev, u_prev]
    of its inputs (post-activation values)."""
    Wp = op.with_data(np.maximum(op.w, 0.0))
    Wm = op.with_data(np.minimum(op.w, 0.0))
    return Wp @ l_prev + Wm @ u_prev + op.b, Wp @ u_prev + Wm @ l_prev + op.b


def _f32_down(x: float) -> float:
    """The largest float32 value <= x."""
    f = np.float32(x)
    if float(f) > x:
        f = np.nextafter(f, np.float32(-np.inf))
    return float(f)


def _f32_up(x: float) -> float:
    """The smallest float32 value >= x."""
    f = np.float32(x)
    if float(f) < x:
        f = np.nextafter(f, np.float32(np.inf))
    return float(f)


def intermediate_bounds(ops: Sequence[LinearOp], l0, u0, prm: SolveParams, fp32_bounds: bool = False):
    """Pre-activation bounds of the ReLU layers 1..n-1 from problem
    eq:primal-intermediates (App. E), its relaxation's dual solved by the
    same schedule as the last layer's bound (Algorithm 3, then Algorithm 1).

    Layer 1: the problem is a box-constrained LP, solved exactly by interval
    propagation.  Layer i >= 2, neuron j: on the sub-network of layers 1..i
    (ReLU layers 1..i-1 with the bounds found before, layer i linear as the
    output) the objective row e_j gives d_j <= min x_hat_i[j] and -e_j gives
    d'_j <= -max x_hat_i[j] (weak duality: any dual point bounds the
    minimum); each is combined with interval propagation of layer i from
    the bounds of layer i-1: lhat_i[j] = max(ibp, d_j), uhat_i[j] =
    min(ibp, -d'_j).  Returns (lhat, uhat), lists over layers 1..n-1.

    fp32_bounds: each layer's bounds are stored as float32 values before the
    next layer uses them (a storage choice of an implementation, not of the
    paper), rounded outward (down for lhat, up for uhat) so that every stored
    bound stays valid.
    """
    l0 = np.asarray(l0, np.float64)
    u0 = np.asarray(u0, np.float64)
    lhat: List[np.ndarray] = []
    uhat: List[np.ndarray] = []
    l_prev, u_prev = l0, u0
    for i in range(1, len(ops)):
        lo, hi = interval_step(ops[i - 1], l_prev, u_prev)
        if fp32_bounds:
            lo = np.array([_f32_down(v) for v in lo])
            hi = np.array([_f32_up(v) for v in hi])
        if i >= 2:
            n_i = ops[i - 1].n_out
            for j in range(n_i):
                e = np.zeros(n_i)
                e[j] = 1.0
                d_lo = solve(make_problem(ops[:i], l0, u0, lhat, uhat, e), prm).bound
                d_hi = solve(make_problem(ops[:i], l0, u0, lhat, uhat, -e), prm).bound
                if fp32_bounds:
                    d_lo, d_hi = _f32_down(d_lo), -_f32_up(-d_hi)
                lo[j] = max(lo[j], d_lo)
                hi[j] = min(hi[j], -d_hi)
        lhat.append(lo)
        uhat.append(hi)
        l_prev, u_prev = np.maximum(lo, 0.0), np.maximum(hi, 0.0)
    return lhat, uhat


# ----------------------------------------------------------------------------
# Lagrangian in constraint form (App. D), used to check dual_functions
# ----------------------------------------------------------------------------


def lagrangian_constraint_form(p: Problem, st: DualState, x, z) -> float:
    """L(x, z, alpha, beta) written constraint by constraint (App. D):

    sum_k alpha_k^T (W_k x_{k-1} + b_k - x_k) + beta_k0^T (x_k - z_k uhat_k)
    + sum_I beta_I^T (LI (1 - z_k) - (W (.) I) x_{k-1} - b_k z_k - UI z_k + x_k)
    + beta_k1^T (x_k - (W_k x_{k-1} + b_k) + (1 - z_k) lhat_k)
    + c^T (W_n x_{n-1} + b_n).
    """
    L = float(p.c @ (p.W(p.n).W @ x[p.n - 1] + p.W(p.n).b))
    for k in range(1, p.n):
        op = p.W(k)
        lh, uh = p.hat(k)
        xh = op.W @ x[k - 1] + op.b
        xk, zk = x[k], z[k - 1]
        L += float(st.alpha[k - 1] @ (xh - xk))
        L += float(st.beta0[k - 1] @ (xk - zk * uh))
        L += float(st.beta1[k - 1] @ (xk - xh + (1.0 - zk) * lh))
        for M in st.masks[k - 1]:
            L += float(M.beta @ (M.LI * (1.0 - zk) - M.WI @ x[k - 1] - op.b * zk
                                 - M.UI * zk + xk))
    return L


# ----------------------------------------------------------------------------
# Gradient of the bound at fixed duals (the adjoint)
# ----------------------------------------------------------------------------


def bound_gradient(p: Problem, st: DualState):
    """Gradient of d_B with respect to every weight, bias and the input box,
    at fixed duals and fixed active sets, the pre-activation bounds l_hat,
    u_hat of layers 1..n-1 held as given inputs.

    d_B = min over the primal box of the Lagrangian (constraint form, App. D);
    it is linear in (x, z) and the minimiser (x*, z*) is a box vertex, so
    (Danskin) its gradient is the Lagrangian's partial derivative at
    (x*, z*) wherever the minimiser is unique:
      dd/dW_k[i,j] = x*_{k-1}[j] (alpha_k[i] - beta_{k,1}[i] - sum_I I[i,j] beta_I[i])
                     + sum_I beta_I[i] ((1 - z*_k[i]) I[i,j] Lchk[i,j]
                                        - z*_k[i] (1 - I[i,j]) Uchk[i,j]),
      dd/db_k[i]   = alpha_k[i] - beta_{k,1}[i] - z*_k[i] sum_I beta_I[i],
    (box input domains only)
    for k = 1..n-1 (LI and UI are the row sums of W . I . Lchk and
    W . (1 - I) . Uchk, Sec. 2.2, with the check entries chosen by the sign
    of W); for the last layer dd/dW_n = c x*_{n-1}^T, dd/db_n = c.  The input
    box enters through x*_0 (dd/du_0 = -f_0 where f_0 >= 0, dd/dl_0 = -f_0
    where f_0 < 0) and through the check entries of layer 1's mask
    constants.  Returns (dW, db, dl0, du0): dW[k-1] and db[k-1] in the shapes
    of layer k's weight tensor and bias (entries of a convolution summed over
    positions)."""
    if p.ball is not None:
        raise ValueError("the bound gradient is defined here for box input domains")
    d, x, z, f, g = evaluate(p, st)
    n = p.n
    dW, db = [], []
    dl0 = np.zeros_like(p.l0)
    du0 = np.zeros_like(p.u0)
    for k in range(1, n + 1):
        op = p.W(k)
        rows, cols, w = op.rows, op.cols, op.w
        xprev = x[k - 1]
        nw = int(op.widx.max()) + 1
        nb = int(op.bidx.max()) + 1
        if k == n:
            ge = p.c[rows] * xprev[cols]
            gb = p.c.copy()
        else:
            a = st.alpha[k - 1] - st.beta1[k - 1]
            ge = a[rows] * xprev[cols]
            zk = z[k - 1]
            gb = a - zk * sum((M.beta for M in st.masks[k - 1]), np.zeros(op.n_out))
            lp, up = p.lu(k - 1)
            Lchk, Uchk = check_matrices(op, lp, up)
            for M in st.masks[k - 1]:
                If = M.I.astype(np.float64)
                br, zr = M.beta[rows], zk[rows]
                ge = ge - If * br * xprev[cols]
                ge = ge + br * ((1.0 - zr) * If * Lchk - zr * (1.0 - If) * Uchk)
                if k == 1:
                    # check entries of the input box: Lchk = l0 (W >= 0) or u0, Uchk = u0 (W >= 0) or l0
                    pos = w >= 0
                    cl = br * ((1.0 - zr) * If * w * pos - zr * (1.0 - If) * w * (~pos))
                    cu = br * ((1.0 - zr) * If * w * (~pos) - zr * (1.0 - If) * w * pos)
                    np.add.at(dl0, cols, cl)
                    np.add.at(du0, cols, cu)
        gw = np.zeros(nw)
        np.add.at(gw, op.widx, ge)
        gbb = np.zeros(nb)
        np.add.at(gbb, op.bidx, gb)
        dW.append(gw)
        db.append(gbb)
    dl0 += np.where(f[0] < 0, -f[0], 0.0)
    du0 += np.where(f[0] >= 0, -f[0], 0.0)
    return dW, db, dl0, du0
