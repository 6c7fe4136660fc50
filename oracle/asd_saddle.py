"""FP64 CPU oracle of the Saddle Point solver (SP-FW on sufficient statistics).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library and imports nothing from it; it builds on asd_oracle.py (the
Active Set / Big-M oracle) for the problem, the check matrices and the dual
functions.

Source: De Palma et al., "Scaling the Convex Barrier with Sparse Dual
Algorithms" (arXiv:2101.05844), Sec. 5 and App. C:

  * sufficient statistics ......... Sec. 5.1, eq:suff-stats, Fact on the
                                    dual at the cost of a backward pass
  * restricted dual domain ........ Sec. 5.1, eq:sp-fw-dual (price caps mu)
  * Saddle Point loop ............. Sec. 5, Algorithm 2 (alg:sp-fw)
  * conditional gradients ......... Sec. 5.2, eq:alphak-condg,
                                    eq:betak-condg and the proposition after it
  * price caps .................... App. C.1, eq:price-caps
  * primal initialisation ......... App. C.2 (simplified form, Big-M duals)
  * step sizes .................... Sec. 7.1 (gamma_t = 1/(t + 10); 100
                                    primal steps from 1e-2 to 1e-5)

Notation.  For ReLU layer k (1..n-1) the multipliers beta_{k,I} of every
mask I (the all-zero mask is beta_{k,0} with bound uhat, the all-one mask
beta_{k,1} with bound lhat) enter the Lagrangian only through four
linearly-sized sums (eq:suff-stats):

  zeta1_k = sum_I beta_{k,I}                                 (layer k)
  zeta2_k = sum_I (W_k (.) I)^T beta_{k,I}                   (layer k-1)
  zeta3_k = beta_{k,1} (lhat_k - b_k) + sum_{I in E_k} LI beta_{k,I}
  zeta4_k = beta_{k,0} (uhat_k - b_k) + sum_{I in E_k} UI beta_{k,I}

with LI = (W (.) I (.) Lchk) <> 1 and UI = (W (.) (1 - I) (.) Uchk) <> 1.
The dual functions then read f_k = alpha_k - zeta1_k - W_{k+1}^T alpha_{k+1}
+ zeta2_{k+1}, g_k = zeta3_k + zeta4_k + b_k zeta1_k, and the constant term
sum_k b_k^T alpha_k + sum_k 1^T zeta3_k, with L = const - sum f^T x - sum g^T z
(the convention of asd_oracle.dual_functions).

Readings (kept with the design notes too):

  S1  The fourth sum of eq:suff-stats takes the complement mask (1 - I)
      with the U-check matrix, as its beta_{k,0} term (uhat - b) and the
      constraint of eq:primal-anderson require; the printed I is read as a
      slip.
  S2  The dual conditional gradient is taken at the current primal iterate
      (x^t, z^t) and the primal one at the current duals (SP-FW's
      simultaneous step); Algorithm 2 computes both before the update.
  S3  The most violated constraint per neuron is chosen among beta_{k,0},
      beta_{k,1} and the oracle's mask I* (eq:oracle over all masks); ties
      go to beta_{k,0}, then beta_{k,1}, then I*.  The vertex puts mu_beta on
      it when its violation is >= 0 (eq:betak-condg), else the vertex is 0.
      The oracle's decision per weight is written as
      (l - x) + z (u - l) >= 0 for W >= 0 and (u - x) - z (u - l) <= 0 for
      W < 0, the same inequality as eq:oracle's
      ((1 - z) Lchk + z Uchk - x) W >= 0, arranged so that a point box
      (l = u = x) gives an exact tie (mask bit 1, reading R6).
  S4  gamma_t = 1 / (t + gamma0) with gamma0 = 10 (Sec. 7.1; Sec. 5.2's
      1 / (1 + t) is gamma0 = 1).
  S5  Price caps (eq:price-caps) per neuron: mu_alpha = alpha^0 where
      alpha^0 > 0, else c_alpha; mu_beta = zeta1^0 (the sum of all beta^0
      of the neuron) where > 0, else c_beta; c_alpha = c_beta = 1e-3 (the
      paper says only "small positive constants").
  S6  The primal initialisation starts at the inner minimiser (x*, z*) of
      the initial duals and takes plain projected subgradient steps on the
      Big-M primal view with the caps above: x_k <- clip(x_k + eta f_k),
      z_k <- clip(z_k + eta g_k) (L carries -f^T x - g^T z), with f, g the
      Big-M dual functions (reading R4) at the inner maximiser (alpha*,
      beta*) given by the conditional-gradient rules restricted to
      beta_{k,0}, beta_{k,1} (ties to beta_{k,0}); eta decreases linearly
      over the steps (reading R10).
  S7  The returned bound is d(alpha^T, zeta^T) (Algorithm 2's return).
  S8  Box input domains only: the l2-ball domain is not combined with
      Saddle Point here.
  S9  The oracle mask's violation is evaluated as
      x - (((W . I) x - LI (1 - z)) + z (b + UI)), the quantity of
      eq:as-supergradient with its terms grouped so that the exact ties with
      beta_{k,0} and beta_{k,1} come out exact in floating point too: at
      z = 1 the oracle's row is full (UI = 0) and the value is computed as
      beta_{k,1}'s x - (W x + b) + (1 - z) lhat; at z = 0 its columns sit at
      their check corners, (W . I) x and LI are the same sum, and the value is
      x, as beta_{k,0}'s x - z uhat.  S3 then picks beta_{k,1} (beta_{k,0})
      whatever the summation order of the products.
  S10 The convex combination of the primal iterate is clipped to the boxes
      ([l_k, u_k], [0, 1]): a no-op in exact arithmetic, it keeps rounding
      from moving an entry one unit outside its box, where the oracle's
      test (S3) would set a bit without the entry sitting at its corner.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import asd_oracle as O


@dataclasses.dataclass
class SPParams:
    iters: int = 100             # T (Algorithm 2)
    gamma0: float = 10.0         # S4
    init_steps: int = 100        # App. C.2 / Sec. 7.1
    init_lr: tuple = (1e-2, 1e-5)
    cap_alpha: float = 1e-3      # S5
    cap_beta: float = 1e-3
    # "exact": the state is kept in FP64; "fp32": after the set-up and after
    # every iteration the state is stored as float32 values (a storage choice
    # of an implementation, not of the paper: it measures how far FP32
    # rounding of the state alone moves a run)
    storage: str = "exact"


@dataclasses.dataclass
class SPState:
    """Duals (alpha, zeta) and the SP-FW primal iterate (x, z), with caps.

    Lists over layers k = 1..n-1 at index k-1, except x over k = 0..n-1.
    """
    alpha: List[np.ndarray]
    zeta1: List[np.ndarray]
    zeta2: List[np.ndarray]      # zeta2[k-1] has the size of layer k-1
    zeta3: List[np.ndarray]
    zeta4: List[np.ndarray]
    mu_alpha: List[np.ndarray]
    mu_beta: List[np.ndarray]
    x: List[np.ndarray]
    z: List[np.ndarray]

    def round_fp32(self):
        """Every stored value rounded to the nearest float32."""
        for f in dataclasses.fields(self):
            setattr(self, f.name, [np.asarray(a, dtype=np.float32).astype(np.float64)
                                   for a in getattr(self, f.name)])

    def copy(self) -> "SPState":
        return dataclasses.replace(self, **{f.name: [a.copy() for a in getattr(self, f.name)]
                                           for f in dataclasses.fields(self)})


# ----------------------------------------------------------------------------
# Sufficient statistics (eq:suff-stats) and the dual through them
# ----------------------------------------------------------------------------


def suff_stats(p: O.Problem, st: O.DualState):
    """zeta(beta) of explicit duals: beta_{k,0}, beta_{k,1} and the masks of B_k."""
    z1, z2, z3, z4 = [], [], [], []
    for k in range(1, p.n):
        op = p.W(k)
        lh, uh = p.hat(k)
        b0, b1 = st.beta0[k - 1], st.beta1[k - 1]
        s1 = b0 + b1
        s2 = op.W.T @ b1
        s3 = b1 * (lh - op.b)
        s4 = b0 * (uh - op.b)
        for M in st.masks[k - 1]:
            s1 = s1 + M.beta
            s2 = s2 + M.WI.T @ M.beta
            s3 = s3 + M.LI * M.beta
            s4 = s4 + M.UI * M.beta
        z1.append(s1)
        z2.append(s2)
        z3.append(s3)
        z4.append(s4)
    return z1, z2, z3, z4


def sp_dual_functions(p: O.Problem, alpha, z1, z2, z3, z4):
    """f_k (k = 0..n-1), g_k (k = 1..n-1) and the constant of L from (alpha, zeta)."""
    n = p.n
    al = lambda k: p.c if k == n else alpha[k - 1]
    f = []
    for k in range(0, n):
        fk = -(p.W(k + 1).W.T @ al(k + 1))
        if k + 1 <= n - 1:
            fk = fk + z2[k]
        if k >= 1:
            fk = fk + alpha[k - 1] - z1[k - 1]
        f.append(fk)
    g = []
    const = float(p.W(n).b @ p.c)
    for k in range(1, n):
        b = p.W(k).b
        g.append(z3[k - 1] + z4[k - 1] + b * z1[k - 1])
        const += float(b @ alpha[k - 1]) + float(np.sum(z3[k - 1]))
    return f, g, const


def sp_evaluate(p: O.Problem, s: SPState):
    """d(alpha, zeta) with its primal minimiser (the primal conditional gradient)."""
    f, g, const = sp_dual_functions(p, s.alpha, s.zeta1, s.zeta2, s.zeta3, s.zeta4)
    x, z = O.inner_min(p, f, g)
    return O.dual_value(f, g, const, x, z), x, z, f, g


# ----------------------------------------------------------------------------
# Conditional gradients (eq:alphak-condg, eq:betak-condg)
# ----------------------------------------------------------------------------


def oracle_mask_continuous(op: O.LinearOp, l_prev, u_prev, x_prev, z):
    """eq:oracle at a fractional z (reading S3's arrangement of the test)."""
    r, j, w = op.rows, op.cols, op.w
    l, u, x = l_prev[j], u_prev[j], x_prev[j]
    zr = z[r]
    pos = (l - x) + zr * (u - l) >= 0.0
    neg = (u - x) - zr * (u - l) <= 0.0
    return np.where(w >= 0, pos, neg)


def violations(p: O.Problem, k: int, x_prev, xk, zk):
    """Constraint violations (the beta gradients of L) at (x, z) for layer k:
    alpha, beta_0, beta_1 and the oracle mask I* with its LI, UI and W (.) I*."""
    op = p.W(k)
    lh, uh = p.hat(k)
    l_prev, u_prev = p.lu(k - 1)
    xh = op.W @ x_prev + op.b
    I = oracle_mask_continuous(op, l_prev, u_prev, x_prev, zk)
    LI, UI = O.mask_constants(op, I, l_prev, u_prev)
    WI = op.with_data(op.w * I.astype(np.float64))
    v_alpha = xh - xk
    v0 = xk - zk * uh
    v1 = xk - xh + (1.0 - zk) * lh
    vI = xk - ((WI @ x_prev - LI * (1.0 - zk)) + zk * (op.b + UI))  # S9
    return v_alpha, v0, v1, vI, I, LI, UI, WI


def vertex_choice(v0, v1, vI):
    """Per neuron: 0 (beta_0), 1 (beta_1) or 2 (I*) by S3's ties, and whether
    the chosen violation is >= 0."""
    best = v0.copy()
    ch = np.zeros(v0.shape, dtype=np.int64)
    m1 = v1 > best
    best = np.where(m1, v1, best)
    ch = np.where(m1, 1, ch)
    m2 = vI > best
    best = np.where(m2, vI, best)
    ch = np.where(m2, 2, ch)
    return ch, best >= 0.0


def dual_conditional_gradient(p: O.Problem, s: SPState):
    """(alpha_bar, zeta_bar) at the primal iterate (x, z) (reading S2)."""
    ab, z1, z2, z3, z4 = [], [], [], [], []
    for k in range(1, p.n):
        op = p.W(k)
        lh, uh = p.hat(k)
        va, v0, v1, vI, I, LI, UI, WI = violations(p, k, s.x[k - 1], s.x[k], s.z[k - 1])
        mua, mub = s.mu_alpha[k - 1], s.mu_beta[k - 1]
        ab.append(np.where(va >= 0.0, mua, 0.0))
        ch, on = vertex_choice(v0, v1, vI)
        w = np.where(on, mub, 0.0)
        w0, w1, w2 = w * (ch == 0), w * (ch == 1), w * (ch == 2)
        z1.append(w)
        z2.append(op.W.T @ w1 + WI.T @ w2)
        z3.append(w1 * (lh - op.b) + w2 * LI)
        z4.append(w0 * (uh - op.b) + w2 * UI)
    return ab, z1, z2, z3, z4


def primal_view_value(p: O.Problem, s: SPState, x=None, z=None) -> float:
    """max over the restricted dual domain of L at a primal point (x, z): the
    objective plus, per neuron, the caps times the positive parts of the
    alpha violation and of the largest beta violation (the domain of
    eq:sp-fw-dual is a box in alpha and a capped simplex per neuron in beta).
    Weak duality: this is >= d(alpha, zeta) for every feasible dual point."""
    x = s.x if x is None else x
    z = s.z if z is None else z
    opn = p.W(p.n)
    val = float(p.c @ (opn.W @ x[p.n - 1] + opn.b))
    for k in range(1, p.n):
        va, v0, v1, vI, *_ = violations(p, k, x[k - 1], x[k], z[k - 1])
        vb = np.maximum(np.maximum(v0, v1), vI)
        val += float(s.mu_alpha[k - 1] @ np.maximum(va, 0.0)) + float(s.mu_beta[k - 1] @ np.maximum(vb, 0.0))
    return val


# ----------------------------------------------------------------------------
# Initialisation: duals to sufficient statistics, caps, primal iterate
# ----------------------------------------------------------------------------


def price_caps(alpha, zeta1, c_alpha: float, c_beta: float):
    """eq:price-caps (reading S5)."""
    mua = [np.where(a > 0.0, a, c_alpha) for a in alpha]
    mub = [np.where(s > 0.0, s, c_beta) for s in zeta1]
    return mua, mub


def bigm_inner_max(p: O.Problem, mua, mub, x, z):
    """Inner maximiser of the Big-M primal view at (x, z): alpha* and beta*_0,
    beta*_1 by the conditional-gradient rules (App. C.2, reading S6)."""
    a, b0, b1 = [], [], []
    for k in range(1, p.n):
        op = p.W(k)
        lh, uh = p.hat(k)
        xh = op.W @ x[k - 1] + op.b
        xk, zk = x[k], z[k - 1]
        va = xh - xk
        v0 = xk - zk * uh
        v1 = xk - xh + (1.0 - zk) * lh
        a.append(np.where(va >= 0.0, mua[k - 1], 0.0))
        pick1 = v1 > v0
        on = np.maximum(v0, v1) >= 0.0
        b0.append(np.where(on & ~pick1, mub[k - 1], 0.0))
        b1.append(np.where(on & pick1, mub[k - 1], 0.0))
    return a, b0, b1


def primal_init(p: O.Problem, mua, mub, x, z, steps: int, lr: tuple):
    """App. C.2, simplified: projected subgradient descent on the Big-M
    primal view (reading S6)."""
    x = [a.copy() for a in x]
    z = [a.copy() for a in z]
    for tau in range(steps):
        eta = O.linear_lr(lr[0], lr[1], tau, steps)
        a, b0, b1 = bigm_inner_max(p, mua, mub, x, z)
        st = O.zero_state(p)
        st.alpha, st.beta0, st.beta1 = a, b0, b1
        f, g, _ = O.dual_functions(p, st)
        for k in range(0, p.n):
            l, u = p.lu(k)
            x[k] = np.clip(x[k] + eta * f[k], l, u)
        for k in range(1, p.n):
            z[k - 1] = np.clip(z[k - 1] + eta * g[k - 1], 0.0, 1.0)
    return x, z


def sp_init(p: O.Problem, st: O.DualState, prm: SPParams) -> SPState:
    """Algorithm 2's set-up from Big-M or Active Set duals: sufficient
    statistics, caps, primal iterate."""
    if p.ball is not None:
        raise ValueError("Saddle Point takes box input domains (reading S8)")
    z1, z2, z3, z4 = suff_stats(p, st)
    alpha = [a.copy() for a in st.alpha]
    mua, mub = price_caps(alpha, z1, prm.cap_alpha, prm.cap_beta)
    s = SPState(alpha, z1, z2, z3, z4, mua, mub, [], [])
    _, s.x, s.z, _, _ = sp_evaluate(p, s)  # the inner minimiser of the initial duals
    s.x, s.z = primal_init(p, mua, mub, s.x, s.z, prm.init_steps, prm.init_lr)
    if prm.storage == "fp32":
        s.round_fp32()
    return s


# ----------------------------------------------------------------------------
# The loop (Algorithm 2)
# ----------------------------------------------------------------------------


def sp_iteration(p: O.Problem, s: SPState, t: int, prm: SPParams):
    """One SP-FW step: both conditional gradients, then the convex
    combination with gamma_t.  Returns d at the duals before the step."""
    d, xb, zb, _, _ = sp_evaluate(p, s)
    ab, b1, b2, b3, b4 = dual_conditional_gradient(p, s)
    gam = 1.0 / (t + prm.gamma0)
    mix = lambda cur, bar: [(1.0 - gam) * c + gam * v for c, v in zip(cur, bar)]
    # S10: the combination stays in the boxes in exact arithmetic
    s.x = [np.clip(v, *p.lu(k)) for k, v in enumerate(mix(s.x, xb))]
    s.z = [np.clip(v, 0.0, 1.0) for v in mix(s.z, zb)]
    s.alpha = mix(s.alpha, ab)
    s.zeta1 = mix(s.zeta1, b1)
    s.zeta2 = mix(s.zeta2, b2)
    s.zeta3 = mix(s.zeta3, b3)
    s.zeta4 = mix(s.zeta4, b4)
    if prm.storage == "fp32":
        s.round_fp32()
    return d


@dataclasses.dataclass
class SPResult:
    bound: float
    init_bound: float
    state: SPState
    trace: List[float]


def sp_solve(p: O.Problem, st: O.DualState, prm: SPParams, trace: bool = False) -> SPResult:
    """Saddle Point from the given duals (Big-M for SP, Active Set for AS-SP)."""
    s = sp_init(p, st, prm)
    d0 = sp_evaluate(p, s)[0]
    tr = []
    for t in range(prm.iters):
        d = sp_iteration(p, s, t, prm)
        if trace:
            tr.append(d)
    return SPResult(sp_evaluate(p, s)[0], d0, s, tr)


def solve_sp(p: O.Problem, prm: O.SolveParams, sprm: SPParams, trace: bool = False) -> SPResult:
    """Big-M (and Active Set when prm.as_iters > 0) followed by Saddle Point."""
    res = O.solve(p, prm)
    return sp_solve(p, res.state, sprm, trace)
