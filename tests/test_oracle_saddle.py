"""Pins of the Saddle Point oracle (Sec. 5, App. C) against facts the paper
and the mathematics fix: the Active Set oracle's dual on explicit
multipliers (itself pinned), brute-force enumeration of the constraints,
a constraint-by-constraint Lagrangian, finite differences, weak duality and
the LP optimum of the relaxation."""
import itertools

import numpy as np
import pytest

from oracle import asd_oracle as O
from oracle import asd_saddle as SP
from oracle import lp
from paper_2101_05844_amd import workloads as WL


def tiny_problem(seed=1000, point_inputs=0):
    w = WL.tiny_config(seed)
    ops = O.ops_from_workload_layers(w.layers)
    l0, u0 = w.l0[0].astype(np.float64), w.u0[0].astype(np.float64)
    if point_inputs:
        u0[:point_inputs] = l0[:point_inputs]
    lh, uh = O.interval_bounds(ops, l0, u0)
    return w, ops, O.make_problem(ops, l0, u0, lh[:-1], uh[:-1], w.c[0])


def random_state(p, rng, n_masks=2):
    st = O.zero_state(p)
    for k in range(1, p.n):
        op = p.W(k)
        n = op.n_out
        st.alpha[k - 1] = rng.uniform(0, 1, n)
        st.beta0[k - 1] = rng.uniform(0, 1, n)
        st.beta1[k - 1] = rng.uniform(0, 1, n)
        lp_, up_ = p.lu(k - 1)
        for _ in range(n_masks):
            I = rng.integers(0, 2, op.w.size).astype(bool)
            M = O.new_mask(op, I, lp_, up_, lp_, np.zeros(n))
            M.beta = rng.uniform(0, 1, n)
            st.masks[k - 1].append(M)
    return st


def random_primal(p, rng):
    x = []
    for k in range(p.n):
        l, u = p.lu(k)
        x.append(l + rng.uniform(0, 1, l.size) * (u - l))
    z = [rng.uniform(0, 1, p.W(k).n_out) for k in range(1, p.n)]
    return x, z


def sp_state_from(p, st, x, z, rng):
    z1, z2, z3, z4 = SP.suff_stats(p, st)
    mua = [a + rng.uniform(0.1, 1, a.size) for a in st.alpha]
    mub = [s + rng.uniform(0.1, 1, s.size) for s in z1]
    return SP.SPState([a.copy() for a in st.alpha], z1, z2, z3, z4, mua, mub,
                      [a.copy() for a in x], [a.copy() for a in z])


# ----------------------------------------------------------------------------
# Fact (Sec. 5.1): the dual through sufficient statistics is the dual
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_suff_stats_dual_equals_explicit_dual(seed):
    _, _, p = tiny_problem()
    rng = np.random.default_rng(seed)
    st = random_state(p, rng, n_masks=3)
    d_ref, x_ref, z_ref, f_ref, g_ref = O.evaluate(p, st)
    z1, z2, z3, z4 = SP.suff_stats(p, st)
    f, g, const = SP.sp_dual_functions(p, st.alpha, z1, z2, z3, z4)
    for a, b in zip(f, f_ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
    for a, b in zip(g, g_ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
    x, z = O.inner_min(p, f, g)
    assert abs(O.dual_value(f, g, const, x, z) - d_ref) <= 1e-12 * (1 + abs(d_ref))
    # and the constraint-by-constraint Lagrangian at any primal point
    xr, zr = random_primal(p, rng)
    L_ref = O.lagrangian_constraint_form(p, st, xr, zr)
    assert abs(O.dual_value(f, g, const, xr, zr) - L_ref) <= 1e-12 * (1 + abs(L_ref))


# ----------------------------------------------------------------------------
# eq:betak-condg and the proposition after it: the vertex is the most violated
# constraint of A_k, found by brute force over every mask and beta_0, beta_1
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("point_inputs", [0, 2])
def test_most_violated_constraint_bruteforce(point_inputs):
    _, _, p = tiny_problem(point_inputs=point_inputs)
    rng = np.random.default_rng(21 + point_inputs)
    for trial in range(4):
        x, z = random_primal(p, rng)
        for k in (1, 2):
            op = p.W(k)
            W = op.W.toarray()
            lh, uh = p.hat(k)
            lp_, up_ = p.lu(k - 1)
            va, v0, v1, vI, I, LI, UI, WI = SP.violations(p, k, x[k - 1], x[k], z[k - 1])
            ch, on = SP.vertex_choice(v0, v1, vI)
            xh = W @ x[k - 1] + op.b
            for i in range(op.n_out):
                cols = op.W.indices[op.W.indptr[i]:op.W.indptr[i + 1]]
                zi, xi = z[k - 1][i], x[k][i]

                def rhs(bits):
                    # x_k[i] <= rhs: the Anderson constraint of mask bits (eq:primal-anderson)
                    v = zi * op.b[i]
                    for t, j in enumerate(cols):
                        Lc = lp_[j] if W[i, j] >= 0 else up_[j]
                        Uc = up_[j] if W[i, j] >= 0 else lp_[j]
                        v += (W[i, j] * x[k - 1][j] - W[i, j] * Lc * (1 - zi)) if bits[t] else W[i, j] * Uc * zi
                    return v

                cands = {("I",) + bits: xi - rhs(bits) for bits in itertools.product((0, 1), repeat=len(cols))}
                cands[("b0",)] = xi - zi * uh[i]                        # x <= z uhat
                cands[("b1",)] = xi - (xh[i] - (1 - zi) * lh[i])        # x <= x_hat - (1 - z) lhat
                best = max(cands.values())
                mine = {0: v0[i], 1: v1[i], 2: vI[i]}[int(ch[i])]
                assert abs(mine - best) <= 1e-12
                assert bool(on[i]) == (best >= 0)
                # the oracle's row attains the best mask violation
                s, e = op.W.indptr[i], op.W.indptr[i + 1]
                assert abs(xi - rhs(tuple(int(b) for b in I[s:e])) - vI[i]) <= 1e-12
                assert vI[i] >= max(v for key, v in cands.items() if key[0] == "I") - 1e-12
                # alpha's violation is the ReLU equality's residual x_hat - x
                assert abs(va[i] - (xh[i] - xi)) <= 1e-12


def test_point_box_columns_tie_to_mask_bit_one():
    # eq:oracle at a point box: both choices give the same violation; the
    # arranged test gives an exact tie, hence bit 1 (readings R6, S3)
    _, _, p = tiny_problem(point_inputs=3)
    rng = np.random.default_rng(5)
    x, z = random_primal(p, rng)
    op = p.W(1)
    I = SP.oracle_mask_continuous(op, p.l0, p.u0, x[0], z[0])
    pt = np.isin(op.cols, np.arange(3))
    assert pt.any() and np.all(I[pt])


# ----------------------------------------------------------------------------
# Algorithm 2 in the space of zeta against the same steps on explicit
# multipliers (every vertex kept as its own mask), evaluated by the Active Set
# oracle's dual
# ----------------------------------------------------------------------------


def test_iterations_match_explicit_multipliers():
    _, _, p = tiny_problem()
    prm = O.params_from_schedule(WL.tiny_config().schedule)
    prm.as_iters = 20
    init = O.solve(p, prm).state
    sprm = SP.SPParams(iters=0, init_steps=30)
    s = SP.sp_init(p, init, sprm)
    ex = init.copy()
    for t in range(25):
        d_ex = O.evaluate(p, ex)[0]
        d_sp = SP.sp_evaluate(p, s)[0]
        assert abs(d_sp - d_ex) <= 1e-11 * (1 + abs(d_ex)), t
        z1, z2, z3, z4 = SP.suff_stats(p, ex)
        for a, b in zip(s.zeta1 + s.zeta2 + s.zeta3 + s.zeta4 + s.alpha, z1 + z2 + z3 + z4 + ex.alpha):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
        # the vertex on explicit multipliers, from the violations
        gam = 1.0 / (t + sprm.gamma0)
        for k in range(1, p.n):
            op = p.W(k)
            lp_, up_ = p.lu(k - 1)
            va, v0, v1, vI, I, LI, UI, WI = SP.violations(p, k, s.x[k - 1], s.x[k], s.z[k - 1])
            ch, on = SP.vertex_choice(v0, v1, vI)
            w = np.where(on, s.mu_beta[k - 1], 0.0)
            ex.alpha[k - 1] = (1 - gam) * ex.alpha[k - 1] + gam * np.where(va >= 0, s.mu_alpha[k - 1], 0.0)
            ex.beta0[k - 1] = (1 - gam) * ex.beta0[k - 1] + gam * w * (ch == 0)
            ex.beta1[k - 1] = (1 - gam) * ex.beta1[k - 1] + gam * w * (ch == 1)
            for M in ex.masks[k - 1]:
                M.beta = (1 - gam) * M.beta
            M = O.new_mask(op, I, lp_, up_, s.x[k - 1], s.z[k - 1])
            M.beta = gam * w * (ch == 2)
            ex.masks[k - 1].append(M)
        SP.sp_iteration(p, s, t, sprm)
        # feasibility in the restricted domain (eq:sp-fw-dual)
        for a, mu in zip(ex.alpha, s.mu_alpha):
            assert np.all(a >= 0) and np.all(a <= mu * (1 + 1e-12))
        for k in range(1, p.n):
            tot = ex.beta0[k - 1] + ex.beta1[k - 1] + sum(M.beta for M in ex.masks[k - 1])
            assert np.all(tot <= s.mu_beta[k - 1] * (1 + 1e-12))


# ----------------------------------------------------------------------------
# Weak duality, validity and convergence of the duality gap
# ----------------------------------------------------------------------------


@pytest.mark.slow
def test_weak_duality_validity_and_gap():
    w, ops, p = tiny_problem()
    v_a = lp.lp_value(ops, p.l0, p.u0, p.lhat, p.uhat, p.c, "anderson")
    prm = O.params_from_schedule(w.schedule)
    init = O.solve(p, prm)
    sprm = SP.SPParams(iters=0)
    s = SP.sp_init(p, init.state, sprm)
    # T = 0 reproduces the bound of the duals it starts from
    assert abs(SP.sp_evaluate(p, s)[0] - init.bound) <= 1e-12 * (1 + abs(init.bound))
    gaps = []
    for t in range(600):
        d = SP.sp_evaluate(p, s)[0]
        pv = SP.primal_view_value(p, s)
        assert pv >= d - 1e-12           # weak duality of eq:sp-fw-dual
        assert d <= v_a + 1e-9           # a dual value bounds the relaxation's optimum
        gaps.append(pv - d)
        SP.sp_iteration(p, s, t, sprm)
    assert gaps[-1] < 0.25 * gaps[10]
    # the iterates improve on the initial bound on this problem
    assert SP.sp_evaluate(p, s)[0] > init.bound


# ----------------------------------------------------------------------------
# App. C: caps and the primal initialisation
# ----------------------------------------------------------------------------


def test_price_caps_contain_the_initial_duals():
    _, _, p = tiny_problem()
    rng = np.random.default_rng(3)
    st = random_state(p, rng)
    for k in range(1, p.n):
        st.alpha[k - 1][::3] = 0.0
        st.beta0[k - 1][::2] = 0.0
        st.beta1[k - 1][::2] = 0.0
        for M in st.masks[k - 1]:
            M.beta[::2] = 0.0
    z1 = SP.suff_stats(p, st)[0]
    mua, mub = SP.price_caps(st.alpha, z1, 1e-3, 2e-3)
    for a, mu in zip(st.alpha, mua):
        assert np.all(mu >= a) and np.all(mu > 0) and np.all(mu[a > 0] == a[a > 0])
        assert np.all(mu[a == 0] == 1e-3)
    for k in range(1, p.n):
        tot = st.beta0[k - 1] + st.beta1[k - 1] + sum(M.beta for M in st.masks[k - 1])
        mu = mub[k - 1]
        assert np.all(mu >= tot * (1 - 1e-15)) and np.all(mu[tot == 0] == 2e-3)


def bigm_view_bruteforce(p, mua, mub, x, z):
    """max over alpha in [0, mu_alpha] and (beta_0, beta_1) in the capped
    simplex of the Big-M Lagrangian, written constraint by constraint, by
    enumerating each neuron's vertices."""
    st = O.zero_state(p)
    base = O.lagrangian_constraint_form(p, st, x, z)
    total = base
    for k in range(1, p.n):
        for i in range(p.W(k).n_out):
            best_a = -np.inf
            for a in (0.0, mua[k - 1][i]):
                s2 = O.zero_state(p)
                s2.alpha[k - 1][i] = a
                best_a = max(best_a, O.lagrangian_constraint_form(p, s2, x, z) - base)
            best_b = -np.inf
            for which in (None, 0, 1):
                s2 = O.zero_state(p)
                if which == 0:
                    s2.beta0[k - 1][i] = mub[k - 1][i]
                elif which == 1:
                    s2.beta1[k - 1][i] = mub[k - 1][i]
                best_b = max(best_b, O.lagrangian_constraint_form(p, s2, x, z) - base)
            total += best_a + best_b
    return total


def test_primal_init_inner_max_and_subgradient():
    _, _, p = tiny_problem()
    rng = np.random.default_rng(9)
    mua = [rng.uniform(0.1, 1, p.W(k).n_out) for k in range(1, p.n)]
    mub = [rng.uniform(0.1, 1, p.W(k).n_out) for k in range(1, p.n)]

    def view(x, z):
        a, b0, b1 = SP.bigm_inner_max(p, mua, mub, x, z)
        st = O.zero_state(p)
        st.alpha, st.beta0, st.beta1 = a, b0, b1
        return O.lagrangian_constraint_form(p, st, x, z), st

    for trial in range(3):
        x, z = random_primal(p, rng)
        val, st = view(x, z)
        assert abs(val - bigm_view_bruteforce(p, mua, mub, x, z)) <= 1e-12 * (1 + abs(val))
        # f and g of the inner maximiser are minus the gradient of the view
        f, g, _ = O.dual_functions(p, st)
        dx = [rng.normal(size=a.size) for a in x]
        dz = [rng.normal(size=a.size) for a in z]
        h = 1e-7
        xp = [a + h * d for a, d in zip(x, dx)]
        zp = [a + h * d for a, d in zip(z, dz)]
        xm = [a - h * d for a, d in zip(x, dx)]
        zm = [a - h * d for a, d in zip(z, dz)]
        fd = (view(xp, zp)[0] - view(xm, zm)[0]) / (2 * h)
        an = -sum(float(a @ d) for a, d in zip(f, dx)) - sum(float(a @ d) for a, d in zip(g, dz))
        assert abs(fd - an) <= 1e-5 * (1 + abs(an))


def test_primal_init_lowers_the_view_and_stays_feasible():
    w, _, p = tiny_problem()
    prm = O.params_from_schedule(w.schedule)
    st = O.solve(p, prm).state
    z1 = SP.suff_stats(p, st)[0]
    mua, mub = SP.price_caps(st.alpha, z1, 1e-3, 1e-3)
    _, x, z, _, _ = O.evaluate(p, st)
    x1, z1_ = SP.primal_init(p, mua, mub, x, z, 100, (1e-2, 1e-5))
    for k in range(p.n):
        l, u = p.lu(k)
        assert np.all(x1[k] >= l) and np.all(x1[k] <= u)
    for a in z1_:
        assert np.all(a >= 0) and np.all(a <= 1)
    v0 = bigm_view_bruteforce(p, mua, mub, x, z)
    v1 = bigm_view_bruteforce(p, mua, mub, x1, z1_)
    assert v1 < v0
