"""GPU (HIP, gfx950) parity against the FP64 oracle, through the C ABI.

Tolerances (EPS = 1e-5 for FP32 plans, 1e-11 for FP64 plans):
  objective at fixed duals:   |d_gpu - d_ora| <= EPS * sum of |terms of d|
  supergradient entries:      <= EPS * row scale, where both sides chose the
                              same primal point for that neuron
  primal choices:             equal wherever |f| (|g|) exceeds EPS/10 * scale
  masks:                      bit-exact wherever the oracle's coefficient
                              margin exceeds 1e-6 (integral points: all bits)
  iteration windows:          duals and bound within EPS (relative), from
                              tie-free starts
  whole runs (FP64 plans):    final bounds within 1e-8 * max(1, |d|)
  whole runs (FP32 plans):    never above a sampled network output, never
                              below the interval bound; agreement with the
                              FP64 oracle within the run's sensitivity to
                              FP32 rounding (see test_end_to_end_fp32)
"""
import numpy as np
import pytest

from oracle import asd_oracle as O
from paper_2101_05844_amd import workloads as WL
from tests import helpers as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL_CONV, SMALL_DENSE, MFMA_CONV, WIDER_CONV = H.SMALL_CONV, H.SMALL_DENSE, H.MFMA_CONV, H.WIDER_CONV
workloads_small, e2e_workloads = H.workloads_small, H.e2e_workloads


def _A():
    from paper_2101_05844_amd import asdual as A
    A.lib()
    return A


EPS = {"fp32": 1e-5, "fp64": 1e-11,
       # BF16 operands: each product term a b is computed from round(a)
       # round(b), within 2 * 2^-9 + 2^-18 < 2^-8 of |a b| (nearest-even
       # rounding to 8 significant bits), so a sum is within 2^-8 of the sum
       # of its terms' magnitudes; plus the FP32 accumulation
       "bf16": 2.0 ** -8 + 2e-5}


def _setup(w, params=None, prec="fp32"):
    A = _A()
    ops, lh, uh = H.oracle_bounds(w)
    probs = H.oracle_problems(w, ops, lh, uh)
    net = A.Net(w.layers)
    prm = params or A.params_from_schedule(w.schedule, A.ASD_PREC_FP64 if prec == "fp64" else A.ASD_PREC_FP32)
    plan = A.Plan(net, w.S, prm)
    l0, u0, lht, uht, c = H.gpu_batch(w, lh, uh)
    plan.init(l0, u0, lht, uht, c)
    return A, ops, probs, net, plan, (l0, u0, lht, uht, c)


@pytest.mark.parametrize("wi", [0, 1])
def test_interval_bounds_match_oracle(wi):
    w = workloads_small()[wi]
    A = _A()
    net = A.Net(w.layers)
    l0 = torch.as_tensor(w.l0, device="cuda")
    u0 = torch.as_tensor(w.u0, device="cuda")
    lh, uh = net.interval_bounds(l0, u0)
    torch.cuda.synchronize()
    ops = O.ops_from_workload_layers(w.layers)
    for s in range(w.S):
        ol, ou = O.interval_bounds(ops, w.l0[s].astype(float), w.u0[s].astype(float))
        for k in range(len(ops)):
            g_l = lh[k][s].cpu().numpy().astype(float)
            g_u = uh[k][s].cpu().numpy().astype(float)
            sc = 1e-5 * (1 + np.abs(ol[k]) + np.abs(ou[k]))
            assert np.all(np.abs(g_l - ol[k]) <= sc) and np.all(np.abs(g_u - ou[k]) <= sc)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("wi", [0, 1, 3])
@pytest.mark.parametrize("n_masks", [0, 3])
def test_fixed_dual_evaluation(wi, n_masks, prec):
    w = workloads_small()[wi]
    A, ops, probs, net, plan, _ = _setup(w, prec=prec)
    eps = EPS[prec]
    rng = np.random.default_rng(100 + 10 * wi + n_masks)
    states = [H.random_integral_state(p, rng, n_masks, scale=0.5) for p in probs]
    H.import_states(plan, probs, states)
    res = plan.eval()
    torch.cuda.synchronize()
    obj = res["obj"].cpu().numpy()
    for s, (p, st) in enumerate(zip(probs, states)):
        d, x, z, f, g = O.evaluate(p, st)
        sc = H.objective_scale(p, st)
        assert abs(obj[s] - d) <= eps * sc, (s, obj[s], d, sc)
        sg = O.supergradient(p, st, x, z)
        for k in range(p.n):
            xg = res["x"][k][s].cpu().numpy().astype(float)
            fsc = eps / 10 * (1 + np.abs(f[k]).max())
            agree_x = np.isclose(xg, x[k], rtol=0, atol=0)
            assert np.all(agree_x | (np.abs(f[k]) <= fsc)), (s, k)
        for k in range(1, p.n):
            zg = res["z"][k][s].cpu().numpy().astype(float)
            gsc = eps / 10 * (1 + np.abs(g[k - 1]).max())
            assert np.all((zg == z[k - 1]) | (np.abs(g[k - 1]) <= gsc)), (s, k)
        # supergradient rows where both sides took the same choices around them
        for k in range(1, p.n):
            op = p.W(k)
            same = (res["z"][k][s].cpu().numpy() == z[k - 1]) & \
                   (res["x"][k][s].cpu().numpy().astype(float) == x[k])
            same_prev_all = np.all(res["x"][k - 1][s].cpu().numpy().astype(float) == x[k - 1])
            if not same_prev_all:
                continue
            lh, uh = p.hat(k)
            absW = op.with_data(np.abs(op.w))
            row = absW @ np.abs(x[k - 1]) + np.abs(op.b) + np.abs(x[k]) + np.abs(lh) + np.abs(uh)
            for M in st.masks[k - 1]:
                row = row + np.abs(M.LI) + np.abs(M.UI)
            tol = eps * (1 + row)
            for key, gk in (("ga", sg["alpha"][k - 1]), ("gb0", sg["beta0"][k - 1]),
                            ("gb1", sg["beta1"][k - 1])):
                gg = res[key][k][s].cpu().numpy().astype(float)
                assert np.all(np.abs(gg - gk)[same] <= tol[same]), (s, k, key)
            for q in range(n_masks):
                gg = res["gm"][k][q][s].cpu().numpy().astype(float)
                assert np.all(np.abs(gg - sg["masks"][k - 1][q])[same] <= tol[same]), (s, k, q)
            # the library re-derived LI/UI from the compact mask
            for q in range(n_masks):
                LI = plan.get(_A().ASD_F_MASK_LI, k, q)[s].cpu().numpy()
                UI = plan.get(_A().ASD_F_MASK_UI, k, q)[s].cpu().numpy()
                M = st.masks[k - 1][q]
                rs = eps * (1 + absW @ (np.abs(p.lu(k - 1)[0]) + np.abs(p.lu(k - 1)[1])))
                assert np.all(np.abs(LI - M.LI) <= rs) and np.all(np.abs(UI - M.UI) <= rs)


def _eval_all_alternatives(A, plan, probs, states, n_masks, eps=EPS["fp32"], eps_grad=None):
    """asd_eval through the iteration kernels under the plan's default kernel
    choices, every single-choice alternative the autotuner may take, and the
    default choices with every kernel launched alone: f, g, x*, z* and the
    supergradient against the oracle (check_eval_against_oracle)."""
    base, alts = _tuning_alternatives(A, plan)
    rows = [(s, p, st) for s, (p, st) in enumerate(zip(probs, states))]
    n_grad = sum(p.W(k).n_out * (3 + n_masks) for p in probs for k in range(1, p.n))
    tot = {}
    for field, idx, val in [(None, None, None)] + alts + [("profile", None, True)]:
        tun = {f: list(v) for f, v in base.items()}
        if field not in (None, "profile"):
            tun[field][idx] = val
        plan.set_tuning(tun)
        plan.profile(A.ASD_PROFILE_KERNELS if field == "profile" else A.ASD_PROFILE_OFF)
        res = plan.eval(path=A.ASD_EVAL_ITERATION)
        torch.cuda.synchronize()
        cnt = H.check_eval_against_oracle(res, rows, eps, eps_grad)
        # every supergradient entry of every subproblem was compared
        assert cnt["grad"] == n_grad, (field, cnt)
        # primal choices: only near-ties of the oracle's f and g are excused
        tie_frac = 0.01 if eps < 1e-4 else 0.1
        assert cnt["x_ties"] <= tie_frac * (cnt["x"] + cnt["x_ties"]) + 2, (field, cnt)
        assert cnt["z_ties"] <= tie_frac * (cnt["z"] + cnt["z_ties"]) + 2, (field, cnt)
        for key, v in cnt.items():
            tot[key] = tot.get(key, 0) + v
    plan.profile(False)
    plan.set_tuning(base)
    return tot


# (precision mode, tolerance of f, g and the primal choices, tolerance of
# the supergradient): BF16 operands in the forward products only, or in
# the transposed products too
PREC_TOL = {"fp32": ("fp32", "fp32"), "mixed": ("fp32", "fp32"), "bf16": ("fp32", "bf16"),
            "bf16_all": ("bf16", "bf16")}


def _mode(A, prec):
    return {"fp32": A.ASD_PREC_FP32, "mixed": A.ASD_PREC_MIXED, "bf16": A.ASD_PREC_BF16,
            "bf16_all": A.ASD_PREC_BF16_ALL}[prec]


@pytest.mark.parametrize("prec", ["fp32", "mixed", "bf16", "bf16_all"])
@pytest.mark.parametrize("wi", [0, 1, 2, 3])
@pytest.mark.parametrize("n_masks", [0, 3])
def test_iteration_kernels_at_fixed_duals(wi, n_masks, prec):
    """The kernels FP32 and mixed-mode iterations run (the (1 + K) products,
    the fused supergradient, the shared launches), evaluated at imported
    duals and masks (asd_eval, ASD_EVAL_ITERATION): f, g, x*, z* and every
    supergradient entry match the oracle (eq:dual-active-set,
    eq:as-primalk-min, eq:as-supergradient) within 1e-5 of their row
    scales, under every kernel choice of the autotuner.  In the BF16 mode
    the matrix-core products take BF16 operands: within 2^-8 of their row
    scales (EPS["bf16"])."""
    w = workloads_small()[wi]
    A = _A()
    A, ops, probs, net, plan, _ = _setup(w, A.params_from_schedule(w.schedule, _mode(A, prec)))
    rng = np.random.default_rng(500 + 10 * wi + n_masks)
    states = [H.random_integral_state(p, rng, n_masks, scale=0.5) for p in probs]
    H.import_states(plan, probs, states)
    ef, eg = PREC_TOL[prec]
    tot = _eval_all_alternatives(A, plan, probs, states, n_masks, EPS[ef], EPS[eg])
    print(w.name, n_masks, prec, tot, flush=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16_all"])
@pytest.mark.parametrize("wi", [0, 1, 2, 3])
def test_iteration_kernels_at_fixed_duals_max_masks(wi, prec):
    """As test_iteration_kernels_at_fixed_duals at the largest mask count
    the library takes (8, above the 7 of the benchmark schedule): the
    iteration kernels' instances for K = 8 under every kernel choice."""
    w = workloads_small()[wi]
    A = _A()
    prm = A.params_from_schedule(w.schedule, _mode(A, prec))
    prm.max_masks = 8
    A, ops, probs, net, plan, _ = _setup(w, prm)
    rng = np.random.default_rng(540 + wi)
    states = [H.random_integral_state(p, rng, 8, scale=0.5) for p in probs]
    H.import_states(plan, probs, states)
    ef, eg = PREC_TOL[prec]
    tot = _eval_all_alternatives(A, plan, probs, states, 8, EPS[ef], EPS[eg])
    print(w.name, 8, prec, tot, flush=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16_all"])
@pytest.mark.parametrize("shape", ["c1x16x8", "c4x16x16", "c2x8x64"])
def test_iteration_kernels_at_fixed_duals_m4(shape, prec):
    """As above on the input layers of the 4-channel matrix-core transposed
    convolution (1, 2 and 4 channels in rows of 8, 16 and 64 positions)."""
    sched = WL.Schedule(bigm_iters=8, as_iters=8, add_every=5, add_count=2, max_masks=3)
    w = WL.custom_config(M4_SHAPES[shape], S=5, seed=31, eps=0.05, schedule=sched, max_fixed=3, name=shape)
    A = _A()
    A, ops, probs, net, plan, _ = _setup(w, A.params_from_schedule(w.schedule, _mode(A, prec)))
    rng = np.random.default_rng(41)
    states = [H.random_integral_state(p, rng, 3, scale=0.5) for p in probs]
    H.import_states(plan, probs, states)
    ef, eg = PREC_TOL[prec]
    _eval_all_alternatives(A, plan, probs, states, 3, EPS[ef], EPS[eg])


def _point_box_workload():
    """The small conv net with point boxes away from zero: some input
    coordinates with l0 = u0 > 0 and, in every ReLU layer, some neurons with
    lhat = uhat > 0 (a fixed positive post-activation value).  At fixed
    duals the bound is a function of the given boxes, valid or not, so both
    sides evaluate the same function."""
    w = workloads_small()[1]
    ops, lh, uh = H.oracle_bounds(w)
    rng = np.random.default_rng(77)
    l0, u0 = w.l0.copy(), w.u0.copy()
    pick = rng.random(l0.shape) < 0.2
    mid = H.f32(np.clip((l0 + u0) / 2, 0.05, None))
    l0 = np.where(pick, mid, l0).astype(np.float32)
    u0 = np.where(pick, mid, u0).astype(np.float32)
    lh2, uh2 = [], []
    for a, b in zip(lh, uh):
        pk = rng.random(a.shape) < 0.2
        val = H.f32(np.abs(b) * 0.5 + 0.01)
        lh2.append(np.where(pk, val, a).astype(np.float32))
        uh2.append(np.where(pk, val, b).astype(np.float32))
    w.l0, w.u0 = l0, u0
    return w, ops, lh2, uh2


@pytest.mark.parametrize("n_masks", [1, 3])
def test_point_boxes_away_from_zero(n_masks):
    """Point boxes away from zero (the W+ x_point correction of the compact
    masks in the iteration kernels, and the general kernels' point-box
    rule): both evaluation paths against the oracle, and one iteration under
    the plain rule against the oracle's step."""
    A = _A()
    w, ops, lh, uh = _point_box_workload()
    probs = H.oracle_problems(w, ops, lh, uh)
    net = A.Net(w.layers)
    prm = A.params_from_schedule(w.schedule, A.ASD_PREC_FP32)
    prm.rule = A.ASD_RULE_SUPERGRADIENT
    prm.bigm_lr0, prm.bigm_lr1, prm.as_lr0, prm.as_lr1 = 1e-3, 1e-4, 1e-4, 1e-5
    plan = A.Plan(net, w.S, prm)
    batch = H.gpu_batch(w, lh, uh)
    plan.init(*batch)
    rng = np.random.default_rng(78 + n_masks)
    states = [H.random_integral_state(p, rng, n_masks, scale=0.5) for p in probs]
    assert any((p.lu(0)[0] == p.lu(0)[1]).any() and (p.lu(0)[0] > 0).any() for p in probs)
    H.import_states(plan, probs, states)
    _eval_all_alternatives(A, plan, probs, states, n_masks)
    res = plan.eval(path=A.ASD_EVAL_GENERAL)
    torch.cuda.synchronize()
    H.check_eval_against_oracle(res, [(s, p, st) for s, (p, st) in enumerate(zip(probs, states))], EPS["fp32"])
    # one step of the plain rule from the imported state (t = 3: no mask
    # addition, 3 mod omega >= V)
    t = 3
    plan.run(A.ASD_PHASE_AS, t, 1)
    torch.cuda.synchronize()
    K = plan.counts().n_masks
    duals = H.export_duals(plan, len(ops), K)
    oprm = O.params_from_schedule(w.schedule)
    lr = O.linear_lr(1e-4, 1e-5, t, oprm.as_iters)
    for s, (p, st) in enumerate(zip(probs, states)):
        d, x, z, _, _ = O.evaluate(p, st)
        e = st.copy()
        O.apply_step(e, O.supergradient(p, st, x, z), lr, "sgd", oprm.adam)
        for k in range(1, p.n):
            pairs = [(duals[("alpha", k)][s], e.alpha[k - 1]), (duals[("beta0", k)][s], e.beta0[k - 1]),
                     (duals[("beta1", k)][s], e.beta1[k - 1])]
            pairs += [(duals[("mask", k, q)][s], e.masks[k - 1][q].beta) for q in range(K)]
            for a, b in pairs:
                assert np.all(np.abs(a - b) <= 1e-5 * (1 + np.abs(b))), (s, k)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("wi", [0, 1])
@pytest.mark.parametrize("integral", [True, False])
def test_separation_oracle_masks(wi, integral, prec):
    w = workloads_small()[wi]
    A, ops, probs, net, plan, _ = _setup(w, prec=prec)
    rng = np.random.default_rng(7 + wi)
    for k in range(1, len(ops)):
        xs, zs = [], []
        for p in probs:
            lp_, up_ = p.lu(k - 1)
            if integral:
                xs.append(np.where(rng.integers(0, 2, lp_.size) == 1, up_, lp_))
                zs.append(rng.integers(0, 2, p.W(k).n_out).astype(float))
            else:
                xs.append(H.f32(lp_ + rng.uniform(0, 1, lp_.size) * (up_ - lp_)).astype(float))
                zs.append(H.f32(rng.uniform(0, 1, p.W(k).n_out)).astype(float))
        bits, LI, UI, fan = plan.oracle(k, torch.as_tensor(H.f32(np.stack(xs)), device="cuda"),
                                        torch.as_tensor(H.f32(np.stack(zs)), device="cuda"))
        torch.cuda.synchronize()
        gb = A.unpack_bits(bits.cpu().numpy().view(np.uint32), fan)
        for s, p in enumerate(probs):
            op = p.W(k)
            lp_, up_ = p.lu(k - 1)
            I = O.oracle_mask(op, lp_, up_, xs[s], zs[s])
            Lc, Uc = O.check_matrices(op, lp_, up_)
            r, j = op.rows, op.cols
            coeff = ((1 - zs[s][r]) * Lc + zs[s][r] * Uc - xs[s][j]) * op.w
            # map pattern entries to receptive-field positions of the library
            L = w.layers[k - 1]
            if L.kind == "dense":
                pos = j
            else:
                sp = L.spec
                co, rem = r // (sp.h_out * sp.w_out), r % (sp.h_out * sp.w_out)
                oy, ox = rem // sp.w_out, rem % sp.w_out
                ci, rem2 = j // (sp.h_in * sp.w_in), j % (sp.h_in * sp.w_in)
                iy, ix = rem2 // sp.w_in, rem2 % sp.w_in
                ky, kx = iy - (oy * sp.stride - sp.pad), ix - (ox * sp.stride - sp.pad)
                pos = (ci * sp.k + ky) * sp.k + kx
            g_bits = gb[s][r, pos]
            sure = np.ones_like(I) if integral else (np.abs(coeff) > 1e-6)
            assert np.array_equal(g_bits[sure], I[sure]), (k, s)
            LIo, UIo = O.mask_constants(op, I, lp_, up_)
            absW = op.with_data(np.abs(op.w))
            rs = EPS[prec] * (1 + absW @ (np.abs(lp_) + np.abs(up_)))
            if integral:
                assert np.all(np.abs(LI[s].cpu().numpy() - LIo) <= rs)
                assert np.all(np.abs(UI[s].cpu().numpy() - UIo) <= rs)


WINDOW_STARTS = [("bigm", 0), ("bigm", 3), ("bigm", 6), ("as", 0), ("as", 2), ("as", 4), ("as", 6), ("as", 9)]


def _window_plan(prec, rule):
    """(starts, window length, bound tolerance) per precision and rule.

    FP64 plans: every start, two iterations, 1e-11.
    FP32 plans compute the same iteration with rounding; where a step is
    decided by the sign of a supergradient entry within rounding of zero the
    FP32 and FP64 iterates part (Adam's first steps of fresh multipliers: the
    phase starts and the iterations right after a mask addition; and the
    step after an addition, where a tiny versus a zero multiplier flips a
    z* choice).  Such entries are common in layer 1, where x_hat = W x* + b
    equals the interval bound up to its rounding whenever x* is the
    maximising corner.  FP32 windows therefore cover one iteration from
    every start under the plain supergradient rule, and one iteration from
    starts whose Adam moments are not fresh under Adam."""
    if prec == "fp64":
        return WINDOW_STARTS, 2, 1e-11
    if rule == "supergradient":
        return WINDOW_STARTS, 1, 1e-5
    return [("bigm", 3), ("bigm", 6), ("as", 4), ("as", 9)], 1, 2e-5


@pytest.mark.parametrize("prec", ["fp32", "fp64", "mixed"])
@pytest.mark.parametrize("rule", ["supergradient", "adam"])
@pytest.mark.parametrize("wi", [0, 1, 2, 3])
def test_iteration_windows_match_oracle(wi, rule, prec):
    """Import the oracle's state at points of its run (the Big-M start, mid
    Big-M, the Active Set start with its mask additions, and later), advance
    the GPU, and compare every subproblem's duals and bound with the
    oracle's state at the end of the same window (see _window_plan).  The
    mixed mode (BF16-stored Adam moments) is compared with the oracle run
    whose Adam step stores its moments rounded to bfloat16; its moments must
    also agree, within one bfloat16 spacing (the GPU rounds the FP32 update,
    the oracle the FP64 one)."""
    if prec == "mixed" and rule != "adam":
        pytest.skip("the plain rule keeps no moments: the mixed mode is the FP32 mode")
    if wi == 3 and prec == "mixed":
        pytest.skip("the mixed mode's moments are covered on the other shapes")
    w = workloads_small()[wi]
    A = _A()
    starts, win, tol = _window_plan("fp32" if prec == "mixed" else prec, rule)
    eps = EPS["fp32" if prec == "mixed" else prec]
    prm = O.params_from_schedule(w.schedule)
    if prec == "mixed":
        prm.adam = O.AdamConsts(prm.adam.beta1, prm.adam.beta2, prm.adam.eps, moments="bf16")
    params = A.params_from_schedule(w.schedule, {"fp32": A.ASD_PREC_FP32, "fp64": A.ASD_PREC_FP64,
                                                 "mixed": A.ASD_PREC_MIXED}[prec])
    if rule == "supergradient":
        prm.rule = "sgd"
        params.rule = A.ASD_RULE_SUPERGRADIENT
        prm.bigm_lr = (1e-3, 1e-4)
        prm.as_lr = (1e-4, 1e-5)
        params.bigm_lr0, params.bigm_lr1, params.as_lr0, params.as_lr1 = 1e-3, 1e-4, 1e-4, 1e-5
    A, ops, probs, net, plan, _ = _setup(w, params)
    want = set(starts) | {(ph, t + win) for ph, t in starts}
    runs = [O.solve(p, prm, snapshot_at=sorted(want, key=str)) for p in probs]
    # FP32 under Adam: Adam's step is the supergradient divided by the root of
    # its second moment, so an entry whose supergradient is zero in exact
    # arithmetic (and whose second moment is still near zero) moves by about
    # one step size in the direction of its rounding residue.  Such an entry
    # may differ, by at most 2.5 step sizes, only where the oracle's
    # supergradient at the window start is within rounding of zero; every
    # other entry must match.
    loose = prec in ("fp32", "mixed") and rule == "adam"
    lr_max = max(prm.bigm_lr[0], prm.as_lr[0])
    n_ent = n_bad = 0
    for ph, t in starts:
        sts = [r.snapshots[(ph, t)] for r in runs]
        ends = [r.snapshots[(ph, t + win)] for r in runs]
        A_ph = A.ASD_PHASE_BIGM if ph == "bigm" else A.ASD_PHASE_AS
        H.import_states(plan, probs, sts)
        plan.run(A_ph, t, win)
        out = plan.bound()
        torch.cuda.synchronize()
        K = plan.counts().n_masks
        assert K == len(ends[0].masks[0])
        duals = H.export_duals(plan, len(ops), K)
        moments = {}
        if prec == "mixed":
            for k in range(1, len(ops)):
                for fld in (A.ASD_F_ALPHA_M, A.ASD_F_ALPHA_V, A.ASD_F_BETA0_M, A.ASD_F_BETA0_V,
                            A.ASD_F_BETA1_M, A.ASD_F_BETA1_V):
                    moments[(fld, k, 0)] = plan.get(fld, k).cpu().numpy().astype(np.float64)
                for q in range(K):
                    for fld in (A.ASD_F_MASK_M, A.ASD_F_MASK_V):
                        moments[(fld, k, q)] = plan.get(fld, k, q).cpu().numpy().astype(np.float64)
        lb = out.cpu().numpy()
        for s, (p, e) in enumerate(zip(probs, ends)):
            d_ora = O.evaluate(p, e)[0]
            bad_before = n_bad
            if loose:
                st0 = sts[s]
                _, x0, z0, _, _ = O.evaluate(p, st0)
                sg0 = O.supergradient(p, st0, x0, z0)
            for k in range(1, len(ops)):
                pairs = [(duals[("alpha", k)][s], e.alpha[k - 1]), (duals[("beta0", k)][s], e.beta0[k - 1]),
                         (duals[("beta1", k)][s], e.beta1[k - 1])]
                pairs += [(duals[("mask", k, q)][s], e.masks[k - 1][q].beta) for q in range(K)]
                names = ["alpha", "beta0", "beta1"] + [f"mask{q}" for q in range(K)]
                if loose:
                    # rounding scale of a supergradient entry of layer k
                    lh_, uh_ = p.hat(k)
                    lp_, up_ = p.lu(k - 1)
                    op = p.W(k)
                    scale = 1 + np.abs(x0[k]) + np.abs(lh_) + np.abs(uh_) + np.abs(op.b) + \
                        op.with_data(np.abs(op.w)) @ (np.abs(lp_) + np.abs(up_))
                    grads = [sg0["alpha"][k - 1], sg0["beta0"][k - 1], sg0["beta1"][k - 1]] + \
                        [sg0["masks"][k - 1][q] for q in range(K)]
                for j, (name, (a, b)) in enumerate(zip(names, pairs)):
                    ok = np.abs(a - b) <= eps * (1 + np.abs(b))
                    n_ent += ok.size
                    n_bad += int((~ok).sum())
                    if loose:
                        tie = np.abs(grads[j]) <= eps * scale
                        assert np.all(ok | tie), (ph, t, s, k, name, np.flatnonzero(~(ok | tie))[:5])
                        assert np.all(np.abs(a - b) <= 2.5 * lr_max + eps * (1 + np.abs(b))), (ph, t, s, k, name)
                    else:
                        assert ok.all(), (ph, t, s, k, name, np.flatnonzero(~ok)[:5])
                    if prec == "mixed":
                        # moments where the dual matched
                        if j < 3:
                            fm, fv = [(A.ASD_F_ALPHA_M, A.ASD_F_ALPHA_V), (A.ASD_F_BETA0_M, A.ASD_F_BETA0_V),
                                      (A.ASD_F_BETA1_M, A.ASD_F_BETA1_V)][j]
                            om, ov = e.m[name][k - 1], e.v[name][k - 1]
                            q = 0
                        else:
                            fm, fv, q = A.ASD_F_MASK_M, A.ASD_F_MASK_V, j - 3
                            om, ov = e.masks[k - 1][q].m, e.masks[k - 1][q].v
                        # one bfloat16 spacing, plus what the FP32 rounding of the
                        # supergradient (eps * scale) moves the updated moment by
                        dg = eps * scale
                        b1, b2 = prm.adam.beta1, prm.adam.beta2
                        for fld, ref, extra in ((fm, om, (1 - b1) * dg),
                                                (fv, ov, (1 - b2) * (2 * np.abs(grads[j]) + dg) * dg)):
                            got = moments[(fld, k, q)][s]
                            close = np.abs(got - ref) <= 2.0 ** -7 * np.abs(ref) + extra
                            assert np.all(close | ~ok), (ph, t, s, k, name, fld,
                                                         np.flatnonzero(~(close | ~ok))[:3])
            # the bound is a function of the duals: compared where every dual
            # matched (a tie entry allowed to differ above moves it further)
            if n_bad == bad_before:
                assert abs(lb[s] - d_ora) <= tol * max(1.0, abs(d_ora)), (ph, t, s, lb[s], d_ora)
    print(f"{n_bad} of {n_ent} entries differ (ties under Adam's normalised step)" if loose else "", flush=True)


def _sampled_min(ops, p, l0, u0, seed, n=400):
    """Smallest sampled network output over the inputs of subproblem p
    (uniform points and the box corners, kept when every pre-activation lies
    within the subproblem's bounds, which encode its fixed ReLU phases)."""
    pts = WL.random_points_in_box(l0.astype(float), u0.astype(float), n, seed)
    x = pts.T
    keep = np.ones(pts.shape[0], dtype=bool)
    for k, op in enumerate(ops[:-1]):
        xh = op.W @ x + op.b[:, None]
        lh, uh = p.hat(k + 1)
        keep &= np.all((xh >= lh[:, None]) & (xh <= uh[:, None]), axis=0)
        x = np.maximum(xh, 0)
    outs = (ops[-1].W @ x + ops[-1].b[:, None]).T @ p.c
    return outs[keep].min() if keep.any() else np.inf


@pytest.mark.parametrize("wi", [0, 1, 2, 3])
def test_end_to_end_fp64(wi):
    """Whole runs (Big-M, Active Set with additions, final bound) in an FP64
    plan agree with the FP64 oracle; sampled outputs bound them from above."""
    w = e2e_workloads()[wi]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp64")
    lb, x0 = plan.solve(*batch, want_x0=True)
    torch.cuda.synchronize()
    lb = lb.cpu().numpy()
    prm = O.params_from_schedule(w.schedule)
    for s, p in enumerate(probs[:12]):
        r = O.solve(p, prm)
        assert abs(lb[s] - r.bound) <= 1e-8 * max(1.0, abs(r.bound)), (s, lb[s], r.bound)
        assert lb[s] <= _sampled_min(ops, p, w.l0[s], w.u0[s], s) + 1e-9


@pytest.mark.parametrize("wi", [0, 1])
def test_end_to_end_fp64_mask_cap(wi):
    """Whole FP64 runs that reach the mask cap of Sec. 7.1 (7 active sets per
    layer: additions of 2 every 5 iterations over 16 Active Set iterations)
    agree with the FP64 oracle run on the same schedule."""
    w = e2e_workloads()[wi]
    sched = WL.Schedule(bigm_iters=10, as_iters=16, add_every=5, add_count=2, max_masks=7)
    w = WL.Workload(w.name, w.layers, w.l0, w.u0, w.c, sched, w.fix_draws, w.meta)
    A = _A()
    A, ops, probs, net, plan, batch = _setup(w, prec="fp64")
    lb = plan.solve(*batch).cpu().numpy()
    assert plan.counts().n_masks == 7
    prm = O.params_from_schedule(sched)
    for s, p in enumerate(probs[:8]):
        r = O.solve(p, prm)
        assert abs(lb[s] - r.bound) <= 1e-8 * max(1.0, abs(r.bound)), (s, lb[s], r.bound)


@pytest.mark.parametrize("wi", [0, 1, 2, 3])
def test_end_to_end_fp32(wi):
    """Whole runs in an FP32 plan.  The final bound (the FP64 evaluation of
    the run's final duals) matches the oracle's evaluation of the same
    exported duals within 1e-10 of the summed term magnitudes, per result.
    The run itself parts from the FP64 oracle's run at the first near-tie
    it meets, so its distance from the oracle's bound is held to a band
    measured from the oracle alone: tests/golden/fp32_band.json records how
    far a model of FP32 arithmetic (state stored as float32, errors of one
    float32 unit of each entry's rounding scale on f, g and the
    supergradient) moves the oracle's own runs on these workloads (max and
    mean over all their subproblems); the band is twice that, at least
    1e-4.  Also: never
    above a sampled output, never below the interval bound."""
    w = e2e_workloads()[wi]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp32")
    lb = plan.solve(*batch).cpu().numpy()
    # the FP64 final bound of the FP32 run is the dual objective of its final
    # duals: per result, against the oracle's evaluation at the same duals
    err = H.final_bound_errors(plan, lb, dict(enumerate(probs[:12])))
    assert all(e[1] <= 1e-10 for e in err.values()), err
    prm = O.params_from_schedule(w.schedule)
    band = H.fp32_band(w.name)
    ora = []
    for s, p in enumerate(probs[:12]):
        r = O.solve(p, prm)
        ora.append(r.bound)
        assert lb[s] <= _sampled_min(ops, p, w.l0[s], w.u0[s], s) + 1e-6
        assert lb[s] >= O.evaluate(p, O.zero_state(p))[0] - 1e-5 * max(1.0, abs(lb[s]))
        assert abs(lb[s] - r.bound) <= band["max"] * max(1.0, abs(r.bound)), (s, lb[s], r.bound, band)
    ora = np.array(ora)
    n = len(ora)
    rel = np.abs(lb[:n] - ora) / np.maximum(1.0, np.abs(ora))
    assert rel.mean() <= band["mean"], (rel.mean(), band)
    print(w.name, "FP32 whole run vs FP64 oracle: max rel", rel.max(), "mean rel", rel.mean(), "band", band,
          "final-bound error (rel. to sum |terms|) max", max(e[1] for e in err.values()), flush=True)


@pytest.mark.parametrize("wi", [0, 1, 2, 3])
def test_end_to_end_mixed(wi):
    """Whole runs with BF16-stored Adam moments: the final bound is the FP64
    evaluation of valid duals (checked per result against the oracle's
    evaluation of the exported duals), so it never exceeds a sampled output
    and never falls below the interval bound.  Its distance from the FP32
    run is held to the sum of the two forms' measured bands against the
    FP64 oracle (tests/golden/fp32_band.json: the oracle's FP32 noise model,
    without and with BF16-stored moments)."""
    w = e2e_workloads()[wi]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp32")
    lb32 = plan.solve(*batch).cpu().numpy()
    prm = A.params_from_schedule(w.schedule, A.ASD_PREC_MIXED)
    plan_m = A.Plan(net, w.S, prm)
    lbm = plan_m.solve(*batch).cpu().numpy()
    err = H.final_bound_errors(plan_m, lbm, dict(enumerate(probs[:12])))
    assert all(e[1] <= 1e-10 for e in err.values()), err
    for s, p in enumerate(probs[:12]):
        assert lbm[s] <= _sampled_min(ops, p, w.l0[s], w.u0[s], s) + 1e-6
        assert lbm[s] >= O.evaluate(p, O.zero_state(p))[0] - 1e-5 * max(1.0, abs(lbm[s]))
    band = H.fp32_band(w.name)
    rel = np.abs(lbm - lb32) / np.maximum(1.0, np.abs(lb32))
    assert np.all(rel <= band["max"] + band["mixed_max"]), (rel.max(), band)
    assert rel.mean() <= band["mean"] + band["mixed_mean"], (rel.mean(), band)
    print(f"mean fp32 - mixed {np.mean(lb32 - lbm):.3e}, max |diff| {np.max(np.abs(lb32 - lbm)):.3e}", flush=True)


@pytest.mark.parametrize("prec", ["bf16", "bf16_all"])
@pytest.mark.parametrize("wi", [0, 1, 2, 3])
def test_end_to_end_bf16(wi, prec):
    """Whole runs with BF16 matrix-core operands (forward products only, or
    all): the final bound is the FP64 evaluation of the run's FP32 duals
    from the FP32 weights (checked per result against the oracle's
    evaluation of the exported duals), so it never exceeds a sampled output
    and never falls below the interval bound; its distance from the FP32
    run is held to the sum of the two forms' measured bands
    (tests/golden/fp32_band.json: the oracle's noise models with FP32 and
    with BF16-sized errors)."""
    w = e2e_workloads()[wi]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp32")
    lb32 = plan.solve(*batch).cpu().numpy()
    plan_b = A.Plan(net, w.S, A.params_from_schedule(w.schedule, _mode(A, prec)))
    lbb = plan_b.solve(*batch).cpu().numpy()
    err = H.final_bound_errors(plan_b, lbb, dict(enumerate(probs[:12])))
    assert all(e[1] <= 1e-10 for e in err.values()), err
    for s, p in enumerate(probs[:12]):
        assert lbb[s] <= _sampled_min(ops, p, w.l0[s], w.u0[s], s) + 1e-6
        assert lbb[s] >= O.evaluate(p, O.zero_state(p))[0] - 1e-5 * max(1.0, abs(lbb[s]))
    band = H.fp32_band(w.name)
    rel = np.abs(lbb - lb32) / np.maximum(1.0, np.abs(lb32))
    assert np.all(rel <= band["max"] + band[prec + "_max"]), (rel.max(), band)
    assert rel.mean() <= band["mean"] + band[prec + "_mean"], (rel.mean(), band)
    print(w.name, prec, "vs FP32: max rel", rel.max(), "mean rel", rel.mean(), "mean fp32 - this",
          float(np.mean(lb32 - lbb)), flush=True)


def test_deterministic_repeat():
    w = workloads_small()[1]
    A, ops, probs, net, plan, batch = _setup(w)
    a = plan.solve(*batch).cpu().numpy()
    b = plan.solve(*batch).cpu().numpy()
    assert np.array_equal(a, b)


def _check_grad(got, ref, mag, tol, what):
    bad = np.abs(got - ref) > tol * (1 + mag)
    assert not bad.any(), (what, np.flatnonzero(bad)[:5], got[bad][:5], ref[bad][:5])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("wi", [0, 1, 2])
@pytest.mark.parametrize("n_masks", [0, 3])
def test_bound_gradient_matches_oracle(wi, n_masks, prec):
    """asd_bound_grad at imported duals and masks against the oracle's Danskin
    gradient (pinned by central differences): weight and bias gradients
    summed over the subproblems with mixed-sign factors, box gradients per
    subproblem.  Both sides sum in FP64 from the same FP32-valued duals, so
    the tolerance (1e-9 of the summed magnitudes) covers summation order."""
    w = workloads_small()[wi]
    A, ops, probs, net, plan, _ = _setup(w, prec=prec)
    rng = np.random.default_rng(300 + 10 * wi + n_masks)
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
            _check_grad(got.cpu().numpy().reshape(-1), ref, mag, 1e-9, ("dW" if i == 0 else "db", k))
    for i, got in ((2, dl0), (3, du0)):
        g = got.cpu().numpy()
        for s in range(w.S):
            ref = gs[s] * ora[s][i]
            _check_grad(g[s], ref, np.abs(ref), 1e-9, ("dl0" if i == 2 else "du0", s))


def test_bound_function_autograd():
    """BoundFunction: the solve's bounds in the forward pass, asd_bound_grad
    in the backward pass (same values as a direct call at the final duals),
    gradients routed to the net's weights and the input box."""
    w = workloads_small()[1]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp64")
    l0, u0, lht, uht, c = batch
    l0 = l0.clone().requires_grad_(True)
    u0 = u0.clone().requires_grad_(True)
    params = [t.requires_grad_(True) for t in net.W + net.b]
    lb = A.BoundFunction.apply(plan, l0, u0, tuple(lht), tuple(uht), c, *params)
    ref_lb = plan.bound()
    assert torch.equal(lb, ref_lb)
    gs = torch.linspace(-1.0, 1.0, w.S, dtype=torch.float64, device="cuda")
    (lb * gs).sum().backward()
    dW, db, dl0, du0 = plan.bound_grad(gs)
    for t, ref in zip(net.W + net.b, dW + db):
        assert torch.equal(t.grad, ref.to(torch.float32))
    assert torch.equal(l0.grad, dl0.to(torch.float32)) and torch.equal(u0.grad, du0.to(torch.float32))
    # repeated evaluation is bit-identical (fixed-order sums)
    dW2, _, dl02, _ = plan.bound_grad(gs)
    assert all(torch.equal(a, b) for a, b in zip(dW, dW2)) and torch.equal(dl0, dl02)
    # after the duals change, a call asking to reuse the minimiser of the last
    # bound recomputes it (the state changed since): same as a fresh call
    plan.run(A.ASD_PHASE_AS, 0, 2)
    dW3, _, dl03, _ = plan.bound_grad(gs, reuse=True)
    dW4, _, dl04, _ = plan.bound_grad(gs)
    assert all(torch.equal(a, b) for a, b in zip(dW3, dW4)) and torch.equal(dl03, dl04)
    assert not all(torch.equal(a, b) for a, b in zip(dW3, dW))


def test_bound_function_refuses_a_stale_plan():
    """Two forward passes through one plan before the first backward pass:
    the first output's backward pass would read the second solve's duals,
    so it raises; the second output's backward pass still matches a direct
    asd_bound_grad."""
    w = workloads_small()[1]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp64")
    l0, u0, lht, uht, c = batch
    params = [t.requires_grad_(True) for t in net.W + net.b]
    l0a = l0.clone().requires_grad_(True)
    lb1 = A.BoundFunction.apply(plan, l0a, u0, tuple(lht), tuple(uht), c, *params)
    mid, rad = (l0 + u0) / 2, (u0 - l0) / 4
    l0b = (mid - rad).contiguous().requires_grad_(True)
    lb2 = A.BoundFunction.apply(plan, l0b, (mid + rad).contiguous(), tuple(lht), tuple(uht), c, *params)
    with pytest.raises(RuntimeError, match="changed after this forward"):
        lb1.sum().backward(retain_graph=True)
    for t in params:
        t.grad = None
    lb2.sum().backward()
    dW, db, dl0, du0 = plan.bound_grad(torch.ones(w.S, dtype=torch.float64, device="cuda"))
    assert torch.equal(l0b.grad, dl0.to(torch.float32))
    assert all(torch.equal(t.grad, r.to(torch.float32)) for t, r in zip(net.W, dW))


def _ragged_budgets(w, seed):
    rng = np.random.default_rng(seed)
    T = w.schedule.as_iters
    b = np.sort(rng.integers(2, T + 1, size=w.S))[::-1].copy()
    b[0] = T
    return [int(v) for v in b]


@pytest.mark.parametrize("wi", [0, 1])
def test_ragged_budgets_match_plain_solves_fp64(wi):
    """Per-subproblem Active Set budgets (FP64 plan): subproblem s of a ragged
    batch ends with the bound of a plain solve whose Active Set phase has
    T = budget[s] iterations (own learning-rate schedule, same additions)."""
    w = workloads_small()[wi]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp64")
    budgets = _ragged_budgets(w, 60 + wi)
    plan.set_budgets(budgets)
    lb = plan.solve(*batch).cpu().numpy()
    for T in sorted(set(budgets)):
        prm = A.params_from_schedule(w.schedule, A.ASD_PREC_FP64)
        prm.as_iters = T
        ref_plan = A.Plan(net, w.S, prm)
        ref = ref_plan.solve(*batch).cpu().numpy()
        rows = [s for s in range(w.S) if budgets[s] == T]
        for s in rows:
            assert abs(lb[s] - ref[s]) <= 1e-12 * max(1.0, abs(ref[s])), (T, s, lb[s], ref[s])
    # and against the oracle's solve with the subproblem's own T
    prm_o = O.params_from_schedule(w.schedule)
    for s in (0, w.S // 2, w.S - 1):
        prm_o.as_iters = budgets[s]
        r = O.solve(probs[s], prm_o)
        assert abs(lb[s] - r.bound) <= 1e-8 * max(1.0, abs(r.bound)), (s, lb[s], r.bound)


@pytest.mark.parametrize("wi", [1, 2, 3])
def test_ragged_budgets_independent_fp32(wi):
    """FP32 plan (matrix-core and column kernels): subproblem s of a ragged
    batch is bit-identical to the same subproblem in a batch where every
    budget equals budget[s]: updating only the prefix within budget changes
    nothing for the others."""
    w = workloads_small()[wi]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp32")
    budgets = _ragged_budgets(w, 70 + wi)
    plan.set_budgets(budgets)
    lb = plan.solve(*batch).cpu().numpy()
    ref_plan = A.Plan(net, w.S, A.params_from_schedule(w.schedule, A.ASD_PREC_FP32))
    for T in sorted(set(budgets)):
        ref_plan.set_budgets([T] * w.S)
        ref = ref_plan.solve(*batch).cpu().numpy()
        rows = [s for s in range(w.S) if budgets[s] == T]
        assert np.array_equal(lb[rows], ref[rows]), (T, rows, lb[rows], ref[rows])
    with pytest.raises(A.AsdError):
        plan.set_budgets(sorted(budgets))  # increasing: rejected


def test_solve_group_matches_separate_solves():
    """asd_solve_group over two plans on different nets (one with budgets),
    each on its own stream: every bound equals that plan's own asd_solve."""
    A = _A()
    outs_sep, plans, batches = [], [], []
    for wi, budgets in ((1, True), (2, False)):
        w = workloads_small()[wi]
        A, ops, probs, net, plan, batch = _setup(w, prec="fp32")
        if budgets:
            plan.set_budgets(_ragged_budgets(w, 80))
        outs_sep.append(plan.solve(*batch).cpu().numpy())
        plans.append(plan)
        batches.append(batch)
    outs = A.solve_group(plans, batches)
    torch.cuda.synchronize()
    for a, b in zip(outs, outs_sep):
        assert np.array_equal(a.cpu().numpy(), b)


def _tuning_alternatives(A, plan):
    """Every single-choice deviation from the plan's default tuning that
    changes a kernel for this net."""
    base = plan.tuning()
    alts = []
    n = plan.net.n
    for L in range(1, n):
        Ly = plan.net.layers[L - 1]
        if Ly.kind == "dense":
            cap = max(1, min(8, Ly.spec.n_in // 128))
            ks = 1
            while ks <= cap:
                if ks != base["ksplit"][L - 1]:
                    alts.append(("ksplit", L - 1, ks))
                ks *= 2
            alts.append(("fwd_kw", L - 1, 4 if base["fwd_kw"][L - 1] == 8 else 8))
        else:
            alts.append(("fwd_mfma", L - 1, 1 - base["fwd_mfma"][L - 1]))
            alts.append(("fwd_kw", L - 1, 4 if base["fwd_kw"][L - 1] == 8 else 8))
    for L in range(1, n + 1):
        Ly = plan.net.layers[L - 1]
        k = L - 1
        if Ly.kind == "conv":
            sp = Ly.spec
            if not ((sp.h_in * sp.w_in) % 64 == 0 and sp.c_in >= 16) and sp.c_in > 4:
                alts.append(("bwd_cb", k, 4 if base["bwd_cb"][k] != 4 else 8))
            if (sp.stride == 2 and sp.c_in <= 4 and (sp.h_in * sp.w_in) % 64 == 0 and sp.w_in % 8 == 0
                    and (sp.w_in % 64 == 0 or 64 % sp.w_in == 0)):
                # matrix-core 4-channel kernel (0) against the VALU column kernel (4)
                alts.append(("bwd_cb", k, 4 if base["bwd_cb"][k] != 4 else 0))
            if (sp.h_in * sp.w_in) % 64 == 0 and sp.c_in >= 16:
                alts.append(("bwd_nt", k, 4 if base["bwd_nt"][k] != 4 else 2))
        else:
            n_in = Ly.spec.n_in
            prev = plan.net.layers[L - 2] if L >= 2 else None
            P_in = prev.spec.h_out * prev.spec.w_out if prev is not None and prev.kind == "conv" else 1
            if P_in % 64 == 0:
                alts.append(("bwd_pos", k, 1 - base["bwd_pos"][k] if base["bwd_pos"][k] < 2 else 1))
                alts.append(("bwd_pos", k, 2 if base["bwd_pos"][k] != 2 else 0))
                alts.append(("bwd_kw", k, 4 if base["bwd_kw"][k] == 8 else 8))
    return base, alts


@pytest.mark.parametrize("wi", [1, 2, 3])
def test_tuning_alternatives_match_oracle(wi):
    """Each kernel alternative the autotuner may pick (dense forward split
    counts, narrow convolution forward on the matrix cores, channels per
    thread of the column transposed convolution, the matrix-core kernel
    into a layer of at most 4 channels, dense backward with positions on
    lanes or on the matrix cores), and the default choices with every kernel
    launched alone instead of sharing launches, one FP32 iteration under the
    plain rule from two oracle snapshots (with and without masks): duals
    within 1e-5."""
    _check_alternatives(workloads_small()[wi])


# first layers for the 4-channel matrix-core transposed convolution: 1 and 4
# input channels, rows of 8, 16 and 64 positions (with 64, a 64-column tile
# is part of one row; with 8 and 16, several whole rows)
M4_SHAPES = {
    "c1x16x8": [WL.ConvSpec(1, 16, 8, 6, 4, 2, 1), WL.DenseSpec(6 * 8 * 4, 9), WL.DenseSpec(9, 3)],
    "c4x16x16": [WL.ConvSpec(4, 16, 16, 8, 4, 2, 1), WL.DenseSpec(8 * 8 * 8, 11), WL.DenseSpec(11, 3)],
    "c2x8x64": [WL.ConvSpec(2, 8, 64, 5, 4, 2, 1), WL.DenseSpec(5 * 4 * 32, 7), WL.DenseSpec(7, 3)],
}


@pytest.mark.parametrize("shape", sorted(M4_SHAPES))
def test_bwd_m4_geometries_match_oracle(shape):
    """The tuning alternatives (among them the matrix-core and the VALU
    transposed convolution into the input) on nets whose input layer has 1,
    2 or 4 channels in rows of 8, 16 or 64 positions: one FP32 iteration from
    oracle snapshots, duals within 1e-5."""
    sched = WL.Schedule(bigm_iters=8, as_iters=8, add_every=5, add_count=2, max_masks=3)
    w = WL.custom_config(M4_SHAPES[shape], S=5, seed=31, eps=0.05, schedule=sched, max_fixed=3, name=shape)
    _check_alternatives(w)


def _check_alternatives(w):
    A = _A()
    prm = O.params_from_schedule(w.schedule)
    prm.rule = "sgd"
    prm.bigm_lr, prm.as_lr = (1e-3, 1e-4), (1e-4, 1e-5)
    params = A.params_from_schedule(w.schedule, A.ASD_PREC_FP32)
    params.rule = A.ASD_RULE_SUPERGRADIENT
    params.bigm_lr0, params.bigm_lr1, params.as_lr0, params.as_lr1 = 1e-3, 1e-4, 1e-4, 1e-5
    A, ops, probs, net, plan, _ = _setup(w, params)
    base, alts = _tuning_alternatives(A, plan)
    assert alts, "no kernel alternative on this net"
    starts = [("bigm", 3), ("as", 4)]
    want = set(starts) | {(ph, t + 1) for ph, t in starts}
    runs = [O.solve(p, prm, snapshot_at=sorted(want, key=str)) for p in probs]
    # and the default choices with every kernel launched alone (as while
    # kernels are timed) instead of sharing launches
    alts = alts + [("profile", None, True)]
    for field, idx, val in alts:
        tun = {f: list(v) for f, v in base.items()}
        if field != "profile":
            tun[field][idx] = val
        plan.set_tuning(tun)
        plan.profile(A.ASD_PROFILE_KERNELS if field == "profile" else A.ASD_PROFILE_OFF)
        for ph, t in starts:
            H.import_states(plan, probs, [r.snapshots[(ph, t)] for r in runs])
            plan.run(A.ASD_PHASE_BIGM if ph == "bigm" else A.ASD_PHASE_AS, t, 1)
            torch.cuda.synchronize()
            K = plan.counts().n_masks
            duals = H.export_duals(plan, len(ops), K)
            for s, r in enumerate(runs):
                e = r.snapshots[(ph, t + 1)]
                for k in range(1, len(ops)):
                    pairs = [(duals[("alpha", k)][s], e.alpha[k - 1]), (duals[("beta0", k)][s], e.beta0[k - 1]),
                             (duals[("beta1", k)][s], e.beta1[k - 1])]
                    pairs += [(duals[("mask", k, q)][s], e.masks[k - 1][q].beta) for q in range(K)]
                    for a, b in pairs:
                        assert np.all(np.abs(a - b) <= 1e-5 * (1 + np.abs(b))), (field, idx, val, ph, t, s, k)
    plan.profile(False)
    plan.set_tuning(base)


def test_autotune_keeps_state():
    """asd_plan_autotune times the kernels without changing the state: the
    bound and every dual and moment are bit-identical before and after, and
    the chosen tuning is one of the valid ones."""
    w = workloads_small()[2]
    A, ops, probs, net, plan, _ = _setup(w, prec="fp32")
    rng = np.random.default_rng(90)
    states = [H.random_integral_state(p, rng, 2, scale=0.5) for p in probs]
    H.import_states(plan, probs, states)
    before = plan.bound().cpu().numpy()
    d0 = H.export_duals(plan, len(ops), 2)
    m0 = plan.get(A.ASD_F_ALPHA_M, 1).cpu().numpy()
    tun = plan.autotune(ktune=2, reps=2)
    after = plan.bound().cpu().numpy()
    d1 = H.export_duals(plan, len(ops), 2)
    assert np.array_equal(before, after)
    assert all(np.array_equal(d0[key], d1[key]) for key in d0)
    assert np.array_equal(m0, plan.get(A.ASD_F_ALPHA_M, 1).cpu().numpy())
    assert plan.counts().n_masks == 2
    assert all(1 <= v <= 8 for v in tun["ksplit"])
    print("tuning", tun, flush=True)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_solve_graph_replays_match_eager(prec):
    """asd_solve_graph: the captured iteration schedule, replayed three times
    with eager work between the replays, on the batch it was captured with
    and on another batch of the same size, and recaptured after budgets are
    set: every result equals the eager asd_solve bit for bit."""
    w = workloads_small()[2]
    A, ops, probs, net, plan, batch = _setup(w, prec=prec)
    lb_e = plan.solve(*batch).cpu().numpy()
    for rep in range(3):
        lb_g = plan.solve_graph(*batch)
        torch.cuda.synchronize()
        assert np.array_equal(lb_g.cpu().numpy(), lb_e), rep
        plan.eval()                       # eager work between replays
        torch.cuda.synchronize()
    l0, u0, lht, uht, c = batch
    mid, rad = (l0 + u0) / 2, (u0 - l0) / 4   # a smaller box: the bounds stay valid
    batch2 = ((mid - rad).contiguous(), (mid + rad).contiguous(), lht, uht, c)
    lb2_e = plan.solve(*batch2).cpu().numpy()
    lb2_g = plan.solve_graph(*batch2).cpu().numpy()
    assert np.array_equal(lb2_g, lb2_e)
    plan.set_budgets(_ragged_budgets(w, 81))
    lb3_e = plan.solve(*batch).cpu().numpy()
    lb3_g = plan.solve_graph(*batch).cpu().numpy()
    assert np.array_equal(lb3_g, lb3_e)


def test_check_finite_flags():
    """asd_check_finite: all zero after a normal solve; a non-finite bound sets
    bit 0 and a non-finite multiplier bit 1 of its subproblem only."""
    w = workloads_small()[1]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp32")
    lb = plan.solve(*batch)
    assert int(plan.check_finite(lb).abs().sum().item()) == 0
    alpha = plan.get(A.ASD_F_ALPHA, 1)
    alpha[3, 2] = float("nan")
    plan.set(A.ASD_F_ALPHA, 1, alpha)
    lb2 = lb.clone()
    lb2[5] = float("inf")
    flags = plan.check_finite(lb2).cpu().numpy()
    want = np.zeros(w.S, dtype=np.int32)
    want[3] |= 2
    want[5] |= 1
    assert np.array_equal(flags, want), flags


def test_invalid_inputs_are_flagged_not_fatal():
    """Subproblems with an empty input interval (l0 > u0), an empty
    pre-activation interval (lhat > uhat: an infeasible subdomain), a NaN
    bound or an infinite objective entry: the solve completes, bit 2 of
    exactly those subproblems' flags is set, and every other subproblem's
    bound is bit-identical to a solve of the clean batch."""
    w = workloads_small()[1]
    A, ops, probs, net, plan, batch = _setup(w, prec="fp32")
    clean = plan.solve(*batch).cpu().numpy()
    assert int(plan.check_finite(torch.as_tensor(clean)).abs().sum().item()) == 0
    l0, u0, lht, uht, c = [t.clone() if isinstance(t, torch.Tensor) else [x.clone() for x in t] for t in batch]
    bad = {2: "l0 > u0", 4: "lhat > uhat", 6: "nan bound", 8: "inf objective"}
    l0[2, 5] = u0[2, 5] + 0.5
    lht[1][4, 3] = uht[1][4, 3] + 1.0
    uht[0][6, 0] = float("nan")
    c[8, 1] = float("inf")
    lb = plan.solve(l0, u0, lht, uht, c)
    torch.cuda.synchronize()
    flags = plan.check_finite(lb).cpu().numpy()
    lb = lb.cpu().numpy()
    for s in range(w.S):
        if s in bad:
            assert flags[s] & 4, (s, bad[s], flags[s])
        else:
            assert flags[s] == 0 and lb[s] == clean[s], (s, flags[s], lb[s], clean[s])
    # the next clean load clears the input flags
    lb2 = plan.solve(*batch)
    assert int(plan.check_finite(lb2).abs().sum().item()) == 0
