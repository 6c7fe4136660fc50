"""GPU parity, through the C ABI, of the l2-ball input domain (Sec. 2 input
set C; eq:as-primal0-min over the ball; reading R20: layer 1 keeps no
masks).  Both sides receive the same float32 centres, radii, box hulls and
interval bounds of the hulls.

Tolerances: FP64 whole runs within 1e-8 * max(1, |d|); at fixed duals the
objective within EPS * (sum of the magnitudes of its terms) and x*_0 within
EPS * (|centre| + radius) (EPS = 1e-5 FP32, 1e-11 FP64); FP32 whole runs
valid against sampled outputs of the ball and within 5e-2 * max(1, |d|) of
the FP64 oracle run (the FP32 whole-run band of the box domain)."""
import numpy as np
import pytest

from oracle import asd_oracle as O
from paper_2101_05844_amd import workloads as WL
from tests import helpers as H
from tests.test_gpu_parity import _A

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = {"fp32": 1e-5, "fp64": 1e-11}


def ball_workloads():
    sched = WL.Schedule(bigm_iters=16, as_iters=18, add_every=6, add_count=2, max_masks=4)
    return [WL.custom_config(H.SMALL_DENSE, S=6, seed=81, eps=0.1, centre_range=(-1.0, 1.0), schedule=sched,
                             name="l2-dense"),
            WL.custom_config(H.MFMA_CONV, S=5, seed=82, eps=0.03, schedule=sched, name="l2-conv")]


def ball_batch(w, scale=2.0):
    """float32 centres and radii (radius = scale * eps of the workload, in l2)
    with the outward-rounded box hulls and their interval bounds."""
    centre = H.f32((w.l0.astype(np.float64) + w.u0.astype(np.float64)) / 2)
    r = np.full(w.S, np.float32(scale * w.meta["eps"]), dtype=np.float32)
    lo = np.nextafter(H.f32(centre - r[:, None]), np.float32(-np.inf), dtype=np.float32)
    hi = np.nextafter(H.f32(centre + r[:, None]), np.float32(np.inf), dtype=np.float32)
    ops = O.ops_from_workload_layers(w.layers)
    per = [O.interval_bounds(ops, lo[s].astype(np.float64), hi[s].astype(np.float64)) for s in range(w.S)]
    n_relu = len(w.layers) - 1
    lh = [np.nextafter(H.f32(np.stack([per[s][0][k] for s in range(w.S)])), np.float32(-np.inf), dtype=np.float32)
          for k in range(n_relu)]
    uh = [np.nextafter(H.f32(np.stack([per[s][1][k] for s in range(w.S)])), np.float32(np.inf), dtype=np.float32)
          for k in range(n_relu)]
    probs = [O.make_problem(ops, lo[s], hi[s], [a[s] for a in lh], [a[s] for a in uh], w.c[s],
                            ball=(centre[s].astype(np.float64), float(r[s]))) for s in range(w.S)]
    return ops, centre, r, lo, hi, lh, uh, probs


def ball_plan(A, w, prec, centre, r, lo, hi, lh, uh):
    net = A.Net(w.layers)
    prm = A.params_from_schedule(w.schedule, A.ASD_PREC_FP64 if prec == "fp64" else A.ASD_PREC_FP32)
    plan = A.Plan(net, w.S, prm)
    t = lambda a: torch.as_tensor(H.f32(a), device="cuda").contiguous()
    plan.set_input_domain(A.ASD_DOMAIN_L2, t(centre), t(r))
    batch = (t(lo), t(hi), [t(a) for a in lh], [t(a) for a in uh], t(w.c))
    plan.init(*batch)
    return plan, batch


def sampled_min(ops, c, centre, radius, rng, m=4000):
    n = centre.size
    d = rng.normal(size=(m, n))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = np.concatenate([centre + radius * d, centre + radius * rng.uniform(0, 1, (m, 1)) ** (1 / n) * d])
    return float((O.network_output(ops, pts) @ c).min())


@pytest.mark.parametrize("wi", [0, 1])
def test_l2_fp64_end_to_end(wi):
    """Whole FP64 runs over l2 balls (Big-M, Active Set with additions at
    layers >= 2, final bound with x*_0 on the ball) agree with the oracle
    within 1e-8 and stay below sampled outputs of the ball."""
    w = ball_workloads()[wi]
    A = _A()
    ops, centre, r, lo, hi, lh, uh, probs = ball_batch(w)
    plan, batch = ball_plan(A, w, "fp64", centre, r, lo, hi, lh, uh)
    lb, x0 = plan.solve(*batch, want_x0=True)
    lb, x0 = lb.cpu().numpy(), x0.cpu().numpy()
    prm = O.params_from_schedule(w.schedule)
    rng = np.random.default_rng(5)
    for s, p in enumerate(probs):
        res = O.solve(p, prm)
        assert abs(lb[s] - res.bound) <= 1e-8 * max(1.0, abs(res.bound)), (s, lb[s], res.bound)
        assert np.abs(np.linalg.norm(x0[s].astype(np.float64) - centre[s]) - r[s]) <= 1e-5 * (1 + r[s])
        assert lb[s] <= sampled_min(ops, w.c[s].astype(np.float64), centre[s].astype(np.float64), float(r[s]),
                                    rng) + 1e-9


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("wi", [0, 1])
def test_l2_fixed_dual_evaluation(wi, prec):
    """At imported duals (masks at every layer, layer 1's with multipliers
    0): the objective through the general kernels and x*_0 through both
    evaluation paths match the oracle's evaluation over the ball."""
    w = ball_workloads()[wi]
    A = _A()
    ops, centre, r, lo, hi, lh, uh, probs = ball_batch(w)
    plan, _ = ball_plan(A, w, prec, centre, r, lo, hi, lh, uh)
    rng = np.random.default_rng(90 + wi)
    states = [H.random_integral_state(p, rng, 2, scale=0.5) for p in probs]
    for st in states:
        for M in st.masks[0]:
            M.beta = np.zeros_like(M.beta)
    H.import_states(plan, probs, states)
    eps = EPS[prec]
    paths = [A.ASD_EVAL_GENERAL] + ([A.ASD_EVAL_ITERATION] if prec == "fp32" else [])
    for path in paths:
        res = plan.eval(path=path)
        torch.cuda.synchronize()
        for s, (p, st) in enumerate(zip(probs, states)):
            d, x, z, f, g = O.evaluate(p, st)
            if res["obj"] is not None and path == A.ASD_EVAL_GENERAL:
                obj = res["obj"].cpu().numpy()
                assert abs(obj[s] - d) <= eps * H.objective_scale(p, st), (path, s, obj[s], d)
            xg = res["x"][0][s].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(xg - x[0]) <= eps * (np.abs(centre[s]) + r[s]) + 1e-7 * (prec == "fp32")), \
                (path, s, np.abs(xg - x[0]).max())


@pytest.mark.parametrize("wi", [0, 1])
def test_l2_fp32_end_to_end(wi):
    """Whole FP32 runs over l2 balls: below sampled outputs of the ball and
    within the FP32 whole-run band of the FP64 oracle's runs."""
    w = ball_workloads()[wi]
    A = _A()
    ops, centre, r, lo, hi, lh, uh, probs = ball_batch(w)
    plan, batch = ball_plan(A, w, "fp32", centre, r, lo, hi, lh, uh)
    lb = plan.solve(*batch).cpu().numpy()
    prm = O.params_from_schedule(w.schedule)
    rng = np.random.default_rng(6)
    for s, p in enumerate(probs):
        res = O.solve(p, prm)
        assert abs(lb[s] - res.bound) <= 5e-2 * max(1.0, abs(res.bound)), (s, lb[s], res.bound)
        assert lb[s] <= sampled_min(ops, w.c[s].astype(np.float64), centre[s].astype(np.float64), float(r[s]),
                                    rng) + 1e-6


def test_l2_domain_switch_and_refusals():
    """Switching back to the box domain gives the box solve bit for bit; an
    l2 plan refuses the bound gradient."""
    w = ball_workloads()[0]
    A = _A()
    ops, centre, r, lo, hi, lh, uh, probs = ball_batch(w)
    plan, batch = ball_plan(A, w, "fp32", centre, r, lo, hi, lh, uh)
    plan.solve(*batch)
    with pytest.raises(A.AsdError, match="box input domains"):
        plan.bound_grad(torch.ones(w.S, dtype=torch.float64, device="cuda"))
    plan.set_input_domain(A.ASD_DOMAIN_BOX)
    lb_box = plan.solve(*batch)
    fresh = A.Plan(A.Net(w.layers), w.S, A.params_from_schedule(w.schedule))
    assert torch.equal(lb_box, fresh.solve(*batch))
