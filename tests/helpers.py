"""Shared test helpers: inputs for both sides, oracle state <-> GPU plan."""
from __future__ import annotations

import numpy as np

from oracle import asd_oracle as O
from paper_2101_05844_amd import workloads as WL


SMALL_CONV = [WL.ConvSpec(2, 7, 9, 5, 3, 1, 1), WL.ConvSpec(5, 7, 9, 6, 4, 2, 1),
              WL.DenseSpec(6 * 3 * 4, 13), WL.DenseSpec(13, 3)]
SMALL_DENSE = [WL.DenseSpec(37, 53), WL.DenseSpec(53, 29), WL.DenseSpec(29, 4)]
# shapes that take the matrix-core kernels of FP32 plans: a 32-channel
# convolution forward (kernel 4, stride 2), a transposed convolution into a
# 16-channel layer of 256 positions, a dense layer fed by 64-position
# channels (forward on matrix cores, backward with positions on lanes)
MFMA_CONV = [WL.ConvSpec(2, 16, 16, 16, 3, 1, 1), WL.ConvSpec(16, 16, 16, 32, 4, 2, 1),
             WL.DenseSpec(32 * 8 * 8, 20), WL.DenseSpec(20, 3)]
# the convolutions of the wider CIFAR variant (32 and 64 channels) with a
# narrow dense head: transposed convolutions from 64 channels on the matrix
# cores, the dense backward with positions on lanes into 64 x 8 x 8
WIDER_CONV = [WL.ConvSpec(3, 32, 32, 32, 4, 2, 1), WL.ConvSpec(32, 16, 16, 64, 4, 2, 1),
              WL.DenseSpec(64 * 8 * 8, 24), WL.DenseSpec(24, 3)]


def workloads_small():
    sched = WL.Schedule(bigm_iters=12, as_iters=14, add_every=5, add_count=2, max_masks=4)
    return [
        WL.custom_config(SMALL_DENSE, S=70, seed=21, eps=0.1, centre_range=(-1.0, 1.0), schedule=sched,
                         max_fixed=3, name="dense-37-53-29-4"),
        WL.custom_config(SMALL_CONV, S=11, seed=22, eps=0.05, schedule=sched, max_fixed=4,
                         name="conv-2x7x9"),
        WL.custom_config(MFMA_CONV, S=9, seed=23, eps=0.03, schedule=sched, max_fixed=6,
                         name="conv-2x16x16"),
        WL.custom_config(WIDER_CONV, S=4, seed=24, eps=0.01, schedule=sched, max_fixed=8,
                         name="conv-3x32x32-wider"),
    ]


def e2e_workloads():
    return workloads_small()[:2] + [WL.mnist_mlp_config(), workloads_small()[2]]


def f32(a):
    return np.asarray(a, dtype=np.float32)


def oracle_bounds(w: WL.Workload):
    """Pre-activation bounds of every ReLU layer, [S, n_k] float32, computed by
    the oracle's interval propagation per subproblem and then the
    workload's subdomain fixes (both sides receive exactly these values)."""
    ops = O.ops_from_workload_layers(w.layers)
    per = [O.interval_bounds(ops, w.l0[s].astype(np.float64), w.u0[s].astype(np.float64))
           for s in range(w.S)]
    n_relu = len(w.layers) - 1
    root_l = [np.stack([per[s][0][k] for s in range(w.S)]) for k in range(n_relu)]
    root_u = [np.stack([per[s][1][k] for s in range(w.S)]) for k in range(n_relu)]
    # round outward to float32 so the bounds stay valid
    root_l = [np.nextafter(f32(a), np.float32(-np.inf), dtype=np.float32) for a in root_l]
    root_u = [np.nextafter(f32(a), np.float32(np.inf), dtype=np.float32) for a in root_u]
    lh, uh = WL.subdomain_bounds(root_l, root_u, w.fix_draws, w.S)
    return ops, lh, uh


def oracle_problems(w: WL.Workload, ops, lh, uh):
    return [O.make_problem(ops, w.l0[s], w.u0[s], [a[s] for a in lh], [a[s] for a in uh], w.c[s])
            for s in range(w.S)]


def gpu_batch(w: WL.Workload, lh, uh):
    import torch
    dev = "cuda"
    t = lambda a: torch.as_tensor(f32(a), device=dev).contiguous()
    return t(w.l0), t(w.u0), [t(a) for a in lh], [t(a) for a in uh], t(w.c)


def random_integral_state(p: O.Problem, rng, n_masks: int, scale: float = 1.0):
    """Random float32-valued duals and masks from the oracle at random integral
    points (as Active Set produces them)."""
    st = O.zero_state(p)
    for k in range(1, p.n):
        n = p.W(k).n_out
        st.alpha[k - 1] = f32(rng.uniform(0, scale, n)).astype(np.float64)
        st.beta0[k - 1] = f32(rng.uniform(0, scale, n)).astype(np.float64)
        st.beta1[k - 1] = f32(rng.uniform(0, scale, n)).astype(np.float64)
        for _ in range(n_masks):
            op = p.W(k)
            lp_, up_ = p.lu(k - 1)
            xprev = np.where(rng.integers(0, 2, op.n_in) == 1, up_, lp_)
            z = rng.integers(0, 2, n).astype(np.float64)
            I = O.oracle_mask(op, lp_, up_, xprev, z)
            M = O.new_mask(op, I, lp_, up_, xprev, z)
            M.beta = f32(rng.uniform(0, scale, n)).astype(np.float64)
            st.masks[k - 1].append(M)
    return st


def import_states(plan, problems, states):
    """Writes oracle states (one per subproblem) into a GPU plan."""
    import torch
    from paper_2101_05844_amd import asdual as A
    n = problems[0].n
    S = len(states)
    dev = "cuda"
    t = lambda rows: torch.as_tensor(np.stack(rows), device=dev).to(plan.dtype)
    K = len(states[0].masks[0]) if n > 1 else 0
    for k in range(1, n):
        plan.set(A.ASD_F_ALPHA, k, t([st.alpha[k - 1] for st in states]))
        plan.set(A.ASD_F_BETA0, k, t([st.beta0[k - 1] for st in states]))
        plan.set(A.ASD_F_BETA1, k, t([st.beta1[k - 1] for st in states]))
        for name, fa, fv in (("alpha", A.ASD_F_ALPHA_M, A.ASD_F_ALPHA_V),
                             ("beta0", A.ASD_F_BETA0_M, A.ASD_F_BETA0_V),
                             ("beta1", A.ASD_F_BETA1_M, A.ASD_F_BETA1_V)):
            plan.set(fa, k, t([st.m[name][k - 1] for st in states]))
            plan.set(fv, k, t([st.v[name][k - 1] for st in states]))
        for q in range(K):
            Ms = [st.masks[k - 1][q] for st in states]
            plan.set(A.ASD_F_MASK_Z, k, t([M.z for M in Ms]), q)
            plan.set(A.ASD_F_MASK_XPREV, k, t([M.x_prev for M in Ms]), q)
            plan.set(A.ASD_F_MASK_BETA, k, t([M.beta for M in Ms]), q)
            plan.set(A.ASD_F_MASK_M, k, t([M.m for M in Ms]), q)
            plan.set(A.ASD_F_MASK_V, k, t([M.v for M in Ms]), q)
    steps = [states[0].masks[0][q].step for q in range(K)] if n > 1 else []
    plan.set_counts(K, states[0].step, steps, recompute=True)
    torch.cuda.synchronize()


def export_duals(plan, n, K):
    from paper_2101_05844_amd import asdual as A
    out = {}
    for k in range(1, n):
        out[("alpha", k)] = plan.get(A.ASD_F_ALPHA, k).cpu().numpy()
        out[("beta0", k)] = plan.get(A.ASD_F_BETA0, k).cpu().numpy()
        out[("beta1", k)] = plan.get(A.ASD_F_BETA1, k).cpu().numpy()
        for q in range(K):
            out[("mask", k, q)] = plan.get(A.ASD_F_MASK_BETA, k, q).cpu().numpy()
    return out


def objective_scale(p: O.Problem, st: O.DualState) -> float:
    """Sum of the absolute values of the terms of d_B (parity scale)."""
    f, g, const = O.dual_functions(p, st)
    x, z = O.inner_min(p, f, g)
    sc = abs(float(p.W(p.n).b @ p.c))
    for k in range(1, p.n):
        lh, _ = p.hat(k)
        b = p.W(k).b
        sc += float(np.abs(b * st.alpha[k - 1]).sum() + np.abs(st.beta1[k - 1] * (lh - b)).sum())
        for M in st.masks[k - 1]:
            sc += float(np.abs(M.LI * M.beta).sum())
    sc += sum(float(np.abs(fk * xk).sum()) for fk, xk in zip(f, x))
    sc += sum(float(np.abs(gk * zk).sum()) for gk, zk in zip(g, z))
    return sc


def _absop(op):
    return op.with_data(np.abs(op.w))


def f_row_scale(p: O.Problem, st: O.DualState, k: int) -> np.ndarray:
    """Sum of the magnitudes of the terms of f_k (eq:dual-anderson-functions
    restricted to the active set): the rounding scale of each entry."""
    n = p.n
    opn = _absop(p.W(k + 1))
    if k + 1 == n:
        v = np.abs(p.c)
    else:
        v = np.abs(st.alpha[k]) + np.abs(st.beta1[k])
        for M in st.masks[k]:
            v = v + np.abs(M.beta)
    sc = opn.T @ v
    if k >= 1:
        sc = sc + np.abs(st.alpha[k - 1]) + np.abs(st.beta0[k - 1]) + np.abs(st.beta1[k - 1])
        for M in st.masks[k - 1]:
            sc = sc + np.abs(M.beta)
    return sc


def g_row_scale(p: O.Problem, st: O.DualState, k: int) -> np.ndarray:
    lh, uh = p.hat(k)
    b = np.abs(p.W(k).b)
    sc = np.abs(st.beta0[k - 1] * uh) + np.abs(st.beta1[k - 1] * lh)
    for M in st.masks[k - 1]:
        sc = sc + np.abs(M.beta) * (np.abs(M.UI) + np.abs(M.LI) + b)
    return sc


def grad_row_scale(p: O.Problem, st: O.DualState, x, k: int) -> np.ndarray:
    """Magnitudes of the terms of the layer-k supergradient entries
    (eq:as-supergradient) at the primal point x."""
    lh, uh = p.hat(k)
    op = p.W(k)
    sc = _absop(op) @ np.abs(x[k - 1]) + np.abs(op.b) + np.abs(x[k]) + np.abs(lh) + np.abs(uh)
    for M in st.masks[k - 1]:
        sc = sc + np.abs(M.LI) + np.abs(M.UI)
    return sc


def check_eval_against_oracle(res, rows, eps, eps_grad=None):
    """Element-wise comparison of an asd_eval result with the oracle.

    rows: iterable of (s, problem, state) (s = the subproblem's row in the
    batch).  f_k and g_k within eps times their row scale (f skipped where
    the neuron's box is a point: the iteration kernels do not form it
    there); x*, z* equal to the oracle's minimiser wherever the oracle's
    |f| (|g|) exceeds eps times its scale; every supergradient entry equal,
    within eps times its row scale, to the oracle's supergradient at the
    GPU's own primal point (x*, z* are valid minimisers at ties too), within
    eps_grad (default eps) times its row scale.  Returns counts of the
    compared and the tie-excused entries."""
    eps_grad = eps if eps_grad is None else eps_grad
    cnt = {"f": 0, "g": 0, "x": 0, "z": 0, "grad": 0, "x_ties": 0, "z_ties": 0, "f_point": 0}
    for s, p, st in rows:
        d, x, z, f, g = O.evaluate(p, st)
        xg = [res["x"][k][s].cpu().numpy().astype(np.float64) for k in range(p.n)]
        zg = [res["z"][k][s].cpu().numpy().astype(np.float64) for k in range(1, p.n)]
        for k in range(p.n):
            lo, hi = p.lu(k)
            point = lo == hi
            fsc = eps * (1.0 + f_row_scale(p, st, k))
            fg = res["f"][k][s].cpu().numpy().astype(np.float64)
            ok = (np.abs(fg - f[k]) <= fsc) | point
            assert ok.all(), ("f", s, k, np.flatnonzero(~ok)[:5], fg[~ok][:5], f[k][~ok][:5])
            cnt["f"] += int((~point).sum())
            cnt["f_point"] += int(point.sum())
            assert np.all((xg[k] == lo) | (xg[k] == hi)), ("x* off the box ends", s, k)
            sure = np.abs(f[k]) > fsc
            assert np.all((xg[k] == x[k]) | ~sure), ("x*", s, k, np.flatnonzero((xg[k] != x[k]) & sure)[:5])
            cnt["x"] += int(sure.sum())
            cnt["x_ties"] += int((~sure).sum())
        for k in range(1, p.n):
            gsc = eps * (1.0 + g_row_scale(p, st, k))
            gg = res["g"][k][s].cpu().numpy().astype(np.float64)
            ok = np.abs(gg - g[k - 1]) <= gsc
            assert ok.all(), ("g", s, k, np.flatnonzero(~ok)[:5])
            cnt["g"] += ok.size
            sure = np.abs(g[k - 1]) > gsc
            assert np.all((zg[k - 1] == z[k - 1]) | ~sure), ("z*", s, k)
            cnt["z"] += int(sure.sum())
            cnt["z_ties"] += int((~sure).sum())
        sg = O.supergradient(p, st, xg, zg)
        for k in range(1, p.n):
            tol = eps_grad * (1.0 + grad_row_scale(p, st, xg, k))
            items = [("ga", sg["alpha"][k - 1]), ("gb0", sg["beta0"][k - 1]), ("gb1", sg["beta1"][k - 1])]
            items += [(("gm", q), sg["masks"][k - 1][q]) for q in range(len(st.masks[k - 1]))]
            for key, ref in items:
                got = res[key[0]][k][key[1]][s] if isinstance(key, tuple) else res[key][k][s]
                got = got.cpu().numpy().astype(np.float64)
                bad = np.abs(got - ref) > tol
                assert not bad.any(), (key, s, k, np.flatnonzero(bad)[:5], got[bad][:5], ref[bad][:5])
                cnt["grad"] += got.size
    return cnt


def oracle_states_from_plan(plan, problems: dict):
    """The plan's current duals and active sets (asd_state_get) as oracle
    states, one per subproblem s in problems ({s: Problem}): multipliers
    as exported (FP32 values for FP32 plans), each mask rebuilt by the
    oracle's own eq:oracle at the primal point the plan recorded for it."""
    from paper_2101_05844_amd import asdual as A
    p0 = next(iter(problems.values()))
    n = p0.n
    K = plan.counts().n_masks
    g = lambda f, k, q=0: plan.get(f, k, q).cpu().numpy().astype(np.float64)
    ex = {}
    for k in range(1, n):
        ex[("alpha", k)] = g(A.ASD_F_ALPHA, k)
        ex[("beta0", k)] = g(A.ASD_F_BETA0, k)
        ex[("beta1", k)] = g(A.ASD_F_BETA1, k)
        for q in range(K):
            ex[("beta", k, q)] = g(A.ASD_F_MASK_BETA, k, q)
            ex[("z", k, q)] = g(A.ASD_F_MASK_Z, k, q)
            ex[("x", k, q)] = g(A.ASD_F_MASK_XPREV, k, q)
    out = {}
    for s, p in problems.items():
        st = O.zero_state(p)
        for k in range(1, n):
            st.alpha[k - 1] = ex[("alpha", k)][s]
            st.beta0[k - 1] = ex[("beta0", k)][s]
            st.beta1[k - 1] = ex[("beta1", k)][s]
            op = p.W(k)
            lp_, up_ = p.lu(k - 1)
            for q in range(K):
                xp, z = ex[("x", k, q)][s], ex[("z", k, q)][s]
                M = O.new_mask(op, O.oracle_mask(op, lp_, up_, xp, z), lp_, up_, xp, z)
                M.beta = ex[("beta", k, q)][s]
                st.masks[k - 1].append(M)
        out[s] = st
    return out


def final_bound_errors(plan, lb, problems: dict):
    """Per-result error of the plan's FP64 final bound (asd_bound, lb [S]) at
    its final duals: |lb[s] - d_B(s)| with d_B evaluated by the oracle at the
    exported duals and masks (eq:dual-active-set), absolute and relative to
    the sum of the magnitudes of d_B's terms."""
    states = oracle_states_from_plan(plan, problems)
    out = {}
    for s, p in problems.items():
        d = O.evaluate(p, states[s])[0]
        sc = objective_scale(p, states[s])
        out[s] = (abs(float(lb[s]) - d), abs(float(lb[s]) - d) / sc, d)
    return out


def fp32_band(name: str, factor: float = 2.0, floor: float = 1e-4):
    """Whole-run band of an FP32 (or mixed-mode) plan against the FP64 oracle
    on workload `name`: factor times the distance the oracle's own FP32
    noise model moves its runs (tests/golden/fp32_band.json, max and mean
    over the workload's subproblems), at least `floor`."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fp32_band.json")) as fh:
        rec = json.load(fh)["workloads"][name]
    out = {}
    for key, pre in (("noise", ""), ("noise_mixed", "mixed_"), ("noise_bf16", "bf16_"),
                     ("noise_bf16_all", "bf16_all_")):
        out[pre + "max"] = max(floor, factor * rec[key]["max_rel"])
        out[pre + "mean"] = max(floor, factor * rec[key]["mean_rel"])
    return out
