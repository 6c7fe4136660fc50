"""Shared test helpers: inputs for both sides, oracle state <-> GPU plan."""
from __future__ import annotations

import numpy as np

from oracle import asd_oracle as O
from paper_2101_05844_amd import workloads as WL


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
