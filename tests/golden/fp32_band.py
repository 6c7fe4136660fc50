"""Writes fp32_band.json: how far FP32 arithmetic may move a whole Active Set
run (Algorithm 1 after Algorithm 3) on the end-to-end test workloads,
measured with the FP64 oracle alone.

For every subproblem of each workload the oracle runs the workload's
schedule in FP64 (the reference run) and in models of reduced-precision
runs:

  storage  every dual, moment and mask constant stored as a float32 value
           after each iteration (the rounding of the state alone: a lower
           model, since an FP32 implementation also rounds its products);
  noise    the storage model plus, in every iteration, a uniform error of up
           to one float32 unit (2^-24) of each entry's rounding scale added
           to f_k and g_k before the inner minimisation and to every
           supergradient entry (the rounding scale of an entry is the sum of
           the magnitudes of the terms that form it: the scale the
           fixed-dual parity tests use); two seeds;
  noise_mixed     the noise model with the Adam moments stored as bfloat16
                  (the mixed mode's storage);
  noise_bf16      the mixed model with errors of 2^-8 units on the
                  supergradient (BF16 operands in the forward products), f
                  and g as in noise;
  noise_bf16_all  and also errors of 2^-8 units on f and g (BF16 operands
                  in the transposed products).

Recorded per workload, for each model: the largest and the mean over the
subproblems (and seeds) of |d_fp64 - d_model| / max(1, |d_fp64|).  The runs
part at near-ties of the minimiser, so the distances are heavy-tailed: the
largest needs every subproblem.

Run from the repository root: python -m tests.golden.fp32_band
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import asd_oracle as O  # noqa: E402
from tests import helpers as H  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp32_band.json")
EPS32 = 2.0 ** -24
EPS_BF16 = 2.0 ** -8  # one BF16 rounding of both operands of a product
SEEDS = (0, 1)


def noisy_solve(p, prm, rng, eps_fg=EPS32, eps_grad=EPS32):
    """The oracle's schedule (Algorithm 3, then Algorithm 1 with additions),
    with the errors of the noise model injected (eps_fg on f and g, eps_grad
    on the supergradient, in units of each entry's rounding scale) and the
    state stored as float32 after every iteration; returns d_B at the final
    duals."""
    st = O.zero_state(p)

    def iteration(t, lr, as_phase):
        f, g, _ = O.dual_functions(p, st)
        f = [fk + rng.uniform(-1, 1, fk.shape) * eps_fg * (1 + H.f_row_scale(p, st, k)) for k, fk in enumerate(f)]
        g = [gk + rng.uniform(-1, 1, gk.shape) * eps_fg * (1 + H.g_row_scale(p, st, k + 1)) for k, gk in enumerate(g)]
        x, z = O.inner_min(p, f, g)
        if as_phase and O.is_addition_iter(t, prm, len(st.masks[0])):
            O.add_masks(p, st, x, z)
        sg = O.supergradient(p, st, x, z)
        for k in range(1, p.n):
            sc = eps_grad * (1 + H.grad_row_scale(p, st, x, k))
            for name in ("alpha", "beta0", "beta1"):
                sg[name][k - 1] = sg[name][k - 1] + rng.uniform(-1, 1, sc.shape) * sc
            sg["masks"][k - 1] = [a + rng.uniform(-1, 1, sc.shape) * sc for a in sg["masks"][k - 1]]
        O.apply_step(st, sg, lr, prm.rule, prm.adam)
        O.round_state_fp32(st)

    for t in range(prm.bigm_iters):
        iteration(t, O.linear_lr(*prm.bigm_lr, t, prm.bigm_iters), False)
    if prm.rule == "adam":
        O.reset_moments(st)
    for t in range(prm.as_iters):
        iteration(t, O.linear_lr(*prm.as_lr, t, prm.as_iters), True)
    return O.evaluate(p, st)[0]


def rel(a, b):
    r = np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(1.0, np.abs(np.asarray(a)))
    return {"max_rel": float(r.max()), "mean_rel": float(r.mean())}


def main():
    res = {}
    for w in H.e2e_workloads():
        ops, lh, uh = H.oracle_bounds(w)
        probs = H.oracle_problems(w, ops, lh, uh)
        prm = O.params_from_schedule(w.schedule)
        prm32 = O.params_from_schedule(w.schedule)
        prm32.storage = "fp32"
        prm_m = O.params_from_schedule(w.schedule)
        prm_m.adam = O.AdamConsts(prm_m.adam.beta1, prm_m.adam.beta2, prm_m.adam.eps, moments="bf16")
        ref = np.array([O.solve(p, prm).bound for p in probs])
        sto = np.array([O.solve(p, prm32).bound for p in probs])
        noi, mix, bfw, bfa = [], [], [], []
        for seed in SEEDS:
            rng = np.random.default_rng(seed)
            noi.append([noisy_solve(p, prm, rng) for p in probs])
            rng = np.random.default_rng(100 + seed)
            mix.append([noisy_solve(p, prm_m, rng) for p in probs])
            rng = np.random.default_rng(200 + seed)
            bfw.append([noisy_solve(p, prm_m, rng, EPS32, EPS_BF16) for p in probs])
            rng = np.random.default_rng(300 + seed)
            bfa.append([noisy_solve(p, prm_m, rng, EPS_BF16, EPS_BF16) for p in probs])
        refs = np.tile(ref, (len(SEEDS), 1))
        res[w.name] = {"storage": rel(ref, sto), "noise": rel(refs, noi), "noise_mixed": rel(refs, mix),
                       "noise_bf16": rel(refs, bfw), "noise_bf16_all": rel(refs, bfa),
                       "subproblems": len(probs), "seeds": len(SEEDS)}
        print(w.name, res[w.name], flush=True)
    doc = {"what": "relative distance of FP32-run models from the FP64 oracle run, per workload "
                   "(storage: state stored as float32; noise: plus errors of one float32 unit of each "
                   "entry's rounding scale on f, g and the supergradient; noise_mixed: the noise model "
                   "with bfloat16 moments; noise_bf16: and errors of 2^-8 units on the supergradient; "
                   "noise_bf16_all: and on f and g)",
           "script": "tests/golden/fp32_band.py", "workloads": res}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
