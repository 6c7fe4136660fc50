"""Writes fp32_band.json: how far FP32 storage of the solver state moves a
whole Active Set run (Algorithm 1 after Algorithm 3) on the end-to-end test
workloads, measured with the FP64 oracle alone.

For the first 12 subproblems of each workload the oracle runs the workload's
schedule twice: with its state in FP64, and with every dual, moment and mask
constant stored as a float32 value after each iteration.  Recorded per
workload: the largest and the mean of |d_fp64 - d_fp32| / max(1, |d_fp64|),
and the same for a third run that also stores its Adam moments as bfloat16
(the mixed mode's storage).
A GPU run in FP32 rounds at least as often as the second run, so these are
the scale of its expected distance from the FP64 oracle's run.

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
N_SUB = 12


def main():
    res = {}
    for w in H.e2e_workloads():
        ops, lh, uh = H.oracle_bounds(w)
        probs = H.oracle_problems(w, ops, lh, uh)[:N_SUB]
        prm = O.params_from_schedule(w.schedule)
        prm32 = O.params_from_schedule(w.schedule)
        prm32.storage = "fp32"
        prm_m = O.params_from_schedule(w.schedule)
        prm_m.storage = "fp32"
        prm_m.adam = O.AdamConsts(prm_m.adam.beta1, prm_m.adam.beta2, prm_m.adam.eps, moments="bf16")
        a = np.array([O.solve(p, prm).bound for p in probs])
        b = np.array([O.solve(p, prm32).bound for p in probs])
        c = np.array([O.solve(p, prm_m).bound for p in probs])
        rel = np.abs(a - b) / np.maximum(1.0, np.abs(a))
        relm = np.abs(a - c) / np.maximum(1.0, np.abs(a))
        res[w.name] = {"max_rel": float(rel.max()), "mean_rel": float(rel.mean()),
                       "mixed_max_rel": float(relm.max()), "mixed_mean_rel": float(relm.mean()),
                       "subproblems": len(probs)}
        print(w.name, res[w.name], flush=True)
    doc = {"what": "FP64 oracle run vs the same run with its state stored as float32 after every iteration "
                   "(mixed_*: and its Adam moments as bfloat16); relative final-bound differences over the "
                   "first 12 subproblems",
           "script": "tests/golden/fp32_band.py", "workloads": res}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
