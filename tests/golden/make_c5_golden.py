"""Writes c5_full_oracle.json: the float64 oracle's answer for accounts 0 and
1 of the large-universe book (8 accounts over N = 384,800 names, k = 100,
50 one-hot groups with bands, 2,000 held names with 4-lot tax, seed 0).

The oracle needs about two minutes per account at this size, too long for a
test, so its answer is stored: objective, budget / cap multipliers and the
support of w* (every weight above 1e-13; the rest are zero to round-off),
with the oracle's own certificate.  Only ``oracle/`` and the seeded input
generator are called.

    python tests/golden/make_c5_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.problem import account  # noqa: E402
from workloads import make_config  # noqa: E402

ACCOUNTS = (0, 1)
OUT = os.path.join(HERE, "c5_full_oracle.json")


def main():
    uni, book = make_config("c5", 0)
    rec = dict(workload="c5 seed 0: 8 x 384,800, k=100, G=50", accounts={})
    for a in ACCOUNTS:
        t0 = time.time()
        out = oracle.solve_account(account(uni, book, a))
        w = out["w"]
        sup = np.flatnonzero(np.abs(w) > 1e-13)
        res = {k: float(v) for k, v in out["res"].items()}
        rec["accounts"][str(a)] = dict(
            obj=float(out["obj"]), nu=float(out["nu"]),
            lam_cap=float(out["lam_cap"]),
            support=[int(i) for i in sup],
            w_support=[float(x) for x in w[sup]],
            res=res, route=out["route"], ipm_iters=int(out["ipm_iters"]),
            seconds=round(time.time() - t0, 1))
        print(a, rec["accounts"][str(a)]["obj"], len(sup), res, flush=True)
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=0, sort_keys=True)


if __name__ == "__main__":
    main()
