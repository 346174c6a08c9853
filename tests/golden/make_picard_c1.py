"""Writes picard_c1.json: the nonlinear residuals ||r^(i)|| / ||f|| of
Picard's method (Alg. 3.1) with exact linear solves and untruncated
iterates on the C1 problem (16 x 48 grid, h = 1/4, m = 2, p = 2, n_t = 10),
from the oracle alone (oracle.solver.picard_direct).  About half an hour on
one host core.  Run from the repository root:

    python tests/golden/make_picard_c1.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.solver import picard_direct  # noqa: E402
from oracle.system import Problem  # noqa: E402
from synthetic_inputs import CONFIGS  # noqa: E402

STEPS = 6


def main():
    P = Problem(CONFIGS["C1"])
    _, res = picard_direct(P, STEPS)
    out = {"config": "C1", "cfg": CONFIGS["C1"], "steps": STEPS,
           "source": "oracle.solver.picard_direct (exact solves, untruncated iterates)",
           "nonlinear_residual": [float(r) for r in res]}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "picard_c1.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out["nonlinear_residual"])


if __name__ == "__main__":
    main()
