"""Write the golden fixtures under tests/golden/ from brute force and closed forms.

Every value stored here comes from oracle.brute (enumeration of basic
solutions, the roots of a quadratic, or a linear solve), never from an
interior-point method and never from the GPU library.  Each fixture is an
instance of the standard-form SDP of eq. sdp-pd (Introduction).

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import brute  # noqa: E402


def main():
    out = {"_source": "eq. sdp-pd instances with optima from oracle.brute (enumeration / quadratic roots / linear solve)"}
    lp = []
    for (n, m, seed) in [(4, 2, 0), (5, 2, 1), (6, 3, 2), (6, 2, 3)]:
        q = brute.lp_instance(n, m, seed)
        val, x = brute.lp_optimum(*q["lp_data"])
        lp.append({"n": n, "m": m, "seed": seed, "optimum": val, "x": x.tolist()})
    out["lp_diagonal"] = {"citation": "eq. sdp-pd with diagonal data reduces to an LP on diag(X)", "cases": lp}
    tb = []
    for seed in range(4):
        q = brute.two_by_two_instance(seed)
        val, X = brute.two_by_two_optimum(q)
        tb.append({"seed": seed, "optimum": val, "X": X.tolist()})
    out["two_by_two"] = {"citation": "eq. sdp-pd with n = 2, m = 2: optimum at a root of det X(t) = 0", "cases": tb}
    det = []
    for (n, seed) in [(3, 0), (4, 1)]:
        q = brute.determined_instance(n, seed)
        X = brute.determined_optimum(q)
        det.append({"n": n, "seed": seed, "X": X.tolist(), "optimum": float(np.sum(q["C"] * X))})
    out["determined"] = {"citation": "eq. sdp-pd with m = n(n+1)/2: X = smat(script-A^{-1} b)", "cases": det}
    with open(os.path.join(HERE, "brute_optima.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
