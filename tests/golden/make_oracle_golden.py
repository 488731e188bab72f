"""Write tests/golden/oracle_config1.json: the oracle's solution summary for the
dense Gaussian sensing workload n=200, r=3, m=2400 (seed 1).

Only oracle/ and workloads/ are called.  The GPU tests compare the library's
objective against the stored primal and dual objectives and its X against
the stored leading eigenpairs, without rerunning the minutes-long oracle.

Run:  python tests/golden/make_oracle_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle import certify, ipm  # noqa: E402


def main():
    p = workloads.config(1)
    t = time.time()
    res = ipm.solve(p)
    el = time.time() - t
    cert = certify.certificate(p, res["X"], res["y"], res["S"])
    w, V = np.linalg.eigh(res["X"])
    top = np.argsort(w)[::-1][:6]
    Xs = p["U"] @ p["U"].T
    out = {
        "workload": "gaussian sensing n=200 r=3 m=2400 seed=1",
        "status": res["status"],
        "iterations": res["iterations"],
        "seconds": el,
        "certificate": cert,
        "recovery_rel_err": float(np.linalg.norm(res["X"] - Xs) / np.linalg.norm(Xs)),
        "X_top_eigenvalues": w[top].tolist(),
        "X_top_eigenvectors": V[:, top[:3]].T.tolist(),
        "history": res["history"],
    }
    with open(os.path.join(HERE, "oracle_config1.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
