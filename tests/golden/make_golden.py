"""Write oracle results for the full-size n = 2^20 - 1 workload (the oracle needs minutes
there). Calls only oracle/ and the seeded input generators.

    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import crossdeim as cd  # noqa: E402


def main(name="n1048575_r30_fp64", seed=0, nrows=200):
    w = workloads.CONFIGS[name]
    U, s, V = workloads.make(w, seed)
    t0 = time.time()
    res = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    rng = np.random.default_rng(12345)
    rows = np.unique(np.concatenate([np.linspace(0, w.n - 1, nrows // 2).astype(np.int64),
                                     rng.integers(0, w.n, nrows // 2)]))
    out = {
        "workload": name,
        "seed": seed,
        "oracle_seconds": time.time() - t0,
        "status": res.status,
        "iters": res.iters,
        "rank": res.rank,
        "I_pre": [t.I_pre for t in res.trace],
        "J_pre": [t.J_pre for t in res.trace],
        "nI": [len(t.I) for t in res.trace],
        "nJ": [len(t.J) for t in res.trace],
        "ranks": [t.rank for t in res.trace],
        "gapI": [t.gapI for t in res.trace],
        "gapJ": [t.gapJ for t in res.trace],
        "S": res.S.tolist(),
        "rows": rows.tolist(),
        "U_rows": res.U[rows].tolist(),
        "V_rows": res.V[rows].tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, out["oracle_seconds"])


if __name__ == "__main__":
    main()
