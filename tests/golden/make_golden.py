"""Write oracle results for the full-size n = 2^20 - 1 workload (the oracle needs minutes
there): per-pass index sets, sizes, ranks, rho and indicator, the singular values, sampled
rows of the factors and Gaussian sketches of the solution. Calls only oracle/ and the seeded
input generators.

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


SKETCH_K = 64
SKETCH_SEEDS = (777, 778)


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
        "rho": [t.rho for t in res.trace],
        "indicator": [t.indicator for t in res.trace],
        "eta1": [t.eta1 for t in res.trace],
        "eta2": [t.eta2 for t in res.trace],
        "S": res.S.tolist(),
        "rows": rows.tolist(),
        "U_rows": res.U[rows].tolist(),
        "V_rows": res.V[rows].tolist(),
    }
    # Gaussian sketches of the solution, A = Om^T U diag(S), B = Om'^T V: a solution W' is
    # compared through ||Om^T (W' - W) Om'||_F / ||Om^T W Om'||_F (Om, Om' regenerated from
    # the seeds by workloads.sketch_matrix)
    for key, mat, sd in (("sketch_U", res.U * res.S[None, :], SKETCH_SEEDS[0]), ("sketch_V", res.V, SKETCH_SEEDS[1])):
        Om = workloads.sketch_matrix(w.n, SKETCH_K, sd)
        out[key] = (Om.T @ mat).tolist()
        del Om
    out["sketch_seeds"] = list(SKETCH_SEEDS)
    out["sketch_k"] = SKETCH_K
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, out["oracle_seconds"])


if __name__ == "__main__":
    main()
