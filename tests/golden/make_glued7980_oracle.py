"""Writes glued7980_oracle.json: what the method itself reaches on the
numerically degenerate clusters of the full-size glued Wilkinson workload
(g = 380 copies of W21+, coupling 1e-8, n = 7980), computed by the CPU oracle
alone.

The Peters-Wilkinson cluster at lambda ~ 5.0 (indices 3421..4180, 760
members) holds two groups of 380 eigenvalues that agree to within 9.2e-13
each.  The oracle runs that one cluster (start vectors are keyed by the
global index, so the arithmetic is that of the full run) for three
start-vector seeds and two iteration counts, and records the largest
per-vector residual ||T z - w z||_2 / ||T||_1, the number of vectors above
1e-12, the out-of-cluster residual ||(I - Z Z^T) T Z||_2 / ||T||_1 and the
orthogonality max |Z^T Z - I|.  Six oracle runs of about 40 s each, in
parallel processes.
"""
from __future__ import annotations

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1209_1910_amd import inputs as G  # noqa: E402

IL, IU = 3421, 4180
SEEDS = (O.DEFAULT_SEED, 1, 2)
ITERS = (3, 5)


def one(args):
    seed, iters = args
    d, e = G.workload_glued()
    norm1 = O.setup(d, e).norm1
    W, Z, _ = O.eigvecs(d, e, IL, IU, iters=iters, seed=seed)
    TZ = d[:, None] * Z
    TZ[1:] += e[:, None] * Z[:-1]
    TZ[:-1] += e[:, None] * Z[1:]
    res = np.linalg.norm(TZ - Z * W[None, :], axis=0) / norm1
    out_of_cluster = np.linalg.norm(TZ - Z @ (Z.T @ TZ), 2) / norm1
    orth = float(np.max(np.abs(Z.T @ Z - np.eye(Z.shape[1]))))
    return {"seed": seed, "iterations": iters, "max_residual_rel_norm1": float(res.max()),
            "columns_above_1e-12": int(np.sum(res > 1e-12)),
            "out_of_cluster_residual_rel_norm1": float(out_of_cluster),
            "max_orthogonality": orth}


def main() -> None:
    runs = [(s, k) for k in ITERS for s in SEEDS]
    with ProcessPoolExecutor(max_workers=len(runs)) as ex:
        rows = list(ex.map(one, runs))
    out = {
        "workload": "glued Wilkinson W21+, g = 380, delta = 1e-8, n = 7980; Peters-Wilkinson "
                    f"cluster {IL}..{IU} (lambda ~ 5.0, 760 members, two groups of 380 "
                    "eigenvalues within 9.2e-13 each)",
        "runs": rows,
    }
    with open(os.path.join(HERE, "glued7980_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
