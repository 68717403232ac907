"""Write medium_backtracking_500.json: the FP64 oracle's run of backtracking
FISTA on the n = 1,000,000, c = 32 workload (ER degree 30, about 3e7 stored
nonzeros, 32 overlapping planted communities, sigma 0.05, seed 0), the values
the GPU replay test compares against.

Alg. 4 with the FISTA backtracking rule the paper cites for it (L0 = 1e4,
eta = 2), 500 iterations, unit diagonal (S + I).  Stored: a fingerprint of the
seeded instance (so a changed generator is caught instead of compared), the
accepted steps tau_n, the trials per iteration, the losses f(Xbar_0..500), the
gradient-mapping norms, and Xbar_500 at 256 seeded sample rows.

Only oracle/ and workloads/ are used.  Run from the repository root:
    python tests/golden/make_medium_replay.py
(about ten minutes on eight cores).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "medium_backtracking_500.json")
ITERS = 500
L0 = 1.0e4
SAMPLE = 256


def fingerprint(rp, ci, v, U0) -> dict:
    """Size and content hashes of the seeded instance."""
    h = hashlib.sha256()
    for a in (rp, ci, v.astype(np.float32), U0.astype(np.float32)):
        h.update(np.ascontiguousarray(a).tobytes())
    return {"n": int(rp.size - 1), "nnz": int(ci.size), "sha256": h.hexdigest(),
            "val_sum": float(v.sum()), "u0_sum": float(U0.sum())}


def sample_rows(n: int) -> np.ndarray:
    return np.sort(np.random.default_rng(2024).choice(n, SAMPLE, replace=False))


def main() -> None:
    wl = W.config_medium(seed=0)
    rp, ci, v, U0 = wl.numpy()
    t0 = time.time()
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=ITERS, backtrack=True,
                       L0=L0)
    secs = time.time() - t0
    assert ref.iters == ITERS
    rows = sample_rows(wl.n)
    doc = {
        "what": "FP64 oracle, backtracking FISTA (Alg. 4), n=1e6, c=32, ER degree 30, seed 0",
        "made_by": "tests/golden/make_medium_replay.py",
        "instance": fingerprint(rp, ci, v, U0),
        "iters": ITERS, "L0": L0, "eta": 2.0, "diag_unit": True,
        "tau": [float(x) for x in ref.tau[1:]],
        "trials": [int(x) for x in ref.trials[1:]],
        "f": [float(x) for x in ref.f],
        "r": [float(x) for x in ref.r[1:]],
        "rows": [int(i) for i in rows],
        "X_rows": [[float(x) for x in ref.X[i]] for i in rows],
        "row_sum_err_max": float(np.abs(ref.X.sum(1) - 1.0).max()),
        "oracle_seconds": secs, "oracle_threads": oracle.num_threads(),
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=0)
        fh.write("\n")
    print(f"wrote {OUT}: {ITERS} iterations, {int(ref.trials[1:].sum())} trials, "
          f"f {ref.f[0]:.10e} -> {ref.f[-1]:.10e}, {secs:.0f} s")


if __name__ == "__main__":
    main()
