"""Write the oracle's solutions of the 256x128 (seed 1) Newton sequence at
sampled entries: tests/golden/newton_256x128_seed1.json.

Calls only the CPU oracle (nested-dissection symbolic + left-looking sparse LU
with threshold partial pivoting, tau = 0.1, and FP64 refinement to omega <=
1e-14) and the seeded input generator.  Takes about 15 minutes on one core.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import splu, sym  # noqa: E402
from vivjac import build_2d, newton_rhs, newton_values  # noqa: E402

NSAMPLE = 2048


def main():
    s = build_2d(256, 128, 1)
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    rng = np.random.default_rng(12345)
    idx = np.sort(np.concatenate([rng.choice(s.n, NSAMPLE, replace=False), s.root]))
    idx = np.unique(idx)
    out = {"mesh": [256, 128], "seed": 1, "n": s.n, "nnz": s.nnz, "sample_rng": 12345,
           "oracle": "oracle.splu.SparseLU(tau=0.1) on the oracle nested-dissection order, refined to 1e-14",
           "index": idx.tolist(), "steps": []}
    for t in range(5):
        v = newton_values(s, t)
        b = newton_rhs(s, t)[0]
        t0 = time.time()
        F = splu.SparseLU(s.n, s.rowptr, s.colind, v, S.perm, tau=0.1)
        x, om, st = F.solve(b, tol=1e-14, max_steps=3)
        print(f"step {t}: {time.time() - t0:.1f}s omega={om[0]:.2e} refinement={st[0]}", flush=True)
        out["steps"].append({"step": t, "x": [float(v_) for v_ in x[idx]], "xinf": float(np.abs(x).max()),
                             "omega": float(om[0])})
    with open(os.path.join(HERE, "newton_256x128_seed1.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
