"""Write the oracle's solutions of the 256x128 (seed 1) Newton sequence at
sampled entries: tests/golden/newton_256x128_seed1.json.

Calls only the CPU oracle (nested-dissection symbolic + left-looking sparse LU
with threshold partial pivoting, tau = 0.1, and FP64 refinement to omega <=
1e-14) and the seeded input generator.  Takes about 15 minutes on one core.

Stored per Newton step: the sampled entries, the infinity norm of the whole
solution and of each unknown block (velocity u, pressure p, mesh displacement
d, multiplier lam, position s), so that errors can be judged per block.  The
"eight_rhs" entry holds the same for eight right-hand sides on the step-0
matrix (the first eight rows of the seeded right-hand-side stream).
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
BLOCKS = ("u", "p", "d", "lam", "s")


def block_inf(s, x):
    return {k: float(np.abs(x[s.blocks[k][0]:s.blocks[k][1]]).max()) for k in BLOCKS}


def main():
    s = build_2d(256, 128, 1)
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    rng = np.random.default_rng(12345)
    idx = np.sort(np.concatenate([rng.choice(s.n, NSAMPLE, replace=False), s.root]))
    idx = np.unique(idx)
    out = {"mesh": [256, 128], "seed": 1, "n": s.n, "nnz": s.nnz, "sample_rng": 12345,
           "oracle": "oracle.splu.SparseLU(tau=0.1) on the oracle nested-dissection order, refined to 1e-14",
           "blocks": {k: list(s.blocks[k]) for k in BLOCKS},
           "index": idx.tolist(), "steps": []}
    for t in range(5):
        v = newton_values(s, t)
        nr = 8 if t == 0 else 1
        B = newton_rhs(s, t, nrhs=nr)
        t0 = time.time()
        F = splu.SparseLU(s.n, s.rowptr, s.colind, v, S.perm, tau=0.1)
        X, om, st = F.solve(B, tol=1e-14, max_steps=3)
        X = np.atleast_2d(X)
        print(f"step {t}: {time.time() - t0:.1f}s omega={np.max(om):.2e} refinement={np.max(st)}", flush=True)
        x = X[0]
        out["steps"].append({"step": t, "x": [float(v_) for v_ in x[idx]], "xinf": float(np.abs(x).max()),
                             "block_inf": block_inf(s, x), "omega": float(om[0])})
        if t == 0:
            out["eight_rhs"] = [{"x": [float(v_) for v_ in X[c][idx]], "xinf": float(np.abs(X[c]).max()),
                                 "block_inf": block_inf(s, X[c]), "omega": float(om[c])} for c in range(nr)]
    with open(os.path.join(HERE, "newton_256x128_seed1.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
