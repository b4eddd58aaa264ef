"""Write the oracle's solution of the 3D box Jacobian (24x12x6 hexahedra, seed 3,
n = 84,825) at sampled entries: tests/golden/box_24x12x6_seed3.json.

Calls only the CPU oracle (nested-dissection symbolic + left-looking sparse LU
with threshold partial pivoting, tau = 0.1, FP64 refinement to omega <= 1e-14)
and the seeded input generator.  Stored: the sampled entries (2,048 random plus
the two position unknowns), the infinity norm of the whole solution and of each
unknown block.  Takes several minutes on one core.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import splu, sym  # noqa: E402
from vivjac import build_3d, newton_rhs, newton_values  # noqa: E402

BLOCKS = ("u", "p", "d", "lam", "s")


def main():
    s = build_3d(24, 12, 6, 3)
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    rng = np.random.default_rng(54321)
    idx = np.unique(np.sort(np.concatenate([rng.choice(s.n, 2048, replace=False), s.root])))
    v = newton_values(s, 0)
    b = newton_rhs(s, 0)[0]
    t0 = time.time()
    F = splu.SparseLU(s.n, s.rowptr, s.colind, v, S.perm, tau=0.1)
    x, om, st = F.solve(b, tol=1e-14, max_steps=3)
    print(f"oracle: {time.time() - t0:.1f}s omega={om[0]:.2e} refinement={st[0]}", flush=True)
    out = {"mesh": [24, 12, 6], "seed": 3, "n": s.n, "nnz": s.nnz, "sample_rng": 54321,
           "oracle": "oracle.splu.SparseLU(tau=0.1) on the oracle nested-dissection order, refined to 1e-14",
           "blocks": {k: list(s.blocks[k]) for k in BLOCKS}, "index": idx.tolist(),
           "x": [float(t) for t in x[idx]], "xinf": float(np.abs(x).max()),
           "block_inf": {k: float(np.abs(x[s.blocks[k][0]:s.blocks[k][1]]).max()) for k in BLOCKS},
           "omega": float(om[0])}
    with open(os.path.join(HERE, "box_24x12x6_seed3.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
