"""Newton-step solves with a factorization kept across steps as the preconditioner.

Each Newton iteration of the paper (Sec. 3.4, eq. NR_iteration) solves a system
with the same pattern and new values.  The paper factors every Jacobian with a
direct solver (Sec. 4.3) and names preconditioned Krylov iterations as its next
step (Sec. 4.3, Sec. 7).  ``ReusedFactorNewton`` is that iterative solver with a
multifrontal preconditioner: one reduced-precision factorization serves several
steps (mf_set_operator: the new Jacobian is the operator of FP64 GMRES-IR, the
old factors its preconditioner), and it is refreshed when reusing it costs more
than factoring again.

Policy (host control only; every step runs in the library):
  * the first step, and any step after a refresh was called for, factors its own
    values in ``prec`` and solves with the library's default refinement for that
    precision (classical FP64 steps while they converge fast, then GMRES-IR; FP64
    fallback enabled);
  * every other step replaces the operator and solves with the kept factors, with
    at most ``reuse_m`` x ``reuse_outer`` GMRES iterations per right-hand side and
    no fallback;
  * a reuse that converges but needs more than ``max_inner`` iterations per
    right-hand side calls for a refresh at the next step;
  * a reuse that does not converge within its cap is discarded, the step is
    factored and solved afresh, and reuse is skipped for the next 1, 2, 4, ...
    steps while failures repeat (reset by a successful reuse).
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass
class StepRecord:
    refactored: bool        # this step factored its own values
    retried: bool           # a reuse failed to converge and the step was factored afresh
    omega: float
    outer_iters: int
    inner_iters: int        # GMRES iterations, summed over right-hand sides (including a failed reuse)


class ReusedFactorNewton:
    def __init__(self, sym, prec="fp32", target_omega=1e-10, max_inner=10, reuse_m=20, reuse_outer=1,
                 stream=None, **factor_opts):
        self.sym = sym
        self.target = target_omega
        self.opts = dict(prec=prec, target_omega=target_omega, **factor_opts)
        self.reuse = dict(target_omega=target_omega, gmres_m=reuse_m, max_outer=reuse_outer, fallback=0)
        self.max_inner = max_inner
        self.stream = stream
        self.num = None
        self.refresh = True
        self.skip = 0           # steps left without a reuse attempt
        self.backoff = 1
        self.history: list[StepRecord] = []

    def _fresh(self, values, b, x):
        self.num = self.sym.factor(values, numeric=self.num, stream=self.stream, **self.opts)
        return self.num.solve(b, x=x, stream=self.stream)

    def step(self, values, b, x=None):
        """Solve J(values) x = b; returns (x, mf_solve_info, StepRecord)."""
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        spent = 0
        retried = False
        if self.refresh or self.num is None or self.skip > 0:
            self.skip = max(0, self.skip - 1)
            x, info = self._fresh(values, b, x)
            refactored = True
        else:
            self.num.set_operator(values, stream=self.stream, **self.reuse)
            x, info = self.num.solve(b, x=x, stream=self.stream, check=False)  # errors still raise
            refactored = False
            if not info.omega <= self.target:
                spent = info.inner_iters
                x, info = self._fresh(values, b, x)
                refactored = retried = True
                self.skip = self.backoff
                self.backoff *= 2
            else:
                self.backoff = 1
        self.refresh = (not refactored) and info.inner_iters > self.max_inner * nrhs
        rec = StepRecord(refactored, retried, info.omega, info.outer_iters, info.inner_iters + spent)
        self.history.append(rec)
        return x, info, rec

    def release(self):
        if self.num is not None:
            self.num.release()
            self.num = None
