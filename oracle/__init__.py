"""CPU oracle for the multifrontal Newton-Jacobian solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library or its Python binding
imports, links or runs anything from this package; only the tests, the smoke
entry point and the benchmark's CPU-baseline leg do.  It shares no code with
the GPU path: the only common module is the seeded input generator ``vivjac``,
which holds none of the solver's arithmetic.

Parts:

* ``oracle.sym``   -- the specified symbolic analysis (nested dissection with
  George-Liu pseudo-peripheral roots, front tree, front rows, elimination tree),
  written independently of the library's C++ implementation so that the two
  can be compared bit for bit.
* ``oracle.splu``  -- plain left-looking sparse LU with partial pivoting
  (Gilbert-Peierls) plus fixed-precision FP64 iterative refinement, in plain C
  (``splu.c``) behind ctypes.  It solves the Newton system J dU = -NL(U) of the
  paper's Newton-Raphson iteration (eq. NR_iteration), the linear problem the
  paper hands to its direct solver (Sec. 4.3).
* ``oracle.check`` -- independent checks used to pin the above: dense LU with
  partial pivoting, exact rational elimination, backward-error measures.
* ``oracle.ale``   -- the full ALE Newton residual NL(U) of the paper (Sec.
  3.1-3.2) on the 2D construction and its Jacobian by complex-step
  differentiation of each element's residual (shape-derivative blocks
  included), for the GPU element assembly.
"""
