"""Seeded synthetic Newton Jacobians shaped like the paper's monolithic VIV system.

This package is *input generation only*: it assembles the linearised coupled
Jacobian (P2-P1 Oseen flow, P2 pseudo-solid mesh block, P2 Lagrange multiplier
on the cylinder boundary, two rigid-position dofs and the spring term) on
structured meshes, and draws the random right-hand sides and Newton-step value
perturbations.  It holds none of the solver's arithmetic (no factorization, no
triangular solves, no residuals): both the solver under test and the CPU oracle
consume its output.

Block structure follows the Jacobian of Sec. 3.2 (zero pressure and multiplier
diagonal blocks), the multiplier weak form of Sec. 3.1 (eq. weak_system), the
force-position coupling of Sec. 4.2 (eq. coupling_constraint) in its single
global-master form, and the spring balance of Sec. 2 (eq. solid_balance).
"""
from .gen2d import System, build_2d, newton_values, newton_rhs
from .gen3d import build_3d, p2_tet
from .parts import build_mesh, value_parts

__all__ = ["System", "build_2d", "build_3d", "build_mesh", "value_parts", "newton_values", "newton_rhs"]
