"""One mesh's Jacobian split into parts that are linear in the viscosity and the
spring stiffness.

Both generators assemble the viscous term as nu times a nu-free matrix and the
spring term as k on the two position diagonals (Sec. 3.2, Sec. 2 eq.
solid_balance), and every other block is independent of nu and k.  The values of
the request (mesh, seed, nu, k) are therefore exactly

    values = base + nu * visc + k * spring

on one fixed pattern, up to the rounding of the two-build difference that
defines ``visc``.  A request stream over a few meshes (the serving workload)
then needs two assemblies per mesh, not one per request.
"""
from __future__ import annotations

import numpy as np

from .gen2d import build_2d
from .gen3d import build_3d


def build_mesh(mesh, seed, nu, k):
    """Assemble ("2d", nx, ny) or ("3d", nx, ny, nz) at the given nu and k."""
    if mesh[0] == "2d":
        return build_2d(int(mesh[1]), int(mesh[2]), seed, nu=nu, k=k)
    if mesh[0] == "3d":
        return build_3d(int(mesh[1]), int(mesh[2]), int(mesh[3]), seed, nu=nu, k=k)
    raise ValueError(f"unknown mesh kind {mesh[0]!r}")


def value_parts(mesh, seed):
    """(system at nu = k = 0, base, visc, spring): float64[nnz] each on the
    system's pattern, with values(nu, k) = base + nu * visc + k * spring."""
    s0 = build_mesh(mesh, seed, 0.0, 0.0)
    s1 = build_mesh(mesh, seed, 1.0, 1.0)
    if not (np.array_equal(s0.rowptr, s1.rowptr) and np.array_equal(s0.colind, s1.colind)):
        raise AssertionError("the pattern must not depend on nu or k")
    spring = np.zeros(s0.nnz)
    for r in s0.root:                     # the (s_c, s_c) entries hold k alone
        lo, hi = int(s0.rowptr[r]), int(s0.rowptr[r + 1])
        spring[lo + int(np.flatnonzero(s0.colind[lo:hi] == r)[0])] = 1.0
    visc = s1.values - s0.values
    visc[spring != 0] = 0.0
    return s0, s0.values.copy(), visc, spring
