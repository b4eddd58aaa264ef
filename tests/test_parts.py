"""The value parts of one mesh (base + nu * visc + k * spring) reproduce a direct
assembly at any nu and k, on the same pattern, in 2D and 3D."""
import numpy as np
import pytest

from vivjac import build_mesh, value_parts


@pytest.mark.parametrize("mesh", [("2d", 16, 8), ("2d", 20, 10), ("3d", 4, 4, 1)])
def test_value_parts_match_direct_assembly(mesh):
    s0, base, visc, spring = value_parts(mesh, 7)
    assert spring.sum() == 2.0                       # the two position diagonals
    for nu, k in [(0.01, 0.5), (1 / 137.0, 3.3)]:
        ref = build_mesh(mesh, 7, nu, k)
        assert np.array_equal(ref.rowptr, s0.rowptr) and np.array_equal(ref.colind, s0.colind)
        got = base + nu * visc + k * spring
        assert np.abs(got - ref.values).max() <= 1e-14 * np.abs(ref.values).max()
        # the spring entries carry k exactly
        assert np.array_equal(got[spring != 0], ref.values[spring != 0])
