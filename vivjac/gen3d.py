"""3D synthetic Jacobian (box of Kuhn-split hexahedra); filled in with the serving workload."""


def build_3d(*args, **kwargs):
    raise NotImplementedError("3D generator not built yet")
