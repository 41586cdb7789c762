"""Seeded synthetic inputs shared by the oracle and the GPU path.

Geometry, labels, permittivity maps, source points, port descriptions and the
non-overlapping partition.  Holds none of the method's arithmetic.
"""
from . import configs, fields, mesh, partition, serving  # noqa: F401
from .mesh import TAG_IMPEDANCE, TAG_PEC, Mesh, PortSpec  # noqa: F401
