"""Seeded synthetic inputs for the shallow-basin solves.

This package produces *data only*: terrain-following tetrahedral (and
hexahedral Q1/Q2) meshes of the
shallow domain of Sec. 2 (surface Gamma_s, depth h, bottom Gamma_b), Dirichlet
node masks for the boundary parts Gamma_0 / Gamma_1 / Gamma_s, nodal forcing
fields (wind tension, Coriolis parameter), random right-hand sides and the
serving workload's arrival stream.  It holds none of the finite element or
solver arithmetic; both the HIP library path and the CPU oracle consume these
arrays as inputs and derive everything else themselves.
"""
from .mesh import (BasinMesh, box_mesh, basin_mesh, bathymetry, node_index,
                   BC_U1, BC_U2, BC_U3, dirichlet_bits,
                   HexMesh, box_hex_mesh, basin_hex_mesh)
from .forcing import (wind_tension, coriolis_parameter, normal_rhs, random_state,
                      wind_scenarios, serving_requests, RHO0, OMEGA_EARTH)
from . import configs

__all__ = [
    "BasinMesh", "box_mesh", "basin_mesh", "bathymetry", "node_index",
    "BC_U1", "BC_U2", "BC_U3", "dirichlet_bits",
    "HexMesh", "box_hex_mesh", "basin_hex_mesh",
    "wind_tension", "coriolis_parameter", "normal_rhs", "random_state", "wind_scenarios",
    "serving_requests", "RHO0", "OMEGA_EARTH", "configs",
]
