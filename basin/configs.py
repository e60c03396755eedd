"""The five benchmark workloads as explicit, seeded parameter sets.

Each entry states the mesh, viscosities, time step, tolerance and seeds; the
functions in `basin.mesh` / `basin.forcing` turn them into arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .mesh import box_mesh, basin_mesh, WALLS
from .forcing import SERVING_MESHES


@dataclass(frozen=True)
class Workload:
    name: str
    Nx: int
    Ny: int
    Nz: int
    nu_h: float
    nu_v: float
    dt: float
    tol: float
    seed: int = 0
    box: bool = False       # unit box of depth H (True) or Gaussian-bump basin
    H: float = 0.01
    L: float = 5.0e6
    extra: dict = field(default_factory=dict)

    def mesh(self):
        if self.box:
            return box_mesh(self.Nx, self.Ny, self.Nz, 1.0, 1.0, self.H, gamma0=WALLS, gamma1=())
        return basin_mesh(self.Nx, self.Ny, self.Nz, self.L, self.seed)


# Plain method, small: anisotropic Laplacian on the unit box of depth 0.01,
# Dirichlet on all of Gamma_b (bottom + walls), Neumann on the surface,
# RHS N(0,1) from seed 0, projected to zero mean, FP64 Jacobi-PCG to 1e-10.
BOX_16x16x4 = Workload("box16x16x4", 16, 16, 4, nu_h=1.0, nu_v=1e-4, dt=1.0,
                       tol=1e-10, seed=0, box=True, H=0.01)

# Atlantic-shaped basin, one projection step with dt = 3600 s, FP64, 1e-10.
BASIN_256x256x20 = Workload("basin256x256x20", 256, 256, 20, nu_h=1e3, nu_v=1e-2,
                            dt=3600.0, tol=1e-10, seed=0)

# Mixed precision on the same operators (same tolerance).
BASIN_256x256x20_MIXED = Workload("basin256x256x20-mixed", 256, 256, 20, nu_h=1e3,
                                  nu_v=1e-2, dt=3600.0, tol=1e-10, seed=0)

# The paper's isotropic pressure operator (nu = 1 in every direction) on the
# same basin, solved with the vertical-line block preconditioner.  Its
# couplings spread over ~8 decades (horizontal cells of 19.5 km, layers of
# 10-275 m), so the FP64 Euclidean residual stalls near 2e-10: tolerance 1e-9.
BASIN_256x256x20_ISO = Workload("basin256x256x20-isotropic", 256, 256, 20, nu_h=1.0,
                                nu_v=1.0, dt=3600.0, tol=1e-9, seed=0)

# Multi-RHS: 3 velocity components x 16 wind scenarios on one 128x128x20 basin.
BASIN_128x128x20_BATCH = Workload("basin128x128x20-batch48", 128, 128, 20, nu_h=1e3,
                                  nu_v=1e-2, dt=3600.0, tol=1e-10, seed=0,
                                  extra={"scenarios": 16, "scenario_seed": 1})

# Serving: 256 requests at 50 req/s over five mesh sizes, tolerance 1e-8.
SERVING = Workload("serving256", 0, 0, 0, nu_h=1e3, nu_v=1e-2, dt=3600.0, tol=1e-8,
                   seed=2, extra={"requests": 256, "rate_hz": 50.0,
                                  "meshes": SERVING_MESHES, "bathymetry_seed_base": 100})

ALL = (BOX_16x16x4, BASIN_256x256x20, BASIN_256x256x20_MIXED, BASIN_128x128x20_BATCH, SERVING)


def serving_mesh(mesh_index: int):
    Nx, Ny, Nz = SERVING_MESHES[mesh_index]
    return basin_mesh(Nx, Ny, Nz, 5.0e6, seed=100 + mesh_index)
