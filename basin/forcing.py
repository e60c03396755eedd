"""Nodal forcing fields, random right-hand sides and request streams (data only).

The wind tensions and bathymetry of the North-Atlantic application (Sec. 6)
are not available, so seeded analytic stand-ins are used:
  * zonal wind stress tau(y) = A cos(pi*y/L + phi) in N/m^2 (A = 0.1, phi = 0
    for the single-step case), converted to the kinematic tension of the
    surface condition of Sec. 2 by theta_1 = tau / rho0, theta_2 = 0;
  * Coriolis parameter f = 2*omega_3 with omega_3 varying from the Equator
    (y = 0) to 70N (y = L): f(y) = 2*Omega*sin(70deg * y / L).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

RHO0 = 1025.0            # reference sea-water density, kg/m^3
OMEGA_EARTH = 7.2921e-5  # Earth's angular velocity, 1/s


def wind_tension(y, L: float, amplitude: float = 0.1, phase: float = 0.0) -> np.ndarray:
    """Kinematic wind tension theta_1 (m^2/s^2) at the given y coordinates."""
    return amplitude * np.cos(np.pi * np.asarray(y, dtype=np.float64) / L + phase) / RHO0


def coriolis_parameter(y, L: float, lat_max_deg: float = 70.0) -> np.ndarray:
    """f = 2*Omega*sin(latitude), latitude linear in y from 0 to lat_max_deg."""
    lat = np.deg2rad(lat_max_deg) * np.asarray(y, dtype=np.float64) / L
    return 2.0 * OMEGA_EARTH * np.sin(lat)


def normal_rhs(n: int, seed: int, zero_mean: bool = False,
               dirichlet: np.ndarray | None = None) -> np.ndarray:
    """iid N(0,1) vector from default_rng(seed), in node order.

    zero_mean subtracts the mean over all n entries; then the entries flagged
    in `dirichlet` (boolean (n,)) are set to zero, in that order.
    """
    b = np.random.default_rng(seed).standard_normal(n)
    if zero_mean:
        b = b - b.mean()
    if dirichlet is not None:
        b = np.where(dirichlet, 0.0, b)
    return b


def random_state(n: int, seed: int, bc: np.ndarray | None = None,
                 velocity_scale: float = 0.1, pressure_scale: float = 1.0):
    """Seeded stand-in for the state (u, p) a time step starts from: u (3, n)
    and p (n,) iid normal from default_rng(seed), drawn in the order u_1, u_2,
    u_3, p and scaled by velocity_scale (m/s) and pressure_scale; u_c is set
    to zero where bit c - 1 of `bc` is set (the component's Dirichlet set)."""
    rng = np.random.default_rng(seed)
    u = velocity_scale * rng.standard_normal((3, n))
    p = pressure_scale * rng.standard_normal(n)
    if bc is not None:
        bc = np.asarray(bc)
        for c in range(3):
            u[c][((bc >> c) & 1) == 1] = 0.0
    return u, p


@dataclass
class WindScenario:
    amplitude: float
    phase: float


def wind_scenarios(count: int = 16, seed: int = 1) -> list[WindScenario]:
    """Wind-forcing scenarios: amplitude ~ U[0.05, 0.2] N/m^2, phase ~ U[0, 2pi)."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.05, 0.2, count)
    phase = rng.uniform(0.0, 2.0 * np.pi, count)
    return [WindScenario(float(a), float(p)) for a, p in zip(amp, phase)]


SERVING_MESHES = ((32, 32, 8), (64, 64, 10), (128, 128, 16), (256, 256, 20), (384, 384, 24))


@dataclass
class SolveRequest:
    index: int
    arrival_s: float
    mesh: tuple           # (Nx, Ny, Nz)
    mesh_index: int
    kind: str             # "poisson" or "helmholtz"
    rhs_seed: int


def serving_requests(count: int = 256, rate_hz: float = 50.0, seed: int = 2,
                     meshes=SERVING_MESHES, poisson_fraction: float = 0.25) -> list[SolveRequest]:
    """Poisson-process arrivals with uniformly drawn mesh sizes and solve kinds.

    Drawn as arrays from default_rng(seed) in the order: inter-arrival gaps
    (exponential, mean 1/rate), mesh index (uniform), kind (Poisson with
    probability poisson_fraction, else Helmholtz for the first velocity
    component).  Request i uses RHS seed 1000 + i.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, count)
    mesh_idx = rng.integers(0, len(meshes), count)
    kind_u = rng.uniform(0.0, 1.0, count)
    t = np.cumsum(gaps)
    return [SolveRequest(index=i, arrival_s=float(t[i]), mesh=tuple(meshes[mesh_idx[i]]),
                         mesh_index=int(mesh_idx[i]),
                         kind="poisson" if kind_u[i] < poisson_fraction else "helmholtz",
                         rhs_seed=1000 + i)
            for i in range(count)]
