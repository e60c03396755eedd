"""One projection time step on the GPU (Sec. 3 of the paper, implicit-Euler form).

Velocity prediction: (M + dt K_nu) ut_c = M u_c + dt (M_s theta_c + C_c + B_c^T p)
for c = 1..3 with the component's Dirichlet set (three PCG solves); pressure
increment: K_nu q = -(1/dt) sum_c B_c ut_c, pure Neumann (one PCG solve);
correction: p += q, u_c = ut_c - dt (B_c q) / m_L.  Every operation runs in
libhns.so; this class only sequences the calls and holds the device state.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .hns import Operator, SolveInfo


@dataclass
class StepResult:
    velocity: list          # SolveInfo of the three prediction solves
    pressure: SolveInfo     # the pressure-increment solve


class ProjectionStep:
    """Device state (u: 3 x n, p: n) and the two resident operators of a
    shallow-basin mesh.

    theta: (2, n) nodal wind tensions (theta_1, theta_2); f: (n,) Coriolis
    parameter.  Both are host arrays, uploaded once.
    """

    def __init__(self, mesh, nu_h: float, nu_v: float, dt: float, theta, f,
                 device=None, keep_fp32: bool = True, fmt: str = "auto"):
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        with torch.cuda.device(self.device):
            self.helm = Operator(mesh, nu_h, nu_v, dt, kind="helmholtz", keep_fp32=keep_fp32,
                                 step_aux=True, fmt=fmt, device=self.device)
            self.pois = Operator(mesh, nu_h, nu_v, kind="poisson", keep_fp32=keep_fp32, fmt=fmt,
                                 device=self.device)
        self.n = self.helm.n
        dd = dict(dtype=torch.float64, device=self.device)
        self.theta = torch.as_tensor(np.ascontiguousarray(theta, dtype=np.float64), **dd)
        self.f = None if f is None else torch.as_tensor(np.ascontiguousarray(f, np.float64), **dd)
        self.u = torch.zeros(3, self.n, **dd)
        self.p = torch.zeros(self.n, **dd)
        self.ut = torch.zeros(3, self.n, **dd)
        self.q = torch.zeros(self.n, **dd)
        self.b_vel = torch.zeros(3, self.n, **dd)
        self.b_q = torch.zeros(self.n, **dd)

    def state(self):
        return self.u.clone(), self.p.clone()

    def set_state(self, u, p):
        self.u.copy_(u)
        self.p.copy_(p)

    def velocity_rhs(self):
        return self.helm.step_velocity_rhs(self.u, self.p, self.theta, self.f, out=self.b_vel)

    def solve_velocity(self, tol: float, mode: str = "fp64", max_iter: int = 100000):
        infos = []
        for c in range(3):
            self.ut[c].zero_()
            _, info = self.helm.solve(self.b_vel[c], self.ut[c], tol=tol, mask_bit=c, mode=mode,
                                      max_iter=max_iter)
            infos.append(info)
        return infos

    def pressure_rhs(self):
        return self.helm.step_pressure_rhs(self.ut, out=self.b_q)

    def solve_pressure(self, tol: float, mode: str = "fp64", max_iter: int = 100000):
        self.q.zero_()
        _, info = self.pois.solve(self.b_q, self.q, tol=tol, mask_bit=-1, mode=mode,
                                  max_iter=max_iter)
        return info

    def correct(self):
        self.helm.step_correct(self.ut, self.q, self.p, out=self.u)

    def step(self, tol: float = 1e-10, mode: str = "fp64") -> StepResult:
        self.velocity_rhs()
        vel = self.solve_velocity(tol, mode)
        self.pressure_rhs()
        prs = self.solve_pressure(tol, mode)
        self.correct()
        return StepResult(vel, prs)
