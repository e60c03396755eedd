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


class ProjectionLoop:
    """Multi-step projection loop on the GPU (Sec. 3 BDF2 scheme with the weak
    forms of Sec. 5): implicit-Euler first step, BDF2 steps after it, explicit
    advection and Coriolis, consistent-mass velocity correction.

    Step k + 1 with (tau, a1, a2) = (dt, 1, 0) first, then (2 dt/3, 4/3, -1/3):
      prediction  (M + tau K_nu) ut_c = a1 M u^k_c + a2 M u^{k-1}_c
                    + tau (M_s theta_c + C_c(u^k) - N_c(u^k) + B_c^T p^k)
      pressure    K_nu q = -(1/tau) sum_c B_c ut_c  (pure Neumann);  p += q
      correction  M u^{k+1}_c = M ut_c - tau B_c q  (PCG on the mass matrix)
    Four resident operators: M + dt K_nu (with the auxiliary forms and the
    mesh), M + (2 dt/3) K_nu, the pressure operator and M.  The pressure
    operator is the isotropic gradient form of eq. fofa_q_cor_h (pressure_nu =
    (1, 1)) with the vertical-line block preconditioner, solved to
    pressure_tol; the anisotropic K_nu makes the loop unstable on thin
    meshes.  Every operation runs in libhns.so.
    """

    def __init__(self, mesh, nu_h: float, nu_v: float, dt: float, theta, f, advect: bool = True,
                 device=None, fmt: str = "auto", velocity_precond: int = 0,
                 pressure_nu=(1.0, 1.0), pressure_line: bool = True):
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.dt = dt
        self.advect = advect
        with torch.cuda.device(self.device):
            self.helm1 = Operator(mesh, nu_h, nu_v, dt, kind="helmholtz", step_aux=True, fmt=fmt,
                                  device=self.device)
            self.helm2 = Operator(mesh, nu_h, nu_v, 2.0 * dt / 3.0, kind="helmholtz", fmt=fmt,
                                  device=self.device)
            self.pois = Operator(mesh, *pressure_nu, kind="poisson", fmt=fmt, device=self.device)
            self.mass = Operator(mesh, 0.0, 0.0, 0.0, kind="helmholtz", fmt=fmt,
                                 device=self.device)
        if pressure_line:
            self.pois.set_param("precond", 1)
        if velocity_precond:
            for op in (self.helm1, self.helm2):
                op.set_param("precond", velocity_precond)
        self.n = self.helm1.n
        dd = dict(dtype=torch.float64, device=self.device)
        self.theta = None if theta is None else torch.as_tensor(
            np.ascontiguousarray(theta, dtype=np.float64), **dd)
        self.f = None if f is None else torch.as_tensor(np.ascontiguousarray(f, np.float64), **dd)
        self.u = torch.zeros(3, self.n, **dd)
        self.u_prev = torch.zeros(3, self.n, **dd)
        self.p = torch.zeros(self.n, **dd)
        self.ut = torch.zeros(3, self.n, **dd)
        self.q = torch.zeros(self.n, **dd)
        self.adv = torch.zeros(3, self.n, **dd)
        self.b_vel = torch.zeros(3, self.n, **dd)
        self.b_q = torch.zeros(self.n, **dd)
        self.b_corr = torch.zeros(3, self.n, **dd)
        self.k = 0

    def set_state(self, u, p, u_prev=None, k: int = 0):
        self.u.copy_(u)
        self.u_prev.copy_(u if u_prev is None else u_prev)
        self.p.copy_(p)
        self.k = k

    def coefficients(self):
        dt = self.dt
        return (dt, 1.0, 0.0) if self.k == 0 else (2.0 * dt / 3.0, 4.0 / 3.0, -1.0 / 3.0)

    def step(self, tol: float = 1e-10, max_iter: int = 100000, pressure_tol: float | None = None):
        tau, a1, a2 = self.coefficients()
        ptol = tol if pressure_tol is None else pressure_tol
        helm = self.helm1 if self.k == 0 else self.helm2
        aux = self.helm1
        if self.advect:
            aux.step_advection(self.u, out=self.adv)
        aux.step_velocity_rhs_bdf(tau, a1, self.u, a2, self.u_prev if a2 != 0.0 else None,
                                  self.p, self.theta, self.f, self.adv if self.advect else None,
                                  out=self.b_vel)
        vel = []
        for c in range(3):
            self.ut[c].zero_()
            _, info = helm.solve(self.b_vel[c], self.ut[c], tol=tol, mask_bit=c,
                                 max_iter=max_iter)
            vel.append(info)
        aux.step_pressure_rhs_tau(tau, self.ut, out=self.b_q)
        self.q.zero_()
        _, prs = self.pois.solve(self.b_q, self.q, tol=ptol, mask_bit=-1, max_iter=max_iter)
        aux.step_correct_rhs(tau, self.ut, self.q, self.p, out=self.b_corr)
        self.u_prev.copy_(self.u)
        corr = []
        for c in range(3):
            self.u[c].zero_()
            _, info = self.mass.solve(self.b_corr[c], self.u[c], tol=tol, mask_bit=c,
                                      max_iter=max_iter)
            corr.append(info)
        self.k += 1
        return LoopResult(vel, prs, corr)

    def close(self):
        for op in (self.helm1, self.helm2, self.pois, self.mass):
            op.close()


@dataclass
class LoopResult:
    velocity: list          # SolveInfo of the three prediction solves
    pressure: SolveInfo     # the pressure-increment solve
    correction: list        # SolveInfo of the three consistent-mass solves
