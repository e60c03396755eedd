"""CPU oracle of one projection time step.  TEST INFRASTRUCTURE ONLY.

Implicit-Euler form of the velocity-correction projection step of Sec. 3
(weak forms of Sec. 4, discretised in Sec. 5), written out with the oracle's
own assembled matrices and its own PCG:

  prediction  (M + dt K_nu) ut_c = M u_c + dt (M_s theta_c + C_c + B_c^T p),
              C_1 = M (f u_2), C_2 = -M (f u_1), C_3 = 0, theta_3 = 0,
              ut_c = 0 on the Dirichlet set of component c;
  pressure    K_nu q = -(1/dt) sum_c B_c ut_c, pure Neumann, zero mass-mean;
  correction  p <- p + q,  u_c = ut_c - dt (B_c q) / m_L  (m_L = M 1),
              zero on the Dirichlet set of component c.

The sign of the correction follows the correction equations of Sec. 3
(u - ut = -(dt) grad q); the paper's closing formula of that section prints
a plus sign, which contradicts them.  Advection is left out of this one-step
form; OracleLoop below is the multi-step BDF2 loop with explicit advection
and the consistent-mass velocity correction.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import (OK, advection, divergence, helmholtz, mass, pcg, stiffness, surface_mass)


@dataclass
class OracleStep:
    mesh: object
    nu_h: float
    nu_v: float
    dt: float

    def __post_init__(self):
        m = self.mesh
        self.A = helmholtz(m, self.nu_h, self.nu_v, self.dt)
        self.K = stiffness(m, self.nu_h, self.nu_v)
        self.M = mass(m)
        self.B = [divergence(m, c) for c in range(3)]
        self.Ms = surface_mass(m)
        self.mL = self.M.matvec(np.ones(m.n))
        self.dirichlet = [((m.bc >> c) & 1) == 1 for c in range(3)]

    def velocity_rhs(self, u, p, theta, f):
        n, dt = self.mesh.n, self.dt
        b = np.zeros((3, n))
        for c in range(3):
            b[c] = self.M.matvec(u[c])
            if theta is not None and c < 2:
                b[c] += dt * self.Ms.matvec(theta[c])
            if p is not None:
                b[c] += dt * self.B[c].rmatvec(p, n)
            if f is not None and c < 2:
                other = u[1] if c == 0 else u[0]
                sign = 1.0 if c == 0 else -1.0
                b[c] += sign * dt * self.M.matvec(f * other)
            b[c][self.dirichlet[c]] = 0.0
        return b

    def pressure_rhs(self, ut):
        return -(1.0 / self.dt) * sum(self.B[c].matvec(ut[c]) for c in range(3))

    def correct(self, ut, q, p):
        u = np.zeros_like(ut)
        for c in range(3):
            u[c] = ut[c] - self.dt * self.B[c].matvec(q) / self.mL
            u[c][self.dirichlet[c]] = 0.0
        return u, (None if p is None else p + q)

    def step(self, u, p, theta, f, tol=1e-10):
        b = self.velocity_rhs(u, p, theta, f)
        ut = np.zeros_like(b)
        vel = []
        for c in range(3):
            r = pcg(self.A, b[c], dirichlet=self.dirichlet[c], tol=tol)
            assert r.status == OK, r.status
            ut[c] = r.x
            vel.append(r)
        bq = self.pressure_rhs(ut)
        rq = pcg(self.K, bq, singular=True, weights=self.mL, tol=tol)
        assert rq.status == OK, rq.status
        u_new, p_new = self.correct(ut, rq.x, p)
        return dict(b_vel=b, ut=ut, b_q=bq, q=rq.x, u=u_new, p=p_new, vel=vel, pres=rq)


@dataclass
class OracleLoop:
    """Multi-step projection loop: the BDF2 scheme of Sec. 3 with the weak
    forms of Sec. 4/5, written out with the oracle's matrices and PCG.

    Step k + 1 (tau = 2 dt / 3, a1 = 4/3, a2 = -1/3; the first step, which the
    paper leaves open, is implicit Euler: tau = dt, a1 = 1, a2 = 0):
      prediction  (M + tau K_nu) ut_c = a1 M u^k_c + a2 M u^{k-1}_c
                    + tau (M_s theta_c + C_c(u^k) - N_c(u^k) + B_c^T p^k),
                  C_1 = M (f u_2), C_2 = -M (f u_1), C_3 = 0 (explicit Coriolis),
                  N_c(u) = int ((u . grad) u_c) phi (explicit advection),
                  ut_c = 0 on the Dirichlet set of component c;
      pressure    K_nu q = -(1/tau) sum_c B_c ut_c, pure Neumann, zero mass-mean;
                  p^{k+1} = p^k + q (eq. fofa_pres_cor_h: the same space);
      correction  M u^{k+1}_c = M ut_c - tau B_c q (eq. fofa_velo_cor_h with the
                  minus sign of the correction equations), solved by PCG on the
                  consistent mass matrix with the Dirichlet set of component c.
    The multiplication of the BDF2 equations by 2 dt / 3 turns the operator
    3/(2dt) M + K_nu into M + tau K_nu.

    The pressure operator is the isotropic gradient form of eq. fofa_q_cor_h
    (pressure_nu = (1, 1)) solved with the vertical-line block preconditioner
    at tolerance pressure_tol (default: the step tolerance); with the
    anisotropic K_nu in its place the loop is unstable on the basin meshes
    (the vertical velocity grows about a hundredfold per step).
    """
    mesh: object
    nu_h: float
    nu_v: float
    dt: float
    advect: bool = True
    pressure_nu: tuple = (1.0, 1.0)
    pressure_line: bool = True
    pressure_tol: float | None = None

    def __post_init__(self):
        m = self.mesh
        self.taus = (self.dt, 2.0 * self.dt / 3.0)
        self.A = [helmholtz(m, self.nu_h, self.nu_v, t) for t in self.taus]
        self.K = stiffness(m, *self.pressure_nu)
        self.M = mass(m)
        self.B = [divergence(m, c) for c in range(3)]
        self.Ms = surface_mass(m)
        self.mL = self.M.matvec(np.ones(m.n))
        self.dirichlet = [((m.bc >> c) & 1) == 1 for c in range(3)]

    @staticmethod
    def coefficients(first: bool, dt: float):
        return (dt, 1.0, 0.0) if first else (2.0 * dt / 3.0, 4.0 / 3.0, -1.0 / 3.0)

    def velocity_rhs(self, tau, a1, u, a2, u_prev, p, theta, f):
        n = self.mesh.n
        adv = advection(self.mesh, u) if self.advect else None
        b = np.zeros((3, n))
        for c in range(3):
            b[c] = a1 * self.M.matvec(u[c])
            if a2 != 0.0:
                b[c] += a2 * self.M.matvec(u_prev[c])
            force = np.zeros(n)
            if theta is not None and c < 2:
                force += self.Ms.matvec(theta[c])
            if f is not None and c < 2:
                other = u[1] if c == 0 else u[0]
                force += (1.0 if c == 0 else -1.0) * self.M.matvec(f * other)
            if adv is not None:
                force -= adv[c]
            if p is not None:
                force += self.B[c].rmatvec(p, n)
            b[c] += tau * force
            b[c][self.dirichlet[c]] = 0.0
        return b

    def step(self, u, u_prev, p, theta, f, first, tol=1e-10, project=True):
        tau, a1, a2 = self.coefficients(first, self.dt)
        A = self.A[0 if first else 1]
        b = self.velocity_rhs(tau, a1, u, a2, u_prev, p, theta, f)
        ut = np.zeros_like(b)
        for c in range(3):
            r = pcg(A, b[c], dirichlet=self.dirichlet[c], tol=tol)
            assert r.status == OK, r.status
            ut[c] = r.x
        if not project:
            return dict(b_vel=b, ut=ut, u=ut.copy(), p=p)
        bq = -(1.0 / tau) * sum(self.B[c].matvec(ut[c]) for c in range(3))
        ptol = tol if self.pressure_tol is None else self.pressure_tol
        rq = pcg(self.K, bq, singular=True, weights=self.mL, tol=ptol,
                 line=(self.mesh.Nz + 1) if self.pressure_line else 0)
        assert rq.status == OK, rq.status
        p_new = (np.zeros(self.mesh.n) if p is None else p) + rq.x
        rhs = np.zeros_like(ut)
        u_new = np.zeros_like(ut)
        for c in range(3):
            rhs[c] = self.M.matvec(ut[c]) - tau * self.B[c].matvec(rq.x)
            rhs[c][self.dirichlet[c]] = 0.0
            r = pcg(self.M, rhs[c], dirichlet=self.dirichlet[c], tol=tol)
            assert r.status == OK, r.status
            u_new[c] = r.x
        return dict(b_vel=b, ut=ut, b_q=bq, q=rq.x, rhs_corr=rhs, u=u_new, p=p_new)

    def run(self, steps, u0, p0, theta, f, tol=1e-10, project=True):
        """States after each of `steps` steps from (u0, p0); u^{-1} = u0."""
        u, u_prev, p = u0.copy(), u0.copy(), p0.copy()
        out = []
        for k in range(steps):
            r = self.step(u, u_prev, p, theta, f, first=(k == 0), tol=tol, project=project)
            u_prev, u, p = u, r["u"], r["p"]
            out.append(r)
        return out
