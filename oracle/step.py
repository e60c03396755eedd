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
a plus sign, which contradicts them.  Advection is left out.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import (OK, divergence, helmholtz, mass, pcg, stiffness, surface_mass)


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
