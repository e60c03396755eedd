"""Pins of the oracle's multi-step projection loop: the advection form, the
BDF2 time discretisation and its consistency with the pinned one-step form."""
import numpy as np
import pytest
import scipy.linalg as sl

import basin
import oracle
from oracle.step import OracleLoop, OracleStep


def test_advection_is_exact_for_linear_fields():
    """For a linear velocity u = A x + c, (u . grad) u_c = sum_d u_d A_cd is
    linear, so the P1 form equals the mass matrix applied to its nodal values."""
    m = basin.basin_mesh(6, 5, 3, seed=1)
    A = np.array([[1e-6, 2e-6, 3e-3], [-2e-6, 5e-7, 1e-3], [4e-7, -1e-6, 2e-3]])
    c0 = np.array([0.1, -0.2, 0.05])
    u = A @ m.xyz.T + c0[:, None]
    N = oracle.advection(m, u)
    M = oracle.mass(m)
    want = np.stack([M.matvec(sum(u[d] * A[c, d] for d in range(3))) for c in range(3)])
    assert np.abs(N - want).max() <= 1e-13 * np.abs(want).max()


def test_advection_is_quadratic_and_bilinear():
    """N(s u) = s^2 N(u); N is the diagonal of the bilinear form
    N(w, v)_c = int ((w . grad) v_c) phi, linear in the advected field."""
    m = basin.box_mesh(4, 3, 2)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((3, m.n))
    N = oracle.advection(m, u)
    scale = np.abs(N).max()
    assert np.abs(oracle.advection(m, 3.0 * u) - 9.0 * N).max() <= 1e-13 * scale
    # polarisation: N(u + v) + N(u - v) = 2 N(u) + 2 N(v)
    v = rng.standard_normal((3, m.n))
    lhs = oracle.advection(m, u + v) + oracle.advection(m, u - v)
    rhs = 2 * N + 2 * oracle.advection(m, v)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def _free_exact(m, loop, u0, F, T, c, d):
    """u(T) of M u' = -K_nu u + F on the free nodes of component c."""
    Mf = loop.M.to_scipy().toarray()[np.ix_(~d, ~d)]
    Kf = loop.K.to_scipy().toarray()[np.ix_(~d, ~d)]
    uinf = np.linalg.solve(Kf, F[~d])
    E = sl.expm(-np.linalg.solve(Mf, Kf) * T)
    out = np.zeros(m.n)
    out[~d] = uinf + E @ (u0[~d] - uinf)
    return out


def _run_prediction(loop, m, u0, theta, steps, bdf1_only):
    u, u_prev = u0.copy(), u0.copy()
    for k in range(steps):
        r = loop.step(u, u_prev, None, theta, None, first=(k == 0 or bdf1_only), tol=1e-14,
                      project=False)
        u_prev, u = u, r["u"]
    return u


def test_bdf2_prediction_is_second_order_in_time():
    """Without the projection the prediction is BDF2 for M u' = -K_nu u + M_s theta
    (implicit Euler first step): the error at a fixed time falls 4x per halving
    of dt, against 2x for implicit Euler at every step."""
    m = basin.box_mesh(3, 3, 2, H=0.1)
    T = 0.02
    d = (m.bc & 1) == 1
    rng = np.random.default_rng(5)
    u0 = np.zeros((3, m.n))
    u0[0] = rng.standard_normal(m.n)
    u0[0][d] = 0.0
    theta = np.stack([np.full(m.n, 0.3), np.zeros(m.n)])
    errs = {False: [], True: []}
    exact = None
    for steps in (64, 128, 256):
        loop = OracleLoop(m, 1.0, 1.0, T / steps, advect=False)
        if exact is None:
            F = loop.Ms.matvec(theta[0])
            exact = _free_exact(m, loop, u0[0], F, T, 0, d)
        for bdf1 in (False, True):
            u = _run_prediction(loop, m, u0, theta, steps, bdf1)
            errs[bdf1].append(np.linalg.norm(u[0] - exact) / np.linalg.norm(exact))
    r2 = [a / b for a, b in zip(errs[False], errs[False][1:])]
    r1 = [a / b for a, b in zip(errs[True], errs[True][1:])]
    assert all(3.5 < r < 4.5 for r in r2), (errs, r2)
    assert all(1.7 < r < 2.3 for r in r1), (errs, r1)


def test_first_loop_step_matches_the_one_step_form():
    """Without advection, step 0 of the loop is the implicit-Euler step: same
    right-hand sides, prediction and pressure increment as OracleStep (whose
    correction uses the lumped mass; the loop's uses the consistent mass)."""
    m = basin.basin_mesh(10, 8, 4, seed=2)
    dt = 3600.0
    theta = np.stack([basin.wind_tension(m.xyz[:, 1], m.Ly), np.zeros(m.n)])
    f = basin.coriolis_parameter(m.xyz[:, 1], m.Ly)
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal((3, m.n)) * 0.01
    for c in range(3):
        u0[c][((m.bc >> c) & 1) == 1] = 0.0
    p0 = rng.standard_normal(m.n)
    one = OracleStep(m, 1e3, 1e-2, dt).step(u0, p0, theta, f, tol=1e-12)
    loop = OracleLoop(m, 1e3, 1e-2, dt, advect=False, pressure_nu=(1e3, 1e-2),
                      pressure_line=False)
    r = loop.step(u0, u0, p0, theta, f, first=True, tol=1e-12)
    assert np.abs(r["b_vel"] - one["b_vel"]).max() <= 1e-12 * np.abs(one["b_vel"]).max()
    assert np.abs(r["ut"] - one["ut"]).max() <= 1e-10 * np.abs(one["ut"]).max()
    assert np.abs(r["q"] - one["q"]).max() <= 1e-9 * np.abs(one["q"]).max()


def test_consistent_correction_satisfies_its_equation():
    """M u_c = M ut_c - tau B_c q on the free nodes of component c, u_c = 0 on
    its Dirichlet set, p^{k+1} = p^k + q; a BDF2 step uses tau = 2 dt / 3."""
    m = basin.basin_mesh(8, 6, 3, seed=3)
    dt = 3600.0
    loop = OracleLoop(m, 1e3, 1e-2, dt, pressure_tol=1e-9)
    theta = np.stack([basin.wind_tension(m.xyz[:, 1], m.Ly), np.zeros(m.n)])
    u0 = np.zeros((3, m.n))
    p0 = np.zeros(m.n)
    rs = loop.run(2, u0, p0, theta, None, tol=1e-12)
    for k, r in enumerate(rs):
        tau = dt if k == 0 else 2 * dt / 3
        for c in range(3):
            d = ((m.bc >> c) & 1) == 1
            lhs = loop.M.matvec(r["u"][c])
            rhs = loop.M.matvec(r["ut"][c]) - tau * loop.B[c].matvec(r["q"])
            assert np.all(r["u"][c][d] == 0.0)
            assert np.abs((lhs - rhs)[~d]).max() <= 1e-10 * np.abs(rhs[~d]).max()
    assert np.allclose(rs[1]["p"], rs[0]["p"] + rs[1]["q"], rtol=0, atol=1e-14 * np.abs(rs[1]["p"]).max())


def test_loop_at_rest_without_forcing_stays_at_rest():
    m = basin.box_mesh(4, 4, 2)
    loop = OracleLoop(m, 1.0, 1e-2, 0.1)
    rs = loop.run(3, np.zeros((3, m.n)), np.zeros(m.n), None, None)
    assert all(np.all(r["u"] == 0.0) and np.all(r["p"] == 0.0) for r in rs)


def test_loop_with_isotropic_pressure_is_stable_and_anisotropic_is_not():
    """Eight wind-driven steps on a small basin: with the paper's isotropic
    pressure operator the velocity grows smoothly and the vertical velocity
    stays small; with the anisotropic K_nu in its place the vertical velocity
    grows by orders of magnitude per step."""
    m = basin.basin_mesh(16, 12, 5, seed=2)
    theta = np.stack([basin.wind_tension(m.xyz[:, 1], m.Ly), np.zeros(m.n)])
    f = basin.coriolis_parameter(m.xyz[:, 1], m.Ly)
    z = (np.zeros((3, m.n)), np.zeros(m.n))
    iso = OracleLoop(m, 1e3, 1e-2, 3600.0, pressure_tol=1e-9).run(8, *z, theta, f, tol=1e-10)
    u1 = [np.abs(r["u"][0]).max() for r in iso]
    u3 = [np.abs(r["u"][2]).max() for r in iso]
    assert all(0 < b / a < 2.5 for a, b in zip(u1, u1[1:]))
    assert max(u3) < 1e-3 * max(u1)
    ani = OracleLoop(m, 1e3, 1e-2, 3600.0, pressure_nu=(1e3, 1e-2), pressure_line=False)
    ra = ani.run(4, *z, theta, f, tol=1e-10)
    assert np.abs(ra[3]["u"][2]).max() > 10.0 * np.abs(ra[3]["u"][0]).max()
