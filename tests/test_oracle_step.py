"""Pins of the oracle's projection-step right-hand sides (CPU)."""
import numpy as np
import pytest

import basin
import oracle
from oracle.step import OracleStep


@pytest.fixture(scope="module")
def small():
    m = basin.basin_mesh(10, 8, 4, seed=2)
    L = m.Ly
    theta = np.stack([basin.wind_tension(m.xyz[:, 1], L), np.zeros(m.n)])
    f = basin.coriolis_parameter(m.xyz[:, 1], L)
    return m, OracleStep(m, 1e3, 1e-2, 3600.0), theta, f


def _masked_random(m, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((3, m.n))
    for c in range(3):
        u[c][((m.bc >> c) & 1) == 1] = 0.0
    return u


def test_rhs_at_rest_is_the_wind_load(small):
    """u = 0, p = 0: only the surface tension load dt M_s theta_1 remains."""
    m, st, theta, f = small
    b = st.velocity_rhs(np.zeros((3, m.n)), np.zeros(m.n), theta, f)
    want = st.dt * st.Ms.matvec(theta[0])
    want[st.dirichlet[0]] = 0.0
    assert np.allclose(b[0], want, rtol=0, atol=1e-14 * np.abs(want).max())
    assert np.all(b[1] == 0) and np.all(b[2] == 0)
    # total load equals dt times the integral of the interpolated tension
    assert st.Ms.matvec(theta[0]).sum() == pytest.approx(
        (st.Ms.to_scipy() @ theta[0]).sum(), rel=1e-14)


def test_pressure_rhs_of_admissible_velocity_sums_to_zero(small):
    """sum_i (sum_c B_c u_c)_i = int div u_h = boundary flux, which vanishes
    when each component is zero where its normal component is not."""
    m, st, _, _ = small
    u = _masked_random(m, 3)
    bq = st.pressure_rhs(u)
    scale = sum(np.abs(st.B[c].matvec(u[c])).sum() for c in range(3)) / st.dt
    assert abs(bq.sum()) <= 1e-12 * scale
    # without the masks the flux does not vanish
    rng = np.random.default_rng(4)
    bq_bad = st.pressure_rhs(rng.standard_normal((3, m.n)))
    assert abs(bq_bad.sum()) > 1e-6 * np.abs(bq_bad).sum()


def test_gradient_of_constant_pressure_lives_on_the_boundary(small):
    """(B_c^T 1)_i = int d phi_i / d x_c: zero at interior nodes, and summing
    to the integral of n_c over the closed boundary (zero)."""
    m, st, _, _ = small
    i, j, k = np.meshgrid(np.arange(m.Nx + 1), np.arange(m.Ny + 1), np.arange(m.Nz + 1),
                          indexing="ij")
    interior = ((i > 0) & (i < m.Nx) & (j > 0) & (j < m.Ny) & (k > 0) & (k < m.Nz)).ravel()
    for c in range(3):
        g = st.B[c].rmatvec(np.ones(m.n), m.n)
        scale = np.abs(g).max()
        assert np.abs(g[interior]).max() <= 1e-12 * scale
        assert abs(g.sum()) <= 1e-12 * np.abs(g).sum()
        # transpose agrees with the library routine
        assert np.allclose(g, st.B[c].to_scipy().T @ np.ones(m.n), rtol=1e-13, atol=0)


def test_coriolis_term_signs(small):
    """C_1 = +M (f u_2), C_2 = -M (f u_1): isolate them with theta = 0, p = 0, u_c = 0."""
    m, st, _, f = small
    u = _masked_random(m, 5)
    base = st.velocity_rhs(u, None, None, None)
    with_f = st.velocity_rhs(u, None, None, f)
    c1 = st.dt * st.M.matvec(f * u[1])
    c1[st.dirichlet[0]] = 0
    c2 = -st.dt * st.M.matvec(f * u[0])
    c2[st.dirichlet[1]] = 0
    assert np.allclose(with_f[0] - base[0], c1, atol=1e-12 * np.abs(c1).max())
    assert np.allclose(with_f[1] - base[1], c2, atol=1e-12 * np.abs(c2).max())
    assert np.array_equal(with_f[2], base[2])


def test_correction_reduces_to_identity_for_zero_increment(small):
    m, st, _, _ = small
    ut = _masked_random(m, 6)
    u, p = st.correct(ut, np.zeros(m.n), np.ones(m.n))
    assert np.array_equal(u, ut) and np.all(p == 1.0)
    # a linear increment q = x_c gives u_c = ut_c - dt (B_c x_c) / m_L = ut_c - dt
    q = m.xyz[:, 0].copy()
    u, _ = st.correct(ut, q, None)
    free = ~st.dirichlet[0]
    assert np.allclose(u[0][free], ut[0][free] - st.dt, rtol=0, atol=1e-9 * st.dt)


def test_step_from_rest_runs(small):
    m, st, theta, f = small
    out = st.step(np.zeros((3, m.n)), np.zeros(m.n), theta, f, tol=1e-12)
    assert np.abs(out["ut"][0]).max() > 0
    assert np.all(out["ut"][1] == 0) and np.all(out["ut"][2] == 0)
    out2 = st.step(out["u"], out["p"], theta, f, tol=1e-12)
    assert np.abs(out2["ut"][1]).max() > 0 and np.abs(out2["ut"][2]).max() > 0
