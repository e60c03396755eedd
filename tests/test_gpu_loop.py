"""GPU multi-step projection loop (BDF2, explicit advection, consistent-mass
correction, isotropic line-preconditioned pressure) against the oracle's
loop on the same seeded inputs."""
import numpy as np
import pytest

import basin
import oracle
from oracle.step import OracleLoop

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_0486_amd.step import ProjectionLoop
    m = basin.basin_mesh(20, 16, 5, seed=6)
    theta = np.stack([basin.wind_tension(m.xyz[:, 1], m.Ly), np.zeros(m.n)])
    f = basin.coriolis_parameter(m.xyz[:, 1], m.Ly)
    gpu = ProjectionLoop(m, 1e3, 1e-2, 3600.0, theta, f)
    ref = OracleLoop(m, 1e3, 1e-2, 3600.0, pressure_tol=1e-9)
    yield m, gpu, ref, theta, f
    gpu.close()


def test_advection_matches_oracle(setup):
    m, gpu, _, _, _ = setup
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3, m.n))
    got = gpu.helm1.step_advection(_t(u)).cpu().numpy()
    want = oracle.advection(m, u)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_advection_exact_for_linear_fields_on_gpu(setup):
    """Independent of the oracle: (u . grad) u_c is linear for linear u, so
    the form equals M times its nodal values (M from the library itself)."""
    m, gpu, _, _, _ = setup
    A = np.array([[1e-6, 2e-6, 3e-3], [-2e-6, 5e-7, 1e-3], [4e-7, -1e-6, 2e-3]])
    u = A @ m.xyz.T + np.array([0.1, -0.2, 0.05])[:, None]
    got = gpu.helm1.step_advection(_t(u)).cpu().numpy()
    nodal = np.stack([sum(u[d] * A[c, d] for d in range(3)) for c in range(3)])
    want = np.stack([gpu.helm1.apply_aux("M", _t(nodal[c])).cpu().numpy() for c in range(3)])
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_bdf_rhs_and_correction_rhs_match_oracle(setup):
    m, gpu, ref, theta, f = setup
    rng = np.random.default_rng(4)
    u, up = rng.standard_normal((3, m.n)) * 0.1, rng.standard_normal((3, m.n)) * 0.1
    p = rng.standard_normal(m.n)
    tau, a1, a2 = ref.coefficients(False, ref.dt)
    adv = gpu.helm1.step_advection(_t(u))
    got = gpu.helm1.step_velocity_rhs_bdf(tau, a1, _t(u), a2, _t(up), _t(p), _t(theta), _t(f),
                                          adv).cpu().numpy()
    want = ref.velocity_rhs(tau, a1, u, a2, up, p, theta, f)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    ut, q = rng.standard_normal((3, m.n)), rng.standard_normal(m.n)
    pd = _t(p)
    got = gpu.helm1.step_correct_rhs(tau, _t(ut), _t(q), pd).cpu().numpy()
    for c in range(3):
        d = ((m.bc >> c) & 1) == 1
        w = ref.M.matvec(ut[c]) - tau * ref.B[c].matvec(q)
        w[d] = 0.0
        assert np.abs(got[c] - w).max() <= 1e-12 * np.abs(w).max()
    assert np.abs(pd.cpu().numpy() - (p + q)).max() <= 1e-15 * np.abs(p + q).max()
    bq = gpu.helm1.step_pressure_rhs_tau(tau, _t(ut)).cpu().numpy()
    wq = -(1.0 / tau) * sum(ref.B[c].matvec(ut[c]) for c in range(3))
    assert np.abs(bq - wq).max() <= 1e-12 * np.abs(wq).max()


def test_three_steps_from_rest_match_oracle(setup):
    """Implicit-Euler first step, then two BDF2 steps; velocity solves to 1e-12,
    the isotropic pressure to 1e-9 (its rounding floor is near 2e-10)."""
    m, gpu, ref, theta, f = setup
    gpu.set_state(torch.zeros(3, m.n, dtype=torch.float64, device="cuda"),
                  torch.zeros(m.n, dtype=torch.float64, device="cuda"))
    outs = ref.run(3, np.zeros((3, m.n)), np.zeros(m.n), theta, f, tol=1e-12)
    for k, out in enumerate(outs):
        res = gpu.step(tol=1e-12, pressure_tol=1e-9)
        assert all(i.status == 0 for i in res.velocity + res.correction), k
        assert res.pressure.status == 0
        for c in range(3):
            if np.abs(out["ut"][c]).max() == 0:
                assert float(gpu.ut[c].abs().max()) == 0.0
            else:
                assert _rel(gpu.ut[c].cpu().numpy(), out["ut"][c]) <= 1e-8, (k, c)
        assert _rel(gpu.q.cpu().numpy(), out["q"]) <= 1e-7, k
        assert _rel(gpu.p.cpu().numpy(), out["p"]) <= 1e-7, k
        assert _rel(gpu.u.cpu().numpy(), out["u"]) <= 1e-7, k
    # the state after three steps: wind-driven, vertical velocity small
    u = gpu.u.cpu().numpy()
    assert np.abs(u[2]).max() < 1e-2 * np.abs(u[0]).max()


def test_paper_constants_stress_case(setup):
    """The paper's run constants: nu = (1e8, 1e8, 250) m^2/s, dt = one month.
    The velocity operator is dominated by the stiffness; two steps against the
    oracle, velocity solves with point Jacobi and with the line blocks."""
    from paper_1207_0486_amd.step import ProjectionLoop
    m, _, _, theta, f = setup
    ref = OracleLoop(m, 1e8, 250.0, 2.592e6, pressure_tol=1e-9)
    outs = ref.run(2, np.zeros((3, m.n)), np.zeros(m.n), theta, f, tol=1e-11)
    for pre in (0, 1):
        gpu = ProjectionLoop(m, 1e8, 250.0, 2.592e6, theta, f, velocity_precond=pre)
        try:
            for k, out in enumerate(outs):
                res = gpu.step(tol=1e-11, pressure_tol=1e-9)
                assert all(i.status == 0 for i in res.velocity + res.correction)
                assert _rel(gpu.u.cpu().numpy(), out["u"]) <= 1e-6, (pre, k)
        finally:
            gpu.close()
