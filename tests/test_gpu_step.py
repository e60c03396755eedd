"""GPU projection-step right-hand sides and a two-step run against the oracle."""
import numpy as np
import pytest

import basin
from oracle.step import OracleStep

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_0486_amd.step import ProjectionStep
    m = basin.basin_mesh(24, 20, 6, seed=4)
    L = m.Ly
    theta = np.stack([basin.wind_tension(m.xyz[:, 1], L), np.zeros(m.n)])
    f = basin.coriolis_parameter(m.xyz[:, 1], L)
    gpu = ProjectionStep(m, 1e3, 1e-2, 3600.0, theta, f)
    ref = OracleStep(m, 1e3, 1e-2, 3600.0)
    return m, gpu, ref, theta, f


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_aux_forms_match_oracle(setup):
    m, gpu, ref, _, _ = setup
    x = np.random.default_rng(1).standard_normal(m.n)
    xt = _t(x)
    assert _rel(gpu.helm.apply_aux("M", xt).cpu().numpy(), ref.M.matvec(x)) <= 1e-13
    assert _rel(gpu.helm.apply_aux("Ms", xt).cpu().numpy(), ref.Ms.matvec(x)) <= 1e-13
    for c in range(3):
        assert _rel(gpu.helm.apply_aux(f"B{c + 1}", xt).cpu().numpy(), ref.B[c].matvec(x)) <= 1e-12
        assert _rel(gpu.helm.apply_aux(f"B{c + 1}T", xt).cpu().numpy(),
                    ref.B[c].rmatvec(x, m.n)) <= 1e-12


def test_step_rhs_and_correction_match_oracle(setup):
    m, gpu, ref, theta, f = setup
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3, m.n)) * 0.1
    p = rng.standard_normal(m.n)
    gpu.set_state(_t(u), _t(p))
    b = gpu.velocity_rhs().cpu().numpy()
    want = ref.velocity_rhs(u, p, theta, f)
    for c in range(3):
        assert _rel(b[c], want[c]) <= 1e-12
    ut = rng.standard_normal((3, m.n))
    gpu.ut.copy_(_t(ut))
    bq = gpu.pressure_rhs().cpu().numpy()
    assert _rel(bq, ref.pressure_rhs(ut)) <= 1e-12
    q = rng.standard_normal(m.n)
    gpu.q.copy_(_t(q))
    gpu.correct()
    u_ref, p_ref = ref.correct(ut, q, p)
    assert _rel(gpu.u.cpu().numpy(), u_ref) <= 1e-12
    assert _rel(gpu.p.cpu().numpy(), p_ref) <= 1e-14


def test_two_steps_from_rest_match_oracle(setup):
    """Step 0 from rest, then step 1 (all three velocity components and the
    pressure increment nontrivial), FP64, tol 1e-12 on both sides."""
    m, gpu, ref, theta, f = setup
    gpu.set_state(torch.zeros(3, m.n, dtype=torch.float64, device="cuda"),
                  torch.zeros(m.n, dtype=torch.float64, device="cuda"))
    u = np.zeros((3, m.n))
    p = np.zeros(m.n)
    for k in range(2):
        res = gpu.step(tol=1e-12)
        out = ref.step(u, p, theta, f, tol=1e-12)
        for c in range(3):
            assert res.velocity[c].status == 0
            if np.abs(out["ut"][c]).max() == 0:
                assert float(gpu.ut[c].abs().max()) == 0.0
            else:
                assert _rel(gpu.ut[c].cpu().numpy(), out["ut"][c]) <= 1e-9
        assert res.pressure.status == 0
        assert _rel(gpu.q.cpu().numpy(), out["q"]) <= 1e-7
        assert _rel(gpu.u.cpu().numpy(), out["u"]) <= 1e-7
        u, p = out["u"], out["p"]


@pytest.mark.parametrize("mode", ["mixed"])
def test_step_mixed_matches_fp64(setup, mode):
    m, gpu, ref, theta, f = setup
    zero3 = torch.zeros(3, m.n, dtype=torch.float64, device="cuda")
    zero = torch.zeros(m.n, dtype=torch.float64, device="cuda")
    gpu.set_state(zero3, zero)
    gpu.step(tol=1e-12)
    u1, p1 = gpu.state()
    gpu.step(tol=1e-12)
    u64 = gpu.u.clone()
    gpu.set_state(u1, p1)
    res = gpu.step(tol=1e-12, mode=mode)
    assert all(i.status == 0 for i in res.velocity) and res.pressure.status == 0
    assert float((gpu.u - u64).abs().max() / u64.abs().max()) <= 1e-7
