"""The allocation-free solve (hns_solve_noalloc, workspace in the library's
static device scratch) against hns_solve on the same inputs: two calls in a
row, the second on a smaller operator, FP64 and mixed precision; the
single-workgroup size; the unscaled fallback; the refusals."""
import numpy as np
import pytest

import basin

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NU = (1e3, 1e-2)
DT = 3600.0


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_0486_amd import hns  # noqa: F401
    return torch.device("cuda", 0)


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _rel(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def _case(mesh, kind, bit, seed, keep_fp32=True):
    from paper_1207_0486_amd.hns import Operator
    op = Operator(mesh, NU[0], NU[1], DT if kind == "helmholtz" else 0.0, kind=kind,
                  keep_fp32=keep_fp32)
    d = None if bit < 0 else ((mesh.bc >> bit) & 1) == 1
    b = basin.normal_rhs(mesh.n, seed, dirichlet=d, zero_mean=bit < 0)
    return op, _t(b)


def _compare(op, b, bit, mode, tol=1e-10):
    x_ref, i_ref = op.solve(b, tol=tol, mask_bit=bit, mode=mode)
    x, info = op.solve_noalloc(b, torch.zeros_like(b), tol=tol, mask_bit=bit, mode=mode)
    assert i_ref.status == 0 and info.status == 0
    assert info.iterations == i_ref.iterations, (info.iterations, i_ref.iterations)
    xr, xn = x_ref.cpu().numpy(), x.cpu().numpy()
    err = _rel(xn, xr)
    assert err <= 1e-10, err
    return err, bool(np.array_equal(xn, xr))


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_two_calls_in_a_row_second_smaller(dev, mode):
    """First a 349,461-row pressure solve (Jacobi-scaled multi-launch path),
    then a 10,619-row velocity solve: each equals hns_solve's answer (the same
    recurrence and launch shapes, so bit for bit here)."""
    from paper_1207_0486_amd.hns import Operator
    big = basin.basin_mesh(128, 128, 20, seed=0)
    small = basin.basin_mesh(40, 36, 6, seed=5)
    op1, b1 = _case(big, "poisson", -1, 61)
    assert op1.noalloc_bytes(mode) <= Operator.noalloc_scratch_bytes()
    e1, same1 = _compare(op1, b1, -1, mode)
    op1.close()
    op2, b2 = _case(small, "helmholtz", 1, 62)
    e2, same2 = _compare(op2, b2, 1, mode)
    op2.close()
    assert same1 and same2, (e1, e2)


def test_unscaled_fallback_and_single_workgroup(dev):
    """An operator that hns_solve never used holds no Jacobi-scaled copy: the
    allocation-free call runs the unscaled recurrence (same iterates up to
    rounding).  A 1,445-row box runs the single-workgroup kernel."""
    from paper_1207_0486_amd.hns import Operator
    m = basin.basin_mesh(40, 36, 6, seed=5)
    op_a, b = _case(m, "helmholtz", 0, 63, keep_fp32=False)
    x, info = op_a.solve_noalloc(b, torch.zeros_like(b), tol=1e-10, mask_bit=0)
    op_a.close()
    op_b, _ = _case(m, "helmholtz", 0, 63, keep_fp32=False)
    x_ref, i_ref = op_b.solve(b, tol=1e-10, mask_bit=0)
    op_b.close()
    assert info.status == 0 and abs(info.iterations - i_ref.iterations) <= 1
    assert _rel(x.cpu().numpy(), x_ref.cpu().numpy()) <= 1e-10
    cfg = basin.configs.BOX_16x16x4
    mb = cfg.mesh()
    d = ~mb.free_mask(basin.BC_U1)
    bb = _t(basin.normal_rhs(mb.n, cfg.seed, zero_mean=True, dirichlet=d))
    opb = Operator(mb, cfg.nu_h, cfg.nu_v, kind="poisson", keep_fp32=True)
    for mode in ("fp64", "mixed"):
        _compare(opb, bb, 0, mode)
    # b = 0: x = 0 after no iteration, whatever the initial guess
    x, info = opb.solve_noalloc(torch.zeros_like(bb), torch.ones_like(bb), mask_bit=0)
    assert info.status == 0 and info.iterations == 0 and float(x.abs().max()) == 0.0
    opb.close()


def test_refusals(dev):
    from paper_1207_0486_amd.hns import HNSError, Operator
    m = basin.basin_mesh(24, 20, 6, seed=4)
    op, b = _case(m, "helmholtz", 0, 64)
    op.set_param("precond", 1)
    with pytest.raises(HNSError, match="point Jacobi"):
        op.solve_noalloc(b, torch.zeros_like(b), mask_bit=0)
    op.close()
    # 3,705,625 rows: more scratch than the static array holds
    big = basin.basin_mesh(384, 384, 24, seed=104)
    opb = Operator(big, NU[0], NU[1], kind="poisson", gpu_assembly=True)
    assert opb.noalloc_bytes("fp64") > Operator.noalloc_scratch_bytes()
    bb = torch.zeros(big.n, dtype=torch.float64, device="cuda")
    with pytest.raises(HNSError, match="static scratch"):
        opb.solve_noalloc(bb, torch.zeros_like(bb))
    opb.close()
