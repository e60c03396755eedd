"""Parity at the full 256x256x20 basin size (1,387,029 nodes), in the launch
configuration the benchmark times: the operator against the oracle's own
assembly, the first CG iterations against the oracle's iterates, and the
converged pressure solve through the oracle's residual (a property that holds
at any size)."""
import numpy as np
import pytest

import basin
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_0486_amd.hns import Operator
    wl = basin.configs.BASIN_256x256x20
    m = wl.mesh()
    op = Operator(m, wl.nu_h, wl.nu_v, kind="poisson")
    K = oracle.stiffness(m, wl.nu_h, wl.nu_v)
    w = oracle.mass(m).matvec(np.ones(m.n))
    yield m, wl, op, K, w
    op.close()


def test_full_size_operator_matches_oracle(full):
    m, wl, op, K, _ = full
    assert op.n == 1387029 and op.nnz == 20192829 and op.format == "sdia"
    x = np.random.default_rng(5).standard_normal(m.n)
    got = op.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    want = K.matvec(x)
    scale = np.abs(K.to_scipy()).sum(axis=1).max() * np.abs(x).max()
    assert np.abs(got - want).max() <= 1e-13 * scale


@pytest.mark.parametrize("fmt", ["csr", "sell"])
def test_full_size_csr_sell_operators_match_oracle(full, fmt):
    """The same operator stored in CSR and in sliced ELL (the formats for
    numberings without diagonal structure): the full-size product against the
    oracle's assembly, and eight iterations of the pressure solve against the
    oracle's iterates."""
    from paper_1207_0486_amd.hns import Operator
    m, wl, _, K, w = full
    op = Operator(m, wl.nu_h, wl.nu_v, kind="poisson", fmt=fmt)
    try:
        assert op.format == fmt and op.nnz == 20192829
        x = np.random.default_rng(6).standard_normal(m.n)
        got = op.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
        scale = np.abs(K.to_scipy()).sum(axis=1).max() * np.abs(x).max()
        assert np.abs(got - K.matvec(x)).max() <= 1e-13 * scale
        b = basin.normal_rhs(m.n, 13, zero_mean=True)
        xs, info = op.solve(torch.as_tensor(b, device="cuda"), tol=1e-300, max_iter=8,
                            check=False)
        assert info.iterations == 8
        ref = oracle.pcg(K, b, singular=True, weights=w, tol=1e-300, maxit=8)
        xh = xs.cpu().numpy()
        assert np.linalg.norm(xh - ref.x) <= 1e-12 * np.linalg.norm(ref.x)
    finally:
        op.close()


def test_full_size_first_iterations_match_oracle(full):
    """Eight CG iterations of the pressure solve from x0 = 0: the GPU iterate
    equals the oracle's to 1e-12 (rounding-order differences only)."""
    m, wl, op, K, w = full
    b = basin.normal_rhs(m.n, 11, zero_mean=True)
    x, info = op.solve(torch.as_tensor(b, device="cuda"), tol=1e-300, max_iter=8, check=False)
    assert info.iterations == 8
    ref = oracle.pcg(K, b, singular=True, weights=w, tol=1e-300, maxit=8)
    assert ref.iterations == 8
    xh = x.cpu().numpy()
    assert np.linalg.norm(xh - ref.x) <= 1e-12 * np.linalg.norm(ref.x)


def test_full_size_pressure_solve_converges(full):
    """The converged solve: the oracle's own residual of the GPU answer meets
    the tolerance, and the answer has zero mass-weighted mean."""
    m, wl, op, K, w = full
    b = basin.normal_rhs(m.n, 12, zero_mean=True)
    x, info = op.solve(torch.as_tensor(b, device="cuda"), tol=wl.tol)
    assert info.status == 0 and info.relres_true <= wl.tol
    xh = x.cpu().numpy()
    bh = b - b.mean()
    r = bh - K.matvec(xh)
    r -= r.mean()
    assert np.linalg.norm(r) <= 1.01 * wl.tol * np.linalg.norm(bh)
    assert abs(w @ xh) <= 1e-12 * np.abs(w).sum() * np.abs(xh).max()


@pytest.fixture(scope="module")
def largest():
    """The largest serving mesh, 384x384x24 (3,705,625 nodes): the SpMV and
    update grids exceed the partials slots there, so the blocks take larger
    chunks than the default launch shape."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_0486_amd.hns import Operator
    wl = basin.configs.BASIN_256x256x20
    m = basin.basin_mesh(384, 384, 24, seed=104)
    yield m, wl, Operator, oracle.helmholtz(m, wl.nu_h, wl.nu_v, wl.dt)


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_largest_mesh_velocity_solve(largest, mode):
    """Dirichlet set 0 on the largest mesh: eight iterations equal the
    oracle's Jacobi-PCG iterate (FP64), and the converged solve meets the
    tolerance in the oracle's residual (FP64 and mixed precision)."""
    m, wl, Operator, A = largest
    assert m.n == 3705625
    op = Operator(m, wl.nu_h, wl.nu_v, wl.dt, kind="helmholtz", keep_fp32=True)
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 13, dirichlet=d)
    bt = torch.as_tensor(b, device="cuda")
    if mode == "fp64":
        x, info = op.solve(bt, tol=1e-300, max_iter=8, mask_bit=0, check=False)
        assert info.iterations == 8
        ref = oracle.pcg(A, b, dirichlet=d, tol=1e-300, maxit=8)
        xh = x.cpu().numpy()
        assert np.linalg.norm(xh - ref.x) <= 1e-12 * np.linalg.norm(ref.x)
    x, info = op.solve(bt, tol=wl.tol, mask_bit=0, mode=mode)
    assert info.status == 0
    assert oracle.relres(A, b, x.cpu().numpy(), d) <= 1.01 * wl.tol
    op.close()
