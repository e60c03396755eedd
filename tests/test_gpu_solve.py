"""GPU parity: the HIP Jacobi-PCG against the FP64 CPU oracle on the same
seeded inputs (same algorithm, same initial guess, same stopping rule)."""
import numpy as np
import pytest

import basin
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_0486_amd import hns  # noqa: F401  (fails loudly without libhns.so)
    return torch.device("cuda", 0)


def _gpu(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)


def _relerr(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def assert_parity(info, x_gpu, A, b, dirichlet=None, singular=False, weights=None, tol=1e-10,
                  ref=None):
    """P-same parity of a GPU FP64 solve with the oracle:
      * converged, and the oracle's own residual of the GPU answer is <= tol;
      * the iteration count is within 1 (or 2 %) of the oracle's;
      * the GPU answer equals the oracle's CG iterate after the same number of
        iterations to relative difference 1e-10 (both run the same recurrence;
        only rounding differs)."""
    assert info.status == 0
    if ref is None:
        ref = oracle.pcg(A, b, dirichlet=dirichlet, singular=singular, weights=weights, tol=tol)
    assert ref.status == oracle.OK
    assert abs(info.iterations - ref.iterations) <= max(1, 0.02 * ref.iterations)
    if singular:
        bh = b - b.mean()
        r = bh - A.matvec(x_gpu)
        r -= r.mean()
        assert np.linalg.norm(r) <= 1.01 * tol * np.linalg.norm(bh)
    else:
        assert oracle.relres(A, b, x_gpu, dirichlet) <= 1.01 * tol
    # the same stopping rule (tolerance, restarts from the true residual),
    # stopped after the GPU's iteration count
    same = oracle.pcg(A, b, dirichlet=dirichlet, singular=singular, weights=weights,
                      tol=tol, maxit=info.iterations)
    if same.iterations < info.iterations:   # the oracle met the tolerance first
        same = oracle.pcg(A, b, dirichlet=dirichlet, singular=singular, weights=weights,
                          tol=1e-300, maxit=info.iterations)
    assert same.iterations == info.iterations
    assert _relerr(x_gpu, same.x) <= 1e-10, _relerr(x_gpu, same.x)
    return ref


BOX = basin.configs.BOX_16x16x4
FORMATS = ["csr", "sell", "sdia"]


@pytest.mark.parametrize("fmt", FORMATS)
def test_box16_poisson_fp64_matches_oracle(dev, fmt):
    """Plain method, small: Dirichlet on Gamma_b, N(0,1) RHS projected to zero mean."""
    from paper_1207_0486_amd.hns import Operator
    m = BOX.mesh()
    d = ~m.free_mask(basin.BC_U1)
    b = basin.normal_rhs(m.n, BOX.seed, zero_mean=True, dirichlet=d)
    A = oracle.stiffness(m, BOX.nu_h, BOX.nu_v)
    op = Operator(m, BOX.nu_h, BOX.nu_v, kind="poisson", fmt=fmt)
    assert op.format == fmt and op.n == 1445 and op.nnz == 18157
    x, info = op.solve(_gpu(b, dev), tol=BOX.tol, mask_bit=0)
    xh = x.cpu().numpy()
    assert info.relres_true <= BOX.tol
    assert np.all(xh[d] == 0)
    ref = assert_parity(info, xh, A, b, dirichlet=d, tol=BOX.tol)
    assert abs(info.iterations - ref.iterations) <= 1
    assert _relerr(xh, ref.x) <= 1e-10


@pytest.fixture(scope="module")
def ragged_basin():
    # 25 x 21 x 7 = 3675 nodes: 58 slices of 64 rows, the last one ragged
    return basin.basin_mesh(24, 20, 6, seed=4)


# small_n = 4096 runs these 3,675 rows in the single-workgroup kernel; 0 runs
# the multi-launch kernels the large solves use (on diagonal storage the
# Jacobi-scaled recurrence)
SMALL_N = [4096, 0]


@pytest.mark.parametrize("small_n", SMALL_N)
@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("bit", [0, 1, 2])
def test_helmholtz_masks_match_oracle(dev, ragged_basin, fmt, bit, small_n):
    from paper_1207_0486_amd.hns import Operator
    m = ragged_basin
    d = (m.bc >> bit) & 1 == 1
    b = basin.normal_rhs(m.n, 20 + bit, dirichlet=d)
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", fmt=fmt)
    op.set_param("small_n", small_n)
    x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=bit)
    xh = x.cpu().numpy()
    assert np.all(xh[d] == 0)
    assert_parity(info, xh, A, b, dirichlet=d)


@pytest.mark.parametrize("small_n", SMALL_N)
@pytest.mark.parametrize("fmt", FORMATS)
def test_neumann_poisson_matches_oracle(dev, ragged_basin, fmt, small_n):
    from paper_1207_0486_amd.hns import Operator
    m = ragged_basin
    b = basin.normal_rhs(m.n, 31)
    w = oracle.mass(m).matvec(np.ones(m.n))
    A = oracle.stiffness(m, 1e3, 1e-2)
    op = Operator(m, 1e3, 1e-2, kind="poisson", fmt=fmt)
    op.set_param("small_n", small_n)
    x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=-1)
    xh = x.cpu().numpy()
    ref = assert_parity(info, xh, A, b, singular=True, weights=w)
    assert info.removed_mean == pytest.approx(ref.removed_mean, rel=1e-12)
    assert abs(w @ xh) <= 1e-12 * np.abs(w).sum() * np.abs(xh).max()


MIXED_VARIANTS = [0, 1, 2]  # FP32 + replacement, restarted refinement, FP32 storage


@pytest.mark.parametrize("variant", MIXED_VARIANTS)
def test_mixed_error_against_tight_oracle(dev, ragged_basin, variant):
    """FP32 inner / FP64 outer: error vs the oracle solved to 1e-13 within 1e-9."""
    from paper_1207_0486_amd.hns import Operator
    m = ragged_basin
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    op.set_param("mixed_variant", variant)
    for bit in (0, 1, 2):
        d = (m.bc >> bit) & 1 == 1
        b = basin.normal_rhs(m.n, 40 + bit, dirichlet=d)
        exact = oracle.pcg(oracle.helmholtz(m, 1e3, 1e-2, 3600.0), b, dirichlet=d, tol=1e-13)
        x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=bit, mode="mixed")
        assert info.status == 0 and info.relres_true <= 1e-10
        assert info.outer_iterations >= 2
        assert _relerr(x.cpu().numpy(), exact.x) <= 1e-9


@pytest.mark.parametrize("variant", MIXED_VARIANTS)
def test_mixed_neumann(dev, ragged_basin, variant):
    from paper_1207_0486_amd.hns import Operator
    m = ragged_basin
    w = oracle.mass(m).matvec(np.ones(m.n))
    b = basin.normal_rhs(m.n, 50)
    exact = oracle.pcg(oracle.stiffness(m, 1e3, 1e-2), b, singular=True, weights=w, tol=1e-13)
    op = Operator(m, 1e3, 1e-2, kind="poisson", keep_fp32=True)
    op.set_param("mixed_variant", variant)
    x, info = op.solve(_gpu(b, dev), tol=1e-10, mode="mixed")
    assert info.status == 0 and info.relres_true <= 1e-10
    assert _relerr(x.cpu().numpy(), exact.x) <= 1e-9


def test_zero_rhs_and_nonfinite(dev, ragged_basin):
    from paper_1207_0486_amd.hns import Operator, HNSError
    m = ragged_basin
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    x0 = _gpu(np.random.default_rng(0).standard_normal(m.n), dev)
    for mode in ("fp64", "mixed"):
        x, info = op.solve(_gpu(np.zeros(m.n), dev), x=x0.clone(), mask_bit=0, mode=mode)
        assert info.status == 0 and info.iterations == 0
        assert torch.count_nonzero(x).item() == 0
    free = np.flatnonzero((m.bc & 1) == 0)
    b = np.ones(m.n)
    b[free[17]] = np.inf
    with pytest.raises(HNSError) as e:
        op.solve(_gpu(b, dev), mask_bit=0)
    assert e.value.status == -1
    # a non-finite value on a Dirichlet node is ignored like any other value there
    b = np.where((m.bc & 1) == 1, np.nan, 1.0)
    x, info = op.solve(_gpu(b, dev), mask_bit=0)
    assert info.status == 0 and bool(torch.isfinite(x).all())


def test_max_iter_returns_last_iterate(dev, ragged_basin):
    """NOT_CONVERGED after exactly max_iter iterations, x = the CG iterate of the oracle."""
    from paper_1207_0486_amd.hns import Operator
    m = ragged_basin
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 60, dirichlet=d)
    A = oracle.stiffness(m, 1e3, 1e-2)
    ref = oracle.pcg(A, b, dirichlet=d, tol=1e-10, maxit=7)
    op = Operator(m, 1e3, 1e-2, kind="poisson")
    x, info = op.solve(_gpu(b, dev), tol=1e-10, max_iter=7, mask_bit=0, check=False)
    assert info.status == 1 and ref.status == oracle.NOT_CONVERGED
    assert info.iterations == 7
    assert _relerr(x.cpu().numpy(), ref.x) <= 1e-12
    assert info.relres_true == pytest.approx(oracle.relres(A, b, x.cpu().numpy(), d), rel=1e-6)


def test_non_spd_operator_reports_breakdown(dev):
    """A negative time step makes M + dt K indefinite; both sides report breakdown."""
    from paper_1207_0486_amd.hns import Operator, HNSError
    m = basin.box_mesh(8, 8, 2, gamma0=("bottom",))
    # largest dt with a positive diagonal is M_ii / K_ii; take most of it
    Ms = oracle.mass(m).to_scipy().diagonal()
    Ks = oracle.stiffness(m, 1.0, 1e-4).to_scipy().diagonal()
    dt = -0.9 * np.min(Ms / Ks)
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 3, dirichlet=d)
    ref = oracle.pcg(oracle.helmholtz(m, 1.0, 1e-4, dt), b, dirichlet=d)
    assert ref.status == oracle.ERR_BREAKDOWN
    op = Operator(m, 1.0, 1e-4, dt, kind="helmholtz")
    with pytest.raises(HNSError) as e:
        op.solve(_gpu(b, dev), mask_bit=0)
    assert e.value.status == -5


def test_apply_matches_oracle_product(dev, ragged_basin):
    from paper_1207_0486_amd.hns import Operator
    m = ragged_basin
    x = np.random.default_rng(5).standard_normal(m.n)
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    for fmt in FORMATS:
        op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", fmt=fmt)
        y = op.apply(_gpu(x, dev)).cpu().numpy()
        ref = A.matvec(x)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
        d = (m.bc & 1) == 1
        ym = op.apply(_gpu(np.where(d, 0.0, x), dev), mask_bit=0).cpu().numpy()
        refm = A.matvec(np.where(d, 0.0, x))
        assert np.all(ym[d] == 0)
        assert np.abs(ym[~d] - refm[~d]).max() <= 1e-13 * np.abs(ref).max()


def test_repeatable_bitwise(dev, ragged_basin):
    """Deterministic reductions: the same solve twice gives identical bits."""
    from paper_1207_0486_amd.hns import Operator
    m = ragged_basin
    b = _gpu(basin.normal_rhs(m.n, 70), dev)
    op = Operator(m, 1e3, 1e-2, kind="poisson")
    x1, i1 = op.solve(b, tol=1e-10)
    x2, i2 = op.solve(b, tol=1e-10)
    assert i1.iterations == i2.iterations
    assert torch.equal(x1, x2)


def test_footprint(dev, ragged_basin):
    from paper_1207_0486_amd.hns import Operator
    op = Operator(ragged_basin, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    f1 = op.footprint(1, "fp64", include_operator=False)
    f4 = op.footprint(4, "fp64", include_operator=False)
    # single solve: r, p, q; batched (k = 4): R, P, Q blocks of n x 4
    assert f1 >= 3 * 8 * op.n and f4 >= 4 * 3 * 8 * op.n
    assert op.footprint(1, "mixed", False) > f1
    # at least the symmetric half of the values (8 bytes each)
    assert op.footprint(1, "fp64", True) > f1 + 4 * op.nnz


def test_unstructured_numbering_falls_back_from_diagonal_storage(dev, ragged_basin):
    """A random node numbering scatters the offsets j - i: the automatic format
    is then not the diagonal one, and the solve still matches the oracle."""
    import copy
    from paper_1207_0486_amd.hns import Operator
    m = copy.deepcopy(ragged_basin)
    perm = np.random.default_rng(9).permutation(m.n)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(m.n)
    m.xyz = m.xyz[perm]
    m.bc = m.bc[perm]
    m.tets = inv[m.tets].astype(np.int32)
    m.surf_tris = inv[m.surf_tris].astype(np.int32)
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz")
    assert op.format in ("sell", "csr")
    with pytest.raises(Exception):
        Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", fmt="sdia")
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 80, dirichlet=d)
    x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=0)
    assert_parity(info, x.cpu().numpy(), oracle.helmholtz(m, 1e3, 1e-2, 3600.0), b, dirichlet=d)


def test_auto_format_is_diagonal_on_structured_mesh(dev, ragged_basin):
    from paper_1207_0486_amd.hns import Operator
    op = Operator(ragged_basin, 1e3, 1e-2, kind="poisson")
    assert op.format == "sdia"


def test_tolerance_below_rounding_floor_stops_early(dev):
    """Same rule as the oracle: restarts from the true residual stop after
    three checks that do not halve the best true residual."""
    from paper_1207_0486_amd.hns import Operator
    m = basin.box_mesh(8, 8, 4)
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 2, dirichlet=d)
    op = Operator(m, 1.0, 1e-4, 0.1, kind="helmholtz")
    x, info = op.solve(_gpu(b, dev), tol=1e-19, max_iter=100000, mask_bit=0)
    assert info.status == 1
    assert info.iterations < 2000
    assert info.relres_true < 1e-14
    A = oracle.helmholtz(m, 1.0, 1e-4, 0.1)
    assert oracle.relres(A, b, x.cpu().numpy(), d) < 1e-14


@pytest.mark.parametrize("case", ["box", "basin"])
def test_error_against_exact_within_condition_bound(dev, case):
    """P-exact: the FP64 GPU answer against the oracle solved to 1e-13 is within
    kappa * tol, kappa estimated by Lanczos from the oracle's CG coefficients."""
    from paper_1207_0486_amd.hns import Operator
    if case == "box":
        m = BOX.mesh()
        d = ~m.free_mask(basin.BC_U1)
        A = oracle.stiffness(m, BOX.nu_h, BOX.nu_v)
        op = Operator(m, BOX.nu_h, BOX.nu_v, kind="poisson")
    else:
        m = basin.basin_mesh(24, 20, 6, seed=4)
        d = (m.bc & 1) == 1
        A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
        op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz")
    b = basin.normal_rhs(m.n, 77, dirichlet=d)
    x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=0)
    exact = oracle.pcg(A, b, dirichlet=d, tol=1e-13, history=True)
    kappa = oracle.lanczos_condition(exact.alphas, exact.betas)
    err = _relerr(x.cpu().numpy(), exact.x)
    assert info.status == 0 and kappa >= 1.0
    assert err <= kappa * 1e-10
