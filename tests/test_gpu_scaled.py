"""Point-Jacobi PCG run as plain CG on the Jacobi-scaled operator
D^-1/2 A D^-1/2 (tunable jacobi_scaling, the default for operators in
symmetric diagonal storage above the single-workgroup size) against the
oracle's unscaled Jacobi-PCG and against the library's unscaled recurrence:
the same method, so the same iterates up to rounding."""
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
    from paper_1207_0486_amd import hns  # noqa: F401
    return torch.device("cuda", 0)


def _gpu(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)


def _rel(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


NU = (1e3, 1e-2)
DT = 3600.0
# (name, mesh factory, small_n): 2,142 rows with the single-workgroup path
# switched off, and 10,619 rows at the default small_n
MESHES = [
    ("basin20x16x5", lambda: basin.basin_mesh(20, 16, 5, seed=3), 0),
    ("basin40x36x6", lambda: basin.basin_mesh(40, 36, 6, seed=5), 4096),
]


def _operator(m, kind, small_n, scaling, fmt="sdia", keep_fp32=False):
    from paper_1207_0486_amd.hns import Operator
    op = Operator(m, NU[0], NU[1], DT if kind == "helmholtz" else 0.0, kind=kind, fmt=fmt,
                  keep_fp32=keep_fp32)
    op.set_param("small_n", small_n)
    op.set_param("jacobi_scaling", scaling)
    return op


def _system(m, bit, seed):
    kind = "poisson" if bit < 0 else "helmholtz"
    A = oracle.helmholtz(m, *NU, DT) if kind == "helmholtz" else oracle.stiffness(m, *NU)
    d = None if bit < 0 else ((m.bc >> bit) & 1) == 1
    b = basin.normal_rhs(m.n, seed, dirichlet=d, zero_mean=bit < 0)
    w = oracle.mass(m).matvec(np.ones(m.n)) if bit < 0 else None
    return kind, A, d, b, w


@pytest.mark.parametrize("mesh", MESHES, ids=[c[0] for c in MESHES])
@pytest.mark.parametrize("bit", [-1, 0, 1, 2])
def test_scaled_fp64_matches_oracle_and_unscaled(dev, mesh, bit):
    _, factory, small_n = mesh
    m = factory()
    kind, A, d, b, w = _system(m, bit, 11 + bit)
    out = {}
    for scaling in (1, 0):
        op = _operator(m, kind, small_n, scaling)
        assert op.format == "sdia"
        x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=bit)
        out[scaling] = (x.cpu().numpy(), info)
        op.close()
    (xs, i_s), (xu, i_u) = out[1], out[0]
    assert i_s.status == 0 and i_u.status == 0
    assert abs(i_s.iterations - i_u.iterations) <= max(1, 0.02 * i_u.iterations)
    ref = oracle.pcg(A, b, dirichlet=d, singular=bit < 0, weights=w, tol=1e-10)
    assert abs(i_s.iterations - ref.iterations) <= max(1, 0.02 * ref.iterations)
    if bit >= 0:
        assert oracle.relres(A, b, xs, d) <= 1.01e-10
        # the oracle's Jacobi-PCG iterate after as many iterations
        same = oracle.pcg(A, b, dirichlet=d, tol=1e-300, maxit=i_s.iterations)
        assert _rel(xs, same.x) <= 1e-10
        assert _rel(xs, xu) <= 1e-10
        assert np.all(xs[d] == 0.0)
    else:
        r = b - A.matvec(xs)
        r -= r.mean()
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
        # the oracle's iterate after as many iterations under the same
        # stopping rule (restarts from the true residual included)
        for xg, ig in ((xs, i_s), (xu, i_u)):
            same = oracle.pcg(A, b, singular=True, weights=w, tol=1e-10, maxit=ig.iterations)
            if same.iterations < ig.iterations:   # the oracle met the tolerance first
                same = oracle.pcg(A, b, singular=True, weights=w, tol=1e-300,
                                  maxit=ig.iterations)
            assert _rel(xg, same.x) <= 1e-10, _rel(xg, same.x)
        assert abs(w @ xs) <= 1e-12 * np.abs(w).sum() * np.abs(xs).max()


@pytest.mark.parametrize("bit", [-1, 0, 2])
@pytest.mark.parametrize("nonzero_x0", [False, True])
def test_scaled_capped_iterate_is_the_jacobi_pcg_iterate(dev, bit, nonzero_x0):
    """Seven iterations from x0: the scaled recurrence's iterate, mapped back
    by D^-1/2, is the oracle's Jacobi-PCG iterate after seven iterations."""
    m = basin.basin_mesh(20, 16, 5, seed=3)
    kind, A, d, b, w = _system(m, bit, 21 + bit)
    x0 = np.random.default_rng(7).standard_normal(m.n) if nonzero_x0 else np.zeros(m.n)
    if d is not None:
        x0[d] = 0.0
    op = _operator(m, kind, 0, 1)
    x, info = op.solve(_gpu(b, dev), x=_gpu(x0, dev), tol=1e-14, max_iter=7, mask_bit=bit,
                       check=False)
    assert info.status == 1 and info.iterations == 7
    same = oracle.pcg(A, b, dirichlet=d, singular=bit < 0, weights=w, x0=x0, tol=1e-300,
                      maxit=7)
    assert _rel(x.cpu().numpy(), same.x) <= 1e-12
    op.close()


@pytest.mark.parametrize("mesh", MESHES, ids=[c[0] for c in MESHES])
@pytest.mark.parametrize("bit", [-1, 0, 1])
def test_scaled_mixed_precision(dev, mesh, bit):
    """FP32 scaled recurrence with FP64 residual replacement: converged in
    FP64 terms, and the error against the oracle's FP64 solution as small as
    the unscaled mixed solve's."""
    _, factory, small_n = mesh
    m = factory()
    kind, A, d, b, w = _system(m, bit, 31 + bit)
    ref = oracle.pcg(A, b, dirichlet=d, singular=bit < 0, weights=w, tol=1e-13).x
    errs = {}
    for scaling in (1, 0):
        op = _operator(m, kind, small_n, scaling, keep_fp32=True)
        x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=bit, mode="mixed")
        assert info.status == 0
        x = x.cpu().numpy()
        if bit >= 0:
            assert oracle.relres(A, b, x, d) <= 1.01e-10
            assert np.all(x[d] == 0.0)
        else:
            r = b - A.matvec(x)
            r -= r.mean()
            assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
        errs[scaling] = _rel(x, ref)
        op.close()
    assert errs[1] <= 10 * errs[0] + 1e-12
    if errs[1] > 1e-9:
        # residual 1e-10 does not bound the error by 1e-9 (error <= kappa *
        # residual): the outer tolerance is tightened until it does
        op = _operator(m, kind, small_n, 1, keep_fp32=True)
        for tol in (1e-11, 1e-12):
            x, info = op.solve(_gpu(b, dev), tol=tol, mask_bit=bit, mode="mixed")
            assert info.status == 0
            errs[tol] = _rel(x.cpu().numpy(), ref)
            if errs[tol] <= 1e-9:
                break
        op.close()
    assert min(errs.values()) <= 1e-9, errs


@pytest.mark.parametrize("fmt", ["csr", "sell"])
def test_scaling_only_on_diagonal_storage(dev, fmt):
    """CSR and sliced ELL keep the unscaled recurrence: the tunable changes
    nothing there, bit for bit; on diagonal storage it changes the rounding."""
    m = basin.basin_mesh(20, 16, 5, seed=3)
    kind, A, d, b, w = _system(m, 0, 41)
    res = {}
    for f in (fmt, "sdia"):
        for scaling in (1, 0):
            op = _operator(m, kind, 0, scaling, fmt=f)
            x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=0)
            assert info.status == 0
            res[f, scaling] = x.cpu().numpy()
            op.close()
    assert np.array_equal(res[fmt, 1], res[fmt, 0])
    assert not np.array_equal(res["sdia", 1], res["sdia", 0])
    assert _rel(res["sdia", 1], res["sdia", 0]) <= 1e-10


def test_scaled_profiled_zero_rhs_and_bad_value(dev):
    from paper_1207_0486_amd.hns import HNSError
    m = basin.basin_mesh(20, 16, 5, seed=3)
    kind, A, d, b, w = _system(m, 1, 51)
    op = _operator(m, kind, 0, 1)
    # per-kernel timing of the scaled iteration (event-recorded launches)
    op.profile(1)
    x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=1)
    prof = op.profile_read()
    op.profile(0)
    assert info.status == 0 and oracle.relres(A, b, x.cpu().numpy(), d) <= 1.01e-10
    assert prof["spmv"][1] == info.iterations and prof["update"][1] == info.iterations
    # b = 0: x = 0 after no iteration, whatever the initial guess
    x, info = op.solve(_gpu(np.zeros(m.n), dev), x=_gpu(np.ones(m.n), dev), mask_bit=1)
    assert info.status == 0 and info.iterations == 0 and float(x.abs().max()) == 0.0
    with pytest.raises(HNSError):
        op.set_param("jacobi_scaling", 2)
    op.close()


# The fused form (fuse_dir): two launches per iteration, the direction update
# inside the next product with every neighbour's r + beta p recomputed where
# it is read, p alternating between two buffers.  Same arithmetic: answers,
# iteration counts and scalars equal the three-launch form's bit for bit,
# whichever buffer a chunk or a stop ends in (odd and one-iteration chunks,
# a budget that ends inside a chunk, the mixed recurrence whose direction is
# kept across residual replacements).
FUSE_CASES = [
    # (bit, mode, check_every, max_iter)
    (-1, "fp64", 32, 100000),
    (-1, "mixed", 32, 100000),
    (0, "fp64", 1, 100000),
    (2, "fp64", 3, 100000),
    (1, "mixed", 7, 100000),
    (-1, "fp64", 32, 37),
]


@pytest.mark.parametrize("rows", [1, 2])   # rows per lane of the FP64 products
@pytest.mark.parametrize("case", FUSE_CASES,
                         ids=[f"bit{c[0]}-{c[1]}-ce{c[2]}-max{c[3]}" for c in FUSE_CASES])
def test_fused_iterations_equal_three_launch_form(dev, case, rows):
    bit, mode, check_every, max_iter = case
    m = basin.basin_mesh(23, 17, 5, seed=7)   # 2,592 rows: ragged against every tile
    kind, A, d, b, w = _system(m, bit, 70 + bit)
    op = _operator(m, kind, 0, 1, keep_fp32=True)
    op.set_param("check_every", check_every)
    op.set_param("spmv_rows64", rows)
    got = {}
    for fuse in (0, 1):
        op.set_param("fuse_dir", fuse)
        x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=bit, mode=mode, max_iter=max_iter,
                           check=False)
        got[fuse] = (x, info)
    op.close()
    (x0, i0), (x1, i1) = got[0], got[1]
    assert i0.status == i1.status and i0.iterations == i1.iterations
    assert i0.outer_iterations == i1.outer_iterations
    assert torch.equal(x0, x1)
    if max_iter < 100000:
        assert i1.iterations == max_iter
    else:
        assert i1.status == 0
        ref = oracle.pcg(A, b, dirichlet=d, singular=bit < 0, weights=w, tol=1e-10)
        assert abs(i1.iterations - ref.iterations) <= max(1, 0.02 * ref.iterations)


@pytest.mark.parametrize("rows", [1, 2])
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_fused_iterations_tiny_mesh(dev, mode, rows):
    """A mesh whose rows all lie within the largest offset of an end (every
    row takes the per-row path of the product): the fused form still equals
    the three-launch form bit for bit."""
    m = basin.box_mesh(2, 2, 1)   # 18 rows, largest offset 9
    kind, A, d, b, w = _system(m, -1, 90)
    op = _operator(m, kind, 0, 1, keep_fp32=True)
    op.set_param("spmv_rows64", rows)
    assert op.format == "sdia" and op.n == 18
    got = {}
    for fuse in (0, 1):
        op.set_param("fuse_dir", fuse)
        got[fuse] = op.solve(_gpu(b, dev), tol=1e-10, mode=mode)
    op.close()
    (x0, i0), (x1, i1) = got[0], got[1]
    assert i0.status == i1.status == 0 and i0.iterations == i1.iterations
    assert torch.equal(x0, x1)


def test_fused_iterations_automatic_by_size(dev):
    """fuse_dir = -1 fuses while a vector takes at most 4 MiB: the timed
    kernels show two launches per iteration (no separate direction update)
    on a small operator, three when fusion is off; a bad value is refused."""
    from paper_1207_0486_amd.hns import HNSError
    m = basin.basin_mesh(23, 17, 5, seed=7)
    kind, A, d, b, w = _system(m, -1, 80)
    op = _operator(m, kind, 0, 1)
    counts = {}
    for fuse in (-1, 0):
        op.set_param("fuse_dir", fuse)
        op.profile(1)
        x, info = op.solve(_gpu(b, dev), tol=1e-10)
        prof = op.profile_read()
        op.profile(0)
        counts[fuse] = (prof["spmv"][1], prof["pupdate"][1], info.iterations)
    assert counts[-1][0] > 0 and counts[-1][1] == 0
    assert counts[0][0] > 0 and counts[0][1] > 0
    assert counts[-1][2] == counts[0][2]
    with pytest.raises(HNSError):
        op.set_param("fuse_dir", 2)
    op.close()


def test_launch_shapes_keep_the_answer(dev):
    """Rows per lane of the FP64 product, passes of the FP32 product and
    packs of the vector updates change the grid (and the summation order of
    the dot products) only: every shape converges in the oracle's
    iteration count to the same answer within the parity tolerance, and bad
    values are refused."""
    from paper_1207_0486_amd.hns import HNSError
    m = basin.basin_mesh(23, 17, 5, seed=7)
    kind, A, d, b, w = _system(m, 0, 95)
    ref = oracle.pcg(A, b, dirichlet=d, tol=1e-10)
    op = _operator(m, kind, 0, 1, keep_fp32=True)
    for mode in ("fp64", "mixed"):
        xs = []
        for rows, it32, vec in ((0, 0, 0), (2, 2, 3), (1, 1, 1), (2, 4, 2)):
            op.set_param("spmv_rows64", rows)
            op.set_param("spmv_it32", it32)
            op.set_param("vec_it", vec)
            x, info = op.solve(_gpu(b, dev), tol=1e-10, mask_bit=0, mode=mode)
            assert info.status == 0
            assert abs(info.iterations - ref.iterations) <= max(1, 0.02 * ref.iterations) \
                or mode == "mixed"
            xs.append(x.cpu().numpy())
        for x in xs[1:]:
            assert _rel(x, xs[0]) <= 1e-9
    for name, bad in (("spmv_rows64", 3), ("spmv_it32", -1), ("vec_it", 65)):
        with pytest.raises(HNSError):
            op.set_param(name, bad)
    op.close()
