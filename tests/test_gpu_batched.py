"""Multi-right-hand-side solves: columns against single solves and the oracle,
graph replay against eager launches, pack widths, status per column."""
import numpy as np
import pytest

import basin
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mesh():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return basin.basin_mesh(24, 20, 6, seed=4)


def _rhs_block(m, bits, seed0):
    cols = []
    for j, bit in enumerate(bits):
        d = None if bit < 0 else ((m.bc >> bit) & 1) == 1
        cols.append(basin.normal_rhs(m.n, seed0 + j, dirichlet=d))
    return np.ascontiguousarray(np.stack(cols, axis=1))


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _rel(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("vec", [1, 2, 4])
def test_batched_helmholtz_fp64_matches_oracle(mesh, vec):
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [0, 1, 2, 0, 1, 2, 0, 1]
    B = _rhs_block(m, bits, 100)
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz")
    op.set_param("bspmm_vec", vec)
    X, infos = op.solve_batched(_t(B), mask_bits=bits, tol=1e-10)
    Xh = X.cpu().numpy()
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    for j, bit in enumerate(bits):
        d = ((m.bc >> bit) & 1) == 1
        ref = oracle.pcg(A, B[:, j], dirichlet=d, tol=1e-10)
        assert infos[j].status == 0 and infos[j].relres_true <= 1e-10
        assert abs(infos[j].iterations - ref.iterations) <= 1
        assert np.all(Xh[d, j] == 0)
        assert oracle.relres(A, B[:, j], Xh[:, j], d) <= 1.01e-10
        same = oracle.pcg(A, B[:, j], dirichlet=d, tol=1e-300, maxit=infos[j].iterations)
        assert _rel(Xh[:, j], same.x) <= 1e-10


def test_batched_columns_equal_single_solves(mesh):
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [0, 1, 2]
    B = _rhs_block(m, bits, 200)
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz")
    X, infos = op.solve_batched(_t(B), mask_bits=bits, tol=1e-10)
    for j, bit in enumerate(bits):
        x1, i1 = op.solve(_t(B[:, j]), tol=1e-10, mask_bit=bit)
        assert abs(i1.iterations - infos[j].iterations) <= 1
        assert _rel(X[:, j].cpu().numpy(), x1.cpu().numpy()) <= 1e-10


def test_batched_poisson_neumann(mesh):
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [-1] * 4
    B = _rhs_block(m, bits, 300)
    op = Operator(m, 1e3, 1e-2, kind="poisson", keep_fp32=True)
    K = oracle.stiffness(m, 1e3, 1e-2)
    w = oracle.mass(m).matvec(np.ones(m.n))
    for mode in ("fp64", "mixed"):
        X, infos = op.solve_batched(_t(B), mask_bits=bits, tol=1e-10, mode=mode)
        Xh = X.cpu().numpy()
        for j in range(len(bits)):
            exact = oracle.pcg(K, B[:, j], singular=True, weights=w, tol=1e-13)
            ref = oracle.pcg(K, B[:, j], singular=True, weights=w, tol=1e-10)
            assert infos[j].status == 0, (mode, j, infos[j])
            assert infos[j].iterations <= 1.35 * ref.iterations + 4, (mode, j, infos[j])
            assert infos[j].removed_mean == pytest.approx(B[:, j].mean(), rel=1e-12)
            assert abs(w @ Xh[:, j]) <= 1e-12 * np.abs(w).sum() * np.abs(Xh[:, j]).max()
            assert _rel(Xh[:, j], exact.x) <= 1e-9


def test_batched_mixed_matches_tight_oracle(mesh):
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [0, 1, 2] * 4
    B = _rhs_block(m, bits, 400)
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    X, infos = op.solve_batched(_t(B), mask_bits=bits, tol=1e-10, mode="mixed")
    Xh = X.cpu().numpy()
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    for j, bit in enumerate(bits):
        d = ((m.bc >> bit) & 1) == 1
        exact = oracle.pcg(A, B[:, j], dirichlet=d, tol=1e-13)
        ref = oracle.pcg(A, B[:, j], dirichlet=d, tol=1e-10)
        assert infos[j].status == 0 and infos[j].relres_true <= 1e-10
        # the replacement keeps the Krylov recurrence: about as many FP32
        # iterations as FP64 ones
        assert infos[j].iterations <= 1.25 * ref.iterations + 4, (j, infos[j], ref.iterations)
        assert _rel(Xh[:, j], exact.x) <= 1e-9


def test_graph_replay_equals_eager(mesh):
    """Captured chunks replay the same kernels: results are bitwise equal, over
    several replays interleaved with eager work."""
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [0, 1, 2, 0]
    B = _t(_rhs_block(m, bits, 500))
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    op.set_param("check_every", 8)
    for mode in ("fp64", "mixed"):
        op.set_param("use_graph", 0)
        X0, i0 = op.solve_batched(B, mask_bits=bits, tol=1e-10, mode=mode)
        op.set_param("use_graph", 1)
        for rep in range(3):
            X1, i1 = op.solve_batched(B, mask_bits=bits, tol=1e-10, mode=mode)
            torch.cuda.synchronize()
            assert torch.equal(X0, X1), (mode, rep)
            assert [a.iterations for a in i0] == [a.iterations for a in i1]
            _ = (B * 2.0).sum().item()  # eager work between replays


def test_zero_and_nonfinite_columns(mesh):
    from paper_1207_0486_amd.hns import Operator, HNSError
    m = mesh
    bits = [0, 1, 2]
    B = _rhs_block(m, bits, 600)
    B[:, 1] = 0.0
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz")
    X0 = _t(np.random.default_rng(1).standard_normal(B.shape))
    X, infos = op.solve_batched(_t(B), X=X0.clone(), mask_bits=bits, tol=1e-10)
    assert [i.status for i in infos] == [0, 0, 0]
    assert infos[1].iterations == 0 and float(X[:, 1].abs().max()) == 0.0
    free = np.flatnonzero((m.bc & 1) == 0)
    B[free[3], 0] = np.nan
    with pytest.raises(HNSError) as e:
        op.solve_batched(_t(B), mask_bits=bits, tol=1e-10)
    assert e.value.status == -1


def test_iteration_cap_per_column(mesh):
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [0, 0]
    B = _rhs_block(m, bits, 700)
    op = Operator(m, 1e3, 1e-2, kind="poisson")
    X, infos = op.solve_batched(_t(B), mask_bits=bits, tol=1e-10, max_iter=5, check=False)
    A = oracle.stiffness(m, 1e3, 1e-2)
    for j in range(2):
        d = (m.bc & 1) == 1
        ref = oracle.pcg(A, B[:, j], dirichlet=d, tol=1e-300, maxit=5)
        assert infos[j].status == 1 and infos[j].iterations == 5
        assert _rel(X[:, j].cpu().numpy(), ref.x) <= 1e-12


@pytest.mark.parametrize("k", [1, 3, 5, 48])
def test_odd_column_counts_and_tuner(mesh, k):
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [j % 3 for j in range(k)]
    B = _rhs_block(m, bits, 800)
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    times, plan = op.tune_batched(k, "mixed")
    V, tile = plan & 7, plan >> 3
    assert f"w{V}" in times and all(t > 0 for t in times.values())
    assert "w1" in times and ("w2" in times) == (k % 2 == 0) and ("w4" in times) == (k % 4 == 0)
    # FP32 tiles: shapes of 32, 16 and 16 columns
    assert ("tile1" in times) == (k % 32 == 0) and ("tile3" in times) == (k % 16 == 0)
    assert tile == 0 or (f"tile{tile}" in times
                         and times[f"tile{tile}"] == min(times.values()))
    X, infos = op.solve_batched(_t(B), mask_bits=bits, tol=1e-10, mode="mixed")
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    for j in (0, k - 1):
        d = ((m.bc >> bits[j]) & 1) == 1
        assert infos[j].status == 0
        assert oracle.relres(A, B[:, j], X[:, j].cpu().numpy(), d) <= 1.01e-10


def test_graph_cache_is_keyed_by_precision(mesh):
    """A pooled workspace serves both precisions: alternating mixed and FP64
    batched solves with graphs must replay the graph of the right precision
    (the freed X block is typically handed back at the same address)."""
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [0, 1, 2, 0]
    B = _t(_rhs_block(m, bits, 900))
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    op.set_param("check_every", 4)
    op.set_param("use_graph", 1)
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    for mode in ("mixed", "fp64", "mixed", "fp64"):
        X, infos = op.solve_batched(B, mask_bits=bits, tol=1e-10, mode=mode, max_iter=500)
        assert all(i.status == 0 for i in infos), (mode, infos)
        assert max(i.iterations for i in infos) < 200
        Xh = X.cpu().numpy()
        for j, bit in enumerate(bits):
            d = ((m.bc >> bit) & 1) == 1
            assert oracle.relres(A, B[:, j].cpu().numpy(), Xh[:, j], d) <= 1.01e-10
        del X


def test_graph_capture_while_other_threads_allocate(mesh):
    """Batched solves capture their iteration chunks while another thread
    allocates device memory and copies synchronously (as the serving loop does
    when it assembles operators): captures stay valid and results match."""
    import threading
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [0, 1, 2, 0]
    B = _t(_rhs_block(m, bits, 950))
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    op.set_param("check_every", 4)
    op.set_param("use_graph", 0)
    X0, _ = op.solve_batched(B, mask_bits=bits, tol=1e-10, mode="mixed")
    op.set_param("use_graph", 1)
    stop = threading.Event()

    def churn():
        while not stop.is_set():
            other = Operator(basin.basin_mesh(6, 5, 2, seed=1), 1.0, 1.0, 1.0, kind="helmholtz")
            t = torch.randn(1 << 16, dtype=torch.float64, device="cuda")
            _ = t.cpu()
            other.close()

    th = threading.Thread(target=churn)
    th.start()
    try:
        for _ in range(4):
            X1, infos = op.solve_batched(B, mask_bits=bits, tol=1e-10, mode="mixed")
            assert all(i.status == 0 for i in infos)
            assert torch.equal(X0, X1)
    finally:
        stop.set()
        th.join()


@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_tiled_product_columns_match_oracle(mesh, tile, mode):
    """The LDS-tiled product (each tile shape; 32 columns, 3,675 rows: a
    ragged last tile) in the whole batched solve: FP64 columns equal the
    oracle's iterate after as many iterations and the grid-stride product's
    answer; mixed columns meet the tolerance by the oracle's residual and
    agree with the grid-stride mixed solve."""
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [j % 3 for j in range(32)]
    B = _t(_rhs_block(m, bits, 1000))
    op = Operator(m, 1e3, 1e-2, 3600.0, kind="helmholtz", keep_fp32=True)
    op.set_param("bspmm_vec", 4)
    op.set_param("bspmm_tile", 0)
    X0, i0 = op.solve_batched(B, mask_bits=bits, tol=1e-10, mode=mode)
    op.set_param("bspmm_tile", tile)
    X1, i1 = op.solve_batched(B, mask_bits=bits, tol=1e-10, mode=mode)
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    X0h, X1h, Bh = X0.cpu().numpy(), X1.cpu().numpy(), B.cpu().numpy()
    for j, bit in enumerate(bits):
        d = ((m.bc >> bit) & 1) == 1
        assert i1[j].status == 0
        assert oracle.relres(A, Bh[:, j], X1h[:, j], d) <= 1.01e-10
        assert np.all(X1h[d, j] == 0)
        assert _rel(X1h[:, j], X0h[:, j]) <= 1e-10
        if mode == "fp64" and j in (0, 13, 31):
            same = oracle.pcg(A, Bh[:, j], dirichlet=d, tol=1e-300, maxit=i1[j].iterations)
            assert _rel(X1h[:, j], same.x) <= 1e-10


def test_tiled_product_neumann_columns(mesh):
    """Pure-Neumann columns through the tiled product (Poisson operator, 16
    columns, FP32 shape 3 and FP64 shape 1)."""
    from paper_1207_0486_amd.hns import Operator
    m = mesh
    bits = [-1] * 16
    B = _t(_rhs_block(m, bits, 1100))
    K = oracle.stiffness(m, 1e3, 1e-2)
    w = oracle.mass(m).matvec(np.ones(m.n))
    op = Operator(m, 1e3, 1e-2, kind="poisson", keep_fp32=True)
    op.set_param("bspmm_vec", 4)
    for mode, tile in (("fp64", 1), ("mixed", 3)):
        op.set_param("bspmm_tile", tile)
        X, infos = op.solve_batched(B, mask_bits=bits, tol=1e-10, mode=mode)
        Xh, Bh = X.cpu().numpy(), B.cpu().numpy()
        for j in (0, 7, 15):
            assert infos[j].status == 0
            bh = Bh[:, j] - Bh[:, j].mean()
            r = bh - K.matvec(Xh[:, j])
            r -= r.mean()
            assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(bh)
            assert abs(w @ Xh[:, j]) <= 1e-12 * np.abs(w).sum() * np.abs(Xh[:, j]).max()
