"""Pins of the oracle's vertical-line (water column) block preconditioner.

The column solve is pinned to a library banded solver; the line-preconditioned
CG is pinned by special cases that reduce to something known: columns of one
node are the point Jacobi preconditioner, an operator with only vertical
couplings is inverted exactly by its column blocks, and on small meshes the
converged result equals a dense direct solve.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import basin
import oracle


def _spd_tridiag(rng, L):
    e = rng.standard_normal(L - 1)
    pad = np.concatenate([[0.0], np.abs(e)]) + np.concatenate([np.abs(e), [0.0]])
    d = pad + rng.uniform(0.1, 2.0, L)
    return d, e


@pytest.mark.parametrize("L", [1, 2, 3, 7, 21, 64])
def test_tridiag_solve_matches_banded_solver(L):
    """Thomas solve against scipy.linalg.solve_banded on diagonally dominant
    symmetric tridiagonal systems."""
    rng = np.random.default_rng(L)
    for _ in range(5):
        d, e = _spd_tridiag(rng, L)
        r = rng.standard_normal(L)
        ab = np.zeros((3, L))
        ab[1] = d
        ab[0, 1:] = e
        ab[2, :-1] = e
        want = sl.solve_banded((1, 1), ab, r)
        got = oracle.tridiag_solve(d, e, r)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_tridiag_solve_is_the_inverse_and_symmetric():
    """T z = r holds row by row, and u^T T^-1 v = v^T T^-1 u (the block
    inverse is symmetric, as CG needs of a preconditioner)."""
    rng = np.random.default_rng(11)
    d, e = _spd_tridiag(rng, 9)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    u, v = rng.standard_normal(9), rng.standard_normal(9)
    zu, zv = oracle.tridiag_solve(d, e, u), oracle.tridiag_solve(d, e, v)
    assert np.abs(T @ zu - u).max() <= 1e-13 * np.abs(u).max()
    assert v @ zu == pytest.approx(u @ zv, rel=1e-13)


def test_tridiag_solve_rejects_indefinite():
    with pytest.raises(oracle.OracleError):
        oracle.tridiag_solve(np.array([1.0, 0.5]), np.array([2.0]), np.ones(2))


def test_line_of_one_node_is_point_jacobi():
    """Columns of one node: z = (1/d) r, the Jacobi preconditioner, bitwise."""
    m = basin.box_mesh(8, 8, 3)
    A = oracle.helmholtz(m, 1.0, 1e-4, 0.1)
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 3, dirichlet=d)
    r0 = oracle.pcg(A, b, dirichlet=d, tol=1e-12)
    r1 = oracle.pcg(A, b, dirichlet=d, tol=1e-12, line=1)
    assert r0.status == 0 and r1.status == 0
    assert r0.iterations == r1.iterations
    assert np.array_equal(r0.x, r1.x)


def test_vertical_only_operator_is_solved_in_one_iteration():
    """On an axis-aligned box every Kuhn tet has one edge per axis, so with
    nu_h = 0 the stiffness couples a node only to its vertical neighbours:
    the matrix is its own column-block diagonal, the line preconditioner is
    its exact inverse, and CG stops after one iteration."""
    m = basin.box_mesh(6, 5, 7)
    K = oracle.stiffness(m, 0.0, 1.0)
    Kd = K.to_scipy().toarray()
    L = m.Nz + 1
    for i in range(m.n):          # the pattern claim itself, exactly
        c = i // L
        off = [j for j in np.flatnonzero(Kd[i]) if j // L != c]
        assert not off
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 4, dirichlet=d)
    r = oracle.pcg(K, b, dirichlet=d, tol=1e-12, line=L)
    assert r.status == 0 and r.iterations == 1
    assert oracle.relres(K, b, r.x, d) <= 1e-13


def _free_direct(A, b, d):
    Ad = A.to_scipy().toarray()
    free = ~d
    x = np.zeros(A.n)
    x[free] = np.linalg.solve(Ad[np.ix_(free, free)], b[free])
    return x


def test_line_pcg_matches_direct_solve_isotropic_dirichlet():
    """Isotropic Laplacian (the pressure form of the paper, nu = 1) with
    Dirichlet bottom and walls on a thin box: converged line-PCG equals the
    dense solve of the free block."""
    m = basin.box_mesh(8, 8, 4, H=0.01)
    K = oracle.stiffness(m, 1.0, 1.0)
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 8, dirichlet=d)
    want = _free_direct(K, b, d)
    r = oracle.pcg(K, b, dirichlet=d, tol=1e-13, line=m.Nz + 1)
    assert r.status == 0
    assert np.linalg.norm(r.x - want) <= 1e-11 * np.linalg.norm(want)


def test_line_pcg_matches_pseudo_inverse_pure_neumann():
    """Pure-Neumann isotropic Laplacian on a small closed box: the normalised
    line-PCG answer equals the minimum-norm least-squares solution shifted to
    zero mass-weighted mean."""
    m = basin.box_mesh(6, 5, 3, H=0.05, gamma0=())
    K = oracle.stiffness(m, 1.0, 1.0)
    w = oracle.mass(m).matvec(np.ones(m.n))
    b = basin.normal_rhs(m.n, 9, zero_mean=True)
    r = oracle.pcg(K, b, singular=True, weights=w, tol=1e-12, line=m.Nz + 1)
    assert r.status == 0
    y = np.linalg.lstsq(K.to_scipy().toarray(), b - b.mean(), rcond=None)[0]
    y -= (w @ y) / w.sum()
    assert np.linalg.norm(r.x - y) <= 1e-11 * np.linalg.norm(y)
    assert abs(w @ r.x) <= 1e-12 * np.abs(w).sum() * np.abs(r.x).max()


def test_line_pcg_energy_error_decreases():
    """With a symmetric positive definite preconditioner CG's A-norm error
    decreases at every iteration."""
    m = basin.basin_mesh(8, 8, 4, seed=5)
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 6, dirichlet=d)
    exact = _free_direct(A, b, d)
    r = oracle.pcg(A, b, dirichlet=d, tol=1e-300, maxit=12, x_history=True, line=m.Nz + 1)
    Ad = A.to_scipy().toarray()
    free = ~d
    errs = []
    for x in r.x_hist:
        e = (x - exact)[free]
        errs.append(e @ Ad[np.ix_(free, free)] @ e)
    assert all(b2 < a2 for a2, b2 in zip(errs, errs[1:]))


def test_line_beats_point_on_thin_isotropic_basin():
    """The isotropic pressure Laplacian on a thin basin (horizontal cells
    ~300 km, layers 10-900 m): point Jacobi needs thousands of iterations,
    the column blocks about a hundred, to the same answer."""
    m = basin.basin_mesh(16, 16, 6, seed=3)
    K = oracle.stiffness(m, 1.0, 1.0)
    w = oracle.mass(m).matvec(np.ones(m.n))
    b = basin.normal_rhs(m.n, 5, zero_mean=True)
    rl = oracle.pcg(K, b, singular=True, weights=w, tol=1e-8, line=m.Nz + 1)
    rp = oracle.pcg(K, b, singular=True, weights=w, tol=1e-8, maxit=20000)
    assert rl.status == 0 and rp.status == 0
    assert rl.iterations * 10 < rp.iterations
    assert np.linalg.norm(rl.x - rp.x) <= 1e-6 * np.linalg.norm(rl.x)


def test_line_len_must_divide_n():
    m = basin.box_mesh(4, 4, 2)
    K = oracle.stiffness(m, 1.0, 1.0)
    d = (m.bc & 1) == 1
    r = oracle.pcg(K, np.ones(m.n), dirichlet=d, line=4)   # n = 75
    assert r.status == oracle.ERR_INVALID


def test_first_iterate_uses_the_column_block_inverse():
    """x_1 = alpha_0 M^-1 b with alpha_0 = (b^T M^-1 b) / (p^T A p), where M is
    the block diagonal of the eliminated matrix on the water columns (identity
    rows and columns at Dirichlet nodes), each block inverted densely here."""
    m = basin.basin_mesh(5, 4, 4, seed=7)
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    d = ((m.bc >> 2) & 1) == 1
    b = basin.normal_rhs(m.n, 12, dirichlet=d)
    L = m.Nz + 1
    Ad = A.to_scipy().toarray()
    Ad[d, :] = 0.0
    Ad[:, d] = 0.0
    Ad[d, d] = 1.0
    Minv = np.zeros_like(Ad)
    for c0 in range(0, m.n, L):
        blk = np.zeros((L, L))
        for k in range(L):
            blk[k, k] = Ad[c0 + k, c0 + k]
            if k + 1 < L:
                blk[k, k + 1] = blk[k + 1, k] = Ad[c0 + k, c0 + k + 1]
        Minv[c0:c0 + L, c0:c0 + L] = np.linalg.inv(blk)
    p = Minv @ b
    alpha = (b @ p) / (p @ Ad @ p)
    r = oracle.pcg(A, b, dirichlet=d, tol=1e-300, maxit=1, x_history=True, line=L)
    assert np.abs(r.x_hist[0] - alpha * p).max() <= 1e-12 * np.abs(alpha * p).max()
