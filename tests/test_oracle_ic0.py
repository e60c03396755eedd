"""Pins of the oracle's IC(0) preconditioner in the greedy multicolour order.

IC(0) is defined by its pattern (that of the lower triangle of the permuted
matrix) and by (L L^T)_ij = B_ij on that pattern; the colouring by having no
two neighbours of one colour.  Both are checked with dense algebra, and the
preconditioned CG against dense solves and its own first iterate."""
import numpy as np
import pytest

import basin
import oracle


def _eliminated_dense(A, d):
    Ad = A.to_scipy().toarray()
    if d is not None:
        Ad[d, :] = 0.0
        Ad[:, d] = 0.0
        Ad[d, d] = 1.0
    return Ad


@pytest.fixture(scope="module")
def case():
    m = basin.basin_mesh(7, 6, 3, seed=4)
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    d = ((m.bc >> 1) & 1) == 1
    return m, A, d


def test_greedy_colouring_is_proper(case):
    m, A, _ = case
    color, k = oracle.greedy_colors(A)
    S = A.to_scipy().tocoo()
    off = S.row != S.col
    assert np.all(color[S.row[off]] != color[S.col[off]])
    assert k == color.max() + 1
    assert k <= 8          # the 15-point Kuhn stencil: the 8 parity classes suffice
    # greedy: every colour below a node's own is taken by a lower neighbour
    for i in range(m.n):
        lower = {color[j] for j in S.col[(S.row == i) & (S.col < i)]}
        assert set(range(color[i])) <= lower


def test_ic0_pattern_and_defining_identity(case):
    m, A, d = case
    perm, L = oracle.ic0_factor(A, d)
    assert sorted(perm) == list(range(m.n))
    B = _eliminated_dense(A, d)[np.ix_(perm, perm)]
    Ld = L.to_scipy().toarray()
    assert np.all(np.triu(Ld, 1) == 0)
    low = np.tril(B) != 0
    assert np.all((Ld != 0) <= low)            # no fill: the pattern of tril(B)
    assert np.all(np.diag(Ld) > 0)
    LLt = Ld @ Ld.T
    assert np.abs((LLt - B)[low]).max() <= 1e-13 * np.abs(B).max()


def test_ic0_first_iterate_uses_the_factor(case):
    """x_1 = alpha_0 M^-1 b with M = P^T L L^T P formed densely."""
    m, A, d = case
    b = basin.normal_rhs(m.n, 12, dirichlet=d)
    perm, L = oracle.ic0_factor(A, d)
    Ld = L.to_scipy().toarray()
    Minv = np.zeros((m.n, m.n))
    inv = np.linalg.inv(Ld @ Ld.T)
    Minv[np.ix_(perm, perm)] = inv
    Ad = _eliminated_dense(A, d)
    p = Minv @ b
    alpha = (b @ p) / (p @ Ad @ p)
    r = oracle.pcg(A, b, dirichlet=d, tol=1e-300, maxit=1, x_history=True, ic0=True)
    assert np.abs(r.x_hist[0] - alpha * p).max() <= 1e-12 * np.abs(alpha * p).max()


def test_ic0_pcg_converges_to_the_direct_solution(case):
    m, A, d = case
    b = basin.normal_rhs(m.n, 13, dirichlet=d)
    Ad = _eliminated_dense(A, d)
    want = np.linalg.solve(Ad, np.where(d, 0.0, b))
    r = oracle.pcg(A, b, dirichlet=d, tol=1e-13, ic0=True)
    assert r.status == oracle.OK
    assert np.linalg.norm(r.x - want) <= 1e-11 * np.linalg.norm(want)
    h = oracle.pcg(A, b, dirichlet=d, tol=1e-300, maxit=r.iterations, x_history=True, ic0=True)
    errs = [(x - want) @ Ad @ (x - want) for x in h.x_hist]
    assert all(b2 < a2 for a2, b2 in zip(errs, errs[1:]) if a2 > 1e-28)


def test_ic0_needs_fewer_iterations_than_jacobi():
    m = basin.basin_mesh(24, 20, 6, seed=4)
    for nu_h, nu_v, dt in ((1e3, 1e-2, 3600.0), (1e8, 250.0, 2.592e6 * 2 / 3)):
        A = oracle.helmholtz(m, nu_h, nu_v, dt)
        d = (m.bc & 1) == 1
        b = basin.normal_rhs(m.n, 40, dirichlet=d)
        rj = oracle.pcg(A, b, dirichlet=d, tol=1e-10)
        ri = oracle.pcg(A, b, dirichlet=d, tol=1e-10, ic0=True)
        assert ri.status == 0 and 2 * ri.iterations < rj.iterations + 2
        assert np.linalg.norm(ri.x - rj.x) <= 1e-8 * np.linalg.norm(rj.x)
