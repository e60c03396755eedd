"""Pins of the oracle's brick elements (Q1 pressure / Q2 velocity spaces of
Sec. 5) against facts fixed by the mathematics, not by the oracle itself:

- on a box element the forms separate: the 3D matrices are Kronecker products
  of the textbook 1D Lagrange mass and stiffness matrices;
- the mass matrix integrates 1 to the exact volume of a brick whose vertical
  edges stand over a rectangle (bilinear top and bottom);
- the coordinate functions x_c lie in both spaces, so x_c^T K_nu x_d equals
  nu_c delta_cd times the volume on any (non-affine) mesh;
- Q2 reproduces quadratics on boxes (closed-form integrals of x^2, x);
- PCG on the assembled operators equals a dense direct solve;
- a manufactured solution converges at the rates the element orders give.
"""
import numpy as np
import pytest

import basin
import oracle

M1_1D = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
K1_1D = np.array([[1.0, -1.0], [-1.0, 1.0]])
M2_1D = np.array([[4.0, 2.0, -1.0], [2.0, 16.0, 2.0], [-1.0, 2.0, 4.0]]) / 30.0
K2_1D = np.array([[7.0, -8.0, 1.0], [-8.0, 16.0, -8.0], [1.0, -8.0, 7.0]]) / 3.0


def _box_corners(x0, h):
    return np.array([[x0[0] + (c & 1) * h[0], x0[1] + ((c >> 1) & 1) * h[1],
                      x0[2] + (c >> 2) * h[2]] for c in range(8)])


@pytest.mark.parametrize("order", [1, 2])
def test_box_element_is_a_kronecker_product_of_1d_matrices(order):
    """Local node (a, b, c) with a fastest: M = Mz (x) My (x) Mx and
    K = nu1 Mz(x)My(x)Kx + nu2 Mz(x)Ky(x)Mx + nu3 Kz(x)My(x)Mx, the 1D
    matrices of the Lagrange elements of degree `order` scaled to each side."""
    h = np.array([0.7, 1.3, 0.05])
    nu = np.array([2.0, 3.0, 1e-3])
    K, M, det = oracle.hex_element(order, _box_corners([0.3, -1.0, -0.2], h), nu)
    m1, k1 = (M1_1D, K1_1D) if order == 1 else (M2_1D, K2_1D)
    Mx, My, Mz = (m1 * s for s in h)
    Kx, Ky, Kz = (k1 / s for s in h)
    Mw = np.kron(Mz, np.kron(My, Mx))
    Kw = (nu[0] * np.kron(Mz, np.kron(My, Kx)) + nu[1] * np.kron(Mz, np.kron(Ky, Mx))
          + nu[2] * np.kron(Kz, np.kron(My, Mx)))
    assert np.abs(M - Mw).max() <= 1e-14 * np.abs(Mw).max()
    assert np.abs(K - Kw).max() <= 1e-12 * np.abs(Kw).max()
    assert det == pytest.approx(np.prod(h) / 8.0, rel=1e-14)


def test_q1_unit_cube_stiffness_textbook_row():
    """The trilinear Laplacian on the unit cube: 12 K row of a corner =
    (4, 0, 0, -1, 0, -1, -1, -1) in the corner order (x fastest)."""
    K, _, _ = oracle.hex_element(1, _box_corners([0, 0, 0], [1, 1, 1]))
    assert np.abs(12.0 * K[0] - [4, 0, 0, -1, 0, -1, -1, -1]).max() <= 1e-14


def _column_brick(rng):
    """Corners over [0,hx]x[0,hy] with vertical edges, random bottom and top."""
    hx, hy = rng.uniform(0.5, 2.0, 2)
    bot = rng.uniform(-3.0, -2.0, 4)
    top = rng.uniform(-1.0, 0.0, 4)
    X8 = np.zeros((8, 3))
    for c in range(8):
        i, j, k = c & 1, (c >> 1) & 1, c >> 2
        X8[c] = [i * hx, j * hy, (top if k else bot)[i + 2 * j]]
    vol = hx * hy * np.mean(top - bot)     # bilinear thickness, exact mean
    return X8, vol


@pytest.mark.parametrize("order", [1, 2])
def test_mass_integrates_one_to_the_exact_volume(order):
    rng = np.random.default_rng(order)
    for _ in range(5):
        X8, vol = _column_brick(rng)
        K, M, det = oracle.hex_element(order, X8, (1.0, 2.0, 0.5))
        assert det > 0
        assert M.sum() == pytest.approx(vol, rel=1e-13)
        assert np.abs(K.sum(axis=1)).max() <= 1e-12 * np.abs(K).max()   # constants
        assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
        assert np.linalg.eigvalsh(M).min() > 0
        assert np.linalg.eigvalsh(K).min() >= -1e-12 * np.abs(K).max()


def _reference_nodes(order):
    t = np.linspace(-1.0, 1.0, order + 1)
    q = order + 1
    pts = np.zeros((q ** 3, 3))
    for c in range(q):
        for b in range(q):
            for a in range(q):
                pts[a + q * b + q * q * c] = [t[a], t[b], t[c]]
    return pts


def _trilinear(X8, s):
    out = np.zeros((s.shape[0], 3))
    for c in range(8):
        w = np.ones(s.shape[0])
        for d, bit in enumerate((c & 1, (c >> 1) & 1, c >> 2)):
            w *= 0.5 * (1.0 + (1.0 if bit else -1.0) * s[:, d])
        out += w[:, None] * X8[c]
    return out


@pytest.mark.parametrize("order", [1, 2])
def test_coordinate_energy_identity_on_a_skewed_brick(order):
    """x_c (nodal values at the images of the reference nodes) lies in the
    space on any trilinear brick, grad x_c = e_c, so x_c^T K_nu x_d =
    nu_c delta_cd |K| and 1^T M x_c = int x_c."""
    rng = np.random.default_rng(10 + order)
    X8 = _box_corners([0, 0, 0], [1, 1, 1]) + rng.uniform(-0.15, 0.15, (8, 3))
    nu = np.array([1.5, 0.25, 4.0])
    K, M, det = oracle.hex_element(order, X8, nu)
    assert det > 0
    vol = M.sum()
    X = _trilinear(X8, _reference_nodes(order))
    E = X.T @ K @ X
    assert np.abs(E - np.diag(nu) * vol).max() <= 1e-12 * nu.max() * vol


def test_q2_reproduces_quadratics_on_a_box():
    """On [x0, x0+hx] x ... the Q2 interpolant of x^2 is exact: x^T K x^2 =
    nu1 int 2x, (x^2)^T K x^2 = nu1 int 4x^2, 1^T M x^2 = int x^2."""
    x0, h = np.array([0.5, -0.25, -1.0]), np.array([1.5, 0.8, 0.3])
    nu = (2.0, 1.0, 1.0)
    K, M, _ = oracle.hex_element(2, _box_corners(x0, h), nu)
    X = _trilinear(_box_corners(x0, h), _reference_nodes(2))
    x, a, b = X[:, 0], x0[0], x0[0] + h[0]
    area = h[1] * h[2]
    int_x = (b ** 2 - a ** 2) / 2 * area
    int_x2 = (b ** 3 - a ** 3) / 3 * area
    assert x @ K @ x ** 2 == pytest.approx(nu[0] * 2 * int_x, rel=1e-12)
    assert x ** 2 @ K @ x ** 2 == pytest.approx(nu[0] * 4 * int_x2, rel=1e-12)
    assert np.ones(27) @ M @ x ** 2 == pytest.approx(int_x2, rel=1e-13)


def test_q1_reproduces_bilinear_xy_on_a_box():
    x0, h = np.array([0.2, 0.1, -0.5]), np.array([1.0, 2.0, 0.5])
    nu = (1.0, 3.0, 7.0)
    K, _, _ = oracle.hex_element(1, _box_corners(x0, h), nu)
    X = _trilinear(_box_corners(x0, h), _reference_nodes(1))
    u = X[:, 0] * X[:, 1]
    a, b, c, d = x0[0], x0[0] + h[0], x0[1], x0[1] + h[1]
    want = h[2] * (nu[0] * (b - a) * (d ** 3 - c ** 3) / 3 + nu[1] * (d - c) * (b ** 3 - a ** 3) / 3)
    assert u @ K @ u == pytest.approx(want, rel=1e-12)


def _mesh_volume(m):
    """Volume of the basin brick mesh: per cell, the rectangle times the mean
    of the four corner depths (bilinear top and bottom)."""
    p = m.order
    My = p * m.Ny + 1
    hc = m.depth.reshape(p * m.Nx + 1, My)[::p, ::p]
    cell = 0.25 * (hc[:-1, :-1] + hc[1:, :-1] + hc[:-1, 1:] + hc[1:, 1:])
    return cell.sum() * (m.Lx / m.Nx) * (m.Ly / m.Ny)


@pytest.mark.parametrize("order", [1, 2])
def test_assembled_basin_operators(order):
    m = basin.basin_hex_mesh(6, 5, 3, order, seed=3)
    vol = _mesh_volume(m)
    M = oracle.hex_mass(m)
    assert M.to_scipy().sum() == pytest.approx(vol, rel=1e-12)
    nu = (1e3, 1e3, 1e-2)
    K = oracle.hex_stiffness(m, nu[0], nu[2])
    Ks = K.to_scipy()
    assert abs(Ks - Ks.T).max() == 0.0 or abs(Ks - Ks.T).max() <= 1e-15 * abs(Ks).max()
    assert np.abs(K.matvec(np.ones(m.n))).max() <= 1e-11 * abs(Ks).max()
    E = np.array([[m.xyz[:, c] @ K.matvec(m.xyz[:, d]) for d in range(3)] for c in range(3)])
    assert np.abs(E - np.diag(nu) * vol).max() <= 1e-10 * max(nu) * vol
    A = oracle.hex_helmholtz(m, nu[0], nu[2], 3600.0)
    diff = A.to_scipy() - (M.to_scipy() + 3600.0 * Ks)
    assert abs(diff).max() <= 1e-15 * abs(A.to_scipy()).max()
    # the pattern: a node couples to every node of the bricks it belongs to
    assert A.nnz == len({(int(a), int(b)) for h in m.hexes for a in h for b in h})


@pytest.mark.parametrize("order", [1, 2])
def test_pcg_on_bricks_matches_dense_solve(order):
    m = basin.basin_hex_mesh(3, 3, 2, order, seed=5)
    A = oracle.hex_helmholtz(m, 1e3, 1e-2, 3600.0)
    d = (m.bc & basin.BC_U1) != 0
    b = basin.normal_rhs(m.n, 17, dirichlet=d)
    r = oracle.pcg(A, b, dirichlet=d, tol=1e-13)
    assert r.status == oracle.OK
    Ad = A.to_scipy().toarray()
    free = ~d
    want = np.zeros(m.n)
    want[free] = np.linalg.solve(Ad[np.ix_(free, free)], b[free])
    assert np.linalg.norm(r.x - want) <= 1e-11 * np.linalg.norm(want)


def _manufactured_error(order, N):
    """-lap u = f on [0,1]^2 x [-1,0], u = sin(pi x) sin(pi y) sin(pi z) = 0 on
    the boundary; load = M f at the nodes; error against the nodal values in
    the mass norm."""
    m = basin.box_hex_mesh(N, N, N, order, H=1.0)
    x, y, z = m.xyz.T
    u = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    K = oracle.hex_stiffness(m, 1.0, 1.0)
    M = oracle.hex_mass(m)
    d = (m.bc & basin.BC_U3) != 0          # walls, bottom and surface
    b = M.matvec(3 * np.pi ** 2 * u)
    b[d] = 0.0
    r = oracle.pcg(K, b, dirichlet=d, tol=1e-12)
    assert r.status == oracle.OK
    e = r.x - u
    return float(np.sqrt(e @ M.matvec(e)))


@pytest.mark.parametrize("order,sizes,rate", [(1, (4, 8, 16), 1.9), (2, (2, 4, 8), 3.7)])
def test_manufactured_solution_convergence(order, sizes, rate):
    """The distance between the discrete solution and the nodal interpolant
    of u, in the mass norm, falls like h^2 for Q1 and like h^4 for Q2 on
    uniform boxes (the Q2 solution is superclose to the interpolant there);
    the finest pair of meshes is checked against those rates."""
    errs = [_manufactured_error(order, N) for N in sizes]
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert rates[-1] >= rate, (errs, rates)
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_inverted_brick_is_a_mesh_error():
    m = basin.box_hex_mesh(2, 2, 1, 1)
    bad = m.hexes.copy()
    bad[0] = bad[0][[1, 0, 3, 2, 5, 4, 7, 6]]       # mirror in x
    with pytest.raises(oracle.OracleError) as e:
        oracle.hex_stiffness(type(m)(**{**m.__dict__, "hexes": bad}), 1.0, 1.0)
    assert e.value.status == oracle.ERR_MESH
