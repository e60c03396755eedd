"""Pins of the CPU oracle against what the mathematics fixes.

The paper prints no discrete value for its solves, so each part of the oracle
is pinned by a closed form, an invariant, an independent construction or a
library routine (see the docstring of each test).
"""
import os

import numpy as np
import pytest

import basin
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
REF = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)


def _golden_blocks(name):
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            s = line.strip()
            if not s or s.startswith("#"):
                continue
            if any(ch.isalpha() for ch in s):
                cur = s
                blocks[cur] = []
            else:
                blocks[cur].append([float(v) for v in s.split()])
    return {k: np.array(v) for k, v in blocks.items()}


# --------------------------------------------------------------------------
# Element level (closed forms)
# --------------------------------------------------------------------------

def test_reference_tet_matches_closed_forms():
    """Reference-tet stiffness, mass and divergence against the hand-derived file."""
    g = _golden_blocks("reference_tet.txt")
    vol, K, M, B = oracle.element(REF)
    assert vol == pytest.approx(1 / 6, abs=1e-16)
    assert np.allclose(6 * K, g["6K"], atol=1e-14)
    assert np.allclose(120 * M, g["120M"], atol=1e-14)
    assert np.allclose(24 * B[0], g["24B1"], atol=1e-14)


def test_reference_tet_anisotropic():
    """nu = (a, a, b): each gradient product is weighted by its direction's nu."""
    a, b = 3.0, 0.25
    _, K, _, _ = oracle.element(REF, (a, a, b))
    want = np.array([[2 * a + b, -a, -a, -b], [-a, a, 0, 0], [-a, 0, a, 0], [-b, 0, 0, b]]) / 6
    assert np.allclose(K, want, atol=1e-15)


def test_element_invariances():
    """Rigid motion leaves K (isotropic) and M unchanged; scaling by s scales
    K by s and M by s^3; the divergence columns sum to the volume integral of
    a derivative of a constant (zero) and B_c x_c = vol/4 for a linear field."""
    rng = np.random.default_rng(7)
    X = REF + rng.uniform(-0.2, 0.2, REF.shape)
    vol, K, M, B = oracle.element(X)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    vol2, K2, M2, _ = oracle.element(X @ Q.T + 5.0)
    assert np.allclose(K, K2, atol=1e-12) and np.allclose(M, M2, atol=1e-14)
    assert vol2 == pytest.approx(vol, rel=1e-12)
    vol3, K3, M3, _ = oracle.element(2.0 * X)
    assert np.allclose(K3, 2 * K, atol=1e-12) and np.allclose(M3, 8 * M, atol=1e-13)
    assert np.allclose(K.sum(axis=1), 0, atol=1e-13)
    assert np.allclose(B.sum(axis=2), 0, atol=1e-14)
    for c in range(3):
        assert np.allclose(B[c] @ X[:, c], vol / 4, atol=1e-14)


def test_inverted_tet_is_a_mesh_error():
    m = basin.box_mesh(2, 2, 1)
    m.tets[0, [2, 3]] = m.tets[0, [3, 2]]
    with pytest.raises(oracle.OracleError) as e:
        oracle.stiffness(m, 1.0, 1.0)
    assert e.value.status == oracle.ERR_MESH


# --------------------------------------------------------------------------
# Assembled operators (invariants and an independent construction)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_basin():
    return basin.basin_mesh(10, 9, 4, seed=5)


def test_stiffness_annihilates_constants(box16, small_basin):
    for m, nu in ((box16, (1.0, 1e-4)), (small_basin, (1e3, 1e-2))):
        K = oracle.stiffness(m, *nu).to_scipy()
        scale = np.abs(K).max()
        assert np.abs(K @ np.ones(m.n)).max() <= 1e-13 * scale


def test_operators_bitwise_symmetric(small_basin):
    for A in (oracle.stiffness(small_basin, 1e3, 1e-2), oracle.helmholtz(small_basin, 1e3, 1e-2, 3600.0),
              oracle.mass(small_basin)):
        S = A.to_scipy()
        assert (S - S.T).count_nonzero() == 0


def test_pattern_is_15_point(box16):
    K = oracle.operator(box16, 1.0, 1.0, 1.0, 1.0)
    assert K.nnz == 18157
    row = K.to_scipy()[basin.node_index(8, 8, 2, 16, 4)]
    assert row.nnz == 15


def test_mass_sums_to_volume(box16, small_basin):
    M = oracle.mass(box16).to_scipy()
    assert M.sum() == pytest.approx(0.01, rel=1e-13)
    # interior lumped mass equals the cell volume (24 tets around the node)
    V = (1 / 16) * (1 / 16) * (0.01 / 4)
    lumped = np.asarray(M.sum(axis=1)).ravel()
    assert lumped[basin.node_index(8, 8, 2, 16, 4)] == pytest.approx(V, rel=1e-12)
    # sigma mesh: (hx hy / 6) sum (2 dz00 + dz10 + dz01 + 2 dz11) per cell
    m = small_basin
    h = m.depth.reshape(m.Nx + 1, m.Ny + 1)
    dz = h / m.Nz
    hx, hy = m.Lx / m.Nx, m.Ly / m.Ny
    want = m.Nz * ((hx * hy / 6.0) * (2 * dz[:-1, :-1] + dz[1:, :-1] + dz[:-1, 1:] + 2 * dz[1:, 1:])).sum()
    assert oracle.mass(m).to_scipy().sum() == pytest.approx(want, rel=1e-12)


def _tridiag(n, last_diag=2.0):
    T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    T[-1, -1] = last_diag
    return T


def test_box_stiffness_equals_finite_difference_kronecker(box16):
    """On an axis-aligned box every Kuhn tet has one edge per axis, so the P1
    anisotropic stiffness couples only axis neighbours with weight V nu_d / h_d^2
    (half on the surface layer).  Built independently with Kronecker products."""
    nu_h, nu_v = 1.0, 1e-4
    hx = hy = 1 / 16
    hz = 0.01 / 4
    V = hx * hy * hz
    T = _tridiag(15)
    I = np.eye(15)
    W = np.diag([1.0, 1.0, 1.0, 0.5])
    N = _tridiag(4, last_diag=1.0)
    want = V * (nu_h / hx ** 2 * np.kron(np.kron(T, I), W)
                + nu_h / hy ** 2 * np.kron(np.kron(I, T), W)
                + nu_v / hz ** 2 * np.kron(np.kron(I, I), N))
    K = oracle.stiffness(box16, nu_h, nu_v).to_scipy()
    free = box16.free_mask(basin.BC_U1)
    Kf = K[free][:, free].toarray()
    assert np.abs(Kf - want).max() <= 1e-13 * np.abs(want).max()


def test_divergence_on_linear_fields(small_basin):
    """B_c 1 = 0 and B_c x_d = delta_cd * (M 1): the derivative of a linear field
    is exact in P1, and int phi_i = (M 1)_i."""
    m = small_basin
    lumped = oracle.mass(m).matvec(np.ones(m.n))
    for c in range(3):
        Bc = oracle.divergence(m, c)
        scale = np.abs(lumped).max()
        assert np.abs(Bc.matvec(np.ones(m.n))).max() <= 1e-12 * scale
        for d in range(3):
            got = Bc.matvec(m.xyz[:, d])
            want = lumped if c == d else np.zeros(m.n)
            assert np.abs(got - want).max() <= 1e-9 * scale


def test_surface_mass(small_basin):
    m = small_basin
    Ms = oracle.surface_mass(m).to_scipy()
    assert Ms.sum() == pytest.approx(m.Lx * m.Ly, rel=1e-13)
    # the load of a linear tension field integrates it exactly
    y = m.xyz[:, 1]
    assert (Ms @ y).sum() == pytest.approx(m.Lx * m.Ly * m.Ly / 2, rel=1e-12)


def test_jacobi_scaled_mass_spectrum(box16):
    """Diagonally scaled P1 tetrahedral mass has its spectrum in [1/2, 5/2]."""
    M = oracle.mass(box16).to_scipy().toarray()
    d = 1 / np.sqrt(np.diag(M))
    ev = np.linalg.eigvalsh(d[:, None] * M * d[None, :])
    assert ev.min() >= 0.5 - 1e-12 and ev.max() <= 2.5 + 1e-12


# --------------------------------------------------------------------------
# Solver pins
# --------------------------------------------------------------------------

def _free_system(A, free):
    S = A.to_scipy()
    return S[free][:, free].toarray()


@pytest.mark.parametrize("dims", [(2, 2, 1), (3, 3, 2), (4, 4, 2), (16, 16, 4)])
def test_pcg_matches_direct_solves(dims):
    m = basin.box_mesh(*dims)
    free = m.free_mask(basin.BC_U1)
    A = oracle.stiffness(m, 1.0, 1e-4)
    b = basin.normal_rhs(m.n, 11, zero_mean=True, dirichlet=~free)
    Af = _free_system(A, free)
    x_np = np.linalg.solve(Af, b[free])
    x_ch = oracle.cholesky_solve(Af, b[free])
    assert np.linalg.norm(x_ch - x_np) <= 1e-12 * np.linalg.norm(x_np)
    r = oracle.pcg(A, b, dirichlet=~free, tol=1e-14, maxit=5000)
    assert r.status == oracle.OK
    assert np.all(r.x[~free] == 0)
    assert np.linalg.norm(r.x[free] - x_np) <= 1e-12 * np.linalg.norm(x_np)


def test_pcg_helmholtz_basin_direct(small_basin):
    m = small_basin
    for bit in (basin.BC_U1, basin.BC_U2, basin.BC_U3):
        free = m.free_mask(bit)
        A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
        b = basin.normal_rhs(m.n, bit, dirichlet=~free)
        x_np = np.linalg.solve(_free_system(A, free), b[free])
        r = oracle.pcg(A, b, dirichlet=~free, tol=1e-14)
        assert r.status == oracle.OK
        assert np.linalg.norm(r.x[free] - x_np) <= 1e-11 * np.linalg.norm(x_np)


def test_pcg_error_within_condition_bound(box16):
    """At tol 1e-10 the error is bounded by kappa(A) * tol (relative)."""
    m = box16
    free = m.free_mask(basin.BC_U1)
    A = oracle.stiffness(m, 1.0, 1e-4)
    b = basin.normal_rhs(m.n, 0, zero_mean=True, dirichlet=~free)
    Af = _free_system(A, free)
    x_np = np.linalg.solve(Af, b[free])
    kappa = np.linalg.cond(Af)
    r = oracle.pcg(A, b, dirichlet=~free, tol=1e-10)
    assert r.status == oracle.OK and r.relres <= 1e-10
    err = np.linalg.norm(r.x[free] - x_np) / np.linalg.norm(x_np)
    assert err <= kappa * 1e-10


def test_pcg_energy_error_decreases(box16):
    """CG minimises the A-norm of the error over growing Krylov spaces, so the
    energy error of successive iterates strictly decreases."""
    m = box16
    free = m.free_mask(basin.BC_U1)
    A = oracle.stiffness(m, 1.0, 1e-4)
    b = basin.normal_rhs(m.n, 3, dirichlet=~free)
    Af = _free_system(A, free)
    x_np = np.linalg.solve(Af, b[free])
    r = oracle.pcg(A, b, dirichlet=~free, tol=1e-12, maxit=400, x_history=True)
    E = r.x_hist[:, free] - x_np
    energy = np.einsum("ki,ij,kj->k", E, Af, E)
    assert np.all(np.diff(energy[energy > 1e-24 * energy[0]]) < 0)


def test_lanczos_estimate_matches_spectrum(box16):
    """The CG coefficients' Lanczos matrix recovers kappa(D^-1 A) from below."""
    m = box16
    free = m.free_mask(basin.BC_U1)
    A = oracle.stiffness(m, 1.0, 1e-4)
    b = basin.normal_rhs(m.n, 0, zero_mean=True, dirichlet=~free)
    r = oracle.pcg(A, b, dirichlet=~free, tol=1e-12, history=True)
    Af = _free_system(A, free)
    d = 1 / np.sqrt(np.diag(Af))
    ev = np.linalg.eigvalsh(d[:, None] * Af * d[None, :])
    k_true = ev[-1] / ev[0]
    k_est = oracle.lanczos_condition(r.alphas, r.betas)
    assert 0.9 * k_true <= k_est <= k_true * (1 + 1e-8)


def test_zero_rhs_and_nonfinite_rhs(box16):
    A = oracle.stiffness(box16, 1.0, 1e-4)
    d = ~box16.free_mask(basin.BC_U1)
    r = oracle.pcg(A, np.zeros(box16.n), dirichlet=d)
    assert r.status == oracle.OK and r.iterations == 0 and np.all(r.x == 0)
    b = np.ones(box16.n)
    b[5] = np.nan
    assert oracle.pcg(A, b, dirichlet=d).status == oracle.ERR_INVALID


def test_indefinite_operator_breaks_down(small_basin):
    """dt < 0 makes M + dt*K indefinite; CG must report breakdown."""
    A = oracle.helmholtz(small_basin, 1e3, 1e-2, -3.6e7)
    free = small_basin.free_mask(basin.BC_U1)
    b = basin.normal_rhs(small_basin.n, 1, dirichlet=~free)
    assert oracle.pcg(A, b, dirichlet=~free).status == oracle.ERR_BREAKDOWN


def test_neumann_projection_and_normalisation(small_basin):
    """Pure Neumann: the RHS is projected to zero sum, and the answer does not
    depend on an added constant in b or x0 once normalised to zero mass-mean."""
    m = small_basin
    K = oracle.stiffness(m, 1e3, 1e-2)
    w = oracle.mass(m).matvec(np.ones(m.n))
    b = basin.normal_rhs(m.n, 9)
    r1 = oracle.pcg(K, b, singular=True, weights=w, tol=1e-12)
    assert r1.status == oracle.OK
    assert r1.removed_mean == pytest.approx(b.mean(), rel=1e-12)
    assert abs(w @ r1.x) <= 1e-12 * np.abs(w).sum() * np.abs(r1.x).max()
    r2 = oracle.pcg(K, b + 3.0, singular=True, weights=w, tol=1e-12)
    assert r2.status == oracle.OK
    assert np.linalg.norm(r2.x - r1.x) <= 1e-9 * np.linalg.norm(r1.x)
    # a constant initial guess of the solution's own size changes nothing either
    r3 = oracle.pcg(K, b, singular=True, weights=w, x0=np.full(m.n, np.abs(r1.x).max()),
                    tol=1e-12)
    assert r3.status == oracle.OK
    assert np.linalg.norm(r3.x - r1.x) <= 1e-9 * np.linalg.norm(r1.x)
    # the normalised answer solves the projected system (pseudo-inverse check)
    Kd = K.to_scipy().toarray()
    bh = b - b.mean()
    x_pinv = np.linalg.lstsq(Kd, bh, rcond=None)[0]
    x_pinv -= (w @ x_pinv) / w.sum()
    assert np.linalg.norm(r1.x - x_pinv) <= 1e-7 * np.linalg.norm(x_pinv)


# --------------------------------------------------------------------------
# Manufactured solutions: second-order nodal convergence
# --------------------------------------------------------------------------

def _mms_error(N, kind):
    H = 0.01
    nu_h, nu_v = 1.0, 1e-4
    m = basin.box_mesh(N, N, N // 4, H=H, gamma0=("bottom", "west", "east", "south", "north"))
    x, y, z = m.xyz.T
    M = oracle.mass(m)
    if kind == "dirichlet":
        u = np.sin(np.pi * x) * np.sin(np.pi * y) * np.cos(np.pi * z / (2 * H))
        lam = 2 * np.pi ** 2 * nu_h + nu_v * np.pi ** 2 / (4 * H ** 2)
        A = oracle.stiffness(m, nu_h, nu_v)
        d = ~m.free_mask(basin.BC_U1)
        r = oracle.pcg(A, M.matvec(lam * u), dirichlet=d, tol=1e-13, maxit=20000)
    elif kind == "helmholtz":
        dt = 0.05
        u = np.sin(np.pi * x) * np.sin(np.pi * y) * np.cos(np.pi * z / (2 * H))
        lam = 2 * np.pi ** 2 * nu_h + nu_v * np.pi ** 2 / (4 * H ** 2)
        A = oracle.helmholtz(m, nu_h, nu_v, dt)
        d = ~m.free_mask(basin.BC_U1)
        r = oracle.pcg(A, M.matvec((1 + dt * lam) * u), dirichlet=d, tol=1e-13, maxit=20000)
    else:  # pure Neumann, zero-mean exact solution
        u = np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z / H)
        lam = 2 * np.pi ** 2 * nu_h + nu_v * np.pi ** 2 / H ** 2
        A = oracle.stiffness(m, nu_h, nu_v)
        w = M.matvec(np.ones(m.n))
        r = oracle.pcg(A, M.matvec(lam * u), singular=True, weights=w, tol=1e-13, maxit=20000)
        u = u - (w @ u) / w.sum()
    assert r.status == oracle.OK
    e = r.x - u
    return np.sqrt(e @ M.matvec(e)) / np.sqrt(u @ M.matvec(u))


@pytest.mark.parametrize("kind", ["dirichlet", "neumann", "helmholtz"])
def test_manufactured_solution_rate(kind):
    errs = [_mms_error(N, kind) for N in (16, 32, 64)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates >= 1.9), (errs, rates)


def test_tolerance_below_rounding_floor_stops_early():
    """A tolerance the rounding of A x cannot reach: CG restarts from the true
    residual until three checks in a row fail to halve the best true residual,
    then reports not-converged long before the iteration cap, with a true
    residual near the floor."""
    m = basin.box_mesh(8, 8, 4)
    A = oracle.helmholtz(m, 1.0, 1e-4, 0.1)
    d = (m.bc & 1) == 1
    b = basin.normal_rhs(m.n, 2, dirichlet=d)
    r = oracle.pcg(A, b, dirichlet=d, tol=1e-19, maxit=100000)
    assert r.status == oracle.NOT_CONVERGED
    assert r.iterations < 2000
    assert r.relres < 1e-14
    assert oracle.relres(A, b, r.x, d) == pytest.approx(r.relres, rel=1e-6)
