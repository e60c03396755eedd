"""Seeded input generator: mesh validity, counts, boundary bits, reproducibility."""
import os

import numpy as np
import pytest

import basin

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _counts():
    rows = []
    with open(os.path.join(GOLDEN, "mesh_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(tuple(int(v) for v in line.split()))
    return rows


def _kuhn_nnz(Nx, Ny, Nz):
    n = (Nx + 1) * (Ny + 1) * (Nz + 1)
    E = 0
    for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)):
        E += (Nx + 1 - d[0]) * (Ny + 1 - d[1]) * (Nz + 1 - d[2])
    return n + 2 * E


@pytest.mark.parametrize("row", _counts())
def test_count_formulas(row):
    Nx, Ny, Nz, n, tets, nnz = row
    assert (Nx + 1) * (Ny + 1) * (Nz + 1) == n
    assert 6 * Nx * Ny * Nz == tets
    assert _kuhn_nnz(Nx, Ny, Nz) == nnz


def test_box16_counts(box16):
    m = box16
    assert m.n == 1445 and m.n_tets == 6144
    assert int(m.free_mask(basin.BC_U1).sum()) == 900
    assert m.surf_tris.shape == (512, 3)
    assert m.tets.min() == 0 and m.tets.max() == m.n - 1


def _signed_volumes(m):
    X = m.xyz[m.tets]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=-1)
    return np.linalg.det(J) / 6.0


def test_tets_positive_and_fill_box(box16):
    vol = _signed_volumes(box16)
    assert np.all(vol > 0)
    assert np.isclose(vol.sum(), 0.01, rtol=1e-13)


def test_basin_volumes_match_sigma_formula():
    m = basin.basin_mesh(12, 10, 5, seed=3)
    vol = _signed_volumes(m)
    assert np.all(vol > 0)
    h = m.depth.reshape(m.Nx + 1, m.Ny + 1)
    dz = h / m.Nz
    hx, hy = m.Lx / m.Nx, m.Ly / m.Ny
    # each cell: (hx*hy/6)(2 dz00 + dz10 + dz01 + 2 dz11), summed over all layers
    per_col = (hx * hy / 6.0) * (2 * dz[:-1, :-1] + dz[1:, :-1] + dz[:-1, 1:] + 2 * dz[1:, 1:])
    assert np.isclose(vol.sum(), m.Nz * per_col.sum(), rtol=1e-12)


def test_node_order_vertical_first():
    m = basin.box_mesh(3, 2, 4)
    i, j, k = 2, 1, 3
    idx = basin.node_index(i, j, k, 2, 4)
    assert np.allclose(m.xyz[idx], [i / 3, j / 2, -0.01 * (1 - k / 4)])


def test_dirichlet_bits_basin():
    m = basin.basin_mesh(4, 5, 3, seed=1)
    i, j, k = np.meshgrid(np.arange(5), np.arange(6), np.arange(4), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    g0 = (k == 0) | (i == 0) | (i == 4)
    g1 = (j == 0) | (j == 5)
    s = k == 3
    assert np.array_equal((m.bc & basin.BC_U1) > 0, g0)
    assert np.array_equal((m.bc & basin.BC_U2) > 0, g0 | g1)
    assert np.array_equal((m.bc & basin.BC_U3) > 0, g0 | s)


def test_surface_triangles_cover_surface():
    m = basin.basin_mesh(6, 7, 2, seed=0)
    P = m.xyz[m.surf_tris]
    assert np.all(P[:, :, 2] == 0.0)
    area = 0.5 * np.abs(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])[:, 2])
    assert np.isclose(area.sum(), m.Lx * m.Ly, rtol=1e-13)


def test_bathymetry_reproducible_and_clipped():
    x = np.linspace(0, 5e6, 50)
    h1 = basin.bathymetry(x, x, 5e6, seed=0)
    h2 = basin.bathymetry(x, x, 5e6, seed=0)
    assert np.array_equal(h1, h2)
    assert h1.min() >= 200.0 and h1.max() <= 5500.0
    assert not np.array_equal(h1, basin.bathymetry(x, x, 5e6, seed=1))


def test_rhs_recipe():
    d = np.zeros(10, bool)
    d[:3] = True
    b = basin.normal_rhs(10, 0, zero_mean=True, dirichlet=d)
    raw = np.random.default_rng(0).standard_normal(10)
    assert np.allclose(b[3:], (raw - raw.mean())[3:]) and np.all(b[:3] == 0)


def test_serving_stream():
    reqs = basin.serving_requests()
    assert len(reqs) == 256
    t = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert 3.0 < t[-1] < 7.5  # 256 arrivals at 50/s
    assert {r.kind for r in reqs} == {"poisson", "helmholtz"}
    assert reqs == basin.serving_requests()


def test_wind_scenarios():
    sc = basin.wind_scenarios()
    assert len(sc) == 16
    assert all(0.05 <= s.amplitude <= 0.2 and 0 <= s.phase < 2 * np.pi for s in sc)
