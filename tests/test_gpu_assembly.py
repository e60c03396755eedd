"""Device assembly of the operator values: bitwise the host assembly, equal to
the oracle's independent assembly, and the same mesh errors."""
import dataclasses

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


def _permuted(m, seed):
    perm = np.random.default_rng(seed).permutation(m.n)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(m.n)
    return dataclasses.replace(m, xyz=m.xyz[perm], bc=m.bc[perm],
                               tets=inv[m.tets].astype(np.int32),
                               surf_tris=inv[m.surf_tris].astype(np.int32))


MESHES = {
    "box16": lambda: basin.box_mesh(16, 16, 4),
    "basin": lambda: basin.basin_mesh(24, 20, 6, seed=4),
    "permuted": lambda: _permuted(basin.basin_mesh(10, 8, 4, seed=2), 5),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("kind", ["poisson", "helmholtz"])
def test_device_values_are_the_host_values(dev, name, kind):
    from paper_1207_0486_amd.hns import Operator
    m = MESHES[name]()
    nu_h, nu_v, dt = 1e3, 1e-2, 3600.0
    host = Operator(m, nu_h, nu_v, dt, kind=kind)
    gpu = Operator(m, nu_h, nu_v, dt, kind=kind, gpu_assembly=True)
    assert (gpu.n, gpu.nnz, gpu.format, gpu.ndiag) == (host.n, host.nnz, host.format, host.ndiag)
    rng = np.random.default_rng(3)
    for _ in range(3):
        x = torch.as_tensor(rng.standard_normal(m.n), device=dev)
        assert torch.equal(gpu.apply(x), host.apply(x))
    # diagonal and lumped mass too: identical solves
    b = torch.as_tensor(basin.normal_rhs(m.n, 9, zero_mean=kind == "poisson"), device=dev)
    bit = -1 if kind == "poisson" else 0
    xh, ih = host.solve(b, tol=1e-10, mask_bit=bit)
    xg, ig = gpu.solve(b, tol=1e-10, mask_bit=bit)
    assert ih.iterations == ig.iterations and torch.equal(xh, xg)
    # against the oracle's own assembly
    A = oracle.helmholtz(m, nu_h, nu_v, dt) if kind == "helmholtz" else \
        oracle.stiffness(m, nu_h, nu_v)
    xr = rng.standard_normal(m.n)
    want = A.matvec(xr)
    got = gpu.apply(torch.as_tensor(xr, device=dev)).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-13 * np.abs(A.to_scipy()).sum(axis=1).max() * \
        np.abs(xr).max()


def test_device_assembly_reports_inverted_tetrahedra(dev):
    from paper_1207_0486_amd.hns import HNSError, Operator
    m = basin.box_mesh(4, 4, 2)
    tets = m.tets.copy()
    tets[17, [1, 2]] = tets[17, [2, 1]]       # negative volume
    bad = dataclasses.replace(m, tets=tets)
    for gpu_assembly in (False, True):
        with pytest.raises(HNSError) as e:
            Operator(bad, 1.0, 1.0, 0.1, kind="helmholtz", gpu_assembly=gpu_assembly)
        assert e.value.status == -4
