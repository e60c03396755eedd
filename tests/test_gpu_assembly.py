"""Device assembly: the whole operator built on the device (incidence,
offsets, diagonal storage) where it fits the unrolled diagonal storage, else
the values on a host pattern; bitwise the host assembly either way, equal to
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


# where the build runs: whole operator on the device (diagonal storage fits),
# or the values only (a random numbering spreads the offsets over the range)
WHERE = {"box16": 2, "basin": 2, "permuted": 1}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("kind", ["poisson", "helmholtz"])
def test_device_values_are_the_host_values(dev, name, kind):
    from paper_1207_0486_amd.hns import Operator
    m = MESHES[name]()
    nu_h, nu_v, dt = 1e3, 1e-2, 3600.0
    host = Operator(m, nu_h, nu_v, dt, kind=kind, keep_fp32=True)
    gpu = Operator(m, nu_h, nu_v, dt, kind=kind, gpu_assembly=True, keep_fp32=True)
    assert host.assembly == 0 and gpu.assembly == WHERE[name]
    assert (gpu.n, gpu.nnz, gpu.format, gpu.ndiag, gpu.line_len) == \
        (host.n, host.nnz, host.format, host.ndiag, host.line_len)
    rng = np.random.default_rng(3)
    for _ in range(3):
        x = torch.as_tensor(rng.standard_normal(m.n), device=dev)
        assert torch.equal(gpu.apply(x), host.apply(x))
    # diagonal, FP32 copies, lumped mass and column blocks too: identical solves
    b = torch.as_tensor(basin.normal_rhs(m.n, 9, zero_mean=kind == "poisson"), device=dev)
    bit = -1 if kind == "poisson" else 0
    for mode in ("fp64", "mixed"):
        xh, ih = host.solve(b, tol=1e-10, mask_bit=bit, mode=mode)
        xg, ig = gpu.solve(b, tol=1e-10, mask_bit=bit, mode=mode)
        assert ih.iterations == ig.iterations and torch.equal(xh, xg), mode
    if host.line_len >= 2:
        for op in (host, gpu):
            op.set_param("precond", 1)
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


def _bad_meshes():
    m = basin.box_mesh(4, 4, 2)
    inverted = m.tets.copy()
    inverted[17, [1, 2]] = inverted[17, [2, 1]]       # negative volume
    outside = m.tets.copy()
    outside[9, 3] = m.n                               # vertex index out of range
    xyz = m.xyz.copy()
    xyz[11, 2] = np.nan                               # non-finite coordinate
    return {"inverted": dataclasses.replace(m, tets=inverted),
            "outside": dataclasses.replace(m, tets=outside),
            "nan": dataclasses.replace(m, xyz=xyz)}


@pytest.mark.parametrize("case", ["inverted", "outside", "nan"])
def test_device_assembly_reports_mesh_errors(dev, case):
    from paper_1207_0486_amd import _lib as L
    from paper_1207_0486_amd.hns import HNSError, Operator
    bad = _bad_meshes()[case]
    msgs = []
    for gpu_assembly in (False, True):
        with pytest.raises(HNSError) as e:
            Operator(bad, 1.0, 1.0, 0.1, kind="helmholtz", gpu_assembly=gpu_assembly)
        assert e.value.status == -4
        msgs.append(L.lib().hns_last_error())
    assert msgs[0] == msgs[1], msgs


def _mesh_of(xyz, tets, bc=None):
    import types
    return types.SimpleNamespace(xyz=np.asarray(xyz, dtype=np.float64),
                                 tets=np.asarray(tets, dtype=np.int32).reshape(-1, 4),
                                 bc=None if bc is None else np.asarray(bc, dtype=np.uint8))


def _pair(m, kind="helmholtz"):
    from paper_1207_0486_amd.hns import Operator
    host = Operator(m, 1.0, 0.5, 0.1, kind=kind)
    gpu = Operator(m, 1.0, 0.5, 0.1, kind=kind, gpu_assembly=True)
    return host, gpu


def test_device_build_edge_meshes(dev):
    """One tetrahedron (every row at the ends of the diagonal storage); a
    mesh with a node no tetrahedron touches (its diagonal is zero: both
    builds report it as a breakdown of the solve); a mesh with no
    tetrahedron at all (no offsets: the host path); each bitwise the host
    build."""
    from paper_1207_0486_amd.hns import HNSError
    rng = np.random.default_rng(4)
    one = _mesh_of([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], [[0, 1, 2, 3]])
    box = basin.box_mesh(2, 2, 1)
    extra = _mesh_of(np.vstack([box.xyz, [[5.0, 5.0, 5.0]]]), box.tets)
    empty = _mesh_of([[0, 0, 0], [1, 0, 0]], np.zeros((0, 4)))
    for m, where in ((one, 2), (extra, 2), (empty, 1)):
        host, gpu = _pair(m)
        assert gpu.assembly == where
        assert (gpu.n, gpu.nnz, gpu.format, gpu.ndiag) == (host.n, host.nnz, host.format,
                                                           host.ndiag)
        x = torch.as_tensor(rng.standard_normal(gpu.n), device=dev)
        assert torch.equal(gpu.apply(x), host.apply(x))
        b = torch.as_tensor(rng.standard_normal(gpu.n), device=dev)
        outs = []
        for op in (host, gpu):
            try:
                xs, info = op.solve(b, tol=1e-10)
                outs.append(("ok", xs))
            except HNSError as e:
                outs.append(("err", e.status))
        assert outs[0][0] == outs[1][0]
        if outs[0][0] == "ok":
            assert torch.equal(outs[0][1], outs[1][1])
        else:
            assert outs[0][1] == outs[1][1] == -5   # breakdown: a zero diagonal
        if m is one:
            assert outs[0][0] == "ok"
