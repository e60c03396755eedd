"""Served results equal the same solves done alone (continuous batching on the GPU)."""
import threading
import time

import numpy as np
import pytest

import basin
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MESHES = [(12, 10, 4), (20, 16, 5)]


def _make(key):
    idx, kind = key
    m = basin.basin_mesh(*MESHES[idx], seed=10 + idx)
    return m, 1e3, 1e-2, 3600.0, kind


@pytest.mark.parametrize("capacity", [2, 4])   # per-slot sessions, shared block
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_served_equals_alone(mode, capacity):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_0486_amd.hns import BatchSession, Operator
    from paper_1207_0486_amd.serve import GpuBackend, Request, Server
    be = GpuBackend(_make, mode=mode, check_every=8)
    srv = Server(be, budget_bytes=4 << 30, capacity=capacity, chunk=16)
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(20):
        idx = int(rng.integers(0, 2))
        kind = "poisson" if rng.uniform() < 0.4 else "helmholtz"
        m = be.make_operator((idx, kind))[0]
        bit = -1 if kind == "poisson" else int(rng.integers(0, 3))
        d = None if bit < 0 else ((m.bc >> bit) & 1) == 1
        b = basin.normal_rhs(m.n, 1000 + i, dirichlet=d)
        reqs.append(Request(key=(idx, kind), b=b, mask_bit=bit, tol=1e-8))
    futs = []
    for r in reqs:   # staggered arrivals: later requests join running sessions
        futs.append(srv.submit(r))
        time.sleep(0.002)
    results = [f.result(timeout=120) for f in futs]
    srv.close()
    assert not srv.errors
    alone_ops = {}
    for r, out in zip(reqs, results):
        m, nu_h, nu_v, dt, kind = _make(r.key)
        if r.key not in alone_ops:
            alone_ops[r.key] = Operator(m, nu_h, nu_v, dt, kind=kind, keep_fp32=True)
        op = alone_ops[r.key]
        x_alone, info = op.solve(torch.as_tensor(r.b, device="cuda"), tol=1e-8,
                                 mask_bit=r.mask_bit, mode=mode)
        x_alone = x_alone.cpu().numpy()
        assert out.info.status == 0, (r.key, out.info)
        # both satisfy the tolerance (oracle's own residual) ...
        A = (oracle.stiffness(m, nu_h, nu_v) if kind == "poisson"
             else oracle.helmholtz(m, nu_h, nu_v, dt))
        if r.mask_bit < 0:
            bh = r.b - r.b.mean()
            res = bh - A.matvec(out.x)
            res -= res.mean()
            assert np.linalg.norm(res) <= 1.01e-8 * np.linalg.norm(bh)
        else:
            d = ((m.bc >> r.mask_bit) & 1) == 1
            assert oracle.relres(A, r.b, out.x, d) <= 1.01e-8
        # ... and agree with each other
        diff = np.linalg.norm(out.x - x_alone) / np.linalg.norm(x_alone)
        if capacity <= 2:
            # per-slot sessions run hns_solve's own recurrence: bit for bit
            assert np.array_equal(out.x, x_alone), (r.key, diff)
        else:
            # the shared block runs the block recurrence: against the same
            # request alone in a block session of the same capacity, within
            # the parity tolerance (the per-column sums of a slot may run in
            # another order than those of the slot it was served in); against
            # hns_solve, both answers meet the tolerance
            assert diff <= 1e-6, (r.key, diff)
            sess = BatchSession(op, capacity, mode)
            bt = torch.as_tensor(r.b, device="cuda")
            sess.add([0], [r.mask_bit], [bt], [1e-8], [r.max_iter])
            while sess.advance(16):
                pass
            x_blk, _ = sess.take(0)
            sess.close()
            xb = x_blk.cpu().numpy()
            d_blk = np.linalg.norm(out.x - xb) / np.linalg.norm(xb)
            assert d_blk <= (1e-10 if mode == "fp64" else 1e-9), (r.key, d_blk)
    st = srv.stats()
    assert st["completed"] == 20 and st["p50_ms"] <= st["p99_ms"]
