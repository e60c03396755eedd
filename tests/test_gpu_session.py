"""Batch sessions (continuous batching) in both forms: per-slot recurrences
(session_mode 2, the default up to two slots) and the shared multi-RHS block
(session_mode 1).  A per-slot session runs hns_solve's own recurrence, so its
answers equal hns_solve's bit for bit whatever the chunking and whenever the
request joined; the block form agrees to the tolerance."""
import numpy as np
import pytest

import basin
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NU = (1e3, 1e-2)
DT = 3600.0


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_0486_amd import hns  # noqa: F401
    return torch.device("cuda", 0)


def _rhs(m, bit, seed):
    d = None if bit < 0 else ((m.bc >> bit) & 1) == 1
    return basin.normal_rhs(m.n, seed, dirichlet=d, zero_mean=bit < 0)


def _run(sess, adds, advance=13, limit=100000):
    """adds: {round: [(slot, bit, b, tol, max_iter), ...]} joined before that
    advance round; returns {slot: (x, info)} of every finished request."""
    out = {}
    rnd = 0
    while True:
        for slot, bit, b, tol, mi in adds.get(rnd, []):
            sess.add([slot], [bit], [b], [tol], [mi])
        active = sess.advance(advance)
        states, _ = sess.poll()
        for j, st in enumerate(states):
            if st == 2:
                out[j] = sess.take(j)
        rnd += 1
        if active == 0 and rnd > max(adds):
            return out
        assert rnd < limit


@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["poisson", "helmholtz"])
def test_per_slot_session_equals_solve_bitwise(dev, mode, kind, precond):
    """Two slots on the 40x36x6 basin (10,619 rows, Jacobi-scaled point
    Jacobi, or the water-column line blocks): the second request joins while
    the first runs; each answer equals hns_solve's."""
    from paper_1207_0486_amd.hns import BatchSession, Operator
    m = basin.basin_mesh(40, 36, 6, seed=5)
    op = Operator(m, *NU, DT if kind == "helmholtz" else 0.0, kind=kind, keep_fp32=True)
    op.set_param("session_mode", 2)
    op.set_param("precond", precond)
    bits = [-1, -1] if kind == "poisson" else [0, 2]
    bs = [torch.as_tensor(_rhs(m, bits[q], 50 + q), device=dev) for q in range(2)]
    sess = BatchSession(op, 2, mode)
    got = _run(sess, {0: [(0, bits[0], bs[0], 1e-9, 100000)],
                      3: [(1, bits[1], bs[1], 1e-9, 100000)]})
    sess.close()
    for q in range(2):
        x, info = got[q]
        ref, rinfo = op.solve(bs[q], tol=1e-9, mask_bit=bits[q], mode=mode)
        assert info.status == 0 and rinfo.status == 0
        assert info.iterations == rinfo.iterations
        assert torch.equal(x, ref)
    op.close()


def test_per_slot_session_edge_cases(dev):
    """b = 0 finishes at once with x = 0; a non-finite right-hand side
    finishes with HNS_ERR_INVALID; an iteration cap finishes with
    NOT_CONVERGED after exactly that many iterations (the oracle's iterate);
    busy, repeated and out-of-range slots are refused."""
    from paper_1207_0486_amd.hns import BatchSession, HNSError, Operator
    m = basin.basin_mesh(20, 16, 5, seed=3)
    op = Operator(m, *NU, DT, kind="helmholtz")
    op.set_param("session_mode", 2)
    op.set_param("small_n", 0)
    sess = BatchSession(op, 2, "fp64")
    zero = torch.zeros(m.n, dtype=torch.float64, device=dev)
    bad = zero.clone()
    free = np.flatnonzero(((m.bc >> 0) & 1) == 0)
    bad[int(free[0])] = float("nan")   # Dirichlet entries of b are ignored; a free one is not
    sess.add([0, 1], [0, 0], [zero, bad], [1e-10, 1e-10], [1000, 1000])
    states, infos = sess.poll()
    assert states == [2, 2]
    x0, i0 = sess.take(0)
    assert i0.status == 0 and i0.iterations == 0 and float(x0.abs().max()) == 0.0
    _, i1 = sess.take(1)
    assert i1.status == -1   # HNS_ERR_INVALID
    b = _rhs(m, 1, 61)
    d = ((m.bc >> 1) & 1) == 1
    sess.add([1], [1], [torch.as_tensor(b, device=dev)], [1e-14], [7])
    with pytest.raises(HNSError):
        sess.add([1], [1], [torch.as_tensor(b, device=dev)], [1e-10], [10])   # busy
    with pytest.raises(HNSError):
        sess.add([0, 0], [1, 1], [zero, zero], [1e-10, 1e-10], [10, 10])      # repeated
    with pytest.raises(HNSError):
        sess.add([2], [1], [zero], [1e-10], [10])                             # out of range
    with pytest.raises(HNSError):
        sess.take(1)                                                          # not finished
    while sess.advance(3) > 0:
        pass
    x, info = sess.take(1)
    assert info.status == 1 and info.iterations == 7
    A = oracle.helmholtz(m, *NU, DT)
    same = oracle.pcg(A, b, dirichlet=d, tol=1e-300, maxit=7)
    xh = x.cpu().numpy()
    assert np.linalg.norm(xh - same.x) <= 1e-12 * np.linalg.norm(same.x)
    sess.close()
    op.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_block_and_per_slot_sessions_agree(dev, mode):
    """The same four requests through a four-slot block session and through
    per-slot sessions of two: both meet the tolerance in the oracle's residual
    and agree with each other."""
    from paper_1207_0486_amd.hns import BatchSession, Operator
    m = basin.basin_mesh(24, 20, 5, seed=8)
    op = Operator(m, *NU, DT, kind="helmholtz", keep_fp32=True)
    A = oracle.helmholtz(m, *NU, DT)
    bits = [0, 1, 2, 0]
    bs = [_rhs(m, bits[q], 70 + q) for q in range(4)]
    bt = [torch.as_tensor(b, device=dev) for b in bs]
    op.set_param("session_mode", 1)
    sess = BatchSession(op, 4, mode)
    block = _run(sess, {0: [(q, bits[q], bt[q], 1e-9, 100000) for q in range(2)],
                        2: [(q, bits[q], bt[q], 1e-9, 100000) for q in range(2, 4)]})
    sess.close()
    op.set_param("session_mode", 2)
    per = {}
    for pair in ((0, 1), (2, 3)):
        sess = BatchSession(op, 2, mode)
        got = _run(sess, {0: [(j, bits[q], bt[q], 1e-9, 100000) for j, q in enumerate(pair)]})
        sess.close()
        for j, q in enumerate(pair):
            per[q] = got[j]
    for q in range(4):
        d = ((m.bc >> bits[q]) & 1) == 1
        xb, ib = block[q]
        xp, ip = per[q]
        assert ib.status == 0 and ip.status == 0
        xb, xp = xb.cpu().numpy(), xp.cpu().numpy()
        assert oracle.relres(A, bs[q], xb, d) <= 1.01e-9
        assert oracle.relres(A, bs[q], xp, d) <= 1.01e-9
        assert np.linalg.norm(xb - xp) <= 1e-7 * np.linalg.norm(xp)
    op.close()
