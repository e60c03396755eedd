"""The OpenMP timing build of the oracle (multi-core CPU baseline): the same
Jacobi-PCG as the plain parity build, with results that do not depend on the
thread count (fixed-order chunked dot products)."""
import numpy as np

import basin
import oracle


def test_openmp_build_matches_plain_build_and_ignores_thread_count():
    m = basin.basin_mesh(24, 20, 6, seed=4)
    K = oracle.stiffness(m, 1e3, 1e-2)
    w = oracle.mass(m).matvec(np.ones(m.n))
    b = basin.normal_rhs(m.n, 1, zero_mean=True)
    plain = oracle.pcg(K, b, singular=True, weights=w, tol=1e-10)
    runs = [oracle.pcg(K, b, singular=True, weights=w, tol=1e-10, threads=t) for t in (1, 2, 3)]
    for r in runs:
        assert r.status == oracle.OK
        assert abs(r.iterations - plain.iterations) <= 1
        assert np.array_equal(r.x, runs[0].x)          # bitwise across thread counts
        assert r.loop_s > 0.0
    assert np.linalg.norm(runs[0].x - plain.x) <= 1e-9 * np.linalg.norm(plain.x)
    A = oracle.helmholtz(m, 1e3, 1e-2, 3600.0)
    d = ((m.bc >> 1) & 1) == 1
    bv = basin.normal_rhs(m.n, 2, dirichlet=d)
    pv = oracle.pcg(A, bv, dirichlet=d, tol=1e-10)
    ov = oracle.pcg(A, bv, dirichlet=d, tol=1e-10, threads=2)
    assert ov.iterations == pv.iterations
    assert np.linalg.norm(ov.x - pv.x) <= 1e-12 * np.linalg.norm(pv.x)
