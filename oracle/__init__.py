"""CPU oracle for the shallow-basin PCG solves.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the HIP library: the
arithmetic lives in `hns_oracle.c` (plain FP64 C, compiled by `build()`), and
this module only marshals arrays to it.  See the header of `hns_oracle.c` for
the paper passages each routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hns_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

OK, NOT_CONVERGED, ERR_INVALID, ERR_NOMEM, ERR_MESH, ERR_BREAKDOWN = 0, 1, -1, -3, -4, -5

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fused multiply-add
    contraction), and the OpenMP timing build of the same file (-O3
    -march=native -fopenmp) used only for the benchmark's multi-core CPU
    baseline and its reference solves."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                        "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_LIB_OMP):
        tmp = _LIB_OMP + ".tmp"
        subprocess.run(["gcc", "-O3", "-march=native", "-fopenmp", "-std=gnu99",
                        "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC,
                        "-lm"], check=True)
        os.replace(tmp, _LIB_OMP)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp, ip, i64p, u8p = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int64), C.POINTER(C.c_uint8))
        vp = C.c_void_p
        L.or_element.restype = C.c_double
        L.or_element.argtypes = [dp, dp, dp, dp, dp]
        L.or_assemble.restype = C.c_int
        L.or_assemble.argtypes = [C.c_int64, dp, C.c_int64, ip, C.c_int, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_int, C.POINTER(vp)]
        L.or_hex_element.restype = C.c_double
        L.or_hex_element.argtypes = [C.c_int, dp, dp, dp, dp]
        L.or_assemble_hex.restype = C.c_int
        L.or_assemble_hex.argtypes = [C.c_int64, dp, C.c_int64, ip, C.c_int, C.c_double,
                                      C.c_double, C.c_double, C.c_double, C.POINTER(vp)]
        L.or_assemble_surface_mass.restype = C.c_int
        L.or_assemble_surface_mass.argtypes = [C.c_int64, dp, C.c_int64, ip, C.POINTER(vp)]
        L.or_csr_free.argtypes = [vp]
        L.or_csr_n.restype = C.c_int64
        L.or_csr_n.argtypes = [vp]
        L.or_csr_nnz.restype = C.c_int64
        L.or_csr_nnz.argtypes = [vp]
        L.or_csr_copy_out.argtypes = [vp, i64p, ip, dp]
        L.or_spmv.argtypes = [vp, dp, dp]
        L.or_spmv_t.argtypes = [vp, dp, dp, C.c_int64]
        L.or_pcg.restype = C.c_int
        L.or_pcg_line.restype = C.c_int
        L.or_pcg_line.argtypes = [vp, u8p, C.c_int, dp, dp, dp, C.c_double, C.c_int, C.c_int64,
                                  C.POINTER(C.c_int), dp, dp, dp, dp, dp]
        L.or_pcg_ic0.restype = C.c_int
        L.or_pcg_ic0.argtypes = [vp, u8p, C.c_int, dp, dp, dp, C.c_double, C.c_int,
                                 C.POINTER(C.c_int), dp, dp, dp, dp, dp]
        L.or_ic0_factor.restype = C.c_int
        L.or_ic0_factor.argtypes = [vp, u8p, ip, C.POINTER(vp)]
        L.or_greedy_colors.restype = C.c_int
        L.or_greedy_colors.argtypes = [vp, ip]
        L.or_advection.restype = C.c_int
        L.or_advection.argtypes = [C.c_int64, dp, C.c_int64, ip, dp, dp]
        L.or_tridiag_solve.restype = C.c_int
        L.or_tridiag_solve.argtypes = [C.c_int64, dp, dp, dp, dp, dp]
        L.or_pcg.argtypes = [vp, u8p, C.c_int, dp, dp, dp, C.c_double, C.c_int,
                             C.POINTER(C.c_int), dp, dp, dp, dp, dp]
        L.or_relres.restype = C.c_double
        L.or_relres.argtypes = [vp, u8p, dp, dp]
        L.or_cholesky_solve.restype = C.c_int
        L.or_cholesky_solve.argtypes = [C.c_int64, dp, dp, dp]
        _declare_timing(L)
        _lib = L
    return _lib


def _declare_timing(L):
    L.or_set_threads.restype = None
    L.or_set_threads.argtypes = [C.c_int]
    L.or_max_threads.restype = C.c_int
    L.or_max_threads.argtypes = []
    L.or_last_loop_seconds.restype = C.c_double
    L.or_last_loop_seconds.argtypes = []


_lib_omp = None


def lib_omp():
    """The OpenMP timing build (same source).  OMP_PROC_BIND / OMP_PLACES are
    read when it is first loaded."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP):
            build()
        L = C.CDLL(_LIB_OMP)
        dp, u8p, vp = C.POINTER(C.c_double), C.POINTER(C.c_uint8), C.c_void_p
        L.or_pcg_line.restype = C.c_int
        L.or_pcg_line.argtypes = [vp, u8p, C.c_int, dp, dp, dp, C.c_double, C.c_int, C.c_int64,
                                  C.POINTER(C.c_int), dp, dp, dp, dp, dp]
        _declare_timing(L)
        _lib_omp = L
    return _lib_omp


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _u8(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_uint8))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Matrix:
    """An oracle-owned CSR matrix (freed with the object)."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)
        self.n = int(lib().or_csr_n(self._h))
        self.nnz = int(lib().or_csr_nnz(self._h))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or_csr_free(self._h)
            self._h = None

    def arrays(self):
        rowptr = np.empty(self.n + 1, np.int64)
        col = np.empty(self.nnz, np.int32)
        val = np.empty(self.nnz, np.float64)
        lib().or_csr_copy_out(self._h, rowptr.ctypes.data_as(C.POINTER(C.c_int64)),
                              _i(col), _d(val))
        return rowptr, col, val

    def to_scipy(self):
        import scipy.sparse as sp
        rowptr, col, val = self.arrays()
        return sp.csr_matrix((val, col, rowptr), shape=(self.n, self.n))

    def matvec(self, x):
        x = _f64(x)
        y = np.empty(self.n, np.float64)
        lib().or_spmv(self._h, _d(x), _d(y))
        return y

    def rmatvec(self, x, ncols):
        x = _f64(x)
        y = np.empty(ncols, np.float64)
        lib().or_spmv_t(self._h, _d(x), _d(y), ncols)
        return y


def element(X, nu=(1.0, 1.0, 1.0)):
    """Element matrices of one tetrahedron: (vol, K 4x4, M 4x4, B 3x4x4)."""
    X = _f64(X).reshape(4, 3)
    nu = _f64(nu)
    K = np.empty(16)
    M = np.empty(16)
    B = np.empty(48)
    vol = lib().or_element(_d(X), _d(nu), _d(K), _d(M), _d(B))
    return vol, K.reshape(4, 4), M.reshape(4, 4), B.reshape(3, 4, 4)


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def _assemble(xyz, tets, form, nu_h=0.0, nu_v=0.0, c_mass=0.0, c_stiff=0.0, comp=0):
    xyz = _f64(xyz)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    h = C.c_void_p()
    st = lib().or_assemble(xyz.shape[0], _d(xyz), tets.shape[0], _i(tets), form, nu_h, nu_v,
                           c_mass, c_stiff, comp, C.byref(h))
    if st != OK:
        raise OracleError(st, "assemble")
    return Matrix(h.value)


def operator(mesh, nu_h, nu_v, c_mass, c_stiff):
    """c_mass * M + c_stiff * K_nu over the mesh (volume forms of Sec. 4/5)."""
    return _assemble(mesh.xyz, mesh.tets, 0, nu_h, nu_v, c_mass, c_stiff)


def helmholtz(mesh, nu_h, nu_v, dt):
    """Velocity-prediction operator M + dt*K_nu (one implicit Euler step)."""
    return operator(mesh, nu_h, nu_v, 1.0, dt)


def stiffness(mesh, nu_h, nu_v):
    """Anisotropic stiffness K_nu (pressure-increment operator)."""
    return operator(mesh, nu_h, nu_v, 0.0, 1.0)


def mass(mesh):
    return operator(mesh, 0.0, 0.0, 1.0, 0.0)


def divergence(mesh, comp):
    """B_c with (B_c)_ij = int phi_i d phi_j / d x_c."""
    return _assemble(mesh.xyz, mesh.tets, 1, comp=comp)


def hex_element(order, X8, nu=(1.0, 1.0, 1.0)):
    """Element matrices (K_nu, M) of one brick of order 1 or 2 from its 8
    corners (corner (c1,c2,c3) at row c1 + 2 c2 + 4 c3) and the smallest
    Jacobian determinant at the quadrature points."""
    X8 = _f64(X8).reshape(8, 3)
    nloc = (order + 1) ** 3
    K = np.empty((nloc, nloc))
    M = np.empty((nloc, nloc))
    det = lib().or_hex_element(order, _d(X8), _d(_f64(nu)), _d(K), _d(M))
    return K, M, det


def hex_operator(mesh, nu_h, nu_v, c_mass, c_stiff):
    """c_mass * M + c_stiff * K_nu over a brick mesh (mesh.hexes, mesh.order)."""
    xyz = _f64(mesh.xyz)
    hexes = np.ascontiguousarray(mesh.hexes, dtype=np.int32)
    h = C.c_void_p()
    st = lib().or_assemble_hex(xyz.shape[0], _d(xyz), hexes.shape[0], _i(hexes), mesh.order,
                               nu_h, nu_v, c_mass, c_stiff, C.byref(h))
    if st != OK:
        raise OracleError(st, "assemble_hex")
    return Matrix(h.value)


def hex_helmholtz(mesh, nu_h, nu_v, dt):
    """Velocity-prediction operator M + dt*K_nu on a brick mesh."""
    return hex_operator(mesh, nu_h, nu_v, 1.0, dt)


def hex_stiffness(mesh, nu_h, nu_v):
    return hex_operator(mesh, nu_h, nu_v, 0.0, 1.0)


def hex_mass(mesh):
    return hex_operator(mesh, 0.0, 0.0, 1.0, 0.0)


def surface_mass(mesh):
    xyz = _f64(mesh.xyz)
    tris = np.ascontiguousarray(mesh.surf_tris, dtype=np.int32)
    h = C.c_void_p()
    st = lib().or_assemble_surface_mass(xyz.shape[0], _d(xyz), tris.shape[0], _i(tris),
                                        C.byref(h))
    if st != OK:
        raise OracleError(st, "surface mass")
    return Matrix(h.value)


@dataclass
class PCGResult:
    x: np.ndarray
    status: int
    iterations: int
    relres: float
    removed_mean: float
    alphas: np.ndarray | None = None
    betas: np.ndarray | None = None
    x_hist: np.ndarray | None = None
    loop_s: float = 0.0


def pcg(A: Matrix, b, dirichlet=None, singular=False, weights=None, x0=None,
        tol=1e-10, maxit=100000, history=False, x_history=False, line=0,
        ic0=False, threads=0) -> PCGResult:
    """Preconditioned CG on A after eliminating `dirichlet` nodes (boolean (n,)
    or None).  line = 0: Jacobi (inverse diagonal); line = L >= 1: inverse of
    the tridiagonal blocks on the consecutive columns of L nodes; ic0: IC(0)
    of the eliminated matrix in the greedy multicolour order.

    threads = 0 runs the plain parity build; threads >= 1 runs the OpenMP
    timing build of the same source with that many threads (Jacobi or line
    blocks only; rounding differs from the plain build in the order of the
    dot-product sums).  The result's loop_s is the wall time of the iteration
    loop."""
    n = A.n
    b = _f64(b)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    dmask = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    w = None if weights is None else _f64(weights)
    it = C.c_int(0)
    rel = np.zeros(1)
    rm = np.zeros(1)
    ah = np.zeros(maxit) if history else None
    bh = np.zeros(maxit) if history else None
    xh = np.zeros((maxit, n)) if x_history else None
    hist = (None if ah is None else _d(ah), None if bh is None else _d(bh),
            None if xh is None else _d(xh))
    if threads and ic0:
        raise ValueError("the OpenMP timing build runs Jacobi or line blocks only")
    L = lib_omp() if threads else lib()
    if threads:
        L.or_set_threads(int(threads))
    if ic0:
        st = L.or_pcg_ic0(A._h, _u8(dmask), int(bool(singular)),
                          None if w is None else _d(w), _d(b), _d(x), tol, maxit,
                          C.byref(it), _d(rel), _d(rm), *hist)
    else:
        st = L.or_pcg_line(A._h, _u8(dmask), int(bool(singular)),
                           None if w is None else _d(w), _d(b), _d(x), tol, maxit, int(line),
                           C.byref(it), _d(rel), _d(rm), *hist)
    k = it.value
    return PCGResult(x=x, status=st, iterations=k, relres=float(rel[0]), removed_mean=float(rm[0]),
                     alphas=None if ah is None else ah[:k], betas=None if bh is None else bh[:k],
                     x_hist=None if xh is None else xh[:k], loop_s=float(L.or_last_loop_seconds()))


def greedy_colors(A: Matrix):
    """Greedy colouring of A's graph in node order: (colours (n,), count)."""
    color = np.empty(A.n, np.int32)
    k = lib().or_greedy_colors(A._h, _i(color))
    if k < 0:
        raise OracleError(k, "greedy_colors")
    return color, k


def ic0_factor(A: Matrix, dirichlet=None):
    """IC(0) of the eliminated A in the greedy multicolour order: (perm, L)
    with perm[k] the node at position k and L a Matrix (lower triangular,
    rows and columns in the permuted order)."""
    dmask = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    perm = np.empty(A.n, np.int32)
    h = C.c_void_p()
    st = lib().or_ic0_factor(A._h, _u8(dmask), _i(perm), C.byref(h))
    if st != OK:
        raise OracleError(st, "ic0_factor")
    return perm, Matrix(h.value)


def advection(mesh, u):
    """(3, n) array of int ((u . grad) u_c) phi_a dx for the P1 velocity u (3, n)."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, -1)
    xyz = _f64(mesh.xyz)
    tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
    n = xyz.shape[0]
    out = np.empty((3, n))
    st = lib().or_advection(n, _d(xyz), tets.shape[0], _i(tets), _d(u), _d(out))
    if st != OK:
        raise OracleError(st, "advection")
    return out


def tridiag_solve(d, e, r):
    """z = T^-1 r for the symmetric tridiagonal T = tridiag(e, d, e) (Thomas)."""
    d = _f64(d)
    e = _f64(e)
    r = _f64(r)
    L = d.shape[0]
    if e.shape[0] < max(L - 1, 0) or r.shape[0] != L:
        raise ValueError("tridiag_solve: need len(e) >= len(d) - 1 and len(r) == len(d)")
    e = np.concatenate([e[:max(L - 1, 0)], np.zeros(1)])
    z = np.empty(L)
    work = np.empty(L)
    st = lib().or_tridiag_solve(L, _d(d), _d(e), _d(r), _d(z), _d(work))
    if st != OK:
        raise OracleError(st, "tridiag_solve")
    return z


def relres(A: Matrix, b, x, dirichlet=None) -> float:
    b = _f64(b)
    x = _f64(x)
    dmask = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    return float(lib().or_relres(A._h, _u8(dmask), _d(b), _d(x)))


def cholesky_solve(A_dense, b):
    A_dense = _f64(A_dense)
    b = _f64(b)
    n = b.shape[0]
    x = np.empty(n)
    st = lib().or_cholesky_solve(n, _d(A_dense), _d(b), _d(x))
    if st != OK:
        raise OracleError(st, "cholesky")
    return x


def lanczos_condition(alphas, betas):
    """Extreme-eigenvalue ratio of the preconditioned operator from the CG
    coefficients (the Lanczos tridiagonal matrix built from alpha and beta)."""
    k = len(alphas)
    if k == 0:
        return 1.0
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(max(betas[j], 0.0)) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    return float(ev[-1] / ev[0])
