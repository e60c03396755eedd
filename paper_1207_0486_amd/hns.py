"""Python binding of the hns library.

Argument marshalling only: every step of assembly and solve runs in libhns.so
(host C++ assembly, HIP kernels for the solves).  PyTorch supplies device
memory and streams.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

KINDS = {"poisson": L.HNS_POISSON, "helmholtz": L.HNS_HELMHOLTZ}
FORMATS = {"auto": L.HNS_FMT_AUTO, "csr": L.HNS_FMT_CSR, "sell": L.HNS_FMT_SELL,
           "sdia": L.HNS_FMT_SDIA}
FORMAT_NAMES = {L.HNS_FMT_CSR: "csr", L.HNS_FMT_SELL: "sell", L.HNS_FMT_SDIA: "sdia",
                L.HNS_MATRIX_FREE: "matrix-free"}
MODES = {"fp64": L.HNS_FP64, "mixed": L.HNS_MIXED}


class HNSError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = L.lib().hns_last_error().decode(errors="replace")
        name = L.lib().hns_status_string(status).decode()
        super().__init__(f"{where}: {name} ({status}): {msg}")
        self.status = status


@dataclass
class SolveInfo:
    iterations: int
    outer_iterations: int
    relres_true: float
    removed_mean: float
    status: int

    @property
    def converged(self) -> bool:
        return self.status == L.HNS_OK

    @classmethod
    def _from(cls, s: L.hns_solve_info) -> "SolveInfo":
        return cls(int(s.iterations), int(s.outer_iterations), float(s.relres_true),
                   float(s.removed_mean), int(s.status))


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_f64(t: torch.Tensor, name: str, n: int | None = None, k: int | None = None,
             rows: int | None = None):
    """Device pointer of a contiguous float64 tensor of shape (n,), (n, k) or
    (rows, n); None passes through as NULL."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if n is not None:
        want = (rows, n) if rows is not None else ((n,) if k is None else (n, k))
        if tuple(t.shape) != want:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {want}")
    return C.c_void_p(t.data_ptr())


class Operator:
    """A device-resident assembled operator.

    kind="helmholtz": A = M + dt K_nu (velocity prediction);
    kind="poisson":   A = K_nu        (pressure increment).
    `mesh` is any object with xyz (n,3) float64, tets (T,4) int32, bc (n,)
    uint8 (optional) and surf_tris (S,3) int32 (optional); or a brick mesh
    with xyz, hexes (E,(order+1)**3) int32, order (1: Q1, 2: Q2) and bc
    (hns_assemble_hex; matrix_free=True: no stored matrix, element-by-element
    products, FP64 solves only).
    """

    def __init__(self, mesh, nu_h: float, nu_v: float, dt: float = 0.0, kind: str = "helmholtz",
                 keep_fp32: bool = False, step_aux: bool = False, fmt: str = "auto",
                 device: int | torch.device | None = None, gpu_assembly: bool = False,
                 keep_host: bool = False, matrix_free: bool = False):
        self._h = None
        self.kind = kind
        flags = KINDS[kind] | FORMATS[fmt]
        if matrix_free:
            flags |= L.HNS_MATRIX_FREE
        if keep_fp32:
            flags |= L.HNS_KEEP_FP32
        if step_aux:
            flags |= L.HNS_STEP_AUX
        if gpu_assembly:
            flags |= L.HNS_GPU_ASSEMBLY
        if keep_host:
            flags |= L.HNS_KEEP_HOST
        xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        bc = getattr(mesh, "bc", None)
        bc = None if bc is None else np.ascontiguousarray(bc, dtype=np.uint8)
        hexes = getattr(mesh, "hexes", None)
        if hexes is not None:
            hexes = np.ascontiguousarray(hexes, dtype=np.int32)
            m = L.hns_hex_mesh()
            m.n_nodes = xyz.shape[0]
            m.xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
            m.n_hex = hexes.shape[0]
            m.order = int(mesh.order)
            m.hex = hexes.ctypes.data_as(C.POINTER(C.c_int32))
            m.bc = None if bc is None else bc.ctypes.data_as(C.POINTER(C.c_uint8))
            assemble = L.lib().hns_assemble_hex
        else:
            tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
            tris = getattr(mesh, "surf_tris", None)
            tris = None if tris is None else np.ascontiguousarray(tris, dtype=np.int32)
            m = L.hns_mesh()
            m.n_nodes = xyz.shape[0]
            m.xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
            m.n_tets = tets.shape[0]
            m.tets = tets.ctypes.data_as(C.POINTER(C.c_int32))
            m.bc = None if bc is None else bc.ctypes.data_as(C.POINTER(C.c_uint8))
            m.n_surf_tris = 0 if tris is None else tris.shape[0]
            m.surf_tris = None if tris is None else tris.ctypes.data_as(C.POINTER(C.c_int32))
            assemble = L.lib().hns_assemble
        if device is None:
            idx = torch.cuda.current_device()
        elif isinstance(device, torch.device):
            idx = device.index or 0
        else:
            idx = int(device)
        self.device = torch.device("cuda", idx)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = assemble(C.byref(m), nu_h, nu_v, dt, flags, C.byref(h))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_assemble_hex" if hexes is not None else "hns_assemble")
        self._h = h
        self.n = int(L.lib().hns_operator_n(h))
        self.nnz = int(L.lib().hns_operator_nnz(h))
        self.format = FORMAT_NAMES.get(int(L.lib().hns_operator_format(h)), "?")
        self.ndiag = int(L.lib().hns_operator_ndiag(h))
        self.line_len = int(L.lib().hns_operator_line_len(h))
        # 0 host, 1 values on the device (host pattern), 2 built on the device
        self.assembly = int(L.lib().hns_operator_assembly(h))
        self.keep_fp32 = keep_fp32

    # -- lifetime -------------------------------------------------------
    def close(self):
        if self._h is not None:
            L.lib().hns_operator_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries ------------------------------------------------------------
    def footprint(self, k: int = 1, mode: str = "fp64", include_operator: bool = True) -> int:
        return int(L.lib().hns_footprint_bytes(self._h, k, MODES[mode], int(include_operator)))

    def set_param(self, name: str, value: float):
        st = L.lib().hns_set_param(self._h, name.encode(), float(value))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_set_param")

    def profile(self, period: int = 1):
        """Time every `period`-th CG iteration with HIP events (0 = off)."""
        st = L.lib().hns_profile_enable(self._h, int(period))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_profile_enable")

    def profile_read(self):
        """{kernel: (total_ms, launches)} for spmv/update/pupdate (fp64, fp32)."""
        names = ["spmv", "update", "pupdate", "spmv32", "update32", "pupdate32"]
        out = {}
        for k, name in enumerate(names):
            ms = C.c_double()
            cnt = C.c_int64()
            st = L.lib().hns_profile_read(self._h, k, C.byref(ms), C.byref(cnt))
            if st != L.HNS_OK:
                raise HNSError(st, "hns_profile_read")
            out[name] = (ms.value, cnt.value)
        return out

    # -- compute ------------------------------------------------------------
    def apply(self, x: torch.Tensor, mask_bit: int = -1, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        xp = _dev_f64(x, "x", self.n)
        y = torch.empty_like(x) if out is None else out
        yp = _dev_f64(y, "out", self.n)
        with torch.cuda.device(self.device):
            st = L.lib().hns_apply(self._h, mask_bit, xp, yp, _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_apply")
        return y

    # -- projection-step right-hand sides (operators with step_aux=True) ----
    def step_velocity_rhs(self, u, p=None, theta=None, f=None, out=None, stream=None):
        """b_c = M u_c + dt (M_s theta_c + C_c + B_c^T p) for c = 1..3 (u: 3 x n)."""
        b = torch.empty_like(u) if out is None else out
        st = L.lib().hns_step_velocity_rhs(
            self._h, _dev_f64(u, "u", self.n, rows=3), _dev_f64(p, "p", self.n),
            _dev_f64(theta, "theta", self.n, rows=2), _dev_f64(f, "f", self.n),
            _dev_f64(b, "out", self.n, rows=3), _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_step_velocity_rhs")
        return b

    def step_pressure_rhs(self, ut, out=None, stream=None):
        """b = -(1/dt) sum_c B_c ut_c (ut: 3 x n)."""
        b = torch.empty(self.n, dtype=torch.float64, device=ut.device) if out is None else out
        st = L.lib().hns_step_pressure_rhs(self._h, _dev_f64(ut, "ut", self.n, rows=3),
                                           _dev_f64(b, "out", self.n), _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_step_pressure_rhs")
        return b

    def step_correct(self, ut, q, p=None, out=None, stream=None):
        """p += q; u_c = ut_c - dt (B_c q) / m_L (masked).  Returns u (3 x n)."""
        u = torch.empty_like(ut) if out is None else out
        st = L.lib().hns_step_correct(self._h, _dev_f64(ut, "ut", self.n, rows=3),
                                      _dev_f64(q, "q", self.n), _dev_f64(p, "p", self.n),
                                      _dev_f64(u, "out", self.n, rows=3), _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_step_correct")
        return u

    def step_advection(self, u, out=None, stream=None):
        """out_c = int ((u . grad) u_c) phi (u: 3 x n).  Returns out (3 x n)."""
        a = torch.empty_like(u) if out is None else out
        st = L.lib().hns_step_advection(self._h, _dev_f64(u, "u", self.n, rows=3),
                                        _dev_f64(a, "out", self.n, rows=3),
                                        _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_step_advection")
        return a

    def step_velocity_rhs_bdf(self, tau, a1, u, a2=0.0, u_prev=None, p=None, theta=None,
                              f=None, adv=None, out=None, stream=None):
        """b_c = a1 M u_c + a2 M u'_c + tau (M_s theta_c + C_c - adv_c + B_c^T p)."""
        b = torch.empty_like(u) if out is None else out
        st = L.lib().hns_step_velocity_rhs_bdf(
            self._h, float(tau), float(a1), _dev_f64(u, "u", self.n, rows=3), float(a2),
            _dev_f64(u_prev, "u_prev", self.n, rows=3), _dev_f64(p, "p", self.n),
            _dev_f64(theta, "theta", self.n, rows=2), _dev_f64(f, "f", self.n),
            _dev_f64(adv, "adv", self.n, rows=3), _dev_f64(b, "out", self.n, rows=3),
            _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_step_velocity_rhs_bdf")
        return b

    def step_pressure_rhs_tau(self, tau, ut, out=None, stream=None):
        """b = -(1/tau) sum_c B_c ut_c."""
        b = torch.empty(self.n, dtype=torch.float64, device=ut.device) if out is None else out
        st = L.lib().hns_step_pressure_rhs_tau(self._h, float(tau),
                                               _dev_f64(ut, "ut", self.n, rows=3),
                                               _dev_f64(b, "out", self.n), _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_step_pressure_rhs_tau")
        return b

    def step_correct_rhs(self, tau, ut, q, p=None, out=None, stream=None):
        """p += q; rhs_c = M ut_c - tau B_c q (masked).  Returns rhs (3 x n)."""
        r = torch.empty_like(ut) if out is None else out
        st = L.lib().hns_step_correct_rhs(self._h, float(tau), _dev_f64(ut, "ut", self.n, rows=3),
                                          _dev_f64(q, "q", self.n), _dev_f64(p, "p", self.n),
                                          _dev_f64(r, "out", self.n, rows=3),
                                          _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_step_correct_rhs")
        return r

    AUX = {"M": 0, "B1": 1, "B2": 2, "B3": 3, "B1T": 4, "B2T": 5, "B3T": 6, "Ms": 7}

    def apply_aux(self, which: str, x, out=None, stream=None):
        y = torch.empty_like(x) if out is None else out
        st = L.lib().hns_apply_aux(self._h, self.AUX[which], _dev_f64(x, "x", self.n),
                                   _dev_f64(y, "out", self.n), _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_apply_aux")
        return y

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-10,
              max_iter: int = 100000, mode: str = "fp64", mask_bit: int = -1, stream=None,
              check: bool = True):
        """Solve A x = b; returns (x, SolveInfo).  x (if given) is the initial
        guess and is overwritten in place."""
        bp = _dev_f64(b, "b", self.n)
        if x is None:
            x = torch.zeros_like(b)
        xp = _dev_f64(x, "x", self.n)
        info = L.hns_solve_info()
        with torch.cuda.device(self.device):
            st = L.lib().hns_solve(self._h, mask_bit, bp, xp, tol, max_iter, MODES[mode],
                                   _stream_handle(stream), C.byref(info))
        if st < 0 and check:
            raise HNSError(st, "hns_solve")
        return x, SolveInfo._from(info)

    def solve_noalloc(self, b: torch.Tensor, x: torch.Tensor, tol: float = 1e-10,
                      max_iter: int = 100000, mode: str = "fp64", mask_bit: int = -1,
                      stream=None, check: bool = True):
        """hns_solve_noalloc: the solve of `solve` with its workspace in the
        library's static device scratch (no device allocation; x, the initial
        guess, is required and overwritten).  Returns (x, SolveInfo)."""
        bp = _dev_f64(b, "b", self.n)
        xp = _dev_f64(x, "x", self.n)
        info = L.hns_solve_info()
        with torch.cuda.device(self.device):
            st = L.lib().hns_solve_noalloc(self._h, mask_bit, bp, xp, tol, max_iter, MODES[mode],
                                           _stream_handle(stream), C.byref(info))
        if st < 0 and check:
            raise HNSError(st, "hns_solve_noalloc")
        return x, SolveInfo._from(info)

    def noalloc_bytes(self, mode: str = "fp64") -> int:
        """Scratch bytes hns_solve_noalloc needs for this operator in `mode`."""
        return int(L.lib().hns_noalloc_bytes(self._h, MODES[mode]))

    @staticmethod
    def noalloc_scratch_bytes() -> int:
        """Size of the static scratch of hns_solve_noalloc (per GPU)."""
        return int(L.lib().hns_noalloc_scratch_bytes())

    def tune_batched(self, k: int, mode: str = "fp64", stream=None):
        """Time the batched product for k columns: the grid-stride product at
        1/2/4 columns per thread and the LDS-tiled product in its shapes 1..3;
        returns ({"w1"/"w2"/"w4"/"tile1".."tile3": microseconds}, plan) with
        plan = width + 8 * tiled shape (0: none)."""
        times = (C.c_double * 6)()
        best = C.c_int()
        with torch.cuda.device(self.device):
            st = L.lib().hns_tune_batched(self._h, k, MODES[mode], _stream_handle(stream), times,
                                          C.byref(best))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_tune_batched")
        names = ("w1", "w2", "w4", "tile1", "tile2", "tile3")
        return {nm: times[i] for i, nm in enumerate(names) if times[i] >= 0}, best.value

    def solve_batched(self, B: torch.Tensor, X: torch.Tensor | None = None, mask_bits=None,
                      tol: float = 1e-10, max_iter: int = 100000, mode: str = "fp64",
                      stream=None, check: bool = True):
        """Solve A X[:, j] = B[:, j] for the k columns of the n x k row-major B."""
        if B.dim() != 2:
            raise ValueError("B must be n x k")
        k = int(B.shape[1])
        Bp = _dev_f64(B, "B", self.n, k)
        if X is None:
            X = torch.zeros_like(B)
        Xp = _dev_f64(X, "X", self.n, k)
        if mask_bits is None:
            mask_bits = [-1] * k
        bits = (C.c_int * k)(*[int(v) for v in mask_bits])
        infos = (L.hns_solve_info * k)()
        with torch.cuda.device(self.device):
            st = L.lib().hns_solve_batched(self._h, k, bits, Bp, Xp, tol, max_iter, MODES[mode],
                                           _stream_handle(stream), infos)
        if st < 0 and check:
            raise HNSError(st, "hns_solve_batched")
        return X, [SolveInfo._from(infos[j]) for j in range(k)]


class BatchSession:
    """Fixed-capacity slots of a continuously batched multi-RHS recurrence on
    one operator (hns_batch_*): requests join free slots at any time, advance
    together, and leave when finished."""

    def __init__(self, op: Operator, capacity: int, mode: str = "fp64"):
        self.op = op
        self.capacity = capacity
        self.mode = mode
        h = C.c_void_p()
        with torch.cuda.device(op.device):
            st = L.lib().hns_batch_open(op._h, capacity, MODES[mode], C.byref(h))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_batch_open")
        self._h = h

    @staticmethod
    def footprint(op: Operator, capacity: int, mode: str = "fp64") -> int:
        return int(L.lib().hns_batch_footprint(op._h, capacity, MODES[mode]))

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lib().hns_batch_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, slots, mask_bits, bs, tols, max_iters, stream=None):
        k = len(slots)
        ptrs = (C.c_void_p * k)(*[_dev_f64(b, "b", self.op.n).value for b in bs])
        with torch.cuda.device(self.op.device):
            st = L.lib().hns_batch_add(
                self._h, k, (C.c_int * k)(*slots), (C.c_int * k)(*mask_bits), ptrs,
                (C.c_double * k)(*tols), (C.c_int * k)(*max_iters), _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_batch_add")

    def advance(self, iterations: int, stream=None) -> int:
        active = C.c_int()
        with torch.cuda.device(self.op.device):
            st = L.lib().hns_batch_advance(self._h, iterations, _stream_handle(stream),
                                           C.byref(active))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_batch_advance")
        return active.value

    def poll(self, stream=None):
        """(states, infos): state 0 free, 1 running, 2 finished per slot."""
        k = self.capacity
        states = (C.c_int * k)()
        infos = (L.hns_solve_info * k)()
        with torch.cuda.device(self.op.device):
            st = L.lib().hns_batch_poll(self._h, states, infos, _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_batch_poll")
        return list(states), [SolveInfo._from(infos[j]) for j in range(k)]

    def take(self, slot: int, out: torch.Tensor | None = None, stream=None):
        x = torch.empty(self.op.n, dtype=torch.float64, device=self.op.device) if out is None \
            else out
        info = L.hns_solve_info()
        with torch.cuda.device(self.op.device):
            st = L.lib().hns_batch_take(self._h, slot, _dev_f64(x, "out", self.op.n),
                                        C.byref(info), _stream_handle(stream))
        if st != L.HNS_OK:
            raise HNSError(st, "hns_batch_take")
        return x, SolveInfo._from(info)
