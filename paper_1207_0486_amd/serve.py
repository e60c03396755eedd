"""Continuous-batching serving loop for PCG solve requests.

Requests (a right-hand side for one resident operator: a mesh and a kind,
Poisson or Helmholtz) arrive at any time.  The server

  * admits an operator by its HBM footprint (operator + batch session) and
    keeps it resident; when the budget is short it evicts idle operators in
    least-recently-used order, otherwise the request waits (first come,
    first served);
  * runs one batch session per resident operator, each on its own worker
    thread and device stream, so different operators' solves overlap on the
    GPU;
  * lets new requests join a session's free slots at every chunk boundary
    while the slots already running keep iterating (continuous batching), and
    hands each result back as soon as its own slot finishes;
  * records per-request latency (arrival to result on the host) and
    throughput.

The device work goes through a backend (the GPU backend drives libhns.so;
tests substitute a fake backend with the same interface to check the
scheduling logic without a GPU).
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    key: tuple                 # operator key, e.g. (mesh_index, "poisson")
    b: np.ndarray              # right-hand side (host, float64)
    mask_bit: int = -1
    tol: float = 1e-8
    max_iter: int = 100000
    arrival: float = 0.0       # time.perf_counter() at submission
    future: Future = field(default_factory=Future)


@dataclass
class Result:
    x: np.ndarray
    info: object
    latency_s: float
    key: tuple


class GpuBackend:
    """Operators and batch sessions on one GPU.

    make_operator(key) -> (mesh, nu_h, nu_v, dt, kind) describes the operator
    of a key; it is assembled on first use.
    """

    def __init__(self, make_operator, device=0, mode="fp64", check_every=16,
                 gpu_assembly=True, line_pressure=False):
        import torch
        self.torch = torch
        self.gpu_assembly = gpu_assembly   # operators built on the device
        # Poisson requests on water-column numberings with the line
        # preconditioner (per-slot sessions run it; see hns_batch_open)
        self.line_pressure = line_pressure
        self._make = make_operator
        self._made = {}
        self._made_lock = threading.Lock()
        self.device = torch.device("cuda", device)
        self.mode = mode
        self.check_every = check_every

    def make_operator(self, key):
        with self._made_lock:
            if key not in self._made:
                self._made[key] = self._make(key)
            return self._made[key]

    def estimate_bytes(self, key, capacity):
        """Upper estimate of operator + session bytes before assembly."""
        mesh = self.make_operator(key)[0]
        n = int(mesh.xyz.shape[0])
        vb = 12 if self.mode == "mixed" else 8
        op_bytes = n * (16 * (vb + 4) + vb + 17)          # generous: 16 nonzeros per row
        sess = n * capacity * (8 * 5 + (16 if self.mode == "mixed" else 0)) + 3 * 2048 * 8 * capacity
        return op_bytes + sess

    def open(self, key, capacity):
        from .hns import BatchSession, Operator
        mesh, nu_h, nu_v, dt, kind = self.make_operator(key)
        with self.torch.cuda.device(self.device):
            op = Operator(mesh, nu_h, nu_v, dt, kind=kind, keep_fp32=self.mode == "mixed",
                          device=self.device, gpu_assembly=self.gpu_assembly)
            op.set_param("check_every", self.check_every)
            op.set_param("use_graph", 1)
            if self.line_pressure and kind == "poisson" and op.line_len >= 2:
                op.set_param("precond", 1)
            sess = BatchSession(op, capacity, self.mode)
            stream = self.torch.cuda.Stream(device=self.device)
        nbytes = op.footprint(1, self.mode, True) + BatchSession.footprint(op, capacity, self.mode)
        return _GpuEntry(self.torch, op, sess, stream, nbytes)


class _GpuEntry:
    def __init__(self, torch, op, sess, stream, nbytes):
        self.torch = torch
        self.op = op
        self.sess = sess
        self.stream = stream
        self.nbytes = nbytes
        self.n = op.n

    def add(self, items):
        """items: list of (slot, Request)."""
        t = self.torch
        with t.cuda.stream(self.stream):
            bs = [t.as_tensor(np.ascontiguousarray(r.b, dtype=np.float64),
                              device=self.op.device) for _, r in items]
            self.stream.synchronize()
            self.sess.add([s for s, _ in items], [r.mask_bit for _, r in items], bs,
                          [r.tol for _, r in items], [r.max_iter for _, r in items],
                          stream=self.stream)

    def advance(self, iterations):
        return self.sess.advance(iterations, stream=self.stream)

    def poll(self):
        return self.sess.poll(stream=self.stream)

    def take(self, slot):
        x, info = self.sess.take(slot, stream=self.stream)
        return x.cpu().numpy(), info

    def close(self):
        self.sess.close()
        self.op.close()


class _Resident:
    """A resident operator with its session, pending queue and worker.

    `pending` and `running` change only under the server's lock.  A request
    moves from `pending` to `running` in the same critical section that
    assigns its slot, so a resident is idle (and may be evicted) only while
    its worker holds no request at all."""

    def __init__(self, key, entry, capacity):
        self.key = key
        self.entry = entry
        self.capacity = capacity
        self.pending = collections.deque()
        self.running = {}            # slot -> Request (being added or iterating)
        self.last_used = time.perf_counter()
        self.thread = None
        self.evicted = False

    @property
    def idle(self):
        return not self.pending and not self.running


class ServerClosed(RuntimeError):
    """The server stopped before the request finished."""


class Server:
    """Continuous-batching server over a backend.

    budget_bytes: device memory the server may hold (operators + sessions);
    capacity: slots per operator session; chunk: iterations between
    admission points.

    Threads: one worker per resident operator (adds, advances and takes its
    session's requests) and one admission thread, which alone assembles
    operators and evicts idle ones, so neither a submitting thread nor a
    worker with running requests ever waits for an assembly.  An evicted
    operator's worker closes its session and operator before the admission
    thread opens the next one, so the device never holds more than the
    budget.  A worker that ends for any reason (eviction, close, an error)
    unregisters its operator and releases its bytes; requests it still held
    fail with the error (or ServerClosed), and later requests for the same
    operator get a fresh one.
    """

    def __init__(self, backend, budget_bytes, capacity=8, chunk=32):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.capacity = capacity
        self.chunk = chunk
        self.lock = threading.Condition()
        self.resident = {}                       # key -> _Resident
        self.waiting = collections.deque()       # requests whose operator is not admitted
        self.used = 0
        self.results = []
        self.events = []                         # (time, what, key) admission log
        self.stop_flag = False
        self.errors = []
        self.peak_used = 0
        self.workers = []                        # every worker thread started
        self._admitter = threading.Thread(target=self._admit_loop, daemon=True)
        self._admitter.start()

    # ------------------------------------------------------------------
    def submit(self, req: Request) -> Future:
        req.arrival = time.perf_counter() if not req.arrival else req.arrival
        with self.lock:
            if self.stop_flag:
                req.future.set_exception(ServerClosed("server is closed"))
                return req.future
            res = self.resident.get(req.key)
            if res is not None:
                res.pending.append(req)
            else:
                self.waiting.append(req)
            self.lock.notify_all()
        return req.future

    def close(self):
        with self.lock:
            self.stop_flag = True
            self.lock.notify_all()
        self._admitter.join()
        for t in list(self.workers):
            t.join()
        with self.lock:
            left = list(self.waiting)
            self.waiting.clear()
        for req in left:
            if not req.future.done():
                req.future.set_exception(ServerClosed("server closed before admission"))

    # ------------------------------------------------------------------
    def _admit_loop(self):
        while True:
            with self.lock:
                if self.stop_flag:
                    return
            progressed = self._admit()
            if not progressed:
                with self.lock:
                    if self.stop_flag:
                        return
                    self.lock.wait(timeout=0.05)

    def _admit(self):
        """Admit the head of the waiting queue (first come, first served):
        hand it to its resident operator, or open the operator when the
        budget allows, evicting idle operators in least-recently-used order.
        Returns whether anything changed."""
        with self.lock:
            if not self.waiting or self.stop_flag:
                return False
            req = self.waiting[0]
            res = self.resident.get(req.key)
            if res is not None:                  # admitted meanwhile
                self.waiting.popleft()
                res.pending.append(req)
                self.lock.notify_all()
                return True
            need = self.backend.estimate_bytes(req.key, self.capacity)
            if need > self.budget:
                self.waiting.popleft()
                req.future.set_exception(MemoryError(
                    f"operator {req.key} needs {need} bytes, budget is {self.budget}"))
                return True
            if self.used + need > self.budget:
                # evict idle operators (least recently used first) until it fits
                victims, freed = [], 0
                for r in sorted((r for r in self.resident.values() if r.idle),
                                key=lambda r: r.last_used):
                    if self.used - freed + need <= self.budget:
                        break
                    victims.append(r)
                    freed += r.entry.nbytes
                if self.used - freed + need > self.budget:
                    return False                 # wait for memory
                for r in victims:
                    self._evict(r)
            else:
                victims = []
                self.used += need                # reserve while assembling
                self.waiting.popleft()
        if victims:
            # the victims' workers close their sessions and release the bytes
            for r in victims:
                r.thread.join()
            return True
        try:
            entry = self.backend.open(req.key, self.capacity)
        except Exception as e:  # noqa: BLE001 - reported through the future
            with self.lock:
                self.used -= need
            req.future.set_exception(e)
            return True
        with self.lock:
            self.used += entry.nbytes - need
            self.peak_used = max(self.peak_used, self.used)
            res = _Resident(req.key, entry, self.capacity)
            res.pending.append(req)
            # requests for the same key that queued behind it join too
            for other in [w for w in self.waiting if w.key == req.key]:
                self.waiting.remove(other)
                res.pending.append(other)
            self.resident[req.key] = res
            self.events.append((time.perf_counter(), "admit", req.key))
            res.thread = threading.Thread(target=self._worker, args=(res,), daemon=True)
            self.workers.append(res.thread)
            res.thread.start()
        return True

    def _evict(self, res):
        # lock held; res is idle, so its worker holds no request and exits at
        # its next look at the flag
        del self.resident[res.key]
        res.evicted = True
        self.events.append((time.perf_counter(), "evict", res.key))
        self.lock.notify_all()

    def _retire(self, res, error):
        """End of a worker: unregister the operator, release its bytes, fail
        the requests it still held, close its session and operator."""
        with self.lock:
            if self.resident.get(res.key) is res:
                del self.resident[res.key]
            held = list(res.running.values()) + list(res.pending)
            res.running.clear()
            res.pending.clear()
        for req in held:
            if not req.future.done():
                req.future.set_exception(
                    error if error is not None else ServerClosed("server closed"))
        try:
            res.entry.close()
        except Exception as e:  # noqa: BLE001
            with self.lock:
                self.errors.append(e)
        with self.lock:
            self.used -= res.entry.nbytes
            self.lock.notify_all()

    def _worker(self, res: _Resident):
        entry = res.entry
        free = list(range(res.capacity))
        error = None
        try:
            while True:
                with self.lock:
                    while (not res.pending and not res.running and not self.stop_flag
                           and not res.evicted):
                        self.lock.wait(timeout=0.05)
                    if self.stop_flag or res.evicted:
                        break
                    batch = []
                    while res.pending and free:
                        slot = free.pop(0)
                        req = res.pending.popleft()
                        res.running[slot] = req
                        batch.append((slot, req))
                    res.last_used = time.perf_counter()
                if batch:
                    entry.add(batch)
                entry.advance(self.chunk)
                states, infos = entry.poll()
                for slot in [s for s in list(res.running) if states[s] == 2]:
                    x, info = entry.take(slot)
                    free.append(slot)
                    with self.lock:
                        req = res.running.pop(slot)
                    r = Result(x, info, time.perf_counter() - req.arrival, req.key)
                    with self.lock:
                        self.results.append(r)
                    req.future.set_result(r)
                with self.lock:
                    res.last_used = time.perf_counter()
                    if res.idle:
                        self.lock.notify_all()
        except Exception as e:  # noqa: BLE001 - surfaced to the waiting requests
            error = e
            with self.lock:
                self.errors.append(e)
        finally:
            self._retire(res, error)

    # ------------------------------------------------------------------
    def stats(self, t0=None, t1=None):
        lat = np.array([r.latency_s for r in self.results])
        out = {"completed": int(lat.size)}
        if lat.size:
            out.update({"p50_ms": float(np.percentile(lat, 50) * 1e3),
                        "p99_ms": float(np.percentile(lat, 99) * 1e3),
                        "mean_ms": float(lat.mean() * 1e3),
                        "max_ms": float(lat.max() * 1e3)})
        if t0 is not None and t1 is not None and t1 > t0:
            out["solves_per_s"] = float(lat.size / (t1 - t0))
        by_key = {}
        for r in self.results:
            by_key.setdefault(r.key, []).append(r.latency_s)
        out["by_key"] = {k: {"completed": len(v),
                             "p50_ms": float(np.percentile(v, 50) * 1e3),
                             "p99_ms": float(np.percentile(v, 99) * 1e3)}
                         for k, v in by_key.items()}
        out["peak_bytes"] = int(self.peak_used)
        out["admissions"] = sum(1 for e in self.events if e[1] == "admit")
        out["evictions"] = sum(1 for e in self.events if e[1] == "evict")
        return out
