"""Benchmark of the projection-step PCG solves on one MI355X.

One step = one projection time step on the 256x256x20 Atlantic-shaped basin
(1,387,029 nodes, Sec. 3 implicit-Euler form): the velocity right-hand sides
(mass, wind-tension load, explicit Coriolis, pressure gradient), three
velocity-prediction solves (M + dt K_nu, one per component with its own
Dirichlet set), the pressure-increment right-hand side, one pure-Neumann
pressure solve (K_nu) and the correction, all solves to relative residual
1e-10.  Every timed step restarts from the state after a first step from
rest (so all three velocity components are nontrivial).  FP64 first, then
mixed precision (FP32 CG with FP64 residual replacement).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PCG time-to-1e-10 and HBM GB/s at 1.3M nodes, FP64 vs mixed; p99 latency"
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def matrix_bytes(fmt, n, nnz, value_bytes):
    """Algorithmic bytes of one read of the operator in the storage format the
    solve runs: symmetric diagonal storage reads the unique values of the
    symmetric matrix ((nnz + n) / 2 of them) and no indices; CSR and sliced
    ELL read every value, its column index and the row pointers."""
    if fmt == "sdia":
        return value_bytes * (nnz + n) // 2
    return (value_bytes + 4) * nnz + 4 * (n + 1)


def bytes_iter(fmt, n, nnz, vb):
    """One CG iteration: one operator read plus 13 vector passes (SpMV reads p
    and writes q; the update reads x, p, r, q, D^-1 and writes x, r; the
    direction update reads r, D^-1, p and writes p)."""
    return matrix_bytes(fmt, n, nnz, vb) + 13 * vb * n


def bytes_spmv(fmt, n, nnz, vb):
    """The SpMV kernel alone: operator + read p + write q."""
    return matrix_bytes(fmt, n, nnz, vb) + 2 * vb * n


def bytes_residual(fmt, n, nnz):
    """FP64 true residual b - A x: operator + read x, b + write r."""
    return matrix_bytes(fmt, n, nnz, 8) + 3 * 8 * n


def solve_bytes(info, fmt, n, nnz, mode):
    if mode == "fp64":
        return info.iterations * bytes_iter(fmt, n, nnz, 8)
    return (info.iterations * bytes_iter(fmt, n, nnz, 4)
            + (info.outer_iterations + 1) * (bytes_residual(fmt, n, nnz) + 8 * 3 * n))


def make_forcing(m):
    import basin
    L = m.Ly
    theta = np.stack([basin.wind_tension(m.xyz[:, 1], L), np.zeros(m.n)])
    f = basin.coriolis_parameter(m.xyz[:, 1], L)
    return theta, f


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--check-every", type=int, default=32)
    ap.add_argument("--cpu-iters", type=int, default=1000,
                    help="oracle PCG iterations in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--fmt", default="auto")
    ap.add_argument("--profile-period", type=int, default=16,
                    help="time every N-th CG iteration with HIP events (0 = off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver "
              "does not shard across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    import basin
    from paper_1207_0486_amd.step import ProjectionStep

    wl = basin.configs.BASIN_256x256x20
    dev = torch.device("cuda", 0)
    t0 = time.time()
    m = wl.mesh()
    theta, f = make_forcing(m)
    log(f"mesh {wl.name}: n={m.n} tets={m.n_tets} ({time.time() - t0:.1f}s)")
    t0 = time.time()
    st = ProjectionStep(m, wl.nu_h, wl.nu_v, wl.dt, theta, f, device=dev, fmt=args.fmt)
    helm, pois = st.helm, st.pois
    for op in (helm, pois):
        op.set_param("check_every", args.check_every)
        op.set_param("mixed_variant", 0)
    helm.set_param("replace_drop", 1e-3)
    pois.set_param("replace_drop", 0.1)
    log(f"assembled: nnz={pois.nnz} format={pois.format} ({time.time() - t0:.1f}s)")
    n, nnz = pois.n, pois.nnz

    # time step 0 from rest (untimed) gives the state every timed step starts from
    t0 = time.time()
    r0 = st.step(tol=wl.tol)
    u1, p1 = st.state()
    log(f"step 0 from rest: iters {[i.iterations for i in r0.velocity]} / "
        f"{r0.pressure.iterations} ({time.time() - t0:.1f}s)")

    def one_step(mode):
        st.set_state(u1, p1)
        res = st.step(tol=wl.tol, mode=mode)
        infos = {f"u{c + 1}": res.velocity[c] for c in range(3)}
        infos["q"] = res.pressure
        return infos

    def timed(mode, steps, warmup, profile):
        for _ in range(warmup):
            one_step(mode)
        for op in (helm, pois):
            op.profile(profile)
        torch.cuda.synchronize()
        t = time.perf_counter()
        per = []
        infos = None
        for _ in range(steps):
            ts = time.perf_counter()
            infos = one_step(mode)
            torch.cuda.synchronize()
            per.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        total = time.perf_counter() - t
        prof = {"helm": helm.profile_read(), "pois": pois.profile_read()}
        for op in (helm, pois):
            op.profile(0)
        return total, per, infos, prof

    total64, per64, infos64, prof64 = timed("fp64", args.steps, args.warmup, args.profile_period)
    u64 = st.u.clone()
    ms64 = 1e3 * total64 / args.steps
    fmt = pois.format
    bytes64 = sum(solve_bytes(i, fmt, n, nnz, "fp64") for i in infos64.values())
    csr_equiv = sum(solve_bytes(i, "csr", n, nnz, "fp64") for i in infos64.values())
    gbs64 = bytes64 / (ms64 * 1e-3) / 1e9
    log(f"fp64: {ms64:.1f} ms/step, {gbs64:.0f} GB/s, iters "
        + ", ".join(f"{k}={i.iterations}" for k, i in infos64.items()))

    # dominant kernel: the SpMV of the pressure solve, timed live with HIP events
    spmv_ms, spmv_n = prof64["pois"]["spmv"]
    spmv_avg_us = 1e3 * spmv_ms / max(spmv_n, 1)
    spmv_bytes = bytes_spmv(fmt, n, nnz, 8)
    spmv_gbs = spmv_bytes / (spmv_avg_us * 1e-6) / 1e9
    kern = {}
    for name in ("spmv", "update", "pupdate"):
        ms_, cnt = prof64["pois"][name]
        kern[name] = {"avg_us": round(1e3 * ms_ / max(cnt, 1), 2), "launches": cnt}
    log(f"pressure-solve kernels: {kern}")

    mixed = None
    if not args.no_mixed:
        totalm, perm, infosm, profm = timed("mixed", args.steps, args.warmup, args.profile_period)
        msm = 1e3 * totalm / args.steps
        diff = float(torch.linalg.norm(st.u - u64) / torch.linalg.norm(u64))
        k32 = {}
        for name in ("spmv32", "update32", "pupdate32"):
            ms_, cnt = profm["pois"][name]
            k32[name] = {"avg_us": round(1e3 * ms_ / max(cnt, 1), 2), "launches": cnt}
        mixed = {
            "ms_per_step": round(msm, 3),
            "speedup_vs_fp64": round(ms64 / msm, 3),
            "variant": "FP32 CG, FP64 residual replacement",
            "velocity_rel_diff_vs_fp64": diff,
            "solves": {k: {"fp32_iters": i.iterations, "replacements": i.outer_iterations,
                           "relres": i.relres_true}
                       for k, i in infosm.items()},
            "pressure_kernels": k32,
        }
        log(f"mixed: {msm:.1f} ms/step (x{ms64 / msm:.2f}), "
            + ", ".join(f"{k}={i.iterations}/{i.outer_iterations}" for k, i in infosm.items()))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.time()
        K = oracle.stiffness(m, wl.nu_h, wl.nu_v)
        w = oracle.mass(m).matvec(np.ones(m.n))
        log(f"oracle assembly {time.time() - t0:.1f}s")
        t = time.perf_counter()
        r = oracle.pcg(K, st.b_q.cpu().numpy(), singular=True, weights=w, tol=wl.tol,
                       maxit=args.cpu_iters)
        el = time.perf_counter() - t
        cpu_gbs = r.iterations * bytes_iter("csr", n, nnz, 8) / el / 1e9
        cpu = {"value": round(cpu_gbs, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"first {r.iterations} Jacobi-PCG iterations of the {wl.name} "
                         f"pressure solve, FP64, 1 thread ({el:.1f} s)",
               "s_per_iter": round(el / max(r.iterations, 1), 5)}
        log(f"cpu oracle: {cpu}")

    out = {
        "metric": METRIC,
        "value": round(gbs64, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "nodes": n, "nnz": nnz, "format": pois.format,
                   "solves": "3 velocity (M+dt*K_nu) + 1 pressure (K_nu, pure Neumann) + RHS",
                   "rhs": "time step 1 after a step from rest (wind, Coriolis, pressure)",
                   "tol": wl.tol, "nu_h": wl.nu_h, "nu_v": wl.nu_v,
                   "dt": wl.dt},
        "value_basis": "algorithmic bytes of the solves in the storage format used (operator "
                       "read + 13 vector passes per CG iteration) / step time",
        "csr_equivalent_GBs": round(csr_equiv / (ms64 * 1e-3) / 1e9, 1),
        "fp64": {k: {"iters": i.iterations, "relres": i.relres_true} for k, i in infos64.items()},
        "step_ms": [round(1e3 * v, 3) for v in per64],
        "roofline": {"bound": "hbm", "achieved": round(spmv_gbs, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(spmv_gbs / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": f"k_spmv_{fmt}<double,double,true>",
                     "bytes_per_launch": spmv_bytes, "avg_us": round(spmv_avg_us, 2)},
        "pressure_kernels": kern,
        "mixed": mixed,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
