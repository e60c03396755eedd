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
import re
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


def matrix_bytes(fmt, n, nnz, value_bytes, unit=False):
    """Algorithmic bytes of one read of the operator in the storage format the
    solve runs: symmetric diagonal storage reads the unique values of the
    symmetric matrix ((nnz + n) / 2 of them; (nnz - n) / 2 for the
    Jacobi-scaled operator, whose unit diagonal is not stored) and no indices;
    CSR and sliced ELL read every value, its column index and the row
    pointers."""
    if fmt == "sdia":
        return value_bytes * ((nnz - n) if unit else (nnz + n)) // 2
    return (value_bytes + 4) * nnz + 4 * (n + 1)


def mf_product_bytes(n, ne, nloc):
    """One matrix-free brick product: per element its node indices and 8
    corners (24 doubles), its nloc results written to the scratch and read
    back by the node gather with their (element, local) indices; per node the
    list start, p read and q written."""
    return ne * (4 * nloc + 8 * 24) + ne * nloc * (8 + 8 + 4) + 8 * (n + 1) + 16 * n


def bytes_iter(fmt, n, nnz, vb):
    """One point-Jacobi CG iteration: one operator read plus 12 vector passes
    (SpMV reads p and writes q; the update reads r, q, D^-1 and writes r; the
    direction update reads x, p, r, D^-1 and writes x, p)."""
    return matrix_bytes(fmt, n, nnz, vb) + 12 * vb * n


def bytes_iter_scaled(n, nnz, vb):
    """The same iteration as CG on the Jacobi-scaled operator: the operator
    without its diagonal, 10 vector passes (no D^-1 reads) and the FP32
    weights diag(A) of the residual norm read by the update."""
    return matrix_bytes("sdia", n, nnz, vb, unit=True) + 10 * vb * n + 4 * n


def bytes_spmv(fmt, n, nnz, vb, unit=False):
    """The SpMV kernel alone: operator + read p + write q."""
    return matrix_bytes(fmt, n, nnz, vb, unit) + 2 * vb * n


def jacobi_scaled(op):
    """Whether point-Jacobi solves of `op` run as CG on the Jacobi-scaled
    operator (tunable jacobi_scaling at its default 1, small_n at 4096)."""
    return op.format == "sdia" and 1 <= op.ndiag <= 16 and op.n > 4096


def bytes_residual(fmt, n, nnz):
    """FP64 true residual b - A x: operator + read x, b + write r."""
    return matrix_bytes(fmt, n, nnz, 8) + 3 * 8 * n


def solve_bytes(info, fmt, n, nnz, mode, scaled=False):
    """Bytes of a solve: by default the plain Jacobi-PCG count (bytes_iter);
    scaled=True: the bytes the Jacobi-scaled recurrence moves."""
    it = (lambda vb: bytes_iter_scaled(n, nnz, vb)) if scaled else (
        lambda vb: bytes_iter(fmt, n, nnz, vb))
    if mode == "fp64":
        return info.iterations * it(8)
    return (info.iterations * it(4)
            + (info.outer_iterations + 1) * (bytes_residual(fmt, n, nnz) + 8 * 3 * n))


def make_forcing(m):
    import basin
    L = m.Ly
    theta = np.stack([basin.wind_tension(m.xyz[:, 1], L), np.zeros(m.n)])
    f = basin.coriolis_parameter(m.xyz[:, 1], L)
    return theta, f


def oracle_threads():
    """Threads of the multi-core CPU baseline: OMP_NUM_THREADS when set (this
    process's share of the host), else the CPUs the process may run on."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    if v.isdigit() and int(v) > 0:
        return int(v)
    return len(os.sched_getaffinity(0))


def host_cpu():
    """CPU model and core counts of this host, from lscpu."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except (OSError, subprocess.SubprocessError):
        return {}
    f = {}
    for line in out.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            f[k.strip()] = v.strip()

    def num(key):
        try:
            return int(f.get(key, "0"))
        except ValueError:
            return 0
    sockets = max(num("Socket(s)"), 1)
    return {"model": f.get("Model name"), "sockets": sockets,
            "physical_cores": sockets * num("Core(s) per socket"),
            "logical_cpus": num("CPU(s)"), "affinity_cpus": len(os.sched_getaffinity(0))}


def oracle_reference(m, wl, theta, f, threads, log):
    """The oracle's own time step 1 on the mesh: its step from rest (FP64
    Jacobi-PCG to the workload tolerance), then the step-1 systems, each
    solved to 1e-13 (the reference the GPU answers are measured against) and
    to the workload tolerance (the CPU time to tolerance).  The pressure
    right-hand side of step 1 comes from the reference velocity predictions.
    Solves run in the OpenMP build of the oracle with `threads` threads."""
    import oracle
    from oracle.step import OracleStep
    t0 = time.time()
    ost = OracleStep(m, wl.nu_h, wl.nu_v, wl.dt)
    log(f"oracle assembly of the step forms {time.time() - t0:.1f}s")
    n = m.n
    zero3, zero = np.zeros((3, n)), np.zeros(n)
    t0 = time.time()
    b0 = ost.velocity_rhs(zero3, zero, theta, f)
    ut0 = np.stack([oracle.pcg(ost.A, b0[c], dirichlet=ost.dirichlet[c], tol=wl.tol,
                               threads=threads).x for c in range(3)])
    q0 = oracle.pcg(ost.K, ost.pressure_rhs(ut0), singular=True, weights=ost.mL, tol=wl.tol,
                    threads=threads).x
    u1, p1 = ost.correct(ut0, q0, zero)
    log(f"oracle step from rest {time.time() - t0:.1f}s")
    t0 = time.time()
    b1 = ost.velocity_rhs(u1, p1, theta, f)
    systems = {}
    ut1 = np.zeros((3, n))

    def solve(name, A, b, d, bit, singular):
        w = ost.mL if singular else None
        ex = oracle.pcg(A, b, dirichlet=d, singular=singular, weights=w, tol=1e-13,
                        history=True, threads=threads)
        at = oracle.pcg(A, b, dirichlet=d, singular=singular, weights=w, tol=wl.tol,
                        threads=threads)
        systems[name] = {"b": b, "bit": bit, "A": A, "d": d, "singular": singular, "w": w,
                         "exact": ex.x, "exact_status": ex.status,
                         "exact_iters": ex.iterations,
                         "kappa": oracle.lanczos_condition(ex.alphas, ex.betas),
                         "cpu_iters": at.iterations, "cpu_s": at.loop_s}
        return ex.x

    for c in range(3):
        ut1[c] = solve(f"u{c + 1}", ost.A, b1[c], ost.dirichlet[c], c, False)
    solve("q", ost.K, ost.pressure_rhs(ut1), None, -1, True)
    log(f"oracle step-1 references {time.time() - t0:.1f}s: "
        + ", ".join(f"{k}: {v['exact_iters']} it to 1e-13 (status {v['exact_status']}), "
                    f"{v['cpu_iters']} it / {v['cpu_s']:.2f}s to {wl.tol:g}, "
                    f"kappa ~{v['kappa']:.3g}" for k, v in systems.items()))
    return systems


ERROR_TARGET = 1e-9
TOL_LADDER = (1e-10, 1e-11, 1e-12)


def bench_errors(torch, log, helm, pois, systems, threads, reps=3):
    """Each step-1 system of the oracle solved on the GPU (FP64 and mixed) at
    the tolerances of TOL_LADDER, until the relative error against the
    oracle's 1e-13 solution is at most ERROR_TARGET: time to the workload
    tolerance (the first rung) and time to that error, separately (median
    of `reps` solves from x0 = 0, operator and b resident).  The FP64 answer
    at the workload tolerance is also compared with the oracle's iterate
    after as many iterations (the OpenMP build, same stopping rule)."""
    import oracle
    out = {}
    for name, sy in systems.items():
        op = pois if name == "q" else helm
        b = torch.as_tensor(sy["b"], device="cuda")
        ex = sy["exact"]
        row = {"kappa_estimate": float("%.4g" % sy["kappa"]), "exact_iters": sy["exact_iters"]}
        for mode in ("fp64", "mixed"):
            ladder = []
            for tol in TOL_LADDER:
                ts = []
                for _ in range(reps):
                    x = torch.zeros_like(b)
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    x, info = op.solve(b, x, tol=tol, mask_bit=sy["bit"], mode=mode)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t)
                xh = x.cpu().numpy()
                err = float(np.linalg.norm(xh - ex) / np.linalg.norm(ex))
                ladder.append({"tol": tol, "ms": round(1e3 * float(np.median(ts)), 3),
                               "iters": info.iterations, "outer": info.outer_iterations,
                               "status": info.status, "rel_err": float("%.4g" % err)})
                if err <= ERROR_TARGET:
                    break
            hit = ladder[-1]["rel_err"] <= ERROR_TARGET
            row[mode] = {"time_to_tol_ms": ladder[0]["ms"], "rel_err_at_tol": ladder[0]["rel_err"],
                         "time_to_1e-9_error_ms": ladder[-1]["ms"] if hit else None,
                         "tol_for_1e-9_error": ladder[-1]["tol"] if hit else None,
                         "ladder": ladder}
            if mode == "fp64":
                x, info = op.solve(b, tol=TOL_LADDER[0], mask_bit=sy["bit"])
                its = info.iterations
                kw = dict(dirichlet=sy["d"], singular=sy["singular"], weights=sy["w"],
                          threads=threads)
                same = oracle.pcg(sy["A"], sy["b"], tol=TOL_LADDER[0], maxit=its, **kw)
                if same.iterations < its:
                    same = oracle.pcg(sy["A"], sy["b"], tol=1e-300, maxit=its, **kw)
                xs = x.cpu().numpy()
                row[mode]["p_same_rel_diff"] = float(
                    "%.4g" % (np.linalg.norm(xs - same.x) / np.linalg.norm(same.x)))
                row[mode]["oracle_iters_at_tol"] = sy["cpu_iters"]
        out[name] = row
        log(f"errors vs oracle {name}: " + json.dumps(row))
    return out


def cpu_baseline(log, wl, systems, threads, m2_bytes_iter):
    """The oracle timed on this host: the four step-1 solves of the 256x256x20
    step to the workload tolerance with `threads` OpenMP threads (loop time;
    the headline figure, in GB/s of the CSR-equivalent Jacobi-PCG bytes),
    a one-thread sample of the plain parity build on the pressure solve, the
    16x16x4 box case, and the 48 right-hand sides of the 128x128x20 basin
    solved one after another."""
    import basin
    import oracle
    from oracle.step import OracleStep
    its = sum(v["cpu_iters"] for v in systems.values())
    secs = sum(v["cpu_s"] for v in systems.values())
    gbs = its * m2_bytes_iter / secs / 1e9
    out = {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"the four time-step-1 solves of {wl.name} (the oracle's own right-hand "
                     f"sides) to {wl.tol:g}, OpenMP build of the oracle, {threads} threads, "
                     f"iteration loops only ({secs:.1f} s)",
           "cpu": host_cpu(), "threads": threads,
           "c2_solves": {k: {"iters": v["cpu_iters"], "s": round(v["cpu_s"], 3)}
                         for k, v in systems.items()},
           "c2_solves_total_s": round(secs, 3)}
    # one thread, plain parity build: the first 300 pressure iterations
    q = systems["q"]
    wlq = basin.configs.BASIN_256x256x20
    m = wlq.mesh()
    K = oracle.stiffness(m, wlq.nu_h, wlq.nu_v)
    w = oracle.mass(m).matvec(np.ones(m.n))
    r = oracle.pcg(K, q["b"], singular=True, weights=w, tol=wlq.tol, maxit=300)
    out["one_thread"] = {"s_per_iter": round(r.loop_s / max(r.iterations, 1), 5),
                         "GBs": round(r.iterations * m2_bytes_iter / r.loop_s / 1e9, 3),
                         "sample": f"first {r.iterations} iterations of the pressure solve, "
                                   "plain parity build"}
    del K
    # the small box case
    cfg = basin.configs.BOX_16x16x4
    mb = cfg.mesh()
    d = ~mb.free_mask(basin.BC_U1)
    bb = basin.normal_rhs(mb.n, cfg.seed, zero_mean=True, dirichlet=d)
    Kb = oracle.stiffness(mb, cfg.nu_h, cfg.nu_v)
    box = {}
    for t in (1, threads):
        rs = [oracle.pcg(Kb, bb, dirichlet=d, tol=cfg.tol, threads=t) for _ in range(3)]
        box[f"threads_{t}"] = {"iters": rs[0].iterations,
                               "us_median": round(1e6 * float(np.median([x.loop_s for x in rs])), 1)}
    out["box16x16x4"] = box
    # 48 right-hand sides on 128x128x20, one solve after another
    wl4 = basin.configs.BASIN_128x128x20_BATCH
    m4 = wl4.mesh()
    ost = OracleStep(m4, wl4.nu_h, wl4.nu_v, wl4.dt)
    f4 = basin.coriolis_parameter(m4.xyz[:, 1], m4.Ly)
    tot_s, tot_it = 0.0, 0
    for s_, sc in enumerate(basin.wind_scenarios(wl4.extra["scenarios"],
                                                 wl4.extra["scenario_seed"])):
        theta = np.stack([basin.wind_tension(m4.xyz[:, 1], m4.Ly, sc.amplitude, sc.phase),
                          np.zeros(m4.n)])
        u, p = basin.random_state(m4.n, 100 + s_, m4.bc)
        b = ost.velocity_rhs(u, p, theta, f4)
        for c in range(3):
            r = oracle.pcg(ost.A, b[c], dirichlet=ost.dirichlet[c], tol=wl4.tol, threads=threads)
            tot_s += r.loop_s
            tot_it += r.iterations
    out["basin128x128x20_48_sequential"] = {
        "s": round(tot_s, 3), "iters": tot_it,
        "rhs": "velocity right-hand sides of 16 wind scenarios from a seeded state per scenario"}
    log(f"cpu baseline: {out}")
    return out


COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "counters_spmv_sdia_fp64_basin256x256x20.md")
KERNEL_SOURCES = ("kernels.hip", "kernels.h", "hns_internal.h")


def kernel_source_hash():
    """SHA-256 over the sources of the CG kernels, to tell whether counter
    figures taken earlier still describe the kernel that runs now."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1207_0486_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed hardware-counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    counter reads for a copy of known size), or None when there is none for
    this kernel or the kernel sources changed since the counters were taken."""
    try:
        with open(COUNTER_SUMMARY) as f:
            text = f.read()
    except OSError:
        return None
    fields = dict(re.findall(r"^- (\w+): `([^`]*)`", text, flags=re.M))
    if fields.get("kernel") != kernel or fields.get("source_sha256") != kernel_source_hash():
        return None
    return int(fields["traffic_bytes_per_launch"])


def bench_batched(torch, log, reps=3):
    """Multi-RHS: 3 velocity components x 16 wind scenarios on the 128x128x20
    basin, each scenario advanced one step from rest to get its time-step-1
    right-hand sides; one batched solve against 48 single FP64 solves."""
    import basin
    from paper_1207_0486_amd.step import ProjectionStep
    wl = basin.configs.BASIN_128x128x20_BATCH
    dev = torch.device("cuda", 0)
    t0 = time.time()
    m = wl.mesh()
    theta0, f = make_forcing(m)
    st = ProjectionStep(m, wl.nu_h, wl.nu_v, wl.dt, theta0, f, device=dev)
    st.pois.set_param("replace_drop", 0.1)
    scen = basin.wind_scenarios(wl.extra["scenarios"], wl.extra["scenario_seed"])
    cols, bits = [], []
    zero3 = torch.zeros(3, m.n, dtype=torch.float64, device=dev)
    zero = torch.zeros(m.n, dtype=torch.float64, device=dev)
    for sc in scen:
        theta = np.stack([basin.wind_tension(m.xyz[:, 1], m.Ly, sc.amplitude, sc.phase),
                          np.zeros(m.n)])
        st.theta.copy_(torch.as_tensor(theta, device=dev))
        st.set_state(zero3, zero)
        st.step(tol=wl.tol, mode="mixed")          # step 0 from rest
        b = st.velocity_rhs()                       # time-step-1 right-hand sides
        for c in range(3):
            cols.append(b[c].clone())
            bits.append(c)
    B = torch.stack(cols, dim=1).contiguous()       # n x 48, row-major
    k = B.shape[1]
    helm = st.helm
    log(f"batched set-up {wl.name}: n={m.n} k={k} ({time.time() - t0:.1f}s)")
    times, plan = helm.tune_batched(k, "mixed")
    times64, plan64 = helm.tune_batched(k, "fp64")
    helm.set_param("use_graph", 1)
    helm.set_param("replace_drop", 1e-3)

    def run_batched(mode):
        X = torch.zeros_like(B)
        torch.cuda.synchronize()
        t = time.perf_counter()
        X, infos = helm.solve_batched(B, X, mask_bits=bits, tol=wl.tol, mode=mode)
        torch.cuda.synchronize()
        return time.perf_counter() - t, X, infos

    def run_single():
        X = torch.zeros_like(B)
        Xc = torch.zeros(m.n, dtype=torch.float64, device=dev)
        infos = []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for j in range(k):
            Xc.zero_()
            _, info = helm.solve(B[:, j].contiguous(), Xc, tol=wl.tol, mask_bit=bits[j])
            X[:, j] = Xc
            infos.append(info)
        torch.cuda.synchronize()
        return time.perf_counter() - t, X, infos

    run_batched("mixed"), run_batched("fp64"), run_single()   # warm-up
    tb = min(run_batched("mixed")[0] for _ in range(reps))
    tb64 = min(run_batched("fp64")[0] for _ in range(reps))
    ts = min(run_single()[0] for _ in range(reps))
    _, Xb, ib = run_batched("mixed")
    _, Xs, isg = run_single()
    diff = float(((Xb - Xs).norm(dim=0) / Xs.norm(dim=0).clamp_min(1e-300)).max())
    out = {
        "workload": wl.name, "nodes": m.n, "rhs": k,
        "rhs_recipe": "3 velocity components x 16 wind scenarios, time step 1 after a step "
                      "from rest",
        "batched_mixed_ms": round(1e3 * tb, 3),
        "batched_fp64_ms": round(1e3 * tb64, 3),
        "sequential_fp64_ms": round(1e3 * ts, 3),
        "speedup_vs_sequential_fp64": round(ts / tb, 2),
        "iterations_max": max(i.iterations for i in ib),
        "relres_max": max(i.relres_true for i in ib),
        "max_rel_diff_vs_sequential_fp64": diff,
        "plan": {"mixed": {"columns_per_thread": plan & 7, "tiled_shape": plan >> 3,
                           "tuned_us": {w: round(t, 2) for w, t in times.items()}},
                 "fp64": {"columns_per_thread": plan64 & 7, "tiled_shape": plan64 >> 3,
                          "tuned_us": {w: round(t, 2) for w, t in times64.items()}}},
        "graph": True,
    }
    log(f"batched: {out}")
    helm.close()
    st.pois.close()
    return out


def bench_formats(torch, log, m, b_q, sdia_us, iters=320, period=8):
    """The headline pressure operator (256x256x20, K_nu, pure Neumann) stored
    in CSR and in sliced ELL instead of symmetric diagonal storage: the same
    point-Jacobi recurrence (unscaled: Jacobi scaling is for diagonal storage),
    `iters` iterations from x0 = 0 (the step's pressure right-hand side) after
    a 32-iteration warm-up.  Per format: the SpMV's average duration over the
    sampled iterations (every `period`-th, HIP events on the solve stream),
    its algorithmic bytes (values, column indices and row pointers of the nnz
    entries plus p in and q out; sliced ELL also reads its padding, which is
    not counted), GB/s and fraction of the 8 TB/s peak, and the wall time per
    iteration of an unprofiled run."""
    import basin
    from paper_1207_0486_amd.hns import Operator
    wl = basin.configs.BASIN_256x256x20
    out = {"workload": wl.name, "iterations": iters,
           "sdia_scaled_spmv_us": sdia_us}
    for fmt in ("csr", "sell"):
        t0 = time.time()
        op = Operator(m, wl.nu_h, wl.nu_v, kind="poisson", fmt=fmt)
        setup = time.time() - t0
        assert op.format == fmt
        op.solve(b_q, tol=1e-30, max_iter=32, check=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info = op.solve(b_q, tol=1e-30, max_iter=iters, check=False)
        torch.cuda.synchronize()
        per_iter = (time.perf_counter() - t) / max(info.iterations, 1)
        op.profile(period)
        op.solve(b_q, tol=1e-30, max_iter=iters, check=False)
        torch.cuda.synchronize()
        prof = op.profile_read()
        op.profile(0)
        ms, cnt = prof["spmv"]
        avg_us = 1e3 * ms / max(cnt, 1)
        nb = bytes_spmv(fmt, op.n, op.nnz, 8)
        gbs = nb / (avg_us * 1e-6) / 1e9
        out[fmt] = {"spmv_avg_us": round(avg_us, 2), "spmv_launches_timed": cnt,
                    "bytes_per_spmv": nb, "spmv_GBs": round(gbs, 1),
                    "frac": round(gbs / 8000.0, 4),
                    "us_per_iteration": round(1e6 * per_iter, 2),
                    "update_us": round(1e3 * prof["update"][0] / max(prof["update"][1], 1), 2),
                    "pupdate_us": round(1e3 * prof["pupdate"][0] / max(prof["pupdate"][1], 1), 2),
                    "setup_s": round(setup, 2)}
        op.close()
    log(f"formats: {out}")
    return out


def bench_shard_share(torch, log, iters=400, reps=3):
    """One GPU's share of the 256x256x20 basin split over 8 GPUs by column
    blocks, stood in for by a 128x64x20 basin (the same 176,085 rows and
    15-point stencil; its cells are twice as long in x): the pressure recurrence's time
    per iteration (`iters` iterations from x0 = 0, median of `reps`), FP64
    and mixed, in two launches per iteration (the default at this size) and
    in three: the per-GPU floor a multi-GPU split would add its halo
    exchange and all-reduces to."""
    import basin
    from paper_1207_0486_amd.hns import Operator
    wl = basin.configs.BASIN_256x256x20
    m = basin.basin_mesh(128, 64, 20, L=wl.L, seed=wl.seed)
    op = Operator(m, wl.nu_h, wl.nu_v, kind="poisson", keep_fp32=True)
    b = torch.as_tensor(basin.normal_rhs(m.n, 0, zero_mean=True), device="cuda")
    out = {"workload": "basin128x64x20 (the row count and stencil of one of 8 column blocks of "
                       "basin256x256x20)",
           "nodes": m.n, "iterations": iters}
    for mode in ("fp64", "mixed"):
        for label, fuse in (("two_launches", -1), ("three_launches", 0)):
            op.set_param("fuse_dir", fuse)
            ts = []
            for k in range(reps + 1):
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, info = op.solve(b, tol=1e-30, max_iter=iters, mode=mode, check=False)
                torch.cuda.synchronize()
                if k:
                    ts.append(time.perf_counter() - t)
            out.setdefault(mode, {})[f"us_per_iteration_{label}"] = round(
                1e6 * float(np.median(ts)) / max(info.iterations, 1), 2)
    op.close()
    log(f"shard share: {out}")
    return out


def bench_isotropic(torch, log, m, b_q, point_cap=3000):
    """The paper's isotropic pressure Laplacian (nu = 1) on the 256x256x20 basin
    with the projection step's pressure right-hand side: vertical-line block
    preconditioner to 1e-9, against point Jacobi capped at `point_cap`
    iterations."""
    import basin
    from paper_1207_0486_amd.hns import Operator
    wl = basin.configs.BASIN_256x256x20_ISO
    t0 = time.time()
    op = Operator(m, wl.nu_h, wl.nu_v, kind="poisson")
    op.set_param("check_every", 32)
    log(f"isotropic pressure operator: line_len={op.line_len} ({time.time() - t0:.1f}s)")
    n, nnz = op.n, op.nnz
    fmt = op.format

    def solve(precond, tol, max_iter, reps):
        op.set_param("precond", precond)
        best, info = None, None
        for _ in range(reps):
            x = torch.zeros_like(b_q)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = op.solve(b_q, x, tol=tol, max_iter=max_iter, check=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            best = el if best is None else min(best, el)
        return best, info

    solve(1, wl.tol, 100000, 1)                       # warm-up (factors, workspace)
    t_line, i_line = solve(1, wl.tol, 100000, 3)
    # bytes per line-preconditioned iteration: operator + 2 (SpMV) + 9 (update
    # reads x, r, p, q, couplings, pivots; writes x, r, z) + 3 (p-update) passes
    line_bytes = i_line.iterations * (matrix_bytes(fmt, n, nnz, 8) + 13 * 8 * n)
    t_pt, i_pt = solve(0, wl.tol, point_cap, 1)
    out = {
        "workload": wl.name, "nu": [wl.nu_h, wl.nu_h, wl.nu_v], "tol": wl.tol,
        "rhs": "pressure right-hand side of time step 1 (the anisotropic step's -(1/dt) B u~)",
        "line": {"ms": round(1e3 * t_line, 3), "iterations": i_line.iterations,
                 "status": i_line.status, "relres": i_line.relres_true,
                 "us_per_iter": round(1e6 * t_line / max(i_line.iterations, 1), 2),
                 "GBs": round(line_bytes / t_line / 1e9, 1)},
        "point_jacobi_capped": {"ms": round(1e3 * t_pt, 3), "iterations": i_pt.iterations,
                                "status": i_pt.status, "relres": i_pt.relres_true},
    }
    op.close()
    log(f"isotropic: {out}")
    return out


def bench_loop(torch, log, m, steps=4, stress_steps=2):
    """Multi-step BDF2 projection loop on the 256x256x20 basin from rest:
    implicit-Euler first step, then BDF2, explicit advection and Coriolis,
    isotropic line-preconditioned pressure (tol 1e-8: the right-hand side of
    the first step from rest has its rounding floor near 2e-9), consistent-mass
    correction; velocity and mass solves to 1e-10.  Then the paper's run
    constants (nu = (1e8, 1e8, 250) m^2/s, dt = one month) with point Jacobi
    and with line blocks for the stiffness-dominated velocity solves (its
    pressure right-hand side is small against the rounding of K q, so its
    pressure tolerance is 1e-6)."""
    import basin
    from paper_1207_0486_amd.step import ProjectionLoop
    theta, f = make_forcing(m)
    zero3 = torch.zeros(3, m.n, dtype=torch.float64, device="cuda")
    zero = torch.zeros(m.n, dtype=torch.float64, device="cuda")

    def run(nu_h, nu_v, dt, nsteps, vprec, ptol):
        t0 = time.time()
        lp = ProjectionLoop(m, nu_h, nu_v, dt, theta, f, velocity_precond=vprec)
        setup = time.time() - t0
        lp.set_state(zero3, zero)
        per, its = [], []
        try:
            for _ in range(nsteps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = lp.step(tol=1e-10, pressure_tol=ptol)
                torch.cuda.synchronize()
                per.append(round(1e3 * (time.perf_counter() - t), 2))
                ok = all(i.status == 0 for i in r.velocity + r.correction) and r.pressure.status == 0
                its.append({"velocity": [i.iterations for i in r.velocity],
                            "pressure": r.pressure.iterations,
                            "pressure_relres": float("%.3g" % r.pressure.relres_true),
                            "mass": [i.iterations for i in r.correction], "ok": ok})
            u = lp.u.abs().amax(dim=1).tolist()
        finally:
            lp.close()
        return {"ms_per_step": per, "iterations": its, "setup_s": round(setup, 1),
                "pressure_tol": ptol, "max_abs_u": [float("%.4g" % v) for v in u]}

    wl = basin.configs.BASIN_256x256x20
    out = {"workload": f"{wl.name} BDF2 loop from rest", "steps": steps,
           "scheme": "implicit Euler first, BDF2 after; explicit advection + Coriolis; "
                     "isotropic pressure with line blocks; consistent-mass correction",
           "workload_constants": run(wl.nu_h, wl.nu_v, wl.dt, steps, 0, 1e-8)}
    log(f"loop: {out['workload_constants']}")
    stress = {}
    for vprec, name in ((0, "velocity_point_jacobi"), (1, "velocity_line_blocks")):
        stress[name] = run(1e8, 250.0, 2.592e6, stress_steps, vprec, 1e-6)
        log(f"loop stress {name}: {stress[name]}")
    out["paper_constants"] = {"nu": [1e8, 1e8, 250.0], "dt_s": 2.592e6, **stress}
    return out


def bench_small_box(torch, log, warm=2, reps=5):
    """The small plain-method case (16x16x4 box, 1445 nodes, anisotropic
    Laplacian, Dirichlet bottom and walls, FP64 Jacobi-PCG to 1e-10):
    launch- and synchronisation-bound, so its figure is the latency of one
    hns_solve call (median of `reps` after `warm` warm-ups), FP64 and mixed."""
    import basin
    from paper_1207_0486_amd.hns import Operator
    cfg = basin.configs.BOX_16x16x4
    m = cfg.mesh()
    d = ~m.free_mask(basin.BC_U1)
    b = torch.as_tensor(basin.normal_rhs(m.n, cfg.seed, zero_mean=True, dirichlet=d),
                        device="cuda")
    op = Operator(m, cfg.nu_h, cfg.nu_v, kind="poisson", keep_fp32=True)
    out = {"workload": cfg.name, "nodes": m.n, "format": op.format, "tol": cfg.tol}
    for mode in ("fp64", "mixed"):
        ts, info = [], None
        for k in range(warm + reps):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = op.solve(b, x, tol=cfg.tol, mask_bit=0, mode=mode)
            torch.cuda.synchronize()
            if k >= warm:
                ts.append(time.perf_counter() - t)
        out[mode] = {"latency_us_median": round(1e6 * float(np.median(ts)), 1),
                     "latency_us_min": round(1e6 * min(ts), 1), "iterations": info.iterations,
                     "relres": float("%.3g" % info.relres_true)}
    op.close()
    log(f"small box: {out}")
    return out


def bench_bricks(torch, log, reps=3):
    """The paper's own discretisation (Sec. 5) over the 256x256x20 basin's
    bathymetry: Q2 velocity operator M + dt K_nu on 128x128x10 bricks
    (1,387,029 nodes, the node lattice of the tetrahedral mesh), the Q1
    pressure operator on the same bricks (the Q2/Q1 pair), and Q1 pressure on
    256x256x20 bricks (1,387,029 nodes).  Jacobi-PCG to 1e-10 from x0 = 0;
    the isotropic Q1 pressure also with the line blocks to 1e-8 (its rounding
    floor is near 1e-9)."""
    import basin
    from paper_1207_0486_amd.hns import Operator
    wl = basin.configs.BASIN_256x256x20
    cases = (
        ("q2_velocity_128x128x10", 2, (128, 128, 10), "helmholtz", (wl.nu_h, wl.nu_v), 0, 0,
         1e-10),
        ("q2_velocity_matrix_free_128x128x10", 2, (128, 128, 10), "helmholtz",
         (wl.nu_h, wl.nu_v), 0, 0, 1e-10),
        ("q1_pressure_128x128x10", 1, (128, 128, 10), "poisson", (wl.nu_h, wl.nu_v), -1, 0,
         1e-10),
        ("q1_pressure_256x256x20", 1, (256, 256, 20), "poisson", (wl.nu_h, wl.nu_v), -1, 0,
         1e-10),
        ("q1_pressure_iso_line_128x128x10", 1, (128, 128, 10), "poisson", (1.0, 1.0), -1, 1,
         1e-8),
    )
    out = {}
    for name, order, (Nx, Ny, Nz), kind, nu, bit, precond, tol in cases:
        m = basin.basin_hex_mesh(Nx, Ny, Nz, order, L=wl.L, seed=wl.seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mfree = "matrix_free" in name
        op = Operator(m, nu[0], nu[1], wl.dt if kind == "helmholtz" else 0.0, kind=kind,
                      matrix_free=mfree)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        op.set_param("precond", precond)
        if bit >= 0:
            d = ((m.bc >> bit) & 1) == 1
            b = basin.normal_rhs(m.n, 31, dirichlet=d)
        else:
            b = basin.normal_rhs(m.n, 31, zero_mean=True)
        b = torch.as_tensor(b, device="cuda")
        best, info = None, None
        for _ in range(reps):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = op.solve(b, x, tol=tol, mask_bit=bit, check=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            best = el if best is None else min(best, el)
        # the product's own time (kernel events on every iteration of one solve)
        op.profile(1)
        op.solve(b, torch.zeros_like(b), tol=tol, mask_bit=bit, check=False)
        prof = op.profile_read()
        op.profile(0)
        product_us = 1e3 * prof["spmv"][0] / max(prof["spmv"][1], 1)
        scaled = precond == 0 and jacobi_scaled(op)
        if mfree:   # element data, the element results written and gathered, p and q
            ne = m.hexes.shape[0]
            prod = mf_product_bytes(op.n, ne, m.hexes.shape[1])
            vec = 10 * 8 * op.n
            by = by_stored = info.iterations * (prod + vec)
        elif scaled:   # bytes the Jacobi-scaled recurrence moves
            by = info.iterations * bytes_iter_scaled(op.n, op.nnz, 8)
            vec = 10 * 8 * op.n + 4 * op.n
        else:
            vec = (12 if precond == 0 else 13) * 8 * op.n
            by = info.iterations * (matrix_bytes(op.format, op.n, op.nnz, 8) + vec)
        if not mfree:
            # diagonal storage also reads the zeros it stores where a row lacks an offset
            stored = ((op.ndiag + (0 if scaled else 1)) * op.n * 8 if op.format == "sdia"
                      else matrix_bytes(op.format, op.n, op.nnz, 8))
            by_stored = info.iterations * (stored + vec)
        out[name] = {"order": order, "bricks": [Nx, Ny, Nz], "nodes": op.n, "nnz": op.nnz,
                     "format": op.format, "ndiag": op.ndiag, "nu": list(nu),
                     "precond": ["jacobi", "line"][precond], "jacobi_scaled": scaled,
                     "tol": tol, "setup_s": round(setup_s, 2), "iterations": info.iterations,
                     "status": info.status, "relres": float("%.3g" % info.relres_true),
                     "ms": round(1e3 * best, 3),
                     "us_per_iter": round(1e6 * best / max(info.iterations, 1), 2),
                     "product_us": round(product_us, 2),
                     "GBs": round(by / best / 1e9, 1),
                     "GBs_stored": round(by_stored / best / 1e9, 1)}
        log(f"bricks {name}: {out[name]}")
        op.close()
        del x, b
    return out


def bench_preconditioners(torch, log, m, b_vel, reps=3):
    """Velocity solve (component 1, its Dirichlet set) on the 256x256x20
    basin with point Jacobi, vertical-line blocks and IC(0) in the greedy
    multicolour order, to 1e-10: the workload operator M + dt K_nu and the
    BDF2 operator of the paper's run constants (nu = (1e8, 1e8, 250), dt = one
    month).  Time to tolerance with the operator resident; the first IC(0)
    solve of a Dirichlet set includes its host factorisation and upload."""
    import basin
    from paper_1207_0486_amd.hns import Operator
    wl = basin.configs.BASIN_256x256x20
    cases = {"workload": (wl.nu_h, wl.nu_v, wl.dt),
             "paper_constants_bdf2": (1e8, 250.0, 2.592e6 * 2.0 / 3.0)}
    out = {"solve": "velocity component 1, Dirichlet set 0, tol 1e-10, FP64",
           "rhs": "the projection step's velocity right-hand side"}
    for name, (nu_h, nu_v, dt) in cases.items():
        op = Operator(m, nu_h, nu_v, dt, kind="helmholtz", keep_host=True)
        res = {}
        for pre, label in ((0, "jacobi"), (1, "line"), (2, "ic0")):
            op.set_param("precond", pre)
            first = None
            best, info = None, None
            for rep in range(reps + 1):
                x = torch.zeros_like(b_vel)
                torch.cuda.synchronize()
                t = time.perf_counter()
                x, info = op.solve(b_vel, x, tol=1e-10, mask_bit=0, check=False)
                torch.cuda.synchronize()
                el = time.perf_counter() - t
                if rep == 0:
                    first = el
                else:
                    best = el if best is None else min(best, el)
            res[label] = {"ms": round(1e3 * best, 3), "iterations": info.iterations,
                          "status": info.status, "relres": float("%.3g" % info.relres_true),
                          "first_solve_ms": round(1e3 * first, 1)}
        op.close()
        out[name] = res
        log(f"preconditioners {name}: {res}")
    # the workload's (anisotropic) pressure operator: point Jacobi against line
    # blocks, FP64 and mixed (FP32 CG with FP64 residual replacement)
    op = Operator(m, wl.nu_h, wl.nu_v, kind="poisson", keep_fp32=True)
    op.set_param("replace_drop", 0.1)
    b_q = torch.as_tensor(basin.normal_rhs(m.n, 21, zero_mean=True), device=b_vel.device)
    res = {}
    for pre, mode, label in ((0, "fp64", "jacobi"), (1, "fp64", "line"),
                             (0, "mixed", "jacobi_mixed"), (1, "mixed", "line_mixed")):
        op.set_param("precond", pre)
        best, info = None, None
        for rep in range(2):
            x = torch.zeros_like(b_q)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = op.solve(b_q, x, tol=1e-10, mode=mode, check=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            best = el if best is None else min(best, el)
        res[label] = {"ms": round(1e3 * best, 3), "iterations": info.iterations,
                      "replacements": info.outer_iterations,
                      "status": info.status, "relres": float("%.3g" % info.relres_true)}
    op.close()
    out["pressure_workload"] = {"rhs": "N(0,1), seed 21, zero mean", **res}
    log(f"preconditioners pressure_workload: {res}")
    return out


def bench_serving(torch, log, budget_gb=1.5, mode="fp64", count=256, capacity=8, chunk=32,
                  check=True, oracle_cache=None, line_pressure=False):
    """Serving: Poisson-process arrivals (50 req/s) of pressure / velocity solve
    requests over five mesh sizes, tolerance 1e-8, continuous batching with
    operators admitted by footprint under an HBM budget (the ten operators
    with two-slot sessions hold about 2.7 GB in FP64 and 3.7 GB in mixed
    precision, so a budget of 1.5 GB makes the server evict idle operators and
    build them again on the device).  check=True: one request
    per mesh size is solved again alone on a fresh operator (the served
    answer must be the same) and checked by the oracle's own residual."""
    import threading
    import basin
    from paper_1207_0486_amd.hns import Operator
    from paper_1207_0486_amd.serve import GpuBackend, Request, Server
    wl = basin.configs.SERVING
    meshes = {}

    def make(key):
        idx, kind = key
        if idx not in meshes:
            meshes[idx] = basin.configs.serving_mesh(idx)
        return meshes[idx], wl.nu_h, wl.nu_v, wl.dt, kind

    reqs = basin.serving_requests(wl.extra["requests"] if count is None else count,
                                  wl.extra["rate_hz"], wl.seed)
    t0 = time.time()
    be = GpuBackend(make, mode=mode, check_every=16, line_pressure=line_pressure)
    srv = Server(be, budget_bytes=int(budget_gb * (1 << 30)), capacity=capacity, chunk=chunk)
    # warm-up: one request per operator (assembly, tuning); with a small
    # budget the early operators are evicted again
    keys = sorted({(r.mesh_index, r.kind) for r in reqs})
    warm = []
    for key in keys:
        m = make(key)[0]
        bit = -1 if key[1] == "poisson" else 0
        d = None if bit < 0 else ((m.bc >> bit) & 1) == 1
        warm.append(srv.submit(Request(key=key, b=basin.normal_rhs(m.n, 7, dirichlet=d),
                                       mask_bit=bit, tol=wl.tol)))
    try:
        for fu in warm:
            fu.result()
    except BaseException:
        srv.close()
        raise
    with srv.lock:
        srv.results.clear()
        ev0 = len(srv.events)
    log(f"serving warm-up ({mode}): {len(keys)} operators, {len(srv.resident)} resident "
        f"({time.time() - t0:.1f}s)")
    # right-hand sides of the stream, generated before it starts
    items = []
    for r in reqs:
        m = make((r.mesh_index, r.kind))[0]
        bit = -1 if r.kind == "poisson" else 0
        d = None if bit < 0 else ((m.bc >> bit) & 1) == 1
        items.append((r, Request(key=(r.mesh_index, r.kind),
                                 b=basin.normal_rhs(m.n, r.rhs_seed, dirichlet=d),
                                 mask_bit=bit, tol=wl.tol)))
    futs = []
    start = time.perf_counter()

    def feeder():
        for r, q in items:
            delay = start + r.arrival_s - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            q.arrival = time.perf_counter()
            futs.append(srv.submit(q))

    try:
        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        results = [fu.result() for fu in futs]
        end = time.perf_counter()
        st = srv.stats(start, end)
        stream_events = srv.events[ev0:]
    finally:
        srv.close()
    nodes = sum(make((r.mesh_index, r.kind))[0].n for r, _ in items)
    bad = sum(1 for x in results if x.info.status != 0)
    per_mesh = {}
    for (r, _), res in zip(items, results):
        per_mesh.setdefault(r.mesh_index, []).append(res.latency_s)
    sizes = basin.forcing.SERVING_MESHES
    by_mesh = {"x".join(map(str, sizes[i])): {
        "requests": len(v), "p50_ms": round(float(np.percentile(v, 50)) * 1e3, 2),
        "p99_ms": round(float(np.percentile(v, 99)) * 1e3, 2)} for i, v in sorted(per_mesh.items())}
    out = {"requests": len(results), "rate_hz": wl.extra["rate_hz"], "tol": wl.tol,
           "mode": mode, "capacity": capacity, "chunk": chunk, "budget_gb": budget_gb,
           "pressure_precond": "line" if line_pressure else "jacobi",
           "p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2),
           "mean_ms": round(st["mean_ms"], 2), "solves_per_s": round(st["solves_per_s"], 2),
           "wall_s": round(end - start, 3), "nodes_solved": int(nodes), "failed": bad,
           "operators": len(keys), "peak_gb": round(st["peak_bytes"] / (1 << 30), 3),
           "admissions_in_stream": sum(1 for e in stream_events if e[1] == "admit"),
           "evictions_in_stream": sum(1 for e in stream_events if e[1] == "evict"),
           "evictions": st["evictions"], "by_mesh": by_mesh,
           "meshes": [list(mm) for mm in sizes]}
    if check:
        out["check"] = serving_check(torch, log, items, results, make, mode, wl.tol,
                                     oracle_cache, line_pressure)
    log(f"serving: {out}")
    return out


def serving_check(torch, log, items, results, make, mode, tol, cache, line_pressure=False):
    """One served request per mesh size (the first of each in the stream):
    the same solve alone on a freshly assembled operator (per-slot sessions
    run hns_solve's recurrence, so the answers should agree bit for bit) and
    the oracle's own residual of the served answer."""
    import oracle
    from paper_1207_0486_amd.hns import Operator
    cache = {} if cache is None else cache
    seen, rows = set(), []
    for (r, q), res in zip(items, results):
        if r.mesh_index in seen:
            continue
        seen.add(r.mesh_index)
        m, nu_h, nu_v, dt, kind = make(q.key)
        op = Operator(m, nu_h, nu_v, dt, kind=kind, keep_fp32=mode == "mixed",
                      gpu_assembly=True)
        op.set_param("check_every", 16)
        if line_pressure and kind == "poisson" and op.line_len >= 2:
            op.set_param("precond", 1)
        x, info = op.solve(torch.as_tensor(q.b, device="cuda"), tol=tol, mask_bit=q.mask_bit,
                           mode=mode)
        alone = x.cpu().numpy()
        op.close()
        diff = float(np.abs(res.x - alone).max() / max(np.abs(alone).max(), 1e-300))
        if q.key not in cache:
            cache[q.key] = (oracle.stiffness(m, nu_h, nu_v) if kind == "poisson"
                            else oracle.helmholtz(m, nu_h, nu_v, dt))
        A = cache[q.key]
        if q.mask_bit < 0:
            bh = q.b - q.b.mean()
            rr = bh - A.matvec(res.x)
            rr -= rr.mean()
            relres = float(np.linalg.norm(rr) / np.linalg.norm(bh))
        else:
            d = ((m.bc >> q.mask_bit) & 1) == 1
            relres = oracle.relres(A, q.b, res.x, d)
        rows.append({"mesh": r.mesh_index, "kind": kind, "nodes": m.n,
                     "served_iters": res.info.iterations, "alone_iters": info.iterations,
                     "max_rel_diff_vs_alone": diff, "oracle_relres": float("%.4g" % relres)})
    ok = all(x["max_rel_diff_vs_alone"] == 0.0 and x["oracle_relres"] <= 1.01 * tol for x in rows)
    log(f"serving check ({mode}): {rows}")
    return {"ok": ok, "samples": rows}


def batched_probe(torch, log, iters=6, k=48):
    """Short run for hardware-counter passes over the batched product: a
    plain 1 GiB device copy (the calibration kernel), then `iters` iterations
    of the FP64 and of the mixed block solve of k seeded N(0,1) columns
    (Dirichlet rows zeroed per column's set) on the 128x128x20 velocity
    operator, with the grid-stride product at 4 columns per thread."""
    import basin
    from paper_1207_0486_amd.hns import Operator
    dev = torch.device("cuda", 0)
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)       # 1 GiB
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    del a, c
    wl = basin.configs.BASIN_128x128x20_BATCH
    m = wl.mesh()
    op = Operator(m, wl.nu_h, wl.nu_v, wl.dt, kind="helmholtz", keep_fp32=True)
    op.set_param("bspmm_vec", 4)
    op.set_param("bspmm_tile", 0)
    bits = [j % 3 for j in range(k)]
    B = np.random.default_rng(0).standard_normal((m.n, k))
    for j, bit in enumerate(bits):
        B[((m.bc >> bit) & 1) == 1, j] = 0.0
    B = torch.as_tensor(B, device=dev)
    out = {"probe": "batched", "nodes": m.n, "rhs": k, "copy_bytes": 2 * (1 << 27) * 8}
    for mode in ("fp64", "mixed"):
        X, infos = op.solve_batched(B, mask_bits=bits, tol=1e-10, max_iter=iters, mode=mode,
                                    check=False)
        torch.cuda.synchronize()
        out[mode] = {"iterations": max(i.iterations for i in infos)}
    op.close()
    print(json.dumps(out), flush=True)


def traffic_probe(torch, log, iters=64, q2_iters=16):
    """Short run for hardware-counter passes: a plain 1 GiB device copy (the
    calibration kernel of known size), 64 iterations of the 256x256x20
    pressure solve (the dominant SpMV kernel), then 16 iterations of the Q2
    velocity solve on 128x128x10 bricks (the wide diagonal SpMV), then the
    same 16 iterations on the matrix-free Q2 operator."""
    import basin
    from paper_1207_0486_amd.hns import Operator
    dev = torch.device("cuda", 0)
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)       # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    wl = basin.configs.BASIN_256x256x20
    m = wl.mesh()
    pois = Operator(m, wl.nu_h, wl.nu_v, kind="poisson")
    rhs = torch.as_tensor(basin.normal_rhs(m.n, 0, zero_mean=True), device=dev)
    x, info = pois.solve(rhs, tol=1e-30, max_iter=iters, check=False)
    torch.cuda.synchronize()
    out = {"probe": "traffic", "copy_bytes": 2 * a.numel() * 8, "nodes": m.n, "nnz": pois.nnz,
           "format": pois.format, "iterations": info.iterations,
           "jacobi_scaled": jacobi_scaled(pois),
           "spmv_algorithmic_bytes": bytes_spmv(pois.format, m.n, pois.nnz, 8,
                                                unit=jacobi_scaled(pois))}
    pois.close()
    del a, b
    mq = basin.basin_hex_mesh(128, 128, 10, 2, L=wl.L, seed=wl.seed)
    q2 = Operator(mq, wl.nu_h, wl.nu_v, wl.dt, kind="helmholtz")
    d = (mq.bc & basin.BC_U1) != 0
    rq = torch.as_tensor(basin.normal_rhs(mq.n, 31, dirichlet=d), device=dev)
    xq, iq = q2.solve(rq, tol=1e-30, max_iter=q2_iters, mask_bit=0, check=False)
    torch.cuda.synchronize()
    out["q2"] = {"nodes": mq.n, "nnz": q2.nnz, "format": q2.format, "ndiag": q2.ndiag,
                 "iterations": iq.iterations,
                 "stored_bytes_per_spmv": (q2.ndiag + 1) * mq.n * 8 + 2 * 8 * mq.n}
    q2.close()
    qf = Operator(mq, wl.nu_h, wl.nu_v, wl.dt, kind="helmholtz", matrix_free=True)
    xf, iff = qf.solve(rq, tol=1e-30, max_iter=q2_iters, mask_bit=0, check=False)
    torch.cuda.synchronize()
    out["q2_matrix_free"] = {"iterations": iff.iterations,
                             "algorithmic_bytes_per_product":
                                 mf_product_bytes(mq.n, mq.hexes.shape[0], mq.hexes.shape[1])}
    qf.close()
    print(json.dumps(out), flush=True)


def main():
    # the OpenMP build of the oracle (CPU baseline) reads these when loaded
    os.environ.setdefault("OMP_PROC_BIND", "close")
    os.environ.setdefault("OMP_PLACES", "cores")
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--check-every", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle: its step-1 references, the per-solve errors and the "
                         "CPU baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-isotropic", action="store_true")
    ap.add_argument("--no-formats", action="store_true",
                    help="skip the CSR / sliced-ELL pressure operator section")
    ap.add_argument("--no-share", action="store_true",
                    help="skip the one-GPU-share (128x64x20) per-iteration section")
    ap.add_argument("--no-loop", action="store_true")
    ap.add_argument("--no-precond", action="store_true")
    ap.add_argument("--no-bricks", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only a 1 GiB copy, 64 pressure iterations and 16 Q2 velocity "
                         "iterations (for counter passes)")
    ap.add_argument("--batched-probe", action="store_true",
                    help="only a 1 GiB copy and 6 iterations of the 48-column FP64 and mixed "
                         "block solves on 128x128x20 (for counter passes)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-budget-gb", type=float, default=1.5,
                    help="HBM budget of the serving stream (its ten operators hold 2.7-3.7 GB)")
    ap.add_argument("--serve-mode", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--serve-capacity", type=int, default=2,
                    help="slots per operator session")
    ap.add_argument("--serve-chunk", type=int, default=32, help="iterations between admissions")
    ap.add_argument("--serve-resident-gb", type=float, default=8.0,
                    help="second serving run with a budget that holds every operator (0: skip)")
    ap.add_argument("--serve-line-pressure", action="store_true",
                    help="serve Poisson requests with the water-column line preconditioner")
    ap.add_argument("--fmt", default="auto")
    ap.add_argument("--param", action="append", default=[], metavar="NAME=VALUE",
                    help="hns_set_param tunable applied to the step's two operators "
                         "(repeatable; for A/B comparisons)")
    ap.add_argument("--profile-period", type=int, default=32,
                    help="time every N-th CG iteration with HIP events (the middle one of each "
                         "N-iteration window of a chunk; at most --check-every)")
    args = ap.parse_args()
    if args.traffic_probe:
        import torch
        traffic_probe(torch, log)
        return
    if args.batched_probe:
        import torch
        batched_probe(torch, log)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver "
              "does not shard across GPUs", file=sys.stderr)
        sys.exit(2)
    if not 1 <= args.profile_period <= args.check_every:
        print("--profile-period must be between 1 and --check-every: the roofline needs "
              "timed SpMV launches", file=sys.stderr)
        sys.exit(2)

    import torch
    import basin
    from paper_1207_0486_amd.hns import Operator
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
    for kv in args.param:
        name, value = kv.split("=", 1)
        for op in (helm, pois):
            op.set_param(name, float(value))
    log(f"assembled: nnz={pois.nnz} format={pois.format} ({time.time() - t0:.1f}s)")
    n, nnz = pois.n, pois.nnz

    # time step 0 from rest (untimed) gives the state every timed step starts from
    t0 = time.time()
    r0 = st.step(tol=wl.tol)
    u1, p1 = st.state()
    log(f"step 0 from rest: iters {[i.iterations for i in r0.velocity]} / "
        f"{r0.pressure.iterations} ({time.time() - t0:.1f}s)")

    def one_step(mode):
        """The step of ProjectionStep.step, with the wall time of each solve
        (hns_solve returns when its answer is final)."""
        st.set_state(u1, p1)
        infos, times = {}, {}
        st.velocity_rhs()
        for c in range(3):
            st.ut[c].zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, infos[f"u{c + 1}"] = helm.solve(st.b_vel[c], st.ut[c], tol=wl.tol, mask_bit=c,
                                               mode=mode)
            times[f"u{c + 1}"] = time.perf_counter() - t
        st.pressure_rhs()
        st.q.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, infos["q"] = pois.solve(st.b_q, st.q, tol=wl.tol, mask_bit=-1, mode=mode)
        times["q"] = time.perf_counter() - t
        st.correct()
        return infos, times

    def timed(mode, steps, warmup, profile):
        for _ in range(warmup):
            one_step(mode)
        for op in (helm, pois):
            op.profile(profile)
        torch.cuda.synchronize()
        t = time.perf_counter()
        per = []
        infos = None
        solve_s = {}
        for _ in range(steps):
            ts = time.perf_counter()
            infos, times = one_step(mode)
            torch.cuda.synchronize()
            per.append(time.perf_counter() - ts)
            for k, v in times.items():
                solve_s.setdefault(k, []).append(v)
        torch.cuda.synchronize()
        total = time.perf_counter() - t
        prof = {"helm": helm.profile_read(), "pois": pois.profile_read()}
        for op in (helm, pois):
            op.profile(0)
        solve_ms = {k: round(1e3 * float(np.median(v)), 3) for k, v in solve_s.items()}
        return total, per, infos, prof, solve_ms

    total64, per64, infos64, prof64, solve_ms64 = timed("fp64", args.steps, args.warmup,
                                                         args.profile_period)
    u64 = st.u.clone()
    ms64 = 1e3 * total64 / args.steps
    fmt = pois.format
    scaled = jacobi_scaled(pois)
    bytes64 = sum(solve_bytes(i, fmt, n, nnz, "fp64") for i in infos64.values())
    moved64 = sum(solve_bytes(i, fmt, n, nnz, "fp64", scaled) for i in infos64.values())
    csr_equiv = sum(solve_bytes(i, "csr", n, nnz, "fp64") for i in infos64.values())
    gbs64 = bytes64 / (ms64 * 1e-3) / 1e9
    log(f"fp64: {ms64:.1f} ms/step, {gbs64:.0f} GB/s, iters "
        + ", ".join(f"{k}={i.iterations}" for k, i in infos64.items()))

    # dominant kernel: the SpMV of the pressure solve, timed live with HIP events
    spmv_ms, spmv_n = prof64["pois"]["spmv"]
    if spmv_n == 0:
        raise RuntimeError("no pressure-solve SpMV launch was timed")
    spmv_avg_us = 1e3 * spmv_ms / max(spmv_n, 1)
    spmv_bytes = bytes_spmv(fmt, n, nnz, 8, unit=scaled)
    spmv_gbs = spmv_bytes / (spmv_avg_us * 1e-6) / 1e9
    spmv_kernel = (f"k_spmv_sdia<double, double, true, {pois.ndiag}, 2, {str(scaled).lower()}>"
                   if fmt == "sdia" else f"k_spmv_{fmt}<double, double, true>")
    traffic = counted_traffic(spmv_kernel)
    kern = {}
    for name in ("spmv", "update", "pupdate"):
        ms_, cnt = prof64["pois"][name]
        kern[name] = {"avg_us": round(1e3 * ms_ / max(cnt, 1), 2), "launches": cnt}
    log(f"pressure-solve kernels: {kern}")

    mixed = None
    if not args.no_mixed:
        totalm, perm, infosm, profm, solve_msm = timed("mixed", args.steps, args.warmup,
                                                       args.profile_period)
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
                           "relres": i.relres_true, "ms": solve_msm[k]}
                       for k, i in infosm.items()},
            "pressure_kernels": k32,
        }
        log(f"mixed: {msm:.1f} ms/step (x{ms64 / msm:.2f}), "
            + ", ".join(f"{k}={i.iterations}/{i.outer_iterations}" for k, i in infosm.items()))

    # per-solve error against the oracle (its own step-1 systems solved to
    # 1e-13), time to the tolerance and time to 1e-9 error, FP64 and mixed
    systems = errors = None
    threads = oracle_threads()
    if not args.no_cpu_baseline:
        systems = oracle_reference(m, wl, theta, f, threads, log)
        errors = bench_errors(torch, log, helm, pois, systems, threads)

    # the same step with the pressure solve preconditioned by the vertical-line
    # blocks (the velocity solves keep point Jacobi): FP64 and mixed precision
    line_step = None
    if not args.no_precond:
        pois.set_param("precond", 1)
        line_step = {}
        for mode in ("fp64",) + (() if args.no_mixed else ("mixed",)):
            tot, per, inf, _, _ = timed(mode, args.steps, args.warmup, 0)
            ms = 1e3 * tot / args.steps
            line_step[mode] = {"ms_per_step": round(ms, 3),
                               "speedup_vs_fp64_jacobi": round(ms64 / ms, 3),
                               "pressure_iters": inf["q"].iterations,
                               "pressure_relres": inf["q"].relres_true}
        pois.set_param("precond", 0)
        log(f"step with line-preconditioned pressure: {line_step}")

    # operator set-up: host assembly against device-computed values (same
    # pattern work on the host, bitwise the same matrix)
    setup = {}
    for gpu_asm in (False, True):
        torch.cuda.synchronize()
        t = time.perf_counter()
        op_a = Operator(m, wl.nu_h, wl.nu_v, kind="poisson", gpu_assembly=gpu_asm)
        torch.cuda.synchronize()
        setup["device_values_s" if gpu_asm else "host_s"] = round(time.perf_counter() - t, 3)
        op_a.close()
    log(f"pressure operator set-up: {setup}")

    share = None
    if not args.no_share:
        share = bench_shard_share(torch, log)

    formats = None
    if not args.no_formats:
        formats = bench_formats(torch, log, m, st.b_q.clone(), kern["spmv"]["avg_us"])

    isotropic = None
    if not args.no_isotropic:
        isotropic = bench_isotropic(torch, log, m, st.b_q.clone())

    precond = None
    if not args.no_precond:
        precond = bench_preconditioners(torch, log, m, st.b_vel[0].clone())

    small_box = bench_small_box(torch, log)

    bricks = None
    if not args.no_bricks:
        bricks = bench_bricks(torch, log)

    loop = None
    if not args.no_loop:
        loop = bench_loop(torch, log, m)

    batched = None
    if not args.no_batched:
        batched = bench_batched(torch, log)

    serving = None
    if not args.no_serving:
        cache = {}
        serving = bench_serving(torch, log, args.serve_budget_gb, args.serve_mode,
                                capacity=args.serve_capacity, chunk=args.serve_chunk,
                                check=not args.no_cpu_baseline, oracle_cache=cache,
                                line_pressure=args.serve_line_pressure)
        other = "mixed" if args.serve_mode == "fp64" else "fp64"
        serving_other = bench_serving(torch, log, args.serve_budget_gb, other,
                                      capacity=args.serve_capacity, chunk=args.serve_chunk,
                                      check=not args.no_cpu_baseline, oracle_cache=cache,
                                      line_pressure=args.serve_line_pressure)
        serving = {args.serve_mode: serving, other: serving_other}
        del cache
        if args.serve_resident_gb > 0:
            # every operator resident: no admission or eviction in the stream
            serving["all_resident"] = {
                md: bench_serving(torch, log, args.serve_resident_gb, md,
                                  capacity=args.serve_capacity, chunk=args.serve_chunk,
                                  check=False, line_pressure=args.serve_line_pressure)
                for md in (args.serve_mode, other)}

    cpu = None
    if systems is not None:
        cpu = cpu_baseline(log, wl, systems, threads, bytes_iter("csr", n, nnz, 8))

    moved_gbs = moved64 / (ms64 * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(moved_gbs, 2),
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
        "value_basis": ("bytes the step's solves move as run / step time: CG on the "
                        "Jacobi-scaled operator (upper diagonals without the unit diagonal, 10 "
                        "vector passes and the FP32 weights per iteration)" if scaled else
                        "bytes the step's solves move as run / step time: operator read + 12 "
                        "vector passes per Jacobi-PCG iteration"),
        "jacobi_scaled": scaled,
        "algorithm_equivalent_GBs": round(gbs64, 1),
        "algorithm_equivalent_basis": "the same iterations priced as plain Jacobi-PCG on the "
                                      "diagonal storage (operator with its diagonal + 12 vector "
                                      "passes) / step time",
        "csr_equivalent_GBs": round(csr_equiv / (ms64 * 1e-3) / 1e9, 1),
        "fp64": {k: {"iters": i.iterations, "relres": i.relres_true, "ms": solve_ms64[k]}
                 for k, i in infos64.items()},
        "pressure_time_to_tol_ms": {"fp64": solve_ms64["q"],
                                    "mixed": None if mixed is None else solve_msm["q"]},
        "errors_vs_oracle": errors,
        "step_ms": [round(1e3 * v, 3) for v in per64],
        "roofline": {"bound": "hbm", "achieved": round(spmv_gbs, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(spmv_gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": spmv_kernel,
                     "bytes_per_launch": spmv_bytes, "avg_us": round(spmv_avg_us, 2),
                     # the same launch priced at the canonical CSR bytes (values, column
                     # indices, row pointers, p, q): what an index-carrying format moves
                     "csr_canonical_bytes_per_launch": bytes_spmv("csr", n, nnz, 8),
                     "frac_csr_canonical": round(bytes_spmv("csr", n, nnz, 8)
                                                 / (spmv_avg_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)},
        "pressure_kernels": kern,
        "mixed": mixed,
        "line_pressure_step": line_step,
        "operator_setup": setup,
        "pressure_formats": formats,
        "shard_share": share,
        "isotropic_pressure": isotropic,
        "velocity_preconditioners": precond,
        "small_box": small_box,
        "bricks_q2_q1": bricks,
        "time_loop": loop,
        "batched": batched,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
