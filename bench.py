#!/usr/bin/env python3
"""Throughput benchmark of the substructuring Schur-complement solver on one MI355X.

One step = one full solve of the hot path on the workload's batch of
right-hand sides: condensation, preconditioned CG on the interface Schur
complement to the tolerance, back substitution, FP64 residual check (and, in
mixed precision, the refinement loop).  The subdomain factorisation is done
once before timing (setup, excluded as in the paper's solve timings).

Default workload: 2D bond-based peridynamics (2 dofs per node), delta = 0.05,
P1 on a structured right-triangle mesh h = 1/160 (50 562 free dofs), 8x8
subdomains from jittered cuts (+-30 % widths), 32 seeded right-hand sides in
one batch, relative residual 1e-9 (the largest tolerance at which every
column stays within 1e-8 relative error of the monolithic FP64 solution).

Prints ONE JSON line.  `value` is the solves/s (right-hand-side columns
solved per second) of the faster of the two paths, mixed precision or plain
FP64 (named in config.path); both are reported under "mixed" and "fp64", each
with its largest per-solve error against the oracle's monolithic solution
(computed in the CPU-baseline leg).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/sec at rel-resid 1e-8 (mixed vs plain FP64, 1 GPU); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of MI355X (TFLOP/s): FP64 and FP32 MFMA
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}

# Relative-residual target per workload: the largest tolerance at which the
# solution stays within 1e-8 relative error of the monolithic FP64 solution
# (at 1e-8 the peridynamic system's columns reach 6e-8 error; checked by the
# GPU parity tests at these tolerances).
WORKLOADS = {
    "cfg2": dict(spec="spec_2d_const", tol=1e-9,
                 desc="2d nonlocal diffusion, constant kernel 4/(pi delta^4), l2 ball "
                      "(barycentre truncation), delta=0.1, P1 h=1/128 (16129 dofs), "
                      "4x4 subdomains, 1 seeded rhs"),
    "cfg3": dict(spec="spec_2d_frac", tol=1e-10,
                 desc="2d fractional-type kernel s=0.5, delta=0.1, P1 h=1/96 (9025 dofs), "
                      "4x4 subdomains, 8 seeded rhs"),
    "cfg4": dict(spec="spec_2d_pd", tol=1e-9,
                 desc="2d bond-based peridynamics, delta=0.05, P1 h=1/160 (50562 dofs), "
                      "8x8 jittered subdomains, 32 seeded rhs"),
}


# Bytes moved beyond L2 per dispatch of the dominant kernels, from two
# rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE) of this benchmark, each
# scaled by what the counter read for an elementwise kernel of known traffic
# (--calibrate-copy).  Valid only for the kernel source they were taken on
# (sha256 prefix of the file holding the kernel) and the workload named;
# reported as null once that source changes.
MEASURED_TRAFFIC = {
    # 2D peridynamics h = 1/160, 32 rhs: medians over the CG iterations' launches
    "k_tile_rows<double,2,true>": dict(src="dd_tiles.h", sha="7e9d81ffc6acec94", workload="cfg4",
                                       fetch_kib=160066.1, write_kib=9624.3,
                                       fetch_scale=262144.0 / 131086.8, write_scale=262144.0 / 262146.9),
    "k_tile_rows<float,2,true>": dict(src="dd_tiles.h", sha="7e9d81ffc6acec94", workload="cfg4",
                                      fetch_kib=82966.3, write_kib=9624.3,
                                      fetch_scale=262144.0 / 131086.8, write_scale=262144.0 / 262146.9),
}


def measured_traffic(kernel: str, workload: str):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None or m["workload"] != workload:
        return None
    src = os.path.join(ROOT, "paper_2306_00094_amd", "csrc", m["src"])
    try:
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    if sha != m["sha"]:
        return None
    return 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gamma_kernel_bytes(dd, nrhs_pad: int, value_bytes: int, gamma_vectors: int = 3) -> float:
    """Algorithmic HBM bytes of one interface-row launch (q = K_GG p - K_GI w):
    every nonzero of [K_GG | K_GI] once (value + int32 column), the row and
    split pointers, the interior vector w read once, and gamma_vectors
    interface-vector passes (three-launch CG iteration: p read, q and D^-1 q
    written; undecomposed system: p read and q written, plus z read and p
    written when the direction is formed at the gathers)."""
    nnz = dd.kgg.nnz + sum(k.nnz for k in dd.kig)
    ni = sum(len(m) for m in dd.i_maps)
    ng = dd.n_gamma
    return (nnz * (value_bytes + 4) + (2 * ng + 1) * 4
            + 8.0 * nrhs_pad * (gamma_vectors * ng + ni))


def tile_format_bytes(dd, nrhs_pad: int, value_bytes: int) -> float:
    """HBM bytes one tiled interface launch streams in its storage format:
    every entry of [K_GG | K_GI] in blocks of 32 interface rows x 8 columns
    (two 16x8 units per entry, zeros included; K_GI columns numbered by the
    interiors one subdomain after the other), its int32 column block, the row
    and split pointers, and the vectors as in gamma_kernel_bytes (p and w
    read, q written)."""
    import numpy as np
    kgg = dd.kgg.tocoo()
    keys = [np.unique((kgg.row.astype(np.int64) // 32) << 32 | (kgg.col.astype(np.int64) // 8))]
    off = 0
    for k, m in enumerate(dd.i_maps):
        kig = dd.kig[k].tocoo()
        g = np.asarray(dd.g_maps[k])[kig.col].astype(np.int64)
        keys.append(np.unique((g // 32) << 32 | ((off + kig.row.astype(np.int64)) // 8) | (1 << 62)))
        off += len(m)
    ent = len(np.unique(np.concatenate(keys)))
    nrb = (dd.n_gamma + 31) // 32
    ni = sum(len(m) for m in dd.i_maps)
    return (ent * (2 * 128 * value_bytes + 4) + (2 * nrb + 1) * 4
            + 8.0 * nrhs_pad * (2 * dd.n_gamma + ni))


def iteration_bytes(dd, nrhs_pad: int, value_bytes: int) -> float:
    """Algorithmic bytes of one CG iteration: K_IG rows (y written), the
    interior inverse blocks (y read, w read and written), the interface rows,
    and the interface-vector updates (r, z, p, q, D^-1 q, x: about 10 passes)."""
    nig = sum(k.nnz for k in dd.kig)
    ni = sum(len(m) for m in dd.i_maps)
    kinv = sum(k.size for k in dd.kii)
    return (nig * (value_bytes + 4) + (ni + 1) * 4 + 8.0 * nrhs_pad * ni
            + kinv * value_bytes + 8.0 * nrhs_pad * 3 * ni
            + gamma_kernel_bytes(dd, nrhs_pad, value_bytes)
            + 8.0 * nrhs_pad * 10 * dd.n_gamma)


def factor_flops(dd) -> float:
    """Arithmetic of one factorisation (MFMA work): per subdomain Cholesky
    n^3/3, X = L^-1 n^3/3 and K^-1 = X^T X n^3/3 flops, and diag(S) from the
    column sums of squares of X K_IG (n^2 n_Gk for the triangle times the
    dense strip of the subdomain's interface columns, 2 n n_Gk for the
    squares)."""
    tot = 0.0
    for K, g in zip(dd.kii, dd.g_maps):
        n, ng = K.shape[0], len(g)
        tot += 3 * n ** 3 / 3.0 + n * n * ng + 2.0 * n * ng
    return float(tot)


# The kernel timing of the roofline is taken on every TIMING_EVERY-th solve of
# the timed region: an event pair recorded by a launch costs about 5 us of
# stream time, which on every launch would slow the timed solves by ~10%.
TIMING_EVERY = 4


def time_path(solver, dd, b, prec, opts, steps, warmup, torch, timing_every=TIMING_EVERY):
    for _ in range(warmup):
        solver.solve(b, prec=prec, opts=opts)
    torch.cuda.synchronize()
    lat = []
    res = None
    mask = (1 << dd.DD_PHASE_GAMMA) | (1 << dd.DD_PHASE_LOOP)
    dd.dd_set_timing(solver.ctx, 0, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        if i % timing_every == 0:
            dd.dd_set_timing(solver.ctx, mask, reset=False)
        res = solver.solve(b, prec=prec, opts=opts)       # returns when complete
        if i % timing_every == 0:
            dd.dd_set_timing(solver.ctx, 0, reset=False)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, n = dd.dd_get_timing(solver.ctx)
    dd.dd_set_timing(solver.ctx, 0)
    return dict(seconds=t1 - t0, lat=lat, info=res.info, u=res.u,
                sampled=(steps + timing_every - 1) // timing_every,
                gamma_ms=ms[dd.DD_PHASE_GAMMA], gamma_launches=n[dd.DD_PHASE_GAMMA],
                loop_ms=ms[dd.DD_PHASE_LOOP], loop_launches=n[dd.DD_PHASE_LOOP])


def pct(v, q):
    v = sorted(v)
    k = max(0, min(len(v) - 1, int(math.ceil(q * len(v))) - 1))
    return v[k]


# State the CPU-baseline workers inherit from the parent (fork): the oracle
# after its setup, the right-hand sides and the tolerance.
_CPU = {}


def _cpu_ready(_):
    return os.getpid()


def _cpu_solve(cols):
    """One worker's share of the CPU baseline: the oracle's substructuring
    solve of a slice of the columns (one call, BLAS on one thread)."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        u, its, conv = _CPU["oracle"].solve(_CPU["b"][:, cols], tol=_CPU["tol"])
        return list(cols), u, [int(i) for i in its], time.perf_counter() - t0


def cpu_baseline(wl, b, tol, workers: int, max_cols: int):
    """The CPU FP64 oracle's substructuring solve (same method, tolerance and
    right-hand sides) on the host's cores: `workers` processes forked before
    anything touches the GPU, each solving a contiguous slice of the first
    max_cols columns in one oracle call with its BLAS on one thread; setup
    excluded, wall time from dispatch to the last result.  Also returns the
    oracle's monolithic solution of every column (Cholesky of the whole
    matrix): the reference of the per-solve error of the GPU paths."""
    import multiprocessing

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    nrhs = b.shape[1]
    ncols = min(nrhs, max_cols)
    workers = max(1, min(workers, ncols))
    with threadpool_limits(limits=1):
        orc = oracle.DDOracle(wl.dd)
        orc.schur_diag()
    _CPU.update(oracle=orc, b=np.ascontiguousarray(b), tol=tol)
    slices = [list(r) for r in np.array_split(np.arange(ncols), workers)]
    ctx = multiprocessing.get_context("fork")
    with ctx.Pool(processes=workers) as pool:
        pool.map(_cpu_ready, range(workers), chunksize=1)       # every worker started
        t0 = time.perf_counter()
        parts = pool.map(_cpu_solve, slices, chunksize=1)
        dt = time.perf_counter() - t0
    _CPU.clear()
    u_dd = np.zeros((b.shape[0], ncols))
    its = [0] * ncols
    for cols, u, it, _ in parts:
        u_dd[:, cols] = u.reshape(b.shape[0], -1)
        for c, i in zip(cols, it):
            its[c] = i
    t1 = time.perf_counter()
    uref = oracle.monolithic_solve(wl.asm.A, b)
    mono_s = time.perf_counter() - t1
    res = dict(value=ncols / dt, unit="solves/s", cores=workers, kind="oracle",
               sample=f"{ncols} of the {nrhs} columns, oracle substructuring PCG (FP64, tol {tol:g}) in "
                      f"{workers} processes x 1 BLAS thread, {dt:.1f} s wall",
               threads_available=os.cpu_count(), iters=its,
               worker_seconds=[round(p[3], 2) for p in parts],
               oracle_dd_max_rel_err=float(oracle.rel_err(u_dd, uref[:, :ncols]).max()),
               monolithic_seconds=mono_s)
    return res, uref


def solve_errors(u, uref):
    """Largest per-column error of u against the oracle's monolithic
    solution: relative 2-norm and relative max-norm."""
    import numpy as np
    d = u - uref
    e2 = np.linalg.norm(d, axis=0) / np.linalg.norm(uref, axis=0)
    einf = np.abs(d).max(axis=0) / np.abs(uref).max(axis=0)
    return dict(max_rel_err_2=float(e2.max()), max_rel_err_inf=float(einf.max()), columns=int(u.shape[1]))


def serving_leg(dd, workloads, wl_main, nreq: int, seed: int = 5000, gather32: int = 1,
                chunk: int = 1000, nreq_load: int = 2000, nreq_budget: int = 1000,
                budget_frac: float = 0.5):
    """Continuous-batching serving run (paper_2306_00094_amd.serving) over
    eleven systems drawn from the first three workloads at mesh scales 0.5 to
    2: the 1D constant kernel at h = 1/512 ... 1/2048 (scales 0.5, 0.75, 1,
    1.5, 2), the 2D constant kernel at h = 1/64, 1/96, 1/128 and the 2D
    fractional kernel at h = 1/48, 1/72, 1/96 (scales 0.5, 0.75, 1; their 1.5
    and 2 scales take 30-60 s of host assembly each and stay out of the
    default run).  Requests carry 1-64 seeded right-hand sides and pick a
    system uniformly.  Three phases, mixed precision with FP32 gathers unless
    gather32 = 0:
      saturated: nreq requests arriving at once, in chunks of `chunk` (each
                 drains before the next), every system resident;
      load:      nreq_load Poisson arrivals at 0.8x the saturated request rate
                 (latency under load);
      budget:    nreq_budget requests arriving at once with an HBM budget of
                 budget_frac of the systems' summed footprint, so that systems
                 are evicted and set up again as requests for them arrive."""
    import numpy as np
    from paper_2306_00094_amd import serving
    specs = {
        "1d-const h=1/512": workloads.spec_1d(n=512),
        "1d-const h=1/768": workloads.spec_1d(n=768),
        "1d-const h=1/1024": workloads.spec_1d(),
        "1d-const h=1/1536": workloads.spec_1d(n=1536),
        "1d-const h=1/2048": workloads.spec_1d(n=2048),
        "2d-const h=1/64": workloads.scaled(workloads.spec_2d_const, 0.5),
        "2d-const h=1/96": workloads.scaled(workloads.spec_2d_const, 0.75),
        "2d-frac h=1/48": workloads.scaled(workloads.spec_2d_frac, 0.5),
        "2d-frac h=1/72": workloads.scaled(workloads.spec_2d_frac, 0.75),
        "2d-frac h=1/96": workloads.spec_2d_frac(),
    }
    systems = {k: workloads.build(sp).dd for k, sp in specs.items()}
    systems["2d-const h=1/128"] = wl_main.dd
    specs["2d-const h=1/128"] = wl_main.spec
    rng = np.random.default_rng(seed)
    keys = sorted(systems)
    loads = {k: workloads.rhs(specs[k], nrhs=64, seed_base=seed + 100 * i) for i, k in enumerate(keys)}

    def requests(arrivals, base=0):
        out = []
        for i, t in enumerate(arrivals):
            k = keys[int(rng.integers(0, len(keys)))]
            m = int(rng.integers(1, 65))
            out.append(serving.Request(key=k, b=np.asfortranarray(loads[k][:, :m]), arrival=float(t),
                                       rid=base + i))
        return out

    # long runs go in chunks of `chunk` requests (each drains before the next
    # starts); seconds add up over the chunks
    def phase(srv, name, n_total, arrivals):
        done, secs = [], 0.0
        for c0 in range(0, n_total, chunk):
            n = min(chunk, n_total - c0)
            t0 = time.perf_counter()
            d = srv.run(requests(arrivals(n, c0), c0), timeout=600, keep_resident=True)
            wall = time.perf_counter() - t0
            secs += wall if name != "load" else serving.summarize(d)["seconds"]
            done += d
            if n_total > chunk:
                log(f"bench: serving {name}: {c0 + n}/{n_total} requests, {secs:.1f} s")
        return serving.summarize(done, wall=secs)

    opts = dd.dd_default_opts(tol=1e-9, gather32=gather32)
    srv = serving.Server(systems, prec=dd.DD_MIXED, opts=opts, iters_per_step=4)
    total_fp = sum(srv.footprint.values())
    try:
        # every system resident (factors formed) before anything is timed
        srv.run(requests(np.zeros(len(keys) * 2)), timeout=300, keep_resident=True)
        burst = phase(srv, "saturated", nreq, lambda n, c0: np.zeros(n))
        rate = 0.8 * burst["requests"] / burst["seconds"]
        load = phase(srv, "load", nreq_load,
                     lambda n, c0: serving.poisson_arrivals(n, rate=rate, seed=seed + 1 + c0))
    finally:
        srv.shutdown()
    budget = int(budget_frac * total_fp)
    srv_b = serving.Server(systems, prec=dd.DD_MIXED, opts=opts, iters_per_step=4, hbm_budget=budget)
    try:
        bud = phase(srv_b, "budget", nreq_budget, lambda n, c0: np.zeros(n))
        evictions = srv_b.evictions
    finally:
        srv_b.shutdown()
    return dict(systems=keys, requests=nreq, rhs_per_request="1-64", rel_resid=1e-9, precision="mixed",
                fp32_gathers=bool(gather32),
                saturated_solves_per_s=burst["solves_per_s"], saturated_p50_ms=burst["p50_ms"],
                saturated_p99_ms=burst["p99_ms"], offered_requests_per_s=rate,
                load_requests=nreq_load,
                solves_per_s=load["solves_per_s"], p50_ms=load["p50_ms"], p99_ms=load["p99_ms"],
                fallbacks=load["fallbacks"] + burst["fallbacks"] + bud["fallbacks"],
                budget=dict(requests=nreq_budget, hbm_budget_bytes=budget, footprint_sum_bytes=total_fp,
                            evictions=evictions, solves_per_s=bud["solves_per_s"], p50_ms=bud["p50_ms"],
                            p99_ms=bud["p99_ms"]),
                note="saturated: requests arrive at once (latency includes queueing); load: Poisson "
                     "arrivals at 0.8x the saturated rate; budget: HBM budget below the summed "
                     "footprint, systems evicted and set up again")


def next_pow2(n: int) -> int:
    ld = 1
    while ld < n:
        ld *= 2
    return ld


def path_roofline(dd, wl, solver, bt, prec, opts, tuned, r, ld, workload, steps, torch):
    """Roofline of the dominant kernel of a path: the interface-row launch
    of the CG iteration (q = K_GG p - K_GI w with the per-column p^T q
    partials).  Its algorithmic bytes are every nonzero of [K_GG | K_GI] once
    (value + int32 column), the row pointers, p and w read and q written.
    The launch duration comes from events the launch records on the solver's
    stream during the timed region; a schedule replayed as a graph hides the
    kernel boundaries, and then a separate pass with per-kernel launches (same
    kernels) times it."""
    vb = 8 if prec == dd.DD_FP64 else 4
    vt = "double" if vb == 8 else "float"
    tiles = bool(tuned.get("three_launch", 0) & 4)
    if tiles:
        ncb = 1 if ld <= 16 else (2 if ld <= 32 else 4)
        key = f"k_tile_rows<{vt},{ncb},true>"
        kname = key + " (16x8 units of [K_GG | K_GI] on MFMA: q = K_GG p - K_GI w, p^T q)"
        algo = gamma_kernel_bytes(wl.dd, ld, vb, 2)
    else:
        key = f"k_gamma_rows<{vt}>"
        kname = key + " (CSR rows of [K_GG | K_GI]: q = K_GG p - K_GI w)"
        algo = gamma_kernel_bytes(wl.dd, ld, vb)
    how = f"events on every {TIMING_EVERY}th solve of the timed region"
    graph = tuned.get("launch") == dd.DD_LAUNCH_GRAPH
    if r["gamma_launches"] > 0 and not graph:
        ms, launches = r["gamma_ms"], r["gamma_launches"]
    else:                 # (a graph schedule times only the launches outside its replays)
        o2 = dd.dd_default_opts(tol=opts.tol, launch=dd.DD_LAUNCH_KERNELS, apply=dd.DD_APPLY_INV,
                                tiles=1 if tiles else 0)
        r2 = time_path(solver, dd, bt, prec, o2, max(3, steps // 4), 1, torch, timing_every=1)
        ms, launches = r2["gamma_ms"], r2["gamma_launches"]
        how = "events on every solve of a separate pass with per-kernel launches (the timed " \
              "schedule replays a graph)"
    if launches <= 0:
        return None
    avg = ms / launches * 1e-3
    ach = algo / avg / 1e9
    out = dict(bound="hbm", kernel=kname, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
               frac=ach / HBM_PEAK_GBS, traffic=measured_traffic(key, workload),
               algo_bytes_per_launch=algo, avg_launch_us=1e6 * avg, launches=launches, timing=how)
    if tiles:
        fb = tile_format_bytes(wl.dd, ld, vb)
        out.update(format_bytes_per_launch=fb, format_gbs=fb / avg / 1e9,
                   format_note="bytes the 32x8-entry unit format streams (zeros of partly filled "
                               "tiles included); achieved/frac use the nonzeros only")
    return out


def solve_leg(dd, torch, wl, b, tol, steps, warmup, launch, workload):
    """Mixed precision against plain FP64 on one system and batch: factor
    (timed on the host, best of 3), autotune each path for the batch width
    (unless a launch mode is fixed), time `steps` solves of each path, and
    the roofline of the dominant kernel.  Returns the per-path summaries and
    the solutions of the last timed solve (n_dof x nrhs, for the error
    against the oracle)."""
    import numpy as np
    nrhs = b.shape[1]
    ld = next_pow2(nrhs)
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda:0").contiguous()
    solver = dd.Solver(wl.dd, max_nrhs=nrhs)
    out, sols = {}, {}
    try:
        for name, prec in (("fp64", dd.DD_FP64), ("mixed", dd.DD_MIXED)):
            solver.factor(prec)                    # first call: allocations, code loading
            reps = []
            for _ in range(3):
                torch.cuda.synchronize()
                t = time.perf_counter()
                solver.factor(prec)
                torch.cuda.synchronize()
                reps.append(time.perf_counter() - t)
            fac = min(reps)
            if launch == "auto":
                opts = dd.dd_default_opts(tol=tol)
                tuned = solver.autotune(prec, nrhs, opts)      # the schedule AUTO solves use
            else:
                mode = {"kernels": dd.DD_LAUNCH_KERNELS, "graph": dd.DD_LAUNCH_GRAPH,
                        "persistent": dd.DD_LAUNCH_PERSISTENT}[launch]
                opts = dd.dd_default_opts(tol=tol, launch=mode, apply=dd.DD_APPLY_INV)
                tuned = dict(apply=dd.DD_APPLY_INV, launch=mode, fixed=True)
            log(f"bench: {workload} {name}: factor {1e3 * fac:.2f} ms, schedule {tuned}")
            r = time_path(solver, dd, bt, prec, opts, steps, warmup, torch)
            fl = factor_flops(wl.dd)
            peak = MFMA_PEAK_TFLOPS["f64" if prec == dd.DD_FP64 else "f32"]
            out[name] = dict(
                value=steps * nrhs / r["seconds"], ms_per_step=1e3 * r["seconds"] / steps,
                p50_ms=1e3 * statistics.median(r["lat"]), p99_ms=1e3 * pct(r["lat"], 0.99),
                iters=[i["iters"] for i in r["info"]],
                refine_steps=[i["refine_steps"] for i in r["info"]],
                used_fallback=[i["used_fallback"] for i in r["info"]],
                rel_resid_max=max(i["rel_resid"] for i in r["info"]),
                schedule=tuned,
                roofline=path_roofline(dd, wl, solver, bt, prec, opts, tuned, r, ld, workload, steps, torch),
                factor=dict(ms=1e3 * fac, gflop=fl / 1e9, achieved_tflops=fl / fac / 1e12, bound="mfma",
                            peak_tflops=peak, frac=fl / fac / 1e12 / peak,
                            note="whole factorisation (Cholesky, L^-1, K^-1, diag(S)) timed on the host"))
            if name == "mixed":
                # the tiled mixed solve with the FP64 factor formed replaces its
                # recurrence residual by the FP64 one instead of refining (one
                # outer step per column)
                out[name]["residual_replacement"] = bool(tuned.get("three_launch", 0) & 4) and \
                    max(out[name]["refine_steps"]) == 1
            sols[name] = r["u"].cpu().numpy().T[:wl.dd.n_dof, :nrhs].copy()
            log(f"bench: {workload} {name}: {out[name]['ms_per_step']:.3f} ms/step "
                f"its={out[name]['iters'][:4]} resid={out[name]['rel_resid_max']:.2e}")
    finally:
        solver.close()
    out["mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    return out, sols


# FP64 vector peak (256 CUs at 2.4 GHz) for the ALU-bound assembly kernel
FP64_VECTOR_PEAK_TFLOPS = 78.6
# FP64 operations per quadrature-point pair of the constant kernel (whose
# value does not depend on the points; the rule weights of the two elements,
# the areas and the constant are combined once per point of F): d_m (1 sub),
# the pair weight (1 mul) times d_m (1 mul), and per vertex of the union of a
# pair without shared vertices (6): d_n (1 sub, E's three vertices only) and
# the accumulation (1 fma: 2)
ASM_FLOPS_PER_QP = 18


def interacting_pairs_per_row(spec) -> int:
    """Ordered element pairs (E holding the node, F) that pass the barycentre
    test, for a free node whose partners all lie on the mesh (the collar is
    at least the search radius, so every free node has the same count)."""
    import math
    h = spec.h
    r1 = int(math.ceil(spec.delta / h)) + 1
    thr = math.floor((3.0 * spec.delta / h) ** 2)

    def tri(a, b, t):
        return [(a, b), (a + 1, b + t), (a + 1 - t, b + 1)]

    m = (0, 0)
    count = 0
    for ca in (-1, 0):
        for cb in (-1, 0):
            for t in (0, 1):
                E = tri(ca, cb, t)
                if m not in E:
                    continue
                be = (sum(v[0] for v in E), sum(v[1] for v in E))
                for fa in range(ca - r1, ca + r1 + 1):
                    for fb in range(cb - r1, cb + r1 + 1):
                        for tf in (0, 1):
                            F = tri(fa, fb, tf)
                            bf = (sum(v[0] for v in F), sum(v[1] for v in F))
                            if (be[0] - bf[0]) ** 2 + (be[1] - bf[1]) ** 2 <= thr:
                                count += 1
    return count


def assembly_leg(dd, workloads, torch, reps=5):
    """Device assembly (dd_assemble_2d) of the benchmark system's stiffness
    windows (2D constant kernel, h = 1/128, delta = 0.1, 16 129 rows of 31 x
    31) against the CPU generator on the host's cores: time, agreement, and
    the FP64 vector rate of the quadrature (ALU-bound)."""
    import numpy as np
    spec = workloads.spec_2d_const()
    R = workloads.window_radius(spec)
    W = 2 * R + 1
    rows = (spec.n - 1) ** 2
    win = torch.empty(rows * W * W, dtype=torch.float64, device="cuda")
    args = (spec.n, spec.collar, spec.delta, spec.kernel, spec.phi, spec.s, R, win)
    dd.dd_assemble_2d(*args)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dd.dd_assemble_2d(*args)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    t0 = time.perf_counter()
    ref = workloads.assemble_windows(spec)
    cpu_ms = 1e3 * (time.perf_counter() - t0)
    got = win.cpu().numpy().reshape(rows, -1)
    ref = ref.reshape(rows, -1)
    err = float((np.abs(got - ref) / np.abs(ref).max(axis=1, keepdims=True)).max())
    pairs = interacting_pairs_per_row(spec) * rows
    qp = pairs * 49
    tflops = qp * ASM_FLOPS_PER_QP / (ms * 1e-3) / 1e12
    return dict(system="2d-const h=1/128 delta=0.1", rows=rows, window=f"{W}x{W}", ms=ms,
                cpu_generator_ms=cpu_ms, cpu_threads=workloads._nthreads(), speedup=cpu_ms / ms,
                max_rel_diff_vs_generator=err, element_pairs=pairs, quad_pairs=qp,
                roofline=dict(bound="alu", achieved=tflops, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                              frac=tflops / FP64_VECTOR_PEAK_TFLOPS,
                              flops_per_quad_pair=ASM_FLOPS_PER_QP))


def jacobi_cg_leg(dd, workloads, wl, b, tol, steps, warmup, torch):
    """The paper's baseline solver on the same system: CG on the whole matrix
    with diag(A) as preconditioner (section "Considered solver strategies"),
    run by the library as the undecomposed problem (no subdomains, S = A).
    Same tolerance, right-hand sides, launch autotuning and timing as the
    substructuring solve; its dominant kernel is the CSR sweep of A."""
    import numpy as np

    und = workloads.undecomposed(wl.asm.A)
    nrhs = b.shape[1]
    ld = next_pow2(nrhs)
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda:0").contiguous()
    s = dd.Solver(und, max_nrhs=nrhs)
    out = {}
    try:
        for name, prec in (("fp64", dd.DD_FP64), ("mixed", dd.DD_MIXED)):
            s.factor(prec)
            opts = dd.dd_default_opts(tol=tol, max_it=20000)
            tuned = s.autotune(prec, nrhs, opts)
            r = time_path(s, dd, bt, prec, opts, steps, warmup, torch)
            vb = 8 if prec == dd.DD_FP64 else 4
            # direction kept by its own kernel: p read, q written; else also z read, p written
            sweep = gamma_kernel_bytes(und, ld, vb, 2 if tuned.get("direction_kernel") else 4)
            roof = None
            if r["gamma_launches"] > 0:
                avg = r["gamma_ms"] / r["gamma_launches"] * 1e-3
                ach = sweep / avg / 1e9
                roof = dict(bound="hbm", kernel="k_gamma_rows<%s> (q = A p)" % ("double" if vb == 8 else "float"),
                            achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                            algo_bytes_per_launch=sweep, avg_launch_us=1e6 * avg,
                            launches=r["gamma_launches"])
            out[name] = dict(value=steps * nrhs / r["seconds"], ms_per_step=1e3 * r["seconds"] / steps,
                             p50_ms=1e3 * statistics.median(r["lat"]), p99_ms=1e3 * pct(r["lat"], 0.99),
                             iters_max=max(i["iters"] for i in r["info"]),
                             rel_resid_max=max(i["rel_resid"] for i in r["info"]),
                             schedule=tuned, roofline=roof)
            log(f"bench: jacobi-cg {name} {out[name]['ms_per_step']:.3f} ms/step its={out[name]['iters_max']}")
    finally:
        s.close()
    out["nnz"] = int(wl.asm.A.nnz)
    return out


def feti_leg(dd, workloads, torch, tol=1e-10, reps=5):
    """One-level FETI (dd_feti_*, Algorithm 1) on the weak-scaling ladder of
    the section "Weak scaling for fixed delta/h": 2D constant kernel,
    delta/h = 4, h = 1/32, 1/64, 1/128 on 2x2, 4x4, 8x8 subdomains, one
    seeded right-hand side.  Beside it the primal Schur-complement PCG
    (FP64, autotuned) and diagonally preconditioned CG on the whole matrix,
    all on the GPU at the same tolerance: iterations and solve time (mean of
    `reps` solves after one warm-up), the counts the paper's Table
    fixedRatio compares."""
    import numpy as np
    rows = []
    for n, cuts in ((32, (2, 2)), (64, (4, 4)), (128, (8, 8))):
        spec = workloads.spec_2d_const(n=n, delta=4.0 / n, cuts=cuts, nrhs=1)
        wl = workloads.build(spec)
        fp = workloads.feti_problem(wl)
        b = workloads.rhs(spec)
        bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda:0").contiguous()
        row = dict(h=f"1/{n}", subdomains=f"{cuts[0]}x{cuts[1]}", n_dof=int(wl.dd.n_dof),
                   n_gamma=int(wl.dd.n_gamma), floating=int(sum(fp.floating)))

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = fn()
            torch.cuda.synchronize()
            return r, 1e3 * (time.perf_counter() - t0) / reps

        fs = dd.FetiSolver(wl.dd, fp, max_nrhs=1)
        try:
            fs.factor()
            r, ms = timed(lambda: fs.solve(bt, tol=tol, max_it=2000))
            row["feti"] = dict(iters=r.info[0]["iters"], ms=ms, rel_resid=r.info[0]["rel_resid"])
        finally:
            fs.close()
        for key, prob in (("primal_schur_pcg", wl.dd), ("jacobi_cg", workloads.undecomposed(wl.asm.A))):
            s = dd.Solver(prob, max_nrhs=1)
            try:
                s.factor(dd.DD_FP64)
                opts = dd.dd_default_opts(tol=tol, max_it=20000)
                s.autotune(dd.DD_FP64, 1, opts)
                r, ms = timed(lambda: s.solve(bt, prec=dd.DD_FP64, opts=opts))
                row[key] = dict(iters=r.info[0]["iters"], ms=ms, rel_resid=r.info[0]["rel_resid"])
            finally:
                s.close()
        log(f"bench: feti ladder h=1/{n}: {row}")
        rows.append(row)
    return dict(kernel="2d constant, delta/h = 4", tol=tol, ladder=rows,
                note="FETI stops on the projected residual of the multipliers, the others on the "
                     "relative residual of their own system; rel_resid is the full system's for all three")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg4", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle baseline (and with it the per-solve error against the oracle)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the CPU baseline (0 = min(16, host CPUs))")
    ap.add_argument("--cpu-max-cols", type=int, default=32,
                    help="columns of the batch the CPU baseline solves (its bounded sample)")
    ap.add_argument("--serving-requests", type=int, default=10000,
                    help="requests of the serving leg (0 = skip it)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the one-rhs leg on the 2D constant-kernel system")
    ap.add_argument("--no-assembly", action="store_true", help="skip the device-assembly leg")
    ap.add_argument("--no-jacobi-cg", action="store_true",
                    help="skip the baseline leg (Jacobi-preconditioned CG on the whole system)")
    ap.add_argument("--no-feti", action="store_true", help="skip the FETI weak-scaling leg")
    ap.add_argument("--launch", default="auto", choices=["auto", "kernels", "graph", "persistent"],
                    help="CG launch mode; auto = the schedule chosen by the library's autotuner")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="run one device-to-device copy of this many MB first (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not supported "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import workloads
    cfg = WORKLOADS[args.workload]
    spec = getattr(workloads, cfg["spec"])()
    tol = cfg["tol"]
    log(f"bench: building workload {args.workload} ...")
    t = time.perf_counter()
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    nrhs = b.shape[1]
    log(f"bench: workload ready in {time.perf_counter() - t:.1f} s: n_dof={wl.dd.n_dof} "
        f"n_gamma={wl.dd.n_gamma} K={wl.dd.n_sub} nrhs={nrhs}")

    # CPU baseline first: its worker processes are forked before anything
    # touches the GPU
    cpu, uref = None, None
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        log(f"bench: CPU oracle baseline ({workers} processes) and monolithic reference ...")
        t = time.perf_counter()
        cpu, uref = cpu_baseline(wl, b, tol, workers, args.cpu_max_cols)
        log(f"bench: CPU leg done in {time.perf_counter() - t:.1f} s: {cpu['value']:.2f} solves/s")

    import numpy as np
    import torch

    import paper_2306_00094_amd as dd
    dd.load_library()
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)         # one elementwise kernel: reads and writes MB each
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {args.calibrate_copy} MB done")
        del src, dst

    head, sols = solve_leg(dd, torch, wl, b, tol, args.steps, args.warmup, args.launch, args.workload)
    mixed, fp64 = head["mixed"], head["fp64"]
    if uref is not None:
        for name in ("mixed", "fp64"):
            head[name]["error_vs_oracle"] = solve_errors(sols[name], uref)
    del sols

    # the headline is the faster of the two paths (both meet the same residual
    # and error gates); the other is reported beside it
    best = "mixed" if mixed["value"] >= fp64["value"] else "fp64"
    other = "fp64" if best == "mixed" else "mixed"
    top = head[best]
    line = {
        "metric": METRIC,
        "value": top["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": top["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if best == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "name": args.workload, "path": best, "rel_resid": tol,
                   "rel_resid_note": "tighter than the metric's 1e-8 so that every column stays within "
                                     "1e-8 relative error of the oracle's monolithic solution",
                   "nrhs": nrhs, "n_dof": wl.dd.n_dof, "n_gamma": wl.dd.n_gamma,
                   "subdomains": wl.dd.n_sub},
        "p50_ms": top["p50_ms"],
        "p99_ms": top["p99_ms"],
        "latency_note": "per batch solve (all nrhs columns), host clock from call to return",
        "mixed": mixed,
        "fp64": fp64,
        "mixed_vs_fp64": head["mixed_vs_fp64"],
        "error_vs_oracle": {k: head[k].get("error_vs_oracle") for k in ("mixed", "fp64")},
        "roofline": dict(top["roofline"] or {}, **{other: head[other]["roofline"]}),
        "paper_context": "14.6x FETI vs Jacobi-CG solve time, fractional kernel, 48x48 subdomains, "
                         "16M dofs, 2304 Broadwell ranks (different method and machine)",
    }
    if not args.no_secondary and args.workload != "cfg2":
        c2 = WORKLOADS["cfg2"]
        log("bench: one-rhs leg (2D constant kernel, h = 1/128) ...")
        wl2 = workloads.build(workloads.spec_2d_const())
        b2 = workloads.rhs(wl2.spec)
        sec, _ = solve_leg(dd, torch, wl2, b2, c2["tol"], max(args.steps, 50), args.warmup, args.launch, "cfg2")
        line["single_rhs"] = dict(workload=c2["desc"], rel_resid=c2["tol"], **sec)
    else:
        wl2 = wl if args.workload == "cfg2" else None
    if not args.no_jacobi_cg:
        log("bench: baseline leg (Jacobi-preconditioned CG on the whole system) ...")
        jcg = jacobi_cg_leg(dd, workloads, wl, b, tol, 3, 1, torch)
        jcg["dd_speedup"] = {k: head[k]["value"] / jcg[k]["value"] for k in ("fp64", "mixed")}
        line["jacobi_cg"] = jcg
    if not args.no_feti:
        log("bench: FETI weak-scaling leg ...")
        t = time.perf_counter()
        line["feti"] = feti_leg(dd, workloads, torch)
        log(f"bench: FETI leg done in {time.perf_counter() - t:.1f} s")
    if not args.no_assembly:
        log("bench: device assembly leg (2D constant kernel, h = 1/128) ...")
        line["assembly"] = assembly_leg(dd, workloads, torch)
        log(f"bench: assembly {line['assembly']['ms']:.2f} ms on the device, "
            f"{line['assembly']['cpu_generator_ms']:.0f} ms for the CPU generator")
    if args.serving_requests > 0:
        log(f"bench: serving leg ({args.serving_requests} requests) ...")
        t = time.perf_counter()
        if wl2 is None:
            wl2 = workloads.build(workloads.spec_2d_const())
        line["serving"] = serving_leg(dd, workloads, wl2, args.serving_requests)
        log(f"bench: serving leg done in {time.perf_counter() - t:.1f} s: {line['serving']}")
    line["cpu_baseline"] = cpu
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
