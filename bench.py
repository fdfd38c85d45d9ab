#!/usr/bin/env python3
"""Throughput benchmark of the substructuring Schur-complement solver on one MI355X.

One step = one full solve of the hot path on the workload's batch of
right-hand sides: condensation, preconditioned CG on the interface Schur
complement to the tolerance, back substitution, FP64 residual check (and, in
mixed precision, the refinement loop).  The subdomain factorisation is done
once before timing (setup, excluded as in the paper's solve timings).

Default workload: 2D nonlocal diffusion on the unit square, constant kernel
4/(pi delta^4) on the Euclidean ball (barycentre pair truncation), delta = 0.1,
P1 on a structured right-triangle mesh h = 1/128 (16 129 free dofs), 4x4
subdomains, one seeded right-hand side per solve, relative residual 1e-9.

Prints ONE JSON line.  `value` is the mixed-precision path's solves/s; the
FP64 path is reported beside it under "fp64".
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
# (checked by the GPU parity tests at this tolerance).
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


# Bytes moved beyond L2 per dispatch of the interface-row kernel, from two
# rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE) of this benchmark on the
# default workload, each scaled by what the counter read for an elementwise
# kernel of known traffic (FETCH x2.000, WRITE x1.000): 256 MiB read and written
# read as about 131085 KiB fetched and 262148 KiB written.  Valid only for the
# kernel source they were taken on (sha256 prefix of csrc/dd_kernels.h);
# reported as null once that source changes.
MEASURED_TRAFFIC = {
    "src_sha256": "c0c496399d23931e",
    "workload": "cfg2",
    # median over the launches of the CG iterations (full [K_GG | K_GI] sweep)
    "k_gamma_rows<float>": dict(fetch_kib=23326.8, write_kib=221.8),
    "k_gamma_rows<double>": dict(fetch_kib=34253.9, write_kib=221.8),
    "fetch_scale": 262144.0 / 131085.4,
    "write_scale": 262144.0 / 262149.4,
}


def measured_traffic(kernel: str, workload: str):
    import hashlib
    src = os.path.join(ROOT, "paper_2306_00094_amd", "csrc", "dd_kernels.h")
    try:
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    m = MEASURED_TRAFFIC
    if sha != m["src_sha256"] or workload != m["workload"] or kernel not in m:
        return None
    k = m[kernel]
    return 1024.0 * (k["fetch_kib"] * m["fetch_scale"] + k["write_kib"] * m["write_scale"])


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
    """Arithmetic of one factorisation of every interior block (MFMA work):
    Cholesky n^3/3, X = L^-1 n^3/3, K^-1 = X^T X n^3/3 flops per subdomain."""
    return float(sum(3 * (k.shape[0] ** 3) / 3.0 for k in dd.kii))


# The kernel timing of the roofline is taken on every TIMING_EVERY-th solve of
# the timed region: an event pair recorded by a launch costs about 5 us of
# stream time, which on every launch would slow the timed solves by ~10%.
TIMING_EVERY = 4


def time_path(solver, dd, b, prec, opts, steps, warmup, torch):
    for _ in range(warmup):
        solver.solve(b, prec=prec, opts=opts)
    torch.cuda.synchronize()
    lat = []
    infos = None
    mask = (1 << dd.DD_PHASE_GAMMA) | (1 << dd.DD_PHASE_LOOP)
    dd.dd_set_timing(solver.ctx, 0, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        if i % TIMING_EVERY == 0:
            dd.dd_set_timing(solver.ctx, mask, reset=False)
        res = solver.solve(b, prec=prec, opts=opts)       # returns when complete
        if i % TIMING_EVERY == 0:
            dd.dd_set_timing(solver.ctx, 0, reset=False)
        lat.append(time.perf_counter() - ts)
        infos = res.info
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, n = dd.dd_get_timing(solver.ctx)
    dd.dd_set_timing(solver.ctx, 0)
    return dict(seconds=t1 - t0, lat=lat, info=infos,
                gamma_ms=ms[dd.DD_PHASE_GAMMA], gamma_launches=n[dd.DD_PHASE_GAMMA],
                loop_ms=ms[dd.DD_PHASE_LOOP], loop_launches=n[dd.DD_PHASE_LOOP])


def pct(v, q):
    v = sorted(v)
    k = max(0, min(len(v) - 1, int(math.ceil(q * len(v))) - 1))
    return v[k]


def cpu_baseline(wl, b, tol, budget_s):
    """The CPU FP64 oracle's substructuring solve on the same system, timed on
    the host (BLAS limited to one thread; the oracle's sparse products are
    single-threaded).  A bounded sample of whole solves (setup excluded)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    with threadpool_limits(limits=1):
        orc = oracle.DDOracle(wl.dd)
        orc.schur_diag()
        col = b[:, :1]
        n = 0
        t0 = time.perf_counter()
        while True:
            orc.solve(col, tol=tol)
            n += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"{n} full oracle solves (1 rhs each, tol {tol:g}) of the same system, "
                       f"{dt:.1f} s", threads_available=os.cpu_count())


def serving_leg(dd, workloads, wl_main, nreq: int, seed: int = 5000, gather32: int = 1,
                chunk: int = 1000):
    """Continuous-batching serving run (paper_2306_00094_amd.serving) over
    six resident systems: the 1D constant kernel at h = 1/1024 and 1/2048,
    the 2D constant kernel at h = 1/64 and 1/128 (the benchmark system), and
    the 2D fractional kernel at h = 1/48 and 1/96 (mesh sizes x0.5 to x2 of
    the three base systems).  Requests carry 1-64 seeded right-hand sides.  First all requests arrive at once (saturated
    throughput), then Poisson arrivals at 0.8x that request rate (latency
    under load); more than `chunk` requests run as consecutive chunks of
    that many.  Mixed precision, with FP32 gathers unless gather32 = 0."""
    import numpy as np
    from paper_2306_00094_amd import serving
    specs = {
        "1d-const h=1/1024": workloads.spec_1d(),
        "1d-const h=1/2048": workloads.spec_1d(n=2048),
        "2d-const h=1/64": workloads.scaled(workloads.spec_2d_const, 0.5),
        "2d-frac h=1/48": workloads.scaled(workloads.spec_2d_frac, 0.5),
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
    def phase(name, arrivals):
        done, secs = [], 0.0
        for c0 in range(0, nreq, chunk):
            n = min(chunk, nreq - c0)
            t0 = time.perf_counter()
            d = srv.run(requests(arrivals(n, c0), c0), timeout=600, keep_resident=True)
            wall = time.perf_counter() - t0
            secs += wall if name == "saturated" else serving.summarize(d)["seconds"]
            done += d
            if nreq > chunk:
                log(f"bench: serving {name}: {c0 + n}/{nreq} requests, {secs:.1f} s")
        return serving.summarize(done, wall=secs)

    opts = dd.dd_default_opts(tol=1e-9, gather32=gather32)
    srv = serving.Server(systems, prec=dd.DD_MIXED, opts=opts, iters_per_step=4)
    try:
        # every system resident (factors formed) before anything is timed
        srv.run(requests(np.zeros(len(keys) * 2)), timeout=300, keep_resident=True)
        burst = phase("saturated", lambda n, c0: np.zeros(n))
        rate = 0.8 * burst["requests"] / burst["seconds"]
        load = phase("load", lambda n, c0: serving.poisson_arrivals(n, rate=rate, seed=seed + 1 + c0))
    finally:
        srv.shutdown()
    return dict(systems=keys, requests=nreq, rhs_per_request="1-64", rel_resid=1e-9, precision="mixed",
                fp32_gathers=bool(gather32),
                saturated_solves_per_s=burst["solves_per_s"], saturated_p50_ms=burst["p50_ms"],
                saturated_p99_ms=burst["p99_ms"], offered_requests_per_s=rate,
                solves_per_s=load["solves_per_s"], p50_ms=load["p50_ms"], p99_ms=load["p99_ms"],
                fallbacks=load["fallbacks"] + burst["fallbacks"])


def wide_batch_leg(dd, workloads, torch, steps=3, warmup=1):
    """Mixed against plain FP64 on a wide batch: the 2D bond-based peridynamic
    system (h = 1/160, 50 562 dofs, 8x8 jittered subdomains) with its 32
    seeded right-hand sides in one batch, each path autotuned for that width
    (the mixed path may choose FP32 gathers), at relative residual 1e-9.
    Reports the time per batch, solves/s (32 per batch), iterations and the
    largest true relative residual of each path."""
    import numpy as np
    cfg = WORKLOADS["cfg4"]
    spec = getattr(workloads, cfg["spec"])()
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    nrhs = b.shape[1]
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda:0").contiguous()
    s = dd.Solver(wl.dd, max_nrhs=nrhs)
    out = dict(workload=cfg["desc"], nrhs=nrhs, rel_resid=cfg["tol"])
    try:
        for name, prec in (("fp64", dd.DD_FP64), ("mixed", dd.DD_MIXED)):
            s.factor(prec)
            opts = dd.dd_default_opts(tol=cfg["tol"])
            tuned = s.autotune(prec, nrhs, opts)
            r = time_path(s, dd, bt, prec, opts, steps, warmup, torch)
            out[name] = dict(ms_per_batch=1e3 * r["seconds"] / steps,
                             solves_per_s=steps * nrhs / r["seconds"],
                             iters_max=max(i["iters"] for i in r["info"]),
                             rel_resid_max=max(i["rel_resid"] for i in r["info"]),
                             schedule=tuned)
            log(f"bench: wide batch prec={prec} {out[name]['ms_per_batch']:.1f} ms/batch "
                f"its={out[name]['iters_max']} schedule={tuned}")
    finally:
        s.close()
    out["mixed_vs_fp64"] = out["mixed"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    return out


# FP64 vector peak (256 CUs at 2.4 GHz) for the ALU-bound assembly kernel
FP64_VECTOR_PEAK_TFLOPS = 78.6
# FP64 operations per quadrature-point pair of the constant kernel (whose
# value does not depend on the points): d_m (1 sub), the weight times the
# kernel value times d_m (5 mul), and per vertex of the pair (6) d_n (1 sub)
# and the accumulation (1 fma: 2)
ASM_FLOPS_PER_QP = 24


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


def jacobi_cg_leg(dd, workloads, wl, bt, b, tol, steps, warmup, torch, cpu_seconds):
    """The paper's baseline solver on the same system: CG on the whole matrix
    with diag(A) as preconditioner (section "Considered solver strategies"),
    run by the library as the undecomposed problem (no subdomains, S = A).
    Same tolerance, right-hand side, launch autotuning and timing as the
    substructuring solve; its dominant kernel is the CSR sweep of A."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    und = workloads.undecomposed(wl.asm.A)
    nrhs = b.shape[1]
    ld = 1
    while ld < nrhs:
        ld *= 2
    s = dd.Solver(und, max_nrhs=nrhs)
    out = {}
    try:
        for name, prec in (("fp64", dd.DD_FP64), ("mixed", dd.DD_MIXED)):
            s.factor(prec)
            opts = dd.dd_default_opts(tol=tol)
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
            elif r["loop_launches"] > 0:
                # graph replay: whole iterations per launch (sweep + update + direction passes)
                its = sum(i["iters"] for i in r["info"]) / max(1, len(r["info"]))
                sampled = (steps + TIMING_EVERY - 1) // TIMING_EVERY
                per_it = sweep + 8.0 * ld * und.n_gamma * (7 + (3 if tuned.get("direction_kernel") else 0))
                algo = per_it * its / max(1, r["loop_launches"] / sampled)
                avg = r["loop_ms"] / r["loop_launches"] * 1e-3
                ach = algo / avg / 1e9
                roof = dict(bound="hbm", kernel="CG loop launch (graph replay)", achieved=ach, peak=HBM_PEAK_GBS,
                            unit="GB/s", frac=ach / HBM_PEAK_GBS, algo_bytes_per_launch=algo,
                            avg_launch_us=1e6 * avg, launches=r["loop_launches"])
            out[name] = dict(value=steps * nrhs / r["seconds"], ms_per_step=1e3 * r["seconds"] / steps,
                             p50_ms=1e3 * statistics.median(r["lat"]), p99_ms=1e3 * pct(r["lat"], 0.99),
                             iters=[i["iters"] for i in r["info"]],
                             rel_resid_max=max(i["rel_resid"] for i in r["info"]),
                             schedule=tuned, roofline=roof)
            log(f"bench: jacobi-cg prec={prec} {out[name]['ms_per_step']:.3f} ms/step its={out[name]['iters'][:4]}")
    finally:
        s.close()
    import oracle
    with threadpool_limits(limits=1):
        n = 0
        t0 = time.perf_counter()
        while True:
            oracle.jacobi_pcg(wl.asm.A, b[:, :1], tol=tol)
            n += 1
            if time.perf_counter() - t0 >= cpu_seconds:
                break
        dt = time.perf_counter() - t0
    out["cpu_oracle"] = dict(value=n / dt, unit="solves/s", cores=1, kind="oracle",
                             sample=f"{n} oracle Jacobi-PCG solves (1 rhs, tol {tol:g}), {dt:.1f} s")
    out["nnz"] = int(wl.asm.A.nnz)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="requests of the serving leg (0 = skip it)")
    ap.add_argument("--no-wide-batch", action="store_true",
                    help="skip the mixed-vs-FP64 leg on the 32-column peridynamic batch")
    ap.add_argument("--no-assembly", action="store_true",
                    help="skip the device-assembly leg")
    ap.add_argument("--no-jacobi-cg", action="store_true",
                    help="skip the baseline leg (Jacobi-preconditioned CG on the whole system)")
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

    import numpy as np
    import torch

    import paper_2306_00094_amd as dd
    import workloads

    dd.load_library()
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)         # one elementwise kernel: reads and writes MB each
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {args.calibrate_copy} MB done")
        del src, dst
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
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda:0").contiguous()
    solver = dd.Solver(wl.dd, max_nrhs=nrhs)
    fac = {}
    for prec in (dd.DD_FP64, dd.DD_MIXED):
        solver.factor(prec)                       # first call: allocations, code loading
        reps = []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            solver.factor(prec)
            torch.cuda.synchronize()
            reps.append(time.perf_counter() - t)
        fac[prec] = min(reps)
    log(f"bench: factor fp64 {1e3 * fac[0]:.2f} ms, fp32 {1e3 * fac[1]:.2f} ms")

    tuned = {}
    if args.launch == "auto":
        opts = dd.dd_default_opts(tol=tol)
        for prec in (dd.DD_FP64, dd.DD_MIXED):
            tuned[prec] = solver.autotune(prec, nrhs, opts)      # schedule used by AUTO solves
            log(f"bench: autotuned prec={prec}: {tuned[prec]}")
    else:
        mode = {"kernels": dd.DD_LAUNCH_KERNELS, "graph": dd.DD_LAUNCH_GRAPH,
                "persistent": dd.DD_LAUNCH_PERSISTENT}[args.launch]
        opts = dd.dd_default_opts(tol=tol, launch=mode, apply=dd.DD_APPLY_INV)
        for prec in (dd.DD_FP64, dd.DD_MIXED):
            tuned[prec] = dict(apply=dd.DD_APPLY_INV, launch=mode, fixed=True)
    res = {}
    for prec in (dd.DD_FP64, dd.DD_MIXED):
        r = time_path(solver, dd, bt, prec, opts, args.steps, args.warmup, torch)
        res[prec] = r
        log(f"bench: prec={prec} {1e3 * r['seconds'] / args.steps:.3f} ms/step "
            f"its={[i['iters'] for i in r['info']][:4]} resid={max(i['rel_resid'] for i in r['info']):.2e}")

    ld = 1
    while ld < nrhs:
        ld *= 2

    def summary(prec):
        r = res[prec]
        solves = args.steps * nrhs
        out = dict(value=solves / r["seconds"], ms_per_step=1e3 * r["seconds"] / args.steps,
                   p50_ms=1e3 * statistics.median(r["lat"]), p99_ms=1e3 * pct(r["lat"], 0.99),
                   iters=[i["iters"] for i in r["info"]],
                   refine_steps=[i["refine_steps"] for i in r["info"]],
                   used_fallback=[i["used_fallback"] for i in r["info"]],
                   rel_resid_max=max(i["rel_resid"] for i in r["info"]),
                   factor_ms=1e3 * fac[prec], schedule=tuned[prec])
        return out

    mixed = summary(dd.DD_MIXED)
    fp64 = summary(dd.DD_FP64)

    # roofline of the dominant kernel (interface rows) on the reported path
    def roof(prec):
        r = res[prec]
        vb = 8 if prec == dd.DD_FP64 else 4
        if r["gamma_launches"] > 0:
            avg = r["gamma_ms"] / r["gamma_launches"] * 1e-3
            algo = gamma_kernel_bytes(wl.dd, ld, vb)
            kname = "k_gamma_rows<%s> (q = K_GG p - K_GI w)" % ("double" if vb == 8 else "float")
            launches = r["gamma_launches"]
            traffic = measured_traffic("k_gamma_rows<%s>" % ("double" if vb == 8 else "float"),
                                       args.workload)
        else:          # graph replay / persistent launch: whole CG iterations per launch
            avg = r["loop_ms"] / max(1, r["loop_launches"]) * 1e-3
            its = sum(i["iters"] for i in r["info"]) / max(1, len(r["info"]))
            per_it = iteration_bytes(wl.dd, ld, vb)
            sampled = (args.steps + TIMING_EVERY - 1) // TIMING_EVERY    # solves with timing on
            algo = per_it * its / max(1, r["loop_launches"] / sampled)
            kname = "CG loop launch (%s)" % r["info"]
            launches = r["loop_launches"]
            traffic = None
        ach = algo / avg / 1e9 if avg > 0 else 0.0
        return dict(bound="hbm", kernel=kname, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=traffic, algo_bytes_per_launch=algo,
                    avg_launch_us=1e6 * avg, launches=launches,
                    timed_solves=f"every {TIMING_EVERY}th solve of the timed region")

    roof_mixed = roof(dd.DD_MIXED)
    roof_fp64 = roof(dd.DD_FP64)

    line = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "name": args.workload, "rel_resid": tol,
                   "nrhs": nrhs, "n_dof": wl.dd.n_dof, "n_gamma": wl.dd.n_gamma,
                   "subdomains": wl.dd.n_sub},
        "p50_ms": mixed["p50_ms"],
        "p99_ms": mixed["p99_ms"],
        "mixed": mixed,
        "fp64": fp64,
        "mixed_vs_fp64": mixed["value"] / fp64["value"],
        "roofline": dict(roof_mixed, fp64=roof_fp64),
        "factor": {
            name: dict(ms=1e3 * fac[prec], gflop=factor_flops(wl.dd) / 1e9,
                       achieved_tflops=factor_flops(wl.dd) / fac[prec] / 1e12, bound="mfma",
                       peak_tflops=MFMA_PEAK_TFLOPS[name],
                       frac=factor_flops(wl.dd) / fac[prec] / 1e12 / MFMA_PEAK_TFLOPS[name],
                       note="whole factorisation (Cholesky, L^-1, K^-1, diag(S)) timed on the host")
            for name, prec in (("f64", dd.DD_FP64), ("f32", dd.DD_MIXED))},
        "paper_context": "14.6x FETI vs Jacobi-CG solve time, fractional kernel, 48x48 subdomains, "
                         "16M dofs, 2304 Broadwell ranks (different method and machine)",
    }
    if not args.no_assembly:
        log("bench: device assembly leg (2D constant kernel, h = 1/128) ...")
        line["assembly"] = assembly_leg(dd, workloads, torch)
        log(f"bench: assembly {line['assembly']['ms']:.2f} ms on the device, "
            f"{line['assembly']['cpu_generator_ms']:.0f} ms for the CPU generator")
    if not args.no_jacobi_cg:
        log("bench: baseline leg (Jacobi-preconditioned CG on the whole system) ...")
        jcg = jacobi_cg_leg(dd, workloads, wl, bt, b, tol, args.steps, args.warmup, torch,
                            min(5.0, args.cpu_seconds))
        jcg["dd_speedup"] = {k: res_v / jcg[k]["value"]
                             for k, res_v in (("fp64", fp64["value"]), ("mixed", mixed["value"]))}
        line["jacobi_cg"] = jcg
    if not args.no_wide_batch:
        log("bench: wide-batch leg (peridynamic system, 32 right-hand sides) ...")
        t = time.perf_counter()
        line["wide_batch"] = wide_batch_leg(dd, workloads, torch)
        log(f"bench: wide-batch leg done in {time.perf_counter() - t:.1f} s")
    if args.serving_requests > 0:
        log(f"bench: serving leg ({args.serving_requests} requests) ...")
        t = time.perf_counter()
        line["serving"] = serving_leg(dd, workloads, wl, args.serving_requests)
        log(f"bench: serving leg done in {time.perf_counter() - t:.1f} s: {line['serving']}")
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle baseline (~{args.cpu_seconds:.0f} s) ...")
        line["cpu_baseline"] = cpu_baseline(wl, b, tol, args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    solver.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
