"""GPU tests of continuous batching: the batch API against dd_solve, and the
serving loop's results alone vs in a mix (bitwise) and against the oracle."""
import functools

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dd():
    import paper_2306_00094_amd as dd
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dd.load_library()
    return dd


@functools.lru_cache(maxsize=None)
def system(name):
    spec = {
        "1d": workloads.spec_1d(n=256, strips=4, nrhs=4, seed_base=1100),
        "2d": workloads.spec_2d_const(n=32, cuts=(2, 2), nrhs=4, seed_base=2100),
        "frac": workloads.spec_2d_frac(n=28, delta=0.15, cuts=(2, 2), nrhs=4, seed_base=3100),
    }[name]
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    return wl, b, oracle.monolithic_solve(wl.asm.A, b)


def dev(b):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(b).T)).to("cuda").contiguous()


def run_batch(dd, s, b, schedule, prec, opts):
    """Admit columns of b at the given step numbers into the given slots."""
    n = b.shape[0]
    dd.dd_batch_begin(s.ctx, prec, opts)
    out = {}
    pending = list(schedule)
    step = 0
    running = {}
    while pending or running:
        for (when, col, slot) in [p for p in pending if p[0] <= step and p[2] not in running]:
            dd.dd_batch_admit(s.ctx, [slot], dev(b[:, col:col + 1]), n)
            running[slot] = col
            pending.remove((when, col, slot))
        st = dd.dd_batch_step(s.ctx, 3, 64)
        for slot, col in list(running.items()):
            if st[slot] in (dd.DD_SLOT_DONE, dd.DD_SLOT_FALLBACK):
                u = torch.empty((1, n), dtype=torch.float64, device="cuda")
                info = dd.dd_batch_retire(s.ctx, [slot], u, n)
                out[col] = (u.cpu().numpy()[0], info[0])
                del running[slot]
        step += 1
        assert step < 2000
    dd.dd_batch_end(s.ctx)
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_api_matches_dd_solve(prec, monkeypatch):
    """The batch API runs the four-launch CG iteration; dd_solve forced to the
    same iteration gives the same bits."""
    dd = _dd()
    wl, b, uref = system("2d")
    print(f"case batch api prec={prec}", flush=True)
    monkeypatch.setenv("DD_CLASSIC_CG", "1")
    s = dd.Solver(wl.dd, max_nrhs=64)
    s.factor(prec)
    opts = dd.dd_default_opts(tol=1e-11)
    ref = s.solve(dev(b), prec=prec, opts=opts).u.cpu().numpy()
    # staggered admissions, a slot that forces a wider batch, reuse of a slot
    out = run_batch(dd, s, b, [(0, 0, 0), (2, 1, 9), (3, 2, 2), (5, 3, 0)], prec, opts)
    for col in range(b.shape[1]):
        u, info = out[col]
        assert info["converged"] == 1
        assert np.array_equal(u, ref[col]), col
        assert oracle.rel_err(u, uref[:, col]).max() <= (1e-10 if prec == 0 else 1e-8)
    s.close()


def test_batch_api_fp32_gathers_match_dd_solve(monkeypatch):
    """Mixed batches with FP32 gathers keep the direction in memory (its own
    kernel) and gather FP32 copies of it and of w; dd_solve forced to the
    same four-launch iteration gives the same bits, and every column meets
    the FP64 tolerance."""
    dd = _dd()
    wl, b, uref = system("2d")
    print("case batch api fp32 gathers", flush=True)
    monkeypatch.setenv("DD_CLASSIC_CG", "1")
    monkeypatch.setenv("DD_DIRECTION_KERNEL", "1")
    s = dd.Solver(wl.dd, max_nrhs=64)
    s.factor(dd.DD_MIXED)
    opts = dd.dd_default_opts(tol=1e-11, gather32=1)
    ref = s.solve(dev(b), prec=dd.DD_MIXED, opts=opts).u.cpu().numpy()
    plain = s.solve(dev(b), prec=dd.DD_MIXED, opts=dd.dd_default_opts(tol=1e-11, gather32=0))
    assert not np.array_equal(ref, plain.u.cpu().numpy())       # the option took effect
    out = run_batch(dd, s, b, [(0, 0, 0), (2, 1, 9), (3, 2, 2), (5, 3, 0)], dd.DD_MIXED, opts)
    for col in range(b.shape[1]):
        u, info = out[col]
        assert info["converged"] == 1
        assert np.array_equal(u, ref[col]), col
        assert oracle.rel_err(u, uref[:, col]).max() <= 1e-8
    s.close()


def test_batch_rejects_solve_while_open():
    dd = _dd()
    wl, b, _ = system("1d")
    s = dd.Solver(wl.dd, max_nrhs=4)
    s.factor(dd.DD_FP64)
    dd.dd_batch_begin(s.ctx, dd.DD_FP64)
    with pytest.raises(dd.DDError) as ei:
        s.solve(dev(b[:, :1]))
    assert ei.value.status == dd.DD_ESTATE
    dd.dd_batch_end(s.ctx)
    s.close()


def test_serving_mix_alone_equal_and_correct():
    """Requests over three systems with Poisson arrivals and an HBM budget that
    forces evictions: every result matches the oracle, and equals, bit for
    bit, the same request served alone on a fresh context."""
    dd = _dd()
    from paper_2306_00094_amd import serving
    names = ["1d", "2d", "frac"]
    systems = {k: system(k)[0].dd for k in names}
    opts = dd.dd_default_opts(tol=1e-11, gather32=1)      # the serving default
    fps = {k: dd.dd_footprint(v, dd.DD_MIXED, 64) for k, v in systems.items()}
    budget = max(fps.values()) * 2           # at most two systems resident
    rng = np.random.default_rng(5)
    arrivals = serving.poisson_arrivals(18, rate=400.0, seed=5)
    reqs = []
    for i, t in enumerate(arrivals):
        k = names[int(rng.integers(0, 3))]
        b = system(k)[1]
        cols = rng.choice(b.shape[1], size=int(rng.integers(1, 4)), replace=False)
        reqs.append(serving.Request(key=k, b=np.asfortranarray(b[:, cols]), arrival=float(t), rid=i))
    print("case serving mix", flush=True)
    srv = serving.Server(systems, prec=dd.DD_MIXED, opts=opts, hbm_budget=budget, iters_per_step=3)
    done = srv.run(reqs, timeout=300)
    assert len(done) == len(reqs)
    stats = serving.summarize(done)
    print("  stats", stats, "evictions", srv.evictions, flush=True)
    for r in done:
        wl, b, uref = system(r.key)
        u_ref = oracle.monolithic_solve(wl.asm.A, r.b)
        assert oracle.rel_err(r.u, u_ref).max() <= 1e-8
    # alone: each request on a fresh context, nothing else in the batch
    for r in done[:6]:
        srv1 = serving.Server({r.key: systems[r.key]}, prec=dd.DD_MIXED, opts=opts, iters_per_step=3)
        alone = serving.Request(key=r.key, b=r.b, arrival=0.0, rid=0)
        d1 = srv1.run([alone], timeout=120)
        assert np.array_equal(d1[0].u, r.u), r.rid


def test_serving_keeps_systems_resident_between_runs():
    """With keep_resident the factors and contexts survive a run: a second run
    reuses the same resident system (no refactorisation) and returns the same
    result, bit for bit, for the same request."""
    dd = _dd()
    from paper_2306_00094_amd import serving
    wl, b, uref = system("2d")
    opts = dd.dd_default_opts(tol=1e-11)
    srv = serving.Server({"2d": wl.dd}, prec=dd.DD_MIXED, opts=opts, iters_per_step=3)
    print("case serving keep_resident", flush=True)
    try:
        r1 = srv.run([serving.Request(key="2d", b=np.asfortranarray(b[:, :2]), rid=0)],
                     timeout=120, keep_resident=True)
        first = srv.resident["2d"]
        r2 = srv.run([serving.Request(key="2d", b=np.asfortranarray(b[:, :2]), rid=1)],
                     timeout=120, keep_resident=True)
        assert srv.resident["2d"] is first
        assert len(r1) == 1 and len(r2) == 1
        assert np.array_equal(r1[0].u, r2[0].u)
        assert oracle.rel_err(r2[0].u, uref[:, :2]).max() <= 1e-8
    finally:
        srv.shutdown()
