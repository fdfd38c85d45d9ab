"""GPU parity of the paper's baseline solver: CG on the whole system with the
diagonal of A as preconditioner (section "Considered solver strategies").

The library runs it as the undecomposed problem (no subdomains): every dof is
an interface dof, S = K_GG = A and diag(S) = diag(A).  Checked against the
oracle's plain Jacobi-PCG (oracle.jacobi_pcg, which shares no code with the
substructuring oracle) and the monolithic FP64 solution.

Gates: FP64 error <= 1e-10 at a tight tolerance, <= 1e-8 at the benchmark's
relative-residual target; mixed path <= 1e-8; iteration counts within one of
the oracle's (the two sum in different orders); launch modes bit-identical.
"""
import functools
import time

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


CASES = {
    "1d": lambda: workloads.spec_1d(n=256, strips=4, nrhs=2),
    "1d-ragged": lambda: workloads.spec_1d(n=100, delta=0.07, strips=3, nrhs=3),
    "2d-const": lambda: workloads.spec_2d_const(n=32, cuts=(2, 2), nrhs=3),
    "2d-pd": lambda: workloads.spec_2d_pd(n=40, delta=0.1, cuts=(3, 3), jitter=0.2, nrhs=2),
}


@functools.lru_cache(maxsize=None)
def case(name):
    t = time.time()
    spec = workloads.SPECS[name]() if name in workloads.SPECS else CASES[name]()
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    print(f"  built {name}: n_dof={wl.dd.n_dof} nrhs={b.shape[1]} in {time.time() - t:.1f} s",
          flush=True)
    return wl, workloads.undecomposed(wl.asm.A), b, uref


def dev(b):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(b).T)).to("cuda:0").contiguous()


@pytest.mark.parametrize("prec", [0, 1])
def test_undecomposed_preconditioner_is_diag_a(prec):
    """diag(S) of the undecomposed problem is diag(A), bit for bit."""
    dd = _dd()
    wl, und, _, _ = case("2d-const")
    print(f"case jcg diag prec={prec}", flush=True)
    s = dd.Solver(und)
    s.factor(prec)
    assert np.array_equal(s.schur_diag(prec), wl.asm.A.diagonal())
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_jacobi_cg_fp64(name):
    dd = _dd()
    wl, und, b, uref = case(name)
    print(f"case jcg fp64 {name}", flush=True)
    nrhs = b.shape[1]
    s = dd.Solver(und, max_nrhs=nrhs)
    s.factor(dd.DD_FP64)
    res = s.solve(dev(b), prec=dd.DD_FP64, opts=dd.dd_default_opts(tol=1e-13))
    u = res.u.cpu().numpy().T
    x, its, _ = oracle.jacobi_pcg(wl.asm.A, b, tol=1e-13)
    got = np.array([i["iters"] for i in res.info])
    print("  iters", got, its, flush=True)
    assert all(i["converged"] for i in res.info)
    assert np.all(np.abs(got - its) <= 1), (got, its)
    assert oracle.rel_err(u, uref).max() <= 1e-10
    assert oracle.rel_err(u, x).max() <= 1e-10
    s.close()


@pytest.mark.parametrize("name", ["1d", "2d-pd"])
def test_jacobi_cg_mixed(name):
    """FP32 matrix values, FP64 vectors, FP64 residual refinement."""
    dd = _dd()
    wl, und, b, uref = case(name)
    print(f"case jcg mixed {name}", flush=True)
    s = dd.Solver(und, max_nrhs=b.shape[1])
    s.factor(dd.DD_MIXED)
    res = s.solve(dev(b), prec=dd.DD_MIXED, opts=dd.dd_default_opts(tol=1e-12))
    err = oracle.rel_err(res.u.cpu().numpy().T, uref)
    print("  err", err, res.info, flush=True)
    assert err.max() <= 1e-8
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_jacobi_cg_launch_modes_bit_identical(prec):
    """Stream launches, the persistent cooperative kernel and graph replays
    give the same bits on the undecomposed problem."""
    dd = _dd()
    wl, und, b, _ = case("1d-ragged")
    print(f"case jcg launch modes prec={prec}", flush=True)
    s = dd.Solver(und, max_nrhs=b.shape[1])
    s.factor(prec)
    o1 = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_KERNELS)
    r1 = s.solve(dev(b), prec=prec, opts=o1)
    for mode, extra in ((dd.DD_LAUNCH_PERSISTENT, {}), (dd.DD_LAUNCH_GRAPH, dict(check_every=4))):
        r2 = s.solve(dev(b), prec=prec, opts=dd.dd_default_opts(tol=1e-12, launch=mode, **extra))
        assert [i["iters"] for i in r1.info] == [i["iters"] for i in r2.info], mode
        assert np.array_equal(r1.u.cpu().numpy(), r2.u.cpu().numpy()), mode
    s.close()


def test_jacobi_cg_batch_api():
    """Continuous batching on the undecomposed problem gives dd_solve's bits."""
    dd = _dd()
    wl, und, b, uref = case("2d-const")
    print("case jcg batch api", flush=True)
    n = b.shape[0]
    s = dd.Solver(und, max_nrhs=4)
    s.factor(dd.DD_FP64)
    opts = dd.dd_default_opts(tol=1e-11)
    ref = s.solve(dev(b), prec=dd.DD_FP64, opts=opts).u.cpu().numpy()
    dd.dd_batch_begin(s.ctx, dd.DD_FP64, opts)
    dd.dd_batch_admit(s.ctx, [0, 3], dev(b[:, :2]), n)
    dd.dd_batch_admit(s.ctx, [1], dev(b[:, 2:3]), n)
    done = {}
    for _ in range(1000):
        st = dd.dd_batch_step(s.ctx, 4, 64)
        for slot, col in ((0, 0), (3, 1), (1, 2)):
            if col not in done and st[slot] == dd.DD_SLOT_DONE:
                u = torch.empty((1, n), dtype=torch.float64, device="cuda:0")
                info = dd.dd_batch_retire(s.ctx, [slot], u, n)
                done[col] = (u.cpu().numpy()[0], info[0])
        if len(done) == 3:
            break
    dd.dd_batch_end(s.ctx)
    assert len(done) == 3
    for col, (u, info) in done.items():
        assert info["converged"] == 1
        assert np.array_equal(u, ref[col]), col
        assert oracle.rel_err(u, uref[:, col]).max() <= 1e-10
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_jacobi_cg_fullsize_bench_setting(prec):
    """The benchmark system (2D constant kernel, h = 1/128, 16 129 dofs) at
    the benchmark's relative residual 1e-9 in the autotuned schedule: error
    <= 1e-8; FP64 iterations within one of the oracle's."""
    dd = _dd()
    wl, und, b, uref = case("cfg2")
    print(f"case jcg fullsize prec={prec}", flush=True)
    s = dd.Solver(und, max_nrhs=b.shape[1])
    s.factor(prec)
    opts = dd.dd_default_opts(tol=1e-9)
    s.autotune(prec, b.shape[1], opts)
    res = s.solve(dev(b), prec=prec, opts=opts)
    err = oracle.rel_err(res.u.cpu().numpy().T, uref)
    print("  err", err, res.info, flush=True)
    assert err.max() <= 1e-8
    if prec == dd.DD_FP64:
        _, its, _ = oracle.jacobi_pcg(wl.asm.A, b, tol=1e-9)
        assert abs(res.info[0]["iters"] - its[0]) <= 1, (res.info, its)
        tight = s.solve(dev(b), prec=prec, opts=dd.dd_default_opts(tol=1e-12))
        assert oracle.rel_err(tight.u.cpu().numpy().T, uref).max() <= 1e-10
    s.close()
