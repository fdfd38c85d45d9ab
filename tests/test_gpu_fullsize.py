"""GPU parity at the full problem sizes of the benchmark workloads, in the
launch configuration the benchmark times (autotuned schedule), plus edge
cases: zero right-hand sides, the widest batch, interface-free problems.

Gates: FP64 path error <= 1e-10 (tight tolerance); both paths <= 1e-8 at the
benchmark's relative-residual target; the error is relative to the monolithic
FP64 solution computed by the CPU oracle."""
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


@functools.lru_cache(maxsize=None)
def full(name):
    t = time.time()
    spec = workloads.SPECS[name]()
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    print(f"  built {name}: n_dof={wl.dd.n_dof} n_gamma={wl.dd.n_gamma} nrhs={b.shape[1]} "
          f"in {time.time() - t:.1f} s", flush=True)
    return wl, b, uref


def dev(b):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(b).T)).to("cuda").contiguous()


# bench tolerance per workload (the largest residual target meeting 1e-8 error)
BENCH_TOL = {"cfg1": 1e-10, "cfg2": 1e-9, "cfg3": 1e-10, "cfg4": 1e-9}


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3", "cfg4"])
def test_fullsize_fp64_tight(name):
    dd = _dd()
    print(f"case fullsize fp64 {name}", flush=True)
    wl, b, uref = full(name)
    s = dd.Solver(wl.dd, max_nrhs=b.shape[1])
    s.factor(dd.DD_FP64)
    r = s.solve(dev(b), prec=dd.DD_FP64, opts=dd.dd_default_opts(tol=1e-13, max_it=3000))
    err = oracle.rel_err(r.u.cpu().numpy().T, uref)
    print(f"  err max {err.max():.2e} its {[i['iters'] for i in r.info][:8]}", flush=True)
    assert err.max() <= 1e-10
    s.close()


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3", "cfg4"])
@pytest.mark.parametrize("prec", [0, 1])
def test_fullsize_bench_setting(name, prec):
    """The benchmark's setting: both factors formed (the mixed solve of wide
    batches then replaces residuals), autotuned schedule, relative residual
    target of the workload; every solve within 1e-8 of the oracle, in the
    2-norm and entry-wise (largest entry error over the largest entry)."""
    dd = _dd()
    print(f"case fullsize bench {name} prec={prec}", flush=True)
    wl, b, uref = full(name)
    nrhs = b.shape[1]
    s = dd.Solver(wl.dd, max_nrhs=nrhs)
    s.factor(dd.DD_FP64)
    s.factor(prec)
    opts = dd.dd_default_opts(tol=BENCH_TOL[name])
    tuned = s.autotune(prec, nrhs, opts)
    print(f"  tuned {tuned}", flush=True)
    r = s.solve(dev(b), prec=prec, opts=opts)
    u = r.u.cpu().numpy().T
    err = oracle.rel_err(u, uref)
    emax = np.abs(u - uref).max(axis=0) / np.abs(uref).max(axis=0)
    res = oracle.full_residual(wl.asm.A, u, b)
    print(f"  err max {err.max():.2e} entry-wise {emax.max():.2e} resid max {res.max():.2e} "
          f"steps {max(i['refine_steps'] for i in r.info)}", flush=True)
    assert err.max() <= 1e-8
    assert emax.max() <= 1e-8
    assert res.max() <= BENCH_TOL[name] * 1.01
    if prec == dd.DD_MIXED and nrhs >= 8 and tuned["three_launch"] & 4:
        assert max(i["refine_steps"] for i in r.info) == 1      # one Krylov space
    for i, rr in zip(r.info, res):
        assert i["converged"] == 1
        assert abs(i["rel_resid"] - rr) <= 1e-3 * rr + 1e-15
    s.close()


def test_zero_and_duplicate_columns():
    """A zero right-hand side gives u = 0 in zero iterations; identical
    columns give identical solutions."""
    dd = _dd()
    wl, b, uref = full("cfg1")
    B = np.zeros((b.shape[0], 3))
    B[:, 1] = b[:, 0]
    B[:, 2] = b[:, 0]
    s = dd.Solver(wl.dd, max_nrhs=3)
    for prec in (0, 1):
        s.factor(prec)
        r = s.solve(dev(B), prec=prec, opts=dd.dd_default_opts(tol=1e-12))
        u = r.u.cpu().numpy()
        assert np.all(u[0] == 0.0) and r.info[0]["iters"] == 0
        assert np.array_equal(u[1], u[2])
        assert oracle.rel_err(u[1], uref[:, 0]).max() <= 1e-8
    s.close()


def test_widest_batch_64_columns():
    """64 right-hand sides (the largest batch) on a small system, both paths."""
    dd = _dd()
    spec = workloads.spec_2d_const(n=32, cuts=(2, 2), nrhs=64, seed_base=7000)
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    s = dd.Solver(wl.dd, max_nrhs=64)
    for prec, gate in ((0, 1e-10), (1, 1e-8)):
        s.factor(prec)
        r = s.solve(dev(b), prec=prec, opts=dd.dd_default_opts(tol=1e-12))
        err = oracle.rel_err(r.u.cpu().numpy().T, uref)
        assert err.max() <= gate
        # a column alone equals the same column inside the 64-wide batch
        r1 = s.solve(dev(b[:, 37:38]), prec=prec, opts=dd.dd_default_opts(tol=1e-12))
        assert np.array_equal(r1.u.cpu().numpy()[0], r.u.cpu().numpy()[37])
    s.close()


def test_bad_arguments_are_rejected():
    dd = _dd()
    wl, b, _ = full("cfg1")
    s = dd.Solver(wl.dd, max_nrhs=2)
    with pytest.raises(dd.DDError) as ei:             # solve before factor
        s.solve(dev(b))
    assert ei.value.status == dd.DD_ESTATE
    s.factor(dd.DD_FP64)
    bt = dev(np.repeat(b, 3, axis=1))
    with pytest.raises(dd.DDError) as ei:             # more columns than max_nrhs
        s.solve(bt)
    assert ei.value.status == dd.DD_EINVAL
    r = s.solve(dev(b), opts=dd.dd_default_opts(tol=1e-14, max_it=3), raise_on_noconv=False)
    assert r.status == dd.DD_ENOCONV and r.info[0]["converged"] == 0 and r.info[0]["iters"] == 3
    s.close()
