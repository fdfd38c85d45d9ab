"""GPU parity of the mixed-precision solve with residual replacement on the
tiled wide-batch path: the directions take S p with the FP32 operators, while
condensation, back substitution and, every `reliable` iterations, the
interface residual g - S x come from the FP64 operators (both factors
formed).  One Krylov space replaces the restarts of iterative refinement.

Gates: error <= 1e-8 relative to the monolithic FP64 solution (the mixed
path's bar) and element-wise; one outer step (no restart) for every column;
iteration counts within a few of the FP64 path's on the same batch; stream
and graph launches bitwise equal; a column's result the same alone and in
a wider batch within the tolerance."""
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


CASES = {
    "2d-const": lambda: workloads.spec_2d_const(n=40, cuts=(3, 2), nrhs=40, seed_base=2100),
    "2d-pd": lambda: workloads.spec_2d_pd(n=40, delta=0.1, cuts=(3, 3), jitter=0.2, nrhs=40,
                                          seed_base=4100),
    "2d-frac": lambda: workloads.spec_2d_frac(n=32, cuts=(2, 2), nrhs=40, seed_base=3100),
}


@functools.lru_cache(maxsize=None)
def problem(name):
    spec = CASES[name]()
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    return wl, b, uref


def dev(b):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(b).T)).to("cuda:0").contiguous()


def solver_both(dd, wl, max_nrhs=64):
    s = dd.Solver(wl.dd, max_nrhs=max_nrhs)
    s.factor(dd.DD_FP64)
    s.factor(dd.DD_MIXED)
    return s


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nrhs", [8, 13, 32, 40])
@pytest.mark.parametrize("period", [-1, 1, 7])
def test_replacement_parity(name, nrhs, period):
    dd = _dd()
    wl, b, uref = problem(name)
    print(f"case replacement {name} nrhs={nrhs} period={period}", flush=True)
    s = solver_both(dd, wl)
    tol = 1e-11
    o64 = dd.dd_default_opts(tol=tol, tiles=1, launch=dd.DD_LAUNCH_KERNELS)
    omx = dd.dd_default_opts(tol=tol, tiles=1, launch=dd.DD_LAUNCH_KERNELS, reliable=period)
    r64 = s.solve(dev(b[:, :nrhs]), prec=dd.DD_FP64, opts=o64)
    rmx = s.solve(dev(b[:, :nrhs]), prec=dd.DD_MIXED, opts=omx)
    u = rmx.u.cpu().numpy().T
    err = oracle.rel_err(u, uref[:, :nrhs])
    emax = np.abs(u - uref[:, :nrhs]).max(axis=0) / np.abs(uref[:, :nrhs]).max(axis=0)
    its64 = [i["iters"] for i in r64.info]
    itsmx = [i["iters"] for i in rmx.info]
    print(f"  err max {err.max():.2e} its fp64 {its64[:4]} mixed {itsmx[:4]}", flush=True)
    assert err.max() <= 1e-8
    assert emax.max() <= 1e-8
    for j in range(nrhs):
        info = rmx.info[j]
        assert info["converged"] == 1 and info["used_fallback"] == 0, (j, info)
        assert info["refine_steps"] == 1, (j, info)          # one Krylov space, no restart
        assert info["rel_resid"] <= tol, (j, info)           # the FP64 residual of dd_solve's check
        # (FP32 directions cost a few iterations on the dense fractional blocks)
        assert itsmx[j] <= its64[j] + 3 + its64[j] // 4, (j, itsmx[j], its64[j])
    s.close()


def test_replacement_needs_fp64_factor():
    """Without the FP64 factor the mixed solve refines as before (restarts),
    and still meets the gate."""
    dd = _dd()
    wl, b, uref = problem("2d-pd")
    s = dd.Solver(wl.dd, max_nrhs=32)
    s.factor(dd.DD_MIXED)
    r = s.solve(dev(b[:, :16]), prec=dd.DD_MIXED,
                opts=dd.dd_default_opts(tol=1e-11, tiles=1, reliable=-1))
    assert oracle.rel_err(r.u.cpu().numpy().T, uref[:, :16]).max() <= 1e-8
    assert max(i["refine_steps"] for i in r.info) >= 2
    s.close()


def test_replacement_graph_matches_kernels():
    """Graph replays (4 iterations each, every second one ending with the
    replacement) equal the stream launches replacing every 8th iteration."""
    dd = _dd()
    wl, b, _ = problem("2d-pd")
    s = solver_both(dd, wl, max_nrhs=32)
    o1 = dd.dd_default_opts(tol=1e-11, tiles=1, launch=dd.DD_LAUNCH_KERNELS, reliable=8)
    o2 = dd.dd_default_opts(tol=1e-11, tiles=1, launch=dd.DD_LAUNCH_GRAPH, check_every=4, reliable=8)
    u1 = s.solve(dev(b[:, :16]), prec=dd.DD_MIXED, opts=o1).u.cpu().numpy()
    for _ in range(3):                     # replays of the captured graphs
        u2 = s.solve(dev(b[:, :16]), prec=dd.DD_MIXED, opts=o2).u.cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(u1, u2)
    s.close()


def test_replacement_columns_alone_and_in_batch():
    """Columns 0..7 solved as an 8-wide batch and inside 13-, 32- and 40-wide
    batches: the replacement points follow the batch (the first column due
    triggers one for all), so the results agree within the tolerance, each
    meeting the gate against the oracle."""
    dd = _dd()
    wl, b, uref = problem("2d-pd")
    s = solver_both(dd, wl)
    opts = dd.dd_default_opts(tol=1e-11, tiles=1, launch=dd.DD_LAUNCH_KERNELS, reliable=-1)
    ref = s.solve(dev(b[:, :8]), prec=dd.DD_MIXED, opts=opts).u.cpu().numpy()
    for w in (13, 32, 40):
        u = s.solve(dev(b[:, :w]), prec=dd.DD_MIXED, opts=opts).u.cpu().numpy()
        assert oracle.rel_err(u[:8].T, ref.T).max() <= 2e-8, w
        assert oracle.rel_err(u[:w].T, uref[:, :w]).max() <= 1e-8, w
    s.close()
