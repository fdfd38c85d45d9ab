"""GPU parity of the primal interface CG with the balancing Neumann-Neumann
preconditioner (dd_bdd_solve) and of the method autotuner (dd_method_*),
against the monolithic FP64 solution and the BDD oracle.

Gates: error <= 1e-10 relative to the monolithic solution at tolerance
1e-12; iteration counts within 2 of the oracle's (same preconditioner, same
stopping rule, different summation order); a column's solution the same
alone and in a batch; flat iteration counts over the delta/h = 4 ladder; every
method of the autotuner reaching the same solution."""
import functools

import numpy as np
import pytest

import oracle
import workloads
from oracle.bdd_oracle import BDDOracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dd():
    import paper_2306_00094_amd as dd
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dd.load_library()
    return dd


CASES = {
    "1d": lambda: workloads.spec_1d(n=160, delta=0.05, strips=4, nrhs=3),
    "2d-const": lambda: workloads.spec_2d_const(n=32, delta=0.15, cuts=(3, 3), nrhs=3),
    "2d-frac": lambda: workloads.spec_2d_frac(n=28, delta=0.15, cuts=(3, 3), nrhs=2),
    "2d-pd": lambda: workloads.spec_2d_pd(n=28, delta=0.15, cuts=(3, 3), jitter=0.15, nrhs=2),
}


@functools.lru_cache(maxsize=None)
def problem(name):
    spec = CASES[name]()
    wl = workloads.build(spec)
    fp = workloads.feti_problem(wl)
    b = workloads.rhs(spec)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    return spec, wl, fp, b, uref


def dev(b):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(b).T)).to("cuda:0").contiguous()


@pytest.mark.parametrize("name", list(CASES))
def test_bdd_parity(name):
    dd = _dd()
    spec, wl, fp, b, uref = problem(name)
    print(f"case bdd {name} K={len(fp.g_sets)} floating={sum(fp.floating)}", flush=True)
    s = dd.FetiSolver(wl.dd, fp, max_nrhs=b.shape[1])
    try:
        s.factor()
        r = s.solve_bdd(dev(b), tol=1e-12, max_it=500)
        u = r.u.cpu().numpy().T
        err = oracle.rel_err(u, uref)
        emax = np.abs(u - uref).max(axis=0) / np.abs(uref).max(axis=0)
        print(f"  err {err.max():.2e} its {[i['iters'] for i in r.info]}", flush=True)
        assert err.max() <= 1e-10 and emax.max() <= 1e-10
        assert all(i["converged"] == 1 and i["rel_resid"] <= 1.01e-12 for i in r.info)
        _, its, _ = BDDOracle(fp).solve(b, tol=1e-12)
        for i, it in zip(r.info, its):
            assert abs(i["iters"] - int(it)) <= 2, (i, its)
        r1 = s.solve_bdd(dev(b[:, 1:2]), tol=1e-12, max_it=500)
        assert np.allclose(r1.u.cpu().numpy()[0], r.u.cpu().numpy()[1], rtol=0, atol=1e-13 * np.abs(uref).max())
    finally:
        s.close()


def test_bdd_iterations_flat_at_fixed_delta_over_h():
    dd = _dd()
    its = []
    for n, cuts in ((32, (2, 2)), (64, (4, 4)), (128, (8, 8))):
        spec = workloads.spec_2d_const(n=n, delta=4.0 / n, cuts=cuts, nrhs=1)
        wl = workloads.build(spec)
        fp = workloads.feti_problem(wl)
        b = workloads.rhs(spec)
        print(f"case bdd ladder n={n}", flush=True)
        s = dd.FetiSolver(wl.dd, fp, max_nrhs=1)
        try:
            s.factor()
            r = s.solve_bdd(dev(b), tol=1e-10, max_it=500)
            assert r.info[0]["converged"] == 1 and r.info[0]["rel_resid"] <= 1.01e-10
            its.append(r.info[0]["iters"])
        finally:
            s.close()
    print(f"  iterations {its}", flush=True)
    assert max(its) <= 1.35 * min(its)


def test_method_autotune_and_every_method():
    dd = _dd()
    spec, wl, fp, b, uref = problem("2d-pd")
    print("case method autotune", flush=True)
    s = dd.FetiSolver(wl.dd, fp, max_nrhs=b.shape[1])
    try:
        s.factor()
        t = s.autotune(b.shape[1], tol=1e-12, max_it=2000)
        print(f"  {t}", flush=True)
        assert t["method"] in (dd.DD_METHOD_FETI, dd.DD_METHOD_BDD, dd.DD_METHOD_JACOBI)
        ms = [t["ms_feti"], t["ms_bdd"], t["ms_jacobi"]]
        assert all(0.0 < m < 1e300 for m in ms) and ms[t["method"] - 1] == min(ms)
        for m in (dd.DD_METHOD_AUTO, dd.DD_METHOD_FETI, dd.DD_METHOD_BDD, dd.DD_METHOD_JACOBI):
            r = s.solve_method(dev(b), method=m, tol=1e-12, max_it=2000)
            assert oracle.rel_err(r.u.cpu().numpy().T, uref).max() <= 1e-10, m
    finally:
        s.close()


def test_bdd_bad_arguments():
    dd = _dd()
    spec, wl, fp, b, uref = problem("1d")
    s = dd.FetiSolver(wl.dd, fp, max_nrhs=1)
    try:
        with pytest.raises(dd.DDError) as ei:              # solve before factor
            s.solve_bdd(dev(b[:, :1]))
        assert ei.value.status == dd.DD_ESTATE
        s.factor()
        r = s.solve_bdd(dev(b[:, :1]), tol=1e-14, max_it=2, raise_on_noconv=False)
        assert r.status == dd.DD_ENOCONV and r.info[0]["converged"] == 0 and r.info[0]["iters"] == 2
        with pytest.raises(dd.DDError) as ei:
            s.solve_method(dev(b[:, :1]), method=7)
        assert ei.value.status == dd.DD_EINVAL
    finally:
        s.close()
