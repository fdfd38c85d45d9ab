"""GPU parity of the tiled matrix-core products of wide batches (8 to 64
right-hand sides): 16x16 tiles of K_IG and [K_GG | K_GI], interior solves on
the matrix cores, against the CPU FP64 oracle.

Gates: FP64 path error <= 1e-10 relative to the monolithic FP64 solution
(tolerance 1e-13), mixed path <= 1e-8; the same iteration counts as the
oracle's substructuring PCG within 2; a column's result bitwise the same at
every batch width the tiled path serves; the tiled and CSR paths agree to
the gate.  The cases span several 16-row blocks with ragged last blocks
(n_gamma and every interior size are not multiples of 16)."""
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
    "1d": lambda: workloads.spec_1d(n=300, delta=0.07, strips=3, nrhs=40, seed_base=1100),
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


def test_cases_are_ragged():
    for name in CASES:
        wl, _, _ = problem(name)
        assert wl.dd.n_gamma % 16 != 0 or any(k.shape[0] % 16 for k in wl.dd.kii), name
        assert wl.dd.n_gamma > 2 * 16


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nrhs", [8, 13, 32, 40])
def test_tiled_solve_parity(name, prec, nrhs):
    dd = _dd()
    wl, b, uref = problem(name)
    print(f"case tiles {name} prec={prec} nrhs={nrhs}", flush=True)
    s = dd.Solver(wl.dd, max_nrhs=64)
    s.factor(prec)
    opts = dd.dd_default_opts(tol=1e-13, tiles=1)
    r = s.solve(dev(b[:, :nrhs]), prec=prec, opts=opts)
    u = r.u.cpu().numpy().T
    err = oracle.rel_err(u, uref[:, :nrhs])
    gate = 1e-10 if prec == dd.DD_FP64 else 1e-8
    print(f"  err max {err.max():.2e} its {[i['iters'] for i in r.info][:4]}", flush=True)
    assert err.max() <= gate
    # element-wise: the largest entry error relative to the largest entry
    emax = np.abs(u - uref[:, :nrhs]).max(axis=0) / np.abs(uref[:, :nrhs]).max(axis=0)
    assert emax.max() <= gate
    if prec == dd.DD_FP64:
        ora = oracle.DDOracle(wl.dd)
        _, its_ref, _ = ora.solve(b[:, :4], tol=1e-13)
        for j in range(4):
            assert abs(r.info[j]["iters"] - int(its_ref[j])) <= 2, (j, r.info[j], its_ref[j])
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_tiled_columns_independent_of_width(prec):
    """Columns 0..7 solved as an 8-wide batch, inside a 13-, 32- and a 40-wide
    (64-column) batch: bitwise the same."""
    dd = _dd()
    wl, b, _ = problem("2d-pd")
    s = dd.Solver(wl.dd, max_nrhs=64)
    s.factor(prec)
    opts = dd.dd_default_opts(tol=1e-11, tiles=1)
    ref = s.solve(dev(b[:, :8]), prec=prec, opts=opts).u.cpu().numpy()
    for w in (13, 32, 40):
        u = s.solve(dev(b[:, :w]), prec=prec, opts=opts).u.cpu().numpy()
        assert np.array_equal(u[:8], ref), w
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_tiled_and_csr_paths_agree(prec):
    """The tiled path and the CSR kernels solve the same batch to the gate."""
    dd = _dd()
    wl, b, uref = problem("2d-const")
    s = dd.Solver(wl.dd, max_nrhs=32)
    s.factor(prec)
    ut = s.solve(dev(b[:, :32]), prec=prec, opts=dd.dd_default_opts(tol=1e-13, tiles=1)).u.cpu().numpy()
    uc = s.solve(dev(b[:, :32]), prec=prec, opts=dd.dd_default_opts(tol=1e-13, tiles=0)).u.cpu().numpy()
    gate = 1e-10 if prec == dd.DD_FP64 else 1e-8
    assert oracle.rel_err(ut.T, uc.T).max() <= 2 * gate
    assert oracle.rel_err(ut.T, uref[:, :32]).max() <= gate
    s.close()


def test_tiled_graph_launch_matches_kernels():
    """Graph-captured iterations of the tiled path equal the stream launches."""
    dd = _dd()
    wl, b, _ = problem("2d-const")
    s = dd.Solver(wl.dd, max_nrhs=32)
    s.factor(dd.DD_FP64)
    o1 = dd.dd_default_opts(tol=1e-12, tiles=1, launch=dd.DD_LAUNCH_KERNELS)
    o2 = dd.dd_default_opts(tol=1e-12, tiles=1, launch=dd.DD_LAUNCH_GRAPH, check_every=4)
    u1 = s.solve(dev(b[:, :16]), opts=o1).u.cpu().numpy()
    for _ in range(3):                     # replays of the captured graph
        u2 = s.solve(dev(b[:, :16]), opts=o2).u.cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(u1, u2)
    s.close()


def test_tiles_ignored_below_eight_columns():
    """tiles = 1 with fewer than 8 columns runs the narrow kernels: bitwise the
    result of tiles = 0."""
    dd = _dd()
    wl, b, _ = problem("2d-const")
    s = dd.Solver(wl.dd, max_nrhs=32)
    s.factor(dd.DD_FP64)
    u1 = s.solve(dev(b[:, :3]), opts=dd.dd_default_opts(tol=1e-12, tiles=1)).u.cpu().numpy()
    u0 = s.solve(dev(b[:, :3]), opts=dd.dd_default_opts(tol=1e-12, tiles=0)).u.cpu().numpy()
    assert np.array_equal(u0, u1)
    s.close()
