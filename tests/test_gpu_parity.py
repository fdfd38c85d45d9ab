"""GPU parity tests: the HIP path (through the C ABI) against the CPU FP64 oracle.

Gates: FP64 path error <= 1e-10 relative to the monolithic FP64 solution,
mixed path error <= 1e-8 after refinement; factors, diag(S) and the Schur
operator element by element against the oracle.
"""
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
    dd.load_library()          # raises if the HIP library is missing
    return dd


SMALL = {
    "1d-4strips": lambda: workloads.spec_1d(n=256, strips=4, nrhs=2),
    "1d-ragged": lambda: workloads.spec_1d(n=100, delta=0.07, strips=3, nrhs=3),
    "2d-const": lambda: workloads.spec_2d_const(n=32, cuts=(2, 2), nrhs=3),
    "2d-const-3x2": lambda: workloads.spec_2d_const(n=40, cuts=(3, 2), nrhs=2),
    "2d-frac": lambda: workloads.spec_2d_frac(n=32, cuts=(2, 2), nrhs=2),
    "2d-pd": lambda: workloads.spec_2d_pd(n=40, delta=0.1, cuts=(3, 3), jitter=0.2, nrhs=2),
}


@functools.lru_cache(maxsize=None)
def problem(name):
    spec = SMALL[name]()
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    return wl, b, uref


def to_dev(b):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(b).T)).to("cuda:0").contiguous()


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("prec", [0, 1])
def test_factor_parity(name, prec):
    dd = _dd()
    wl, _, _ = problem(name)
    print(f"case factor {name} prec={prec}", flush=True)
    s = dd.Solver(wl.dd, max_nrhs=1)
    s.factor(prec)
    tol = 1e-12 if prec == dd.DD_FP64 else 2e-5
    for k in range(wl.dd.n_sub):
        K = wl.dd.kii[k]
        L_ref = np.linalg.cholesky(K)
        L = s.factor_block(k, prec)
        err = np.abs(L - L_ref).max() / np.abs(L_ref).max()
        assert err <= tol, (k, err)
    d_ref = oracle.DDOracle(wl.dd).schur_diag()
    d = s.schur_diag(prec)
    derr = np.abs(d - d_ref).max() / np.abs(d_ref).max()
    assert derr <= (1e-12 if prec == dd.DD_FP64 else 1e-4), derr
    s.close()


# interior blocks past the sizes of the small cases: 853 rows (54 row tiles,
# sixteen tiles per wave in the one-launch Cholesky) and 1138 rows (72 row
# tiles: the per-panel Cholesky, and an L^-1 block column that just fills the
# 160 KB of LDS in FP64)
LARGE = {
    "1d-853": lambda: workloads.spec_1d(n=1800, strips=2, nrhs=1),
    "1d-1138": lambda: workloads.spec_1d(n=2400, strips=2, nrhs=1),
}


@pytest.mark.parametrize("name", list(LARGE))
@pytest.mark.parametrize("prec", [0, 1])
def test_factor_large_blocks(name, prec):
    dd = _dd()
    spec = LARGE[name]()
    wl = workloads.build(spec)
    b = workloads.rhs(spec)
    print(f"case factor large {name} prec={prec} n_i={[k.shape[0] for k in wl.dd.kii]}", flush=True)
    s = dd.Solver(wl.dd, max_nrhs=1)
    s.factor(prec)
    tol = 1e-12 if prec == dd.DD_FP64 else 2e-5
    for k in range(wl.dd.n_sub):
        L_ref = np.linalg.cholesky(wl.dd.kii[k])
        L = s.factor_block(k, prec)
        err = np.abs(L - L_ref).max() / np.abs(L_ref).max()
        assert err <= tol, (k, err)
    d_ref = oracle.DDOracle(wl.dd).schur_diag()
    derr = np.abs(s.schur_diag(prec) - d_ref).max() / np.abs(d_ref).max()
    assert derr <= (1e-12 if prec == dd.DD_FP64 else 1e-4), derr
    res = s.solve(to_dev(b), prec=prec, opts=dd.dd_default_opts(tol=1e-12))
    uref = oracle.monolithic_solve(wl.asm.A, b)
    err = oracle.rel_err(res.u.cpu().numpy().T, uref).max()
    assert err <= (1e-10 if prec == dd.DD_FP64 else 1e-8), err
    s.close()


def test_single_launch_cholesky_wait_bound(monkeypatch):
    """With the wait bound forced to zero from the host, block columns give up
    at once on predecessors that are still running: the launch still drains
    and dd_factor reports DD_EHIP instead of returning a factor.  A context
    with the normal bound then factors and solves correctly."""
    dd = _dd()
    wl, b, uref = problem("2d-const")
    print("case cholesky wait bound", flush=True)
    monkeypatch.setenv("DD_FLOW_SPIN", "0")
    s = dd.Solver(wl.dd, max_nrhs=b.shape[1])
    with pytest.raises(dd.DDError) as ei:
        s.factor(dd.DD_FP64)
    assert ei.value.status == dd.DD_EHIP and "waited too long" in str(ei.value)
    s.close()
    monkeypatch.delenv("DD_FLOW_SPIN")
    s = dd.Solver(wl.dd, max_nrhs=b.shape[1])
    s.factor(dd.DD_FP64)
    res = s.solve(to_dev(b), prec=dd.DD_FP64, opts=dd.dd_default_opts(tol=1e-12))
    assert oracle.rel_err(res.u.cpu().numpy().T, uref).max() <= 1e-10
    s.close()


@pytest.mark.parametrize("lag", [1, 4])
def test_interface_row_timing_counts_sweeps(lag):
    """Phase timing of the interface-row launches counts the launches that
    swept the matrix: iteration 0 and every iteration before the last (whose
    interior-solve launch stops the column), not the launches enqueued after
    the column stopped, which return at once.  The solution does not depend
    on the polling lag."""
    dd = _dd()
    wl, b, uref = problem("2d-const")
    print(f"case gamma timing lag={lag}", flush=True)
    s = dd.Solver(wl.dd, max_nrhs=1)
    s.factor(dd.DD_FP64)
    bd = to_dev(b[:, :1])
    o = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_KERNELS, check_every=lag, apply=dd.DD_APPLY_INV)
    ref = s.solve(bd, prec=dd.DD_FP64, opts=dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_KERNELS,
                                                                 check_every=1, apply=dd.DD_APPLY_INV))
    dd.dd_set_timing(s.ctx, 1 << dd.DD_PHASE_GAMMA, reset=True)
    res = s.solve(bd, prec=dd.DD_FP64, opts=o)
    ms, n = dd.dd_get_timing(s.ctx)
    dd.dd_set_timing(s.ctx, 0)
    its = res.info[0]["iters"]
    print("  iters", its, "timed launches", n[dd.DD_PHASE_GAMMA], "ms", ms[dd.DD_PHASE_GAMMA], flush=True)
    assert n[dd.DD_PHASE_GAMMA] == its
    assert np.array_equal(res.u.cpu().numpy(), ref.u.cpu().numpy())
    assert oracle.rel_err(res.u.cpu().numpy().T, uref[:, :1]).max() <= 1e-10
    s.close()


def test_factor_vector_vs_mfma(monkeypatch):
    """The MFMA trailing update and the vector-FMA one give the same factor,
    and the two formulations of diag(S) agree."""
    dd = _dd()
    wl, _, _ = problem("2d-const-3x2")
    print("case factor mfma/vector", flush=True)
    s1 = dd.Solver(wl.dd)
    s1.factor(dd.DD_FP64)
    monkeypatch.setenv("DD_NO_MFMA", "1")
    s2 = dd.Solver(wl.dd)
    s2.factor(dd.DD_FP64)
    for k in range(wl.dd.n_sub):
        a, b = s1.factor_block(k), s2.factor_block(k)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    # diag(S): column sums of squares of L^-1 K_IG (matrix cores) against the
    # quadratic forms with K_II^-1 (vector path)
    d1, d2 = s1.schur_diag(dd.DD_FP64), s2.schur_diag(dd.DD_FP64)
    assert np.abs(d1 - d2).max() <= 1e-13 * np.abs(d2).max()
    s1.close()
    s2.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_single_launch_cholesky_vs_panels(monkeypatch, prec):
    """The one-launch left-looking Cholesky (block columns waiting on flags)
    and the two-launches-per-panel right-looking one give the same factor,
    diag(S) and solution, on blocks of uneven size."""
    dd = _dd()
    wl, b, _ = problem("2d-pd")
    print(f"case cholesky flow/panels prec={prec}", flush=True)
    opts = dd.dd_default_opts(tol=1e-12)
    out = []
    for env in ("0", "1"):
        monkeypatch.setenv("DD_PANEL_POTRF", env)
        s = dd.Solver(wl.dd, max_nrhs=b.shape[1])
        s.factor(prec)
        u = s.solve(torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda:0"), prec=prec, opts=opts).u
        out.append(([s.factor_block(k, prec) for k in range(wl.dd.n_sub)], s.schur_diag(prec),
                    u.cpu().numpy()))
        s.close()
    (l1, d1, u1), (l2, d2, u2) = out
    tol = 1e-13 if prec == dd.DD_FP64 else 1e-5
    for a, c in zip(l1, l2):
        assert np.abs(a - c).max() <= tol * np.abs(c).max()
    assert np.abs(d1 - d2).max() <= tol * np.abs(d2).max()
    assert np.abs(u1 - u2).max() <= 1e-10 * np.abs(u2).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_inverse_factor_panel_vs_blockwave(monkeypatch, prec):
    """L^-1 by LDS-resident block columns (four waves, inverted diagonal blocks)
    and by one wave per block column give the same diag(S) and solution."""
    dd = _dd()
    wl, b, _ = problem("2d-pd")
    print(f"case trtri panel/blockwave prec={prec}", flush=True)
    opts = dd.dd_default_opts(tol=1e-12)
    out = []
    for env in ("0", "1"):
        monkeypatch.setenv("DD_BLOCKWAVE_TRTRI", env)
        s = dd.Solver(wl.dd, max_nrhs=b.shape[1])
        s.factor(prec)
        u = s.solve(torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda:0"), prec=prec, opts=opts).u
        out.append((s.schur_diag(prec), u.cpu().numpy()))
        s.close()
    (d1, u1), (d2, u2) = out
    tol = 1e-13 if prec == dd.DD_FP64 else 1e-5
    assert np.abs(d1 - d2).max() <= tol * np.abs(d2).max()
    assert np.abs(u1 - u2).max() <= 1e-10 * np.abs(u2).max()


@pytest.mark.parametrize("name", list(SMALL))
def test_schur_apply_parity(name):
    dd = _dd()
    wl, _, _ = problem(name)
    print(f"case schur_apply {name}", flush=True)
    orc = oracle.DDOracle(wl.dd)
    rng = np.random.default_rng(7)
    P = rng.uniform(-1, 1, size=(wl.dd.n_gamma, 3))
    Q_ref = orc.schur_apply(P)
    s = dd.Solver(wl.dd, max_nrhs=3)
    s.factor(dd.DD_FP64)
    Q = s.schur_apply(to_dev(P)).cpu().numpy().T
    err = np.abs(Q - Q_ref).max() / np.abs(Q_ref).max()
    assert err <= 1e-12, err
    s.close()


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("apply", [1, 2])
def test_solve_fp64(name, apply):
    dd = _dd()
    wl, b, uref = problem(name)
    print(f"case solve fp64 {name} apply={apply}", flush=True)
    nrhs = b.shape[1]
    s = dd.Solver(wl.dd, max_nrhs=nrhs)
    s.factor(dd.DD_FP64)
    opts = dd.dd_default_opts(tol=1e-14, apply=apply)
    res = s.solve(to_dev(b), prec=dd.DD_FP64, opts=opts)
    u = res.u.cpu().numpy().T
    err = oracle.rel_err(u, uref)
    assert err.max() <= 1e-10, err
    # iteration counts match the oracle's CG (same preconditioner and stopping rule)
    _, its, _ = oracle.DDOracle(wl.dd).solve(b, tol=1e-14)
    got = np.array([i["iters"] for i in res.info])
    assert np.all(np.abs(got - its) <= 2), (got, its)
    assert all(i["converged"] for i in res.info)
    s.close()


@pytest.mark.parametrize("name", list(SMALL))
def test_solve_mixed(name):
    dd = _dd()
    wl, b, uref = problem(name)
    print(f"case solve mixed {name}", flush=True)
    nrhs = b.shape[1]
    s = dd.Solver(wl.dd, max_nrhs=nrhs)
    s.factor(dd.DD_MIXED)
    opts = dd.dd_default_opts(tol=1e-12)
    res = s.solve(to_dev(b), prec=dd.DD_MIXED, opts=opts)
    u = res.u.cpu().numpy().T
    err = oracle.rel_err(u, uref)
    print("  err", err, res.info, flush=True)
    assert err.max() <= 1e-8, err
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_invariance(prec):
    """Each column solved inside a batch equals the same column solved alone."""
    dd = _dd()
    wl, b, _ = problem("2d-const")
    print(f"case batch invariance prec={prec}", flush=True)
    s = dd.Solver(wl.dd, max_nrhs=3)
    s.factor(prec)
    opts = dd.dd_default_opts(tol=1e-12)
    ub = s.solve(to_dev(b), prec=prec, opts=opts).u.cpu().numpy()
    for j in range(b.shape[1]):
        uj = s.solve(to_dev(b[:, j:j + 1]), prec=prec, opts=opts).u.cpu().numpy()
        assert np.array_equal(uj[0], ub[j]), j
    s.close()


@pytest.mark.parametrize("name", ["1d-ragged", "2d-const", "2d-pd"])
@pytest.mark.parametrize("prec", [0, 1])
def test_persistent_launch_matches_kernels(name, prec, monkeypatch):
    """One cooperative persistent kernel for the CG loop gives the same
    solution, bit for bit, as one launch per phase of the same four-phase
    iteration (forced here; by default stream launches use three per
    iteration)."""
    dd = _dd()
    wl, b, uref = problem(name)
    print(f"case persistent {name} prec={prec}", flush=True)
    nrhs = b.shape[1]
    monkeypatch.setenv("DD_CLASSIC_CG", "1")
    s = dd.Solver(wl.dd, max_nrhs=nrhs)
    s.factor(prec)
    o1 = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_KERNELS)
    o2 = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_PERSISTENT)
    r1 = s.solve(to_dev(b), prec=prec, opts=o1)
    r2 = s.solve(to_dev(b), prec=prec, opts=o2)
    assert [i["iters"] for i in r1.info] == [i["iters"] for i in r2.info]
    assert np.array_equal(r1.u.cpu().numpy(), r2.u.cpu().numpy())
    s.close()


@pytest.mark.parametrize("name", ["1d-ragged", "2d-const", "2d-pd"])
@pytest.mark.parametrize("prec", [0, 1])
def test_graph_launch_matches_kernels(name, prec):
    """CG iterations captured in a hipGraph and replayed give the same
    solution, bit for bit, as stream launches (converged columns are frozen,
    so extra replayed iterations change nothing)."""
    dd = _dd()
    wl, b, uref = problem(name)
    print(f"case graph {name} prec={prec}", flush=True)
    nrhs = b.shape[1]
    s = dd.Solver(wl.dd, max_nrhs=nrhs)
    s.factor(prec)
    o1 = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_KERNELS)
    o2 = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_GRAPH, check_every=4)
    r1 = s.solve(to_dev(b), prec=prec, opts=o1)
    for _ in range(3):          # replays of the cached graph, eager work in between
        r2 = s.solve(to_dev(b), prec=prec, opts=o2)
        assert [i["iters"] for i in r1.info] == [i["iters"] for i in r2.info]
        assert np.array_equal(r1.u.cpu().numpy(), r2.u.cpu().numpy())
        r1 = s.solve(to_dev(b), prec=prec, opts=o1)
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_then_auto_solve(prec):
    """The autotuner times its candidate schedules, records the fastest, and
    AUTO solves then use it and still meet the parity gate."""
    dd = _dd()
    wl, b, uref = problem("2d-const-3x2")
    print(f"case autotune prec={prec}", flush=True)
    nrhs = b.shape[1]
    s = dd.Solver(wl.dd, max_nrhs=nrhs)
    s.factor(prec)
    res = s.autotune(prec, nrhs, dd.dd_default_opts(tol=1e-12))
    print("  tuned", res, flush=True)
    assert res["candidates"] >= 7 and res["ms_per_solve"] > 0
    assert res["launch"] in (1, 2, 3) and res["apply"] in (1, 2)
    assert res["three_launch"] in ((0, 1) if prec == 0 else (0, 1, 2, 3))   # bit 1: FP32 gathers (mixed)
    if prec == 1:        # the mixed path also tunes its inner tolerance
        assert res["inner_tol"] in (1e-4, 1e-5, 1e-6)
    else:
        assert res["inner_tol"] == 0.0
    r = s.solve(to_dev(b), prec=prec, opts=dd.dd_default_opts(tol=1e-12))
    err = oracle.rel_err(r.u.cpu().numpy().T, uref)
    assert err.max() <= (1e-10 if prec == 0 else 1e-8)
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_factor_rejects_indefinite_block(prec):
    """A subdomain block that is not positive definite is reported by
    dd_factor as DD_ENOTSPD naming the subdomain and the failing column; the
    context stays usable after the error (a valid problem factors and solves
    on a fresh context)."""
    import copy
    dd = _dd()
    wl, b, uref = problem("1d-4strips")
    bad = copy.deepcopy(wl.dd)
    K = np.array(bad.kii[2], order="F", copy=True)
    K[7, 7] = -10.0 * abs(K[7, 7])
    bad.kii[2] = K
    print(f"case indefinite block prec={prec}", flush=True)
    s = dd.Solver(bad, max_nrhs=1)
    with pytest.raises(dd.DDError) as ei:
        s.factor(prec)
    assert ei.value.status == dd.DD_ENOTSPD
    assert "subdomain 2" in str(ei.value) and "column 7" in str(ei.value)
    with pytest.raises(dd.DDError) as ei:          # no factors: solve refuses
        s.solve(to_dev(b[:, :1]), prec=prec)
    assert ei.value.status == dd.DD_ESTATE
    s.close()
    s = dd.Solver(wl.dd, max_nrhs=1)
    s.factor(prec)
    r = s.solve(to_dev(b[:, :1]), prec=prec, opts=dd.dd_default_opts(tol=1e-12))
    assert oracle.rel_err(r.u.cpu().numpy().T, uref[:, :1]).max() <= (1e-10 if prec == 0 else 1e-8)
    s.close()


@pytest.mark.parametrize("name", ["1d-4strips", "2d-const-3x2", "2d-pd"])
@pytest.mark.parametrize("prec", [0, 1])
def test_three_launch_iteration_matches_four_launch(name, prec, monkeypatch):
    """The three-launch CG iteration (interior-solve recurrence, update fused
    into the K_IG launch) and the four-launch one are the same method: the
    same iteration counts (up to one, from rounding) and solutions that agree
    to the parity gate; both meet it against the monolithic solution."""
    dd = _dd()
    wl, b, uref = problem(name)
    print(f"case three vs four launches {name} prec={prec}", flush=True)
    nrhs = b.shape[1]
    opts = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_KERNELS, apply=dd.DD_APPLY_INV)
    s3 = dd.Solver(wl.dd, max_nrhs=nrhs)
    s3.factor(prec)
    r3 = s3.solve(to_dev(b), prec=prec, opts=opts)
    monkeypatch.setenv("DD_CLASSIC_CG", "1")
    s4 = dd.Solver(wl.dd, max_nrhs=nrhs)
    s4.factor(prec)
    r4 = s4.solve(to_dev(b), prec=prec, opts=opts)
    i3 = np.array([i["iters"] for i in r3.info])
    i4 = np.array([i["iters"] for i in r4.info])
    print("  iters", i3, i4, flush=True)
    assert np.all(np.abs(i3 - i4) <= 1 + 2 * (prec == 1)), (i3, i4)
    u3, u4 = r3.u.cpu().numpy().T, r4.u.cpu().numpy().T
    gate = 1e-10 if prec == 0 else 1e-8
    assert oracle.rel_err(u3, uref).max() <= gate
    assert oracle.rel_err(u4, uref).max() <= gate
    assert oracle.rel_err(u3, u4).max() <= 2 * gate
    s3.close()
    s4.close()


@pytest.mark.parametrize("iteration", ["three", "four"])
@pytest.mark.parametrize("name", ["1d-ragged", "2d-const", "2d-pd"])
def test_mixed_fp32_gathers(name, iteration, monkeypatch):
    """The mixed path with its FP32-data products gathering FP32 copies of
    the vectors they multiply (three-launch iteration: z, D^-1 q, p, w;
    four-launch iteration with the direction kernel: p, w): the refined
    solution meets the mixed gate against the monolithic solution, graph
    replays give the bits of stream launches, and every column of a
    16-column batch equals, bit for bit, the same column solved alone."""
    dd = _dd()
    wl, b, uref = problem(name)
    print(f"case mixed fp32 gathers {name} {iteration} launches", flush=True)
    monkeypatch.setenv("DD_GATHER32", "1")
    if iteration == "four":
        monkeypatch.setenv("DD_CLASSIC_CG", "1")
        monkeypatch.setenv("DD_DIRECTION_KERNEL", "1")
    s = dd.Solver(wl.dd, max_nrhs=16)
    s.factor(dd.DD_MIXED)
    o1 = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_KERNELS, apply=dd.DD_APPLY_INV)
    o2 = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_GRAPH, check_every=4, apply=dd.DD_APPLY_INV)
    r1 = s.solve(to_dev(b), prec=dd.DD_MIXED, opts=o1)
    err = oracle.rel_err(r1.u.cpu().numpy().T, uref)
    print("  err", err, [i["iters"] for i in r1.info], flush=True)
    assert err.max() <= 1e-8
    r2 = s.solve(to_dev(b), prec=dd.DD_MIXED, opts=o2)
    assert [i["iters"] for i in r1.info] == [i["iters"] for i in r2.info]
    assert np.array_equal(r1.u.cpu().numpy(), r2.u.cpu().numpy())
    b16 = np.tile(b, (1, 16))[:, :16]
    r16 = s.solve(to_dev(b16), prec=dd.DD_MIXED, opts=o1).u.cpu().numpy()
    for j in (0, 7, 15):
        one = s.solve(to_dev(b16[:, j:j + 1]), prec=dd.DD_MIXED, opts=o1).u.cpu().numpy()
        assert np.array_equal(r16[j], one[0]), j
    s.close()


def test_three_launch_wide_batch(monkeypatch):
    """16 columns (wide-batch kernels of the three-launch iteration): the same
    iterations (up to one) and solutions as the four-launch iteration within
    the gate, and every column equal, bit for bit, to the same column solved
    alone."""
    dd = _dd()
    wl, b, uref = problem("2d-const")
    print("case three-launch wide batch, 16 columns", flush=True)
    b16 = np.tile(b, (1, 6))[:, :16]
    opts = dd.dd_default_opts(tol=1e-12, launch=dd.DD_LAUNCH_KERNELS, apply=dd.DD_APPLY_INV)
    s = dd.Solver(wl.dd, max_nrhs=16)
    s.factor(dd.DD_FP64)
    r = s.solve(to_dev(b16), prec=dd.DD_FP64, opts=opts)
    u = r.u.cpu().numpy()
    assert oracle.rel_err(u.T[:, :3], uref).max() <= 1e-10
    for j in (0, 5, 15):
        r1 = s.solve(to_dev(b16[:, j:j + 1]), prec=dd.DD_FP64, opts=opts)
        assert np.array_equal(r1.u.cpu().numpy()[0], u[j]), j
    monkeypatch.setenv("DD_CLASSIC_CG", "1")
    s4 = dd.Solver(wl.dd, max_nrhs=16)
    s4.factor(dd.DD_FP64)
    r4 = s4.solve(to_dev(b16), prec=dd.DD_FP64, opts=opts)
    i3 = np.array([i["iters"] for i in r.info])
    i4 = np.array([i["iters"] for i in r4.info])
    assert np.all(np.abs(i3 - i4) <= 1), (i3, i4)
    assert oracle.rel_err(u.T, r4.u.cpu().numpy().T).max() <= 2e-10
    s.close()
    s4.close()
