"""GPU tests of the paths that are not taken on the benchmark systems:

- the mixed-precision refinement falling back to the FP64 path, forced by a
  step cap and reached naturally on a system too ill-conditioned for the FP32
  operators, through dd_solve and through the serving loop (DD_SLOT_FALLBACK);
- the CG breakdown p^T S p <= 0 on an indefinite interface operator, reported
  as DD_ENOTSPD (the oracle's PCG breaks down on the same system);
- a problem without interface (one subdomain holding every dof: the solve is
  the interior solve alone).

The modified systems are built on the CPU from a generated one: a diagonal
shift of the whole matrix (A - sigma I, still positive definite, condition
number about 3e7) or of the interface block only (K_GG - sigma I with
lambda_min(S) < sigma < min diag(S): diag(S) stays positive, S becomes
indefinite)."""
import copy
import functools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dd():
    import paper_2306_00094_amd as dd
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dd.load_library()
    return dd


def dev(b):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(b).T)).to("cuda:0").contiguous()


@functools.lru_cache(maxsize=None)
def base():
    spec = workloads.spec_1d(n=160, delta=0.05, strips=3, nrhs=3, seed_base=1500)
    wl = workloads.build(spec)
    return spec, wl, workloads.rhs(spec)


def shifted(dd, sigma, interface_only=False):
    d2 = copy.deepcopy(dd)
    if not interface_only:
        d2.kii = [np.asfortranarray(K - sigma * np.eye(K.shape[0])) for K in dd.kii]
    d2.kgg = (dd.kgg - sigma * sp.eye(dd.n_gamma)).tocsr()
    d2.kgg.sort_indices()
    return d2


def full_matrix(dd):
    """A assembled back from the blocks (for the oracle's monolithic solve)."""
    n = dd.n_dof
    A = sp.lil_matrix((n, n))
    g = dd.gamma_map
    A[np.ix_(g, g)] = dd.kgg.toarray()
    for k in range(dd.n_sub):
        I = dd.i_maps[k]
        A[np.ix_(I, I)] = dd.kii[k]
        G = g[dd.g_maps[k]]
        kig = dd.kig[k].toarray()
        A[np.ix_(I, G)] = kig
        A[np.ix_(G, I)] = kig.T
    return A.tocsr()


@functools.lru_cache(maxsize=None)
def ill_conditioned():
    spec, wl, b = base()
    ev = np.linalg.eigvalsh(wl.asm.A.toarray())
    sigma = ev[0] - ev[-1] / 3e7                 # lambda_min(A - sigma I) = lambda_max / 3e7
    d2 = shifted(wl.dd, sigma)
    A2 = full_matrix(d2)
    e2 = np.linalg.eigvalsh(A2.toarray())
    assert 1e7 < e2[-1] / e2[0] < 1e8
    return d2, A2, b, e2[-1] / e2[0]


def test_fallback_forced_by_step_cap():
    """max_refine = 1 with a tolerance one FP32-operator step cannot reach:
    every column finishes on the FP64 path, within the FP64 gate."""
    dd = _dd()
    spec, wl, b = base()
    print("case fallback step cap", flush=True)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    s = dd.Solver(wl.dd, max_nrhs=b.shape[1])
    s.factor(dd.DD_MIXED)
    opts = dd.dd_default_opts(tol=1e-13, max_refine=1, inner_tol=1e-3)
    r = s.solve(dev(b), prec=dd.DD_MIXED, opts=opts)
    u = r.u.cpu().numpy().T
    assert all(i["used_fallback"] == 1 and i["converged"] == 1 for i in r.info), r.info
    assert oracle.rel_err(u, uref).max() <= 1e-10
    assert (np.abs(u - uref).max(axis=0) / np.abs(uref).max(axis=0)).max() <= 1e-10
    # without the fallback the step cap leaves the tolerance unmet
    r2 = s.solve(dev(b), prec=dd.DD_MIXED, raise_on_noconv=False,
                 opts=dd.dd_default_opts(tol=1e-13, max_refine=1, inner_tol=1e-3, fp64_fallback=0))
    assert r2.status == dd.DD_ENOCONV and all(i["used_fallback"] == 0 for i in r2.info)
    s.close()


def test_fallback_on_stalled_refinement():
    """Condition number 3e7: FP32 operators (relative error about kappa u_32 > 1)
    cannot reduce the FP64 residual by 1/2 per step, the refinement stalls and
    the FP64 path finishes every column to the tolerance (1e-8: the FP64
    floor of the relative residual is about kappa u_64 = 7e-9)."""
    dd = _dd()
    d2, A2, b, kappa = ill_conditioned()
    print(f"case fallback stall kappa={kappa:.2e}", flush=True)
    uref = oracle.monolithic_solve(A2, b)
    s = dd.Solver(d2, max_nrhs=b.shape[1])
    s.factor(dd.DD_MIXED)
    tol = 1e-8
    r = s.solve(dev(b), prec=dd.DD_MIXED, opts=dd.dd_default_opts(tol=tol, max_it=5000))
    u = r.u.cpu().numpy().T
    print(f"  info {r.info}", flush=True)
    assert all(i["used_fallback"] == 1 and i["converged"] == 1 for i in r.info), r.info
    res = oracle.full_residual(A2, u, b)
    assert res.max() <= tol * 1.01
    # error bound of a relative residual tol at condition number kappa
    assert oracle.rel_err(u, uref).max() <= kappa * tol
    s.close()


def test_serving_fallback_slots():
    """The serving loop on the ill-conditioned system: the batch API marks the
    stalled slots DD_SLOT_FALLBACK and the loop finishes them with FP64
    factors; every request within the residual tolerance, flagged."""
    dd = _dd()
    from paper_2306_00094_amd import serving
    d2, A2, b, kappa = ill_conditioned()
    print("case serving fallback", flush=True)
    tol = 1e-8
    srv = serving.Server({"ill": d2}, prec=dd.DD_MIXED,
                         opts=dd.dd_default_opts(tol=tol, max_it=5000, gather32=1))
    reqs = [serving.Request("ill", b[:, j:j + 1].copy(), arrival=0.0, rid=j) for j in range(b.shape[1])]
    done = srv.run(reqs, timeout=120)
    assert len(done) == len(reqs)
    for r in done:
        assert r.fallback and r.info[0]["used_fallback"] == 1
        assert oracle.full_residual(A2, r.u, r.b).max() <= tol * 1.01
    # the admission count of a mixed system reserves its FP64 fallback context
    assert srv.footprint["ill"] >= dd.dd_footprint(d2, dd.DD_MIXED, serving.MAX_SLOTS) + \
        dd.dd_footprint(d2, dd.DD_FP64, serving.MAX_SLOTS)


def test_breakdown_on_indefinite_interface_operator():
    dd = _dd()
    spec, wl, b = base()
    ora = oracle.DDOracle(wl.dd)
    n = wl.dd.n_gamma
    S = np.column_stack([ora.schur_apply(np.eye(n)[:, j]) for j in range(n)])
    lam = np.linalg.eigvalsh(S)[0]
    sigma = 0.5 * (lam + S.diagonal().min())
    d2 = shifted(wl.dd, sigma, interface_only=True)
    with pytest.raises(ArithmeticError):           # the oracle's PCG breaks down
        oracle.DDOracle(d2).solve(b, tol=1e-12)
    print("case breakdown", flush=True)
    s = dd.Solver(d2, max_nrhs=b.shape[1])
    s.factor(dd.DD_FP64)                           # diag(S) is positive: the factor succeeds
    assert (s.schur_diag(dd.DD_FP64) > 0).all()
    for launch in (dd.DD_LAUNCH_KERNELS, dd.DD_LAUNCH_GRAPH):
        with pytest.raises(dd.DDError) as ei:
            s.solve(dev(b), prec=dd.DD_FP64, opts=dd.dd_default_opts(tol=1e-12, launch=launch))
        assert ei.value.status == dd.DD_ENOTSPD and "p^T S p" in str(ei.value)
    s.close()


def test_interface_free_problem():
    """One subdomain holding every dof: no interface, the solve is K_II^-1 b."""
    dd = _dd()
    spec, wl, b = base()
    A = wl.asm.A.tocsr()
    n = A.shape[0]
    one = workloads.DDProblem(n_dof=n, n_gamma=0, gamma_map=np.zeros(0, np.int32),
                              kgg=sp.csr_matrix((0, 0)))
    one.i_maps.append(np.arange(n, dtype=np.int32))
    one.g_maps.append(np.zeros(0, np.int32))
    one.kii.append(np.asfortranarray(A.toarray()))
    one.kig.append(sp.csr_matrix((n, 0)))
    uref = oracle.monolithic_solve(A, b)
    print("case interface-free", flush=True)
    s = dd.Solver(one, max_nrhs=b.shape[1])
    for prec, gate in ((dd.DD_FP64, 1e-10), (dd.DD_MIXED, 1e-8)):
        s.factor(prec)
        r = s.solve(dev(b), prec=prec, opts=dd.dd_default_opts(tol=1e-12))
        u = r.u.cpu().numpy().T
        assert oracle.rel_err(u, uref).max() <= gate
        assert all(i["iters"] == 0 for i in r.info) or prec == dd.DD_MIXED
    s.close()


def test_replacement_on_ill_conditioned_wide_batch():
    """The wide-batch mixed solve with both factors formed (FP32 directions,
    FP64 residual replacement) on the system too ill-conditioned for the
    FP32 operators: whatever the FP32 directions do (slow progress or a
    breakdown), the final FP64 check, the refinement behind it and the FP64
    fallback bring every column to the tolerance."""
    dd = _dd()
    d2, A2, _, kappa = ill_conditioned()
    spec, _, _ = base()
    b = workloads.rhs(spec, nrhs=8)
    print(f"case replacement ill-conditioned kappa={kappa:.2e}", flush=True)
    uref = oracle.monolithic_solve(A2, b)
    s = dd.Solver(d2, max_nrhs=8)
    s.factor(dd.DD_FP64)
    s.factor(dd.DD_MIXED)
    tol = 1e-8
    r = s.solve(dev(b), prec=dd.DD_MIXED, raise_on_noconv=False,
                opts=dd.dd_default_opts(tol=tol, max_it=5000, tiles=1))
    u = r.u.cpu().numpy().T
    print(f"  info {r.info}", flush=True)
    assert r.status == dd.DD_OK
    assert all(i["converged"] == 1 for i in r.info), r.info
    assert oracle.full_residual(A2, u, b).max() <= tol * 1.01
    assert oracle.rel_err(u, uref).max() <= kappa * tol
    s.close()
