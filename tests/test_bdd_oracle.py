"""Pins of the balancing Neumann-Neumann (BDD) oracle for the primal interface
problem (oracle/bdd_oracle.py).  CPU only.

What mathematics fixes, independently of the code:
  * the multiplicity scaling is a partition of unity: sum_k R_k^T D_k R_k = I;
  * balanced residuals are orthogonal to the coarse space: N^T (I - S P_0) r = 0;
  * M^-1 is symmetric, and the spectrum of M^-1 S lies in [1, C(1 + log H/h)^2]
    with 1 attained on the coarse space (M^-1 S N c = N c); a wrong scaling,
    pseudoinverse or sign moves eigenvalues below 1;
  * every S_k^+ in M_NN sees a compatible right-hand side: Z_k^T D_k R_k of a
    balanced residual vanishes, and S_k S_k^+ returns it;
  * the PCG reaches the monolithic solution;
  * at fixed delta/h and H/h the iteration count stays nearly flat as the
    number of subdomains grows, where diagonally preconditioned CG on S does
    not (the behaviour of the paper's Table fixedRatio for its dual method).
"""
import functools

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.bdd_oracle import BDDOracle

CASES = {
    "1d": lambda: W.spec_1d(n=96, delta=0.06, strips=4, nrhs=2),
    "2d-const": lambda: W.spec_2d_const(n=24, delta=0.15, cuts=(3, 3), nrhs=2),
    "2d-frac": lambda: W.spec_2d_frac(n=24, delta=0.15, cuts=(3, 3), nrhs=1),
    "2d-pd": lambda: W.spec_2d_pd(n=24, delta=0.15, cuts=(3, 3), jitter=0.15, nrhs=1),
}


@functools.lru_cache(maxsize=None)
def case(name):
    spec = CASES[name]()
    wl = W.build(spec)
    fp = W.feti_problem(wl)
    return spec, wl, fp, BDDOracle(fp)


@functools.lru_cache(maxsize=None)
def dense_ops(name):
    spec, wl, fp, bo = case(name)
    E = np.eye(wl.dd.n_gamma)
    S = np.column_stack([bo.ddo.schur_apply(e) for e in E])
    M = np.column_stack([bo.precond(e) for e in E])
    return S, M


@pytest.mark.parametrize("name", list(CASES))
def test_scaling_is_a_partition_of_unity(name):
    _, _, fp, bo = case(name)
    assert np.all(bo.partition_of_unity() == 1.0)
    assert bo.N.shape[1] == sum(np.asarray(fp.z[k]).shape[1] for k in range(len(fp.g_sets)) if fp.floating[k])


@pytest.mark.parametrize("name", ["1d", "2d-pd"])
def test_balanced_residuals_are_compatible(name):
    """N^T (I - S P_0) r = 0, so for every floating k the right-hand side
    D_k R_k r of S_k^+ is orthogonal to ker S_k and S_k S_k^+ returns it."""
    _, wl, fp, bo = case(name)
    r = np.random.default_rng(5).standard_normal(wl.dd.n_gamma)
    t = bo.balance(r)
    assert np.abs(bo.N.T @ t).max() <= 1e-12 * np.abs(bo.N.T @ r).max()
    for k, G in enumerate(fp.g_sets):
        if not fp.floating[k]:
            continue
        v = t[G] / bo.mult[G]
        assert np.abs(np.asarray(fp.z[k]).T @ v).max() <= 1e-11 * np.abs(v).max()
        w = bo.fo.schur_pinv_k(k, v)
        assert np.abs(bo.fo.schur_k(k, w) - v).max() <= 1e-9 * np.abs(v).max()


@pytest.mark.parametrize("name", list(CASES))
def test_preconditioned_spectrum_starts_at_one(name):
    S, M = dense_ops(name)
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    ev = np.sort(np.linalg.eigvals(M @ S).real)
    assert abs(ev[0] - 1.0) <= 1e-9, ev[:3]
    assert ev[-1] < 20.0
    # the Jacobi-preconditioned operator of the same system is far worse conditioned
    d = np.diag(S)
    ej = np.sort(np.linalg.eigvals(S / d[:, None]).real)
    assert ej[-1] / ej[0] > 2.0 * ev[-1] / ev[0]


def test_coarse_space_is_the_eigenvalue_one():
    """M^-1 S N c = N c for every coarse vector."""
    _, wl, fp, bo = case("2d-pd")
    S, M = dense_ops("2d-pd")
    c = np.random.default_rng(9).standard_normal(bo.N.shape[1])
    v = bo.N @ c
    assert np.abs(M @ (S @ v) - v).max() <= 1e-10 * np.abs(v).max()


@pytest.mark.parametrize("name", list(CASES))
def test_bdd_solution_equals_monolithic(name):
    spec, wl, fp, bo = case(name)
    b = W.rhs(spec)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    u, its, conv = bo.solve(b, tol=1e-12)
    assert conv.all()
    assert oracle.rel_err(u, uref).max() <= 1e-10
    _, its_j, _ = bo.ddo.solve(b, tol=1e-12)
    assert its.max() < its_j.min()


def test_bdd_iterations_flat_at_fixed_delta_over_h():
    its_b, its_j = [], []
    for n, cuts in ((32, (2, 2)), (64, (4, 4))):
        spec = W.spec_2d_const(n=n, delta=4.0 / n, cuts=cuts, nrhs=1)
        wl = W.build(spec)
        bo = BDDOracle(W.feti_problem(wl))
        b = W.rhs(spec)
        u, its, _ = bo.solve(b, tol=1e-10)
        assert oracle.full_residual(wl.asm.A, u, b).max() <= 1e-9
        its_b.append(int(its[0]))
        its_j.append(int(bo.ddo.solve(b, tol=1e-10)[1][0]))
    assert its_b[1] <= 1.35 * its_b[0]
    assert its_j[1] >= 1.7 * its_j[0]
