"""Pins of the dual-method (FETI) oracle and of the subdomain data it reads:
the zeta-weighted subdomain matrices (eqs. zeta, bilinear-multi1), the
constraint matrices of the section "FETI", the pseudoinverse by pinned
Neumann solves (section "Pseudoinverse and Cholesky decomposition"), the
natural coarse space and the solution of Algorithm 1 against the monolithic
solve.  CPU only."""
import functools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W
from oracle.feti_oracle import FETIOracle, constraint_matrix

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
    return spec, wl, fp, FETIOracle(fp)


def restriction(G, n_gamma):
    return sp.csr_matrix((np.ones(G.size), (np.arange(G.size), G)), shape=(G.size, n_gamma))


@pytest.mark.parametrize("name", list(CASES))
def test_zeta_weighted_subdomain_matrices(name):
    """Sum_k R_k^T A^k_GG R_k = A_GG (the zeta weights are a partition of
    unity on the support of the kernel); the interface-interior blocks equal
    the global matrix's; a floating subdomain's matrix annihilates its kernel
    (constants, or the rigid motions for peridynamics: remark "floating")."""
    spec, wl, fp, _ = case(name)
    dd = wl.dd
    tot = sp.csr_matrix((dd.n_gamma, dd.n_gamma))
    scale = abs(dd.kgg).max()
    assert any(fp.floating) and not all(fp.floating)
    for k, G in enumerate(fp.g_sets):
        Rk = restriction(G, dd.n_gamma)
        tot = tot + Rk.T @ fp.agg[k] @ Rk
        assert abs(fp.agi[k] - fp.kig[k].T).max() <= 1e-13 * scale
        assert abs(fp.agg[k] - fp.agg[k].T).max() <= 1e-13 * scale
        if fp.floating[k]:
            I = dd.i_maps[k]
            if spec.ncomp == 1:
                ZI = np.ones((I.size, 1))
            else:
                xy = wl.asm.coords[I // 2]
                comp = I % 2
                ZI = np.zeros((I.size, 3))
                ZI[comp == 0, 0] = 1.0
                ZI[comp == 1, 1] = 1.0
                ZI[:, 2] = np.where(comp == 0, -xy[:, 1], xy[:, 0])
            Ak = sp.bmat([[sp.csr_matrix(dd.kii[k]), fp.kig[k]], [fp.agi[k], fp.agg[k]]]).tocsr()
            assert abs(Ak @ np.vstack([ZI, fp.z[k]])).max() <= 1e-12 * scale
    assert abs(tot - dd.kgg).max() <= 1e-13 * scale


@pytest.mark.parametrize("name", ["1d", "2d-pd"])
def test_zeta_weighted_loads_sum_to_global_load(name):
    """Eq. bilinear-multi5: sum_k R_k^T f~_Gamma^k = b_Gamma."""
    spec, wl, fp, _ = case(name)
    b = W.rhs(spec)
    fG = W.feti_loads(fp)
    tot = np.zeros((wl.dd.n_gamma, b.shape[1]))
    for k, G in enumerate(fp.g_sets):
        tot[G] += fG[k]
    assert np.abs(tot - b[wl.dd.gamma_map]).max() <= 1e-14 * np.abs(b).max()


def test_constraint_matrix_rows_and_kernel():
    """Each row of B holds exactly one +1 and one -1 (section "Implementation");
    zeta(x,x) - 1 rows per interface dof (eq. constraintSpace); B u = 0 exactly
    when all copies of every dof agree; B_D B^T = I."""
    spec, wl, fp, fo = case("2d-const")
    B = fo.B.tocsr()
    assert np.all(np.diff(B.indptr) == 2)
    assert np.all(np.sort(B.data.reshape(-1, 2), axis=1) == [-1.0, 1.0])
    assert B.shape[0] == int((fp.zeta_nodes - 1).sum())
    rng = np.random.default_rng(7)
    ug = rng.integers(-50, 50, wl.dd.n_gamma).astype(float)
    uU = np.concatenate([ug[G] for G in fp.g_sets])
    assert np.abs(B @ uU).max() == 0.0
    uU[5] += 1.0
    assert np.abs(B @ uU).max() == 1.0
    assert abs(fo.BD @ B.T - sp.eye(B.shape[0])).max() <= 1e-13
    # the construction on a hand-made three-copy dof
    B3, offs, mult = constraint_matrix([np.array([0]), np.array([0, 1]), np.array([0])], 2)
    assert B3.toarray().tolist() == [[1, -1, 0, 0], [0, 1, 0, -1]] and mult.tolist() == [3, 1]


@pytest.mark.parametrize("name", ["1d", "2d-const", "2d-pd"])
def test_pinned_neumann_solve_is_the_pseudoinverse(name):
    """S_k^+ from the pinned Cholesky factor: S_k S_k^+ v = v on range(S_k),
    S_k^+ Z_k = 0, S_k^+ symmetric, and equal to the dense Moore-Penrose
    pseudoinverse (SVD, a library routine as a cross-check)."""
    spec, wl, fp, fo = case(name)
    rng = np.random.default_rng(11)
    for k in range(fo.K):
        if not fp.floating[k]:
            continue
        n = fp.g_sets[k].size
        S = np.column_stack([fo.schur_k(k, e) for e in np.eye(n)])
        Sp = np.column_stack([fo.schur_pinv_k(k, e) for e in np.eye(n)])
        assert np.abs(S @ fp.z[k]).max() <= 1e-11 * np.abs(S).max()
        ref = np.linalg.pinv(S, rcond=1e-12, hermitian=True)
        assert np.abs(Sp - ref).max() <= 1e-9 * np.abs(ref).max()
        assert np.abs(Sp - Sp.T).max() <= 1e-11 * np.abs(Sp).max()
        assert np.abs(Sp @ fp.z[k]).max() <= 1e-11 * np.abs(Sp).max()
        v = fo.project_kernel(k, rng.standard_normal(n))
        assert np.abs(S @ (Sp @ v) - v).max() <= 1e-10 * np.abs(v).max()


def test_initial_multiplier_meets_the_coarse_constraint():
    """lambda_0 = G (G^T G)^-1 e satisfies G^T lambda_0 = e (eq. FETIproblem),
    and P maps into ker G^T."""
    spec, wl, fp, fo = case("2d-pd")
    b = W.rhs(spec)
    f = fo.forcing(b, W.feti_loads(fp))[:, 0]
    e = fo.Z.T @ f
    import scipy.linalg as sla
    lam0 = fo.G @ sla.cho_solve(fo.GtG_fac, e)
    assert np.abs(fo.G.T @ lam0 - e).max() <= 1e-12 * np.abs(e).max()
    x = np.random.default_rng(3).standard_normal(fo.B.shape[0])
    assert np.abs(fo.G.T @ fo.P(x)).max() <= 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("name", list(CASES))
def test_feti_solution_equals_monolithic(name):
    spec, wl, fp, fo = case(name)
    b = W.rhs(spec)
    uref = oracle.monolithic_solve(wl.asm.A, b)
    u, its = fo.solve(b, W.feti_loads(fp), tol=1e-12)
    assert oracle.rel_err(u, uref).max() <= 1e-10
    assert its.max() < fo.B.shape[0]


def test_iterations_flat_at_fixed_delta_over_h():
    """Weak scaling at delta/h = 4 (section "Weak scaling for fixed delta/h"):
    from h = 1/32 on 2x2 subdomains to h = 1/64 on 4x4 the FETI iteration
    count stays nearly constant while diagonally preconditioned CG on the
    whole system about doubles -- the behaviour of Table fixedRatio (the
    counts themselves are not comparable: other h, delta and tolerance)."""
    its_f, its_j = [], []
    for n, cuts in ((32, (2, 2)), (64, (4, 4))):
        spec = W.spec_2d_const(n=n, delta=4.0 / n, cuts=cuts, nrhs=1)
        wl = W.build(spec)
        fp = W.feti_problem(wl)
        b = W.rhs(spec)
        u, its = FETIOracle(fp).solve(b, W.feti_loads(fp), tol=1e-10)
        assert oracle.full_residual(wl.asm.A, u, b).max() <= 1e-9
        its_f.append(int(its[0]))
        its_j.append(int(oracle.jacobi_pcg(wl.asm.A, b, tol=1e-10)[1][0]))
    assert its_f[1] <= 1.35 * its_f[0]
    assert its_j[1] >= 1.7 * its_j[0]
