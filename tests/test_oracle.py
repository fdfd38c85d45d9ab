"""Pins of the CPU FP64 oracle against the definitions it follows: explicit
dense Schur complements and inverses on small systems, monolithic solves,
CG termination, DD-vs-monolithic agreement.  CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W

CASES = {
    "1d": lambda: W.spec_1d(n=128, strips=4, nrhs=2),
    "2d-const": lambda: W.spec_2d_const(n=24, delta=0.15, cuts=(2, 2), nrhs=2),
    "2d-frac": lambda: W.spec_2d_frac(n=24, delta=0.15, cuts=(3, 2), nrhs=2),
    "2d-pd": lambda: W.spec_2d_pd(n=20, delta=0.15, cuts=(2, 2), jitter=0.0, nrhs=2),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    spec = CASES[request.param]()
    wl = W.build(spec)
    b = W.rhs(spec)
    return wl, b


def dense_blocks(wl):
    """Full matrix in (interior..., interface) order and the index sets."""
    dd = wl.dd
    A = wl.asm.A.toarray()
    I = np.concatenate(dd.i_maps)
    G = dd.gamma_map
    return A, I, G


def test_monolithic_matches_dense_solve(case):
    wl, b = case
    A = wl.asm.A.toarray()
    u = oracle.monolithic_solve(wl.asm.A, b)
    ref = np.linalg.solve(A, b)
    assert oracle.rel_err(u, ref).max() <= 1e-12


def test_schur_apply_matches_explicit_schur_complement(case):
    """S = A_GG - A_GI A_II^{-1} A_IG formed densely (eq. subSchurComplement
    with the block-diagonal A_II) against the matrix-free operator."""
    wl, _ = case
    A, I, G = dense_blocks(wl)
    S = A[np.ix_(G, G)] - A[np.ix_(G, I)] @ np.linalg.solve(A[np.ix_(I, I)], A[np.ix_(I, G)])
    orc = oracle.DDOracle(wl.dd)
    rng = np.random.default_rng(11)
    P = rng.standard_normal((len(G), 3))
    Q = orc.schur_apply(P)
    assert np.abs(Q - S @ P).max() <= 1e-12 * np.abs(S).max() * np.abs(P).max() * len(G) ** 0.5
    # symmetric operator
    v, w = P[:, 0], P[:, 1]
    assert abs(v @ orc.schur_apply(w) - w @ orc.schur_apply(v)) <= 1e-12 * np.abs(S).max() * len(G)
    # exact diagonal used as preconditioner
    assert np.allclose(orc.schur_diag(), np.diag(S), rtol=1e-12, atol=0)
    # positive definite (the global A is)
    assert np.linalg.eigvalsh(S).min() > 0


def test_condensation_and_back_substitution(case):
    """g = b_G - A_GI A_II^{-1} b_I (eq. subForcing summed) and
    u_I = A_II^{-1}(b_I - A_IG u_G) (eq. backwardSubstitution) reproduce the
    monolithic solution when u_G is exact."""
    wl, b = case
    A, I, G = dense_blocks(wl)
    orc = oracle.DDOracle(wl.dd)
    g_ref = b[G] - A[np.ix_(G, I)] @ np.linalg.solve(A[np.ix_(I, I)], b[I])
    g = orc.condense(b)
    assert np.abs(g - g_ref).max() <= 1e-12 * np.abs(g_ref).max()
    u = np.linalg.solve(A, b)
    u2 = orc.back_substitute(b, u[G])
    assert oracle.rel_err(u2, u).max() <= 1e-12


def test_cholesky_factor(case):
    wl, _ = case
    for K in wl.dd.kii:
        L = oracle.cholesky(K)
        assert np.allclose(np.triu(L, 1), 0)
        assert np.abs(L @ L.T - K).max() <= 1e-14 * K.shape[0] * np.abs(K).max()


def test_dd_solution_matches_monolithic(case):
    wl, b = case
    u_ref = oracle.monolithic_solve(wl.asm.A, b)
    orc = oracle.DDOracle(wl.dd)
    u, its, conv = orc.solve(b, tol=1e-14)
    assert conv.all()
    assert oracle.rel_err(u, u_ref).max() <= 1e-11
    # CG on an SPD n_G x n_G system terminates within n_G steps (in exact arithmetic)
    assert its.max() <= wl.dd.n_gamma
    assert oracle.full_residual(wl.asm.A, u, b).max() <= 1e-13


def test_unpreconditioned_cg_also_converges(case):
    wl, b = case
    u_ref = oracle.monolithic_solve(wl.asm.A, b)
    orc = oracle.DDOracle(wl.dd)
    u, its, conv = orc.solve(b, tol=1e-13, precond=False, max_it=20000)
    assert conv.all()
    assert oracle.rel_err(u, u_ref).max() <= 1e-9
    _, its_p, _ = orc.solve(b, tol=1e-13)
    assert its_p.max() <= its.max()


def test_stopping_rule_is_relative_full_residual():
    """The CG stops on ||r_G|| <= tol ||b||; after back substitution the full
    residual ||b - A u|| equals ||r_G||, so the reported relative residual is
    at most tol (up to rounding)."""
    spec = W.spec_2d_const(n=24, delta=0.15, cuts=(2, 2), nrhs=3)
    wl = W.build(spec)
    b = W.rhs(spec)
    orc = oracle.DDOracle(wl.dd)
    for tol in (1e-6, 1e-9):
        u, its, conv = orc.solve(b, tol=tol)
        assert conv.all()
        assert oracle.full_residual(wl.asm.A, u, b).max() <= tol * 1.01


def test_zero_rhs_column():
    spec = W.spec_1d(n=64, strips=2)
    wl = W.build(spec)
    b = np.zeros((wl.dd.n_dof, 2))
    b[:, 1] = W.rhs(spec)[:, 0]
    u, its, conv = oracle.DDOracle(wl.dd).solve(b, tol=1e-12)
    assert conv.all() and its[0] == 0 and np.all(u[:, 0] == 0)


def test_multi_rhs_columns_independent():
    spec = W.spec_2d_const(n=24, delta=0.15, cuts=(2, 2), nrhs=3)
    wl = W.build(spec)
    b = W.rhs(spec)
    orc = oracle.DDOracle(wl.dd)
    U, its, _ = orc.solve(b, tol=1e-12)
    for j in range(3):
        u, it, _ = orc.solve(b[:, j:j + 1], tol=1e-12)
        assert it[0] == its[j]
        assert np.abs(u[:, 0] - U[:, j]).max() <= 1e-14 * np.abs(U[:, j]).max()


# ------------------------------------------------ baseline: Jacobi-PCG on A --
def test_jacobi_pcg_first_iterates_worked_by_hand():
    """A = [[4, 1], [1, 3]], b = [1, 2], D = diag(4, 3), x0 = 0, by hand:
    z0 = p0 = [1/4, 2/3], r0.z0 = 19/12, A p0 = [5/3, 9/4], p0.A p0 = 23/12,
    alpha0 = 19/23, x1 = [19/92, 38/69]; CG ends after n = 2 steps at
    A^{-1} b = [1/11, 7/11]."""
    import scipy.sparse as sp
    A = sp.csr_matrix(np.array([[4.0, 1.0], [1.0, 3.0]]))
    b = np.array([1.0, 2.0])
    x1, its, _ = oracle.jacobi_pcg(A, b, tol=1e-300, max_it=1)
    assert its[0] == 1
    assert np.allclose(x1, [19 / 92, 38 / 69], rtol=1e-15, atol=0)
    x2, its, _ = oracle.jacobi_pcg(A, b, tol=1e-300, max_it=2)
    assert np.allclose(x2, [1 / 11, 7 / 11], rtol=4e-16, atol=0)
    _, its, conv = oracle.jacobi_pcg(A, b, tol=1e-14)
    assert conv[0] and its[0] == 2


def test_jacobi_pcg_diagonal_system_one_step():
    """With A diagonal the preconditioned residual is the exact solution:
    one step, x = b / diag(A)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(7)
    d = rng.uniform(0.5, 3.0, 50)
    b = rng.uniform(-1, 1, (50, 2))
    x, its, conv = oracle.jacobi_pcg(sp.diags(d).tocsr(), b, tol=1e-14)
    assert conv.all() and np.all(its == 1)
    assert np.abs(x - b / d[:, None]).max() <= 1e-15 * np.abs(b / d[:, None]).max()


def test_jacobi_pcg_matches_monolithic(case):
    """kappa(A) is a few hundred on these systems, so a 1e-13 relative
    residual bounds the error by about 1e-10; CG ends within n steps."""
    wl, b = case
    A = wl.asm.A
    x, its, conv = oracle.jacobi_pcg(A, b, tol=1e-13)
    uref = oracle.monolithic_solve(A, b)
    assert conv.all() and np.all(its <= A.shape[0])
    assert oracle.rel_err(x, uref).max() <= 1e-9
    assert oracle.full_residual(A, x, b).max() <= 1e-12


def test_undecomposed_dd_is_jacobi_pcg(case):
    """With no subdomains the interface Schur complement is A and its exact
    diagonal is diag(A): the substructuring oracle and the plain Jacobi-PCG
    (no shared code) take the same iterations to the same iterate."""
    wl, b = case
    A = wl.asm.A
    und = W.undecomposed(A)
    assert und.n_sub == 0 and und.n_gamma == A.shape[0]
    orc = oracle.DDOracle(und)
    assert np.array_equal(orc.schur_diag(), A.diagonal())
    u0, it0, c0 = orc.solve(b, tol=1e-11)
    x, its, conv = oracle.jacobi_pcg(A, b, tol=1e-11)
    assert c0.all() and conv.all() and np.array_equal(it0, its)
    assert oracle.rel_err(u0, x).max() <= 1e-12
