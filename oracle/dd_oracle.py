"""FP64 reference computations (test infrastructure only; see package doc)."""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def rel_err(u: np.ndarray, uref: np.ndarray) -> np.ndarray:
    """Per-column ||u - uref||_2 / ||uref||_2."""
    u = np.asarray(u).reshape(uref.shape[0], -1)
    uref = np.asarray(uref).reshape(uref.shape[0], -1)
    return np.linalg.norm(u - uref, axis=0) / np.linalg.norm(uref, axis=0)


def full_residual(A: sp.spmatrix, u: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per-column ||b - A u||_2 / ||b||_2 (the system of the section
    "A discretized weak formulation", homogeneous Dirichlet data)."""
    b = np.asarray(b).reshape(A.shape[0], -1)
    u = np.asarray(u).reshape(A.shape[0], -1)
    return np.linalg.norm(b - A @ u, axis=0) / np.linalg.norm(b, axis=0)


def monolithic_solve(A: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    """u* = A^{-1} b by Cholesky of the banded matrix A (natural order).

    A is symmetric positive definite (stated after the definition of the
    discrete system); entries outside the band of a banded SPD matrix never
    fill, so the banded factorisation performs the dense algorithm's nonzero
    operations."""
    A = sp.tril(A.tocsr()).tocoo()
    n = A.shape[0]
    bw = int((A.row - A.col).max())
    ab = np.zeros((bw + 1, n), dtype=np.float64)
    ab[A.row - A.col, A.col] = A.data
    cb = sla.cholesky_banded(ab, lower=True, overwrite_ab=True, check_finite=False)
    b2 = np.asarray(b, dtype=np.float64).reshape(n, -1)
    x = sla.cho_solve_banded((cb, True), b2, check_finite=False)
    return x.reshape(np.asarray(b).shape)


def jacobi_pcg(A: sp.spmatrix, b: np.ndarray, tol: float = 1e-10, max_it: int = 100000):
    """Conjugate gradients on the whole system A u = b with the diagonal of A
    as preconditioner: the baseline solver of the paper's experiments (section
    "Considered solver strategies"; the rows are not split into subdomains).

    x0 = 0; column c stops when ||b_c - A x_c||_2 (recurrence residual) <=
    tol * ||b_c||_2, every column an independent CG.  Returns (x, iterations,
    converged)."""
    A = A.tocsr()
    b2 = np.asarray(b, dtype=np.float64).reshape(A.shape[0], -1)
    n, m = b2.shape
    dinv = 1.0 / A.diagonal()
    x = np.zeros((n, m))
    its = np.zeros(m, dtype=np.int64)
    conv = np.zeros(m, dtype=bool)
    for c in range(m):
        r = b2[:, c].copy()
        stop = tol * np.linalg.norm(b2[:, c])
        z = dinv * r
        p = z.copy()
        rz = r @ z
        it = 0
        while np.linalg.norm(r) > stop and it < max_it:
            q = A @ p
            pq = p @ q
            if pq <= 0.0:
                raise ArithmeticError("p^T A p <= 0: A not positive definite")
            alpha = rz / pq
            x[:, c] += alpha * p
            r -= alpha * q
            it += 1
            z = dinv * r
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        its[c] = it
        conv[c] = np.linalg.norm(r) <= stop
    return x.reshape(np.asarray(b).shape), its, conv


def cholesky(K: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor L with K = L L^T (LAPACK potrf as one step)."""
    return np.linalg.cholesky(np.asarray(K, dtype=np.float64))


class DDOracle:
    """Primal substructuring on the interface Schur complement.

    ``dd`` is a workloads.DDProblem: per subdomain K_II^k (dense), K_IG^k
    (CSR over local interface columns), maps i_map (interior local -> global
    dof) and g_map (local interface column -> interface index), and the
    global K_GG with gamma_map (interface index -> global dof)."""

    def __init__(self, dd):
        self.dd = dd
        # eq. splittingBlockCholesky: A^k_{Omega Omega} is non-singular for
        # every subdomain (also floating ones), so its Cholesky factor exists.
        self.L = [cholesky(K) for K in dd.kii]
        self.kgi = [K.T.tocsr() for K in dd.kig]
        self._dinv = None

    # -- K_II^{-1} through the factor: two triangular solves ---------------
    def kii_solve(self, k: int, v: np.ndarray) -> np.ndarray:
        L = self.L[k]
        w = sla.solve_triangular(L, v, lower=True, check_finite=False)
        return sla.solve_triangular(L.T, w, lower=False, check_finite=False)

    # -- S applied matrix-free (eq. subSchurComplement summed over k) ------
    def schur_apply(self, p: np.ndarray) -> np.ndarray:
        dd = self.dd
        p2 = np.asarray(p, dtype=np.float64).reshape(dd.n_gamma, -1)
        q = dd.kgg @ p2
        for k in range(dd.n_sub):
            pk = p2[dd.g_maps[k]]                       # R_k p
            yk = dd.kig[k] @ pk                         # K_IG^k R_k p
            zk = self.kii_solve(k, yk)                  # (K_II^k)^{-1} ...
            np.subtract.at(q, dd.g_maps[k], self.kgi[k] @ zk)   # - R_k^T K_GI^k ...
        return q.reshape(np.asarray(p).shape)

    # -- exact diagonal of S (Jacobi preconditioner) ------------------------
    def schur_diag(self) -> np.ndarray:
        """diag(S)_j = (K_GG)_jj - sum_k || L_k^{-1} K_IG^k e_j ||^2."""
        if self._dinv is None:
            dd = self.dd
            d = dd.kgg.diagonal().copy()
            for k in range(dd.n_sub):
                W = sla.solve_triangular(self.L[k], dd.kig[k].toarray(), lower=True,
                                         check_finite=False)
                np.subtract.at(d, dd.g_maps[k], (W * W).sum(axis=0))
            self._dinv = d
        return self._dinv

    # -- eq. subForcing, summed over subdomains -----------------------------
    def condense(self, b: np.ndarray) -> np.ndarray:
        dd = self.dd
        b2 = np.asarray(b, dtype=np.float64).reshape(dd.n_dof, -1)
        g = b2[dd.gamma_map].copy()
        for k in range(dd.n_sub):
            zk = self.kii_solve(k, b2[dd.i_maps[k]])
            np.subtract.at(g, dd.g_maps[k], self.kgi[k] @ zk)
        return g

    # -- eq. backwardSubstitution -------------------------------------------
    def back_substitute(self, b: np.ndarray, uG: np.ndarray) -> np.ndarray:
        dd = self.dd
        b2 = np.asarray(b, dtype=np.float64).reshape(dd.n_dof, -1)
        uG = uG.reshape(dd.n_gamma, -1)
        u = np.zeros_like(b2)
        u[dd.gamma_map] = uG
        for k in range(dd.n_sub):
            rhs = b2[dd.i_maps[k]] - dd.kig[k] @ uG[dd.g_maps[k]]
            u[dd.i_maps[k]] = self.kii_solve(k, rhs)
        return u

    # -- preconditioned CG, one independent CG per column --------------------
    def pcg(self, g: np.ndarray, stop: np.ndarray, tol: float, max_it: int,
            precond: bool = True):
        """Solve S x = g column by column.  Column c stops when
        ||r_c||_2 <= tol * stop[c].  Returns (x, iterations, converged)."""
        n, m = g.shape
        dinv = 1.0 / self.schur_diag() if precond else np.ones(n)
        x = np.zeros((n, m))
        r = g.copy()
        z = dinv[:, None] * r
        p = z.copy()
        rz = np.einsum("ij,ij->j", r, z)
        its = np.zeros(m, dtype=np.int64)
        done = np.linalg.norm(r, axis=0) <= tol * stop
        for it in range(1, max_it + 1):
            if done.all():
                break
            act = ~done
            q = self.schur_apply(p[:, act])
            pq = np.einsum("ij,ij->j", p[:, act], q)
            if np.any(pq <= 0.0):
                raise ArithmeticError("p^T S p <= 0: S not positive definite")
            alpha = rz[act] / pq
            x[:, act] += alpha * p[:, act]
            r[:, act] -= alpha * q
            its[act] = it
            now = np.linalg.norm(r[:, act], axis=0) <= tol * stop[act]
            idx = np.nonzero(act)[0]
            done[idx[now]] = True
            z[:, act] = dinv[:, None] * r[:, act]
            rz_new = np.einsum("ij,ij->j", r[:, act], z[:, act])
            beta = rz_new / rz[act]
            rz[act] = rz_new
            p[:, act] = z[:, act] + beta * p[:, act]
        return x, its, done

    def solve(self, b: np.ndarray, tol: float = 1e-10, max_it: int = 5000,
              precond: bool = True):
        """Full substructuring solve: condensation, PCG, back substitution."""
        b2 = np.asarray(b, dtype=np.float64).reshape(self.dd.n_dof, -1)
        g = self.condense(b2)
        stop = np.linalg.norm(b2, axis=0)
        xG, its, conv = self.pcg(g, stop, tol, max_it, precond)
        u = self.back_substitute(b2, xG)
        return u.reshape(np.asarray(b).shape), its, conv
