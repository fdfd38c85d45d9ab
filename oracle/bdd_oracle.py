"""Balancing Neumann-Neumann preconditioner for the primal interface problem.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It shares no code with
the GPU path.

The paper preconditions its dual problem with the scaled Dirichlet operator
B_D S B_D^T (eq. preconditioner, section "Preconditioning").  The primal
interface problem S u_G = g (the Schur complement of eq. SchurComplement,
summed over subdomains) has the mirror image: the Neumann-Neumann operator

    M_NN = sum_k R_k^T D_k S_k^+ D_k R_k,

with R_k the restriction to Gamma_k, D_k the diagonal of 1 / zeta(x_m, x_m)
(the multiplicity scaling D of the paper, inverted: sum_k R_k^T D_k R_k = I)
and S_k^+ the pseudoinverse of the zeta-weighted subdomain Schur complement
(eq. subSchurComplement), by pinned Neumann solves (section "Pseudoinverse and
Cholesky decomposition", the same S_k^+ as in the FETI oracle).  Floating
subdomains make S_k singular; the balancing coarse space of Mandel (1993),

    N = [R_k^T D_k Z_k] over the floating subdomains,  S_0 = N^T S N,
    P_0 = N S_0^-1 N^T,
    M^-1 = P_0 + (I - P_0 S) M_NN (I - S P_0),

hands M_NN only residuals orthogonal to every D_k Z_k, so each S_k^+ sees a
right-hand side in the range of S_k.  The PCG, the stopping rule, the
condensation and the back substitution are those of DDOracle; only the
preconditioner differs.  (This is the primal counterpart named in the
paper's discussion of preconditioners; the paper itself does not build it.)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .dd_oracle import DDOracle
from .feti_oracle import FETIOracle


class BDDOracle:
    def __init__(self, fp):
        self.fp = fp
        self.dd = fp.dd
        self.ddo = DDOracle(fp.dd)
        self.fo = FETIOracle(fp)
        nG = self.dd.n_gamma
        self.mult = self.fo.mult.astype(np.float64)          # zeta(x, x) per interface dof
        cols = []
        for k, G in enumerate(fp.g_sets):
            if not fp.floating[k]:
                continue
            Z = np.asarray(fp.z[k], dtype=np.float64)
            for m in range(Z.shape[1]):
                c = np.zeros(nG)
                c[G] = Z[:, m] / self.mult[G]
                cols.append(c)
        self.N = np.array(cols).T if cols else np.zeros((nG, 0))
        self.SN = self.ddo.schur_apply(self.N) if self.N.shape[1] else self.N
        self.S0 = self.N.T @ self.SN
        self.S0_fac = sla.cho_factor(self.S0, lower=True) if self.S0.size else None

    # -- pieces ------------------------------------------------------------------
    def partition_of_unity(self) -> np.ndarray:
        """sum_k R_k^T D_k R_k as a vector (its diagonal; it is diagonal)."""
        d = np.zeros(self.dd.n_gamma)
        for G in self.fp.g_sets:
            d[G] += 1.0 / self.mult[G]
        return d

    def nn(self, r: np.ndarray) -> np.ndarray:
        """M_NN r = sum_k R_k^T D_k S_k^+ D_k R_k r."""
        out = np.zeros_like(r)
        for k, G in enumerate(self.fp.g_sets):
            v = r[G] / self.mult[G][:, None] if r.ndim == 2 else r[G] / self.mult[G]
            w = self.fo.schur_pinv_k(k, v)
            out[G] += w / self.mult[G][:, None] if r.ndim == 2 else w / self.mult[G]
        return out

    def coarse(self, r: np.ndarray) -> np.ndarray:
        """P_0 r = N S_0^-1 N^T r."""
        if self.N.shape[1] == 0:
            return np.zeros_like(r)
        return self.N @ sla.cho_solve(self.S0_fac, self.N.T @ r)

    def balance(self, r: np.ndarray) -> np.ndarray:
        """(I - S P_0) r: orthogonal to the columns of N."""
        if self.N.shape[1] == 0:
            return r
        return r - self.SN @ sla.cho_solve(self.S0_fac, self.N.T @ r)

    def precond(self, r: np.ndarray) -> np.ndarray:
        """M^-1 r = P_0 r + (I - P_0 S) M_NN (I - S P_0) r."""
        u = self.nn(self.balance(r))
        if self.N.shape[1] == 0:
            return u
        return self.coarse(r) + u - self.N @ sla.cho_solve(self.S0_fac, self.SN.T @ u)

    # -- preconditioned CG (DDOracle's, with M^-1 in place of diag(S)^-1) --------
    def pcg(self, g: np.ndarray, stop: np.ndarray, tol: float, max_it: int):
        n, m = g.shape
        x = np.zeros((n, m))
        its = np.zeros(m, dtype=np.int64)
        done = np.zeros(m, dtype=bool)
        for c in range(m):
            r = g[:, c].copy()
            if np.linalg.norm(r) <= tol * stop[c]:
                done[c] = True
                continue
            z = self.precond(r)
            p = z.copy()
            rz = r @ z
            for it in range(1, max_it + 1):
                q = self.ddo.schur_apply(p)
                pq = p @ q
                if pq <= 0.0:
                    raise ArithmeticError("p^T S p <= 0")
                a = rz / pq
                x[:, c] += a * p
                r -= a * q
                its[c] = it
                if np.linalg.norm(r) <= tol * stop[c]:
                    done[c] = True
                    break
                z = self.precond(r)
                rz_new = r @ z
                p = z + (rz_new / rz) * p
                rz = rz_new
        return x, its, done

    def solve(self, b: np.ndarray, tol: float = 1e-10, max_it: int = 1000):
        """Condensation, BDD-preconditioned CG on S u_G = g, back substitution."""
        b2 = np.asarray(b, dtype=np.float64).reshape(self.dd.n_dof, -1)
        g = self.ddo.condense(b2)
        stop = np.linalg.norm(b2, axis=0)
        xG, its, conv = self.pcg(g, stop, tol, max_it)
        u = self.ddo.back_substitute(b2, xG)
        return u.reshape(np.asarray(b).shape), its, conv
