"""One-level FETI (section "FETI", Algorithm 1) in plain FP64 numpy/scipy.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It shares no code with
the GPU path.

Input: a workloads.FetiProblem -- per subdomain k the blocks of the
subdomain stiffness matrix A^k (eq. subStiffnessMatrix, assembled with the
zeta-weighted form of eq. bilinear-multi1) on I_k u Gamma_k, whether
hat-Omega_k is floating, and a basis Z_k of the kernel of S_k on Gamma_k
(constants for scalar kernels, two translations and the rotation for
peridynamics).  The steps, in the order of Algorithm 1:

1. constraints B (signed Boolean, each row one +1 and one -1: consecutive
   copies of an interface dof must agree, zeta(x, x) - 1 rows per dof, the
   non-redundant count of eq. constraintSpace), the multiplicity scaling
   D^k_mm = zeta(x_m, x_m) and B_D = (B D^-1 B^T)^-1 B D^-1 (section
   "Preconditioning");
2. the subdomain forcing f_k of eq. subForcing from the zeta-weighted loads
   of eq. bilinear-multi5;
3. d = B S^+ f, e = Z^T f, G = B Z (eqs. FETIproblem, forU);
4. Cholesky factors: A^k itself when Gamma^D_k is non-empty, else A^k with
   pinned dofs (the rows and columns of the pins replaced by unit vectors,
   section "Pseudoinverse and Cholesky decomposition"); (G^T G);
5. F = B S^+ B^T, P = I - G (G^T G)^-1 G^T (eq. P), M^-1 = B_D S B_D^T
   (eq. preconditioner), all applied matrix-free;
6. lambda_0 = G (G^T G)^-1 e;
7. projected preconditioned CG on P F lambda = P d;
8. alpha = (G^T G)^-1 G^T (d - F lambda) (eq. forAlpha);
9. u = S^+ (f - B^T lambda) - Z alpha (eq. forU), then the interiors by eq.
   backwardSubstitution.

S_k^+ v (the Moore-Penrose inverse): the Neumann problem of eq.
neumannSubproblem with right-hand side (0, v) is solved with the pinned
factor; the interface part is then made orthogonal to ker S_k (for scalar
kernels: the mean is subtracted).  The argument of the section needs v to be
orthogonal to the kernel, so v is projected first: S^+ = P_Z S^+ P_Z.  For
several pins (peridynamics) the same argument holds when the kernel basis
restricted to the pinned dofs is non-singular, which decides the pins.

Readings (paper silent): the norm of the stopping rule -- the projected
residual ||P r||_2 relative to its initial value; the global interface value
after the solve -- the mean of the subdomain copies (they agree to the
tolerance).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def constraint_matrix(g_sets, n_gamma):
    """B over the stacked copies U = (Gamma_1, ..., Gamma_K): for every
    interface dof with copies in subdomains k_1 < k_2 < ... one row per
    consecutive pair, +1 on the copy in k_i and -1 on the copy in k_{i+1}."""
    offs = np.concatenate([[0], np.cumsum([g.size for g in g_sets])])
    copies = [[] for _ in range(n_gamma)]
    for k, G in enumerate(g_sets):
        for j, gi in enumerate(G):
            copies[gi].append(offs[k] + j)
    rows, cols, vals = [], [], []
    r = 0
    for cp in copies:
        for a, b in zip(cp[:-1], cp[1:]):
            rows += [r, r]
            cols += [a, b]
            vals += [1.0, -1.0]
            r += 1
    B = sp.csr_matrix((vals, (rows, cols)), shape=(r, offs[-1]))
    mult = np.array([len(cp) for cp in copies])
    return B, offs, mult


def choose_pins(Zg, nz):
    """Dofs of Gamma_k whose kernel rows are well conditioned: greedy pivoting
    over the rows of Z (largest remaining row norm, then orthogonalise the
    others against it)."""
    Z = np.array(Zg, dtype=np.float64, copy=True)
    pins = []
    for _ in range(nz):
        j = int(np.argmax(np.einsum("ij,ij->i", Z, Z)))
        pins.append(j)
        q = Z[j] / np.linalg.norm(Z[j])
        Z = Z - np.outer(Z @ q, q)
    return pins


class FETIOracle:
    def __init__(self, fp):
        self.fp = fp
        dd = fp.dd
        self.dd = dd
        self.K = len(fp.g_sets)
        self.B, self.offs, self.mult = constraint_matrix(fp.g_sets, dd.n_gamma)
        nU = self.offs[-1]
        # D^-1 on U: 1 / zeta(x, x) of every copy
        dinv = np.concatenate([1.0 / self.mult[G] for G in fp.g_sets])
        BDB = (self.B @ sp.diags(dinv) @ self.B.T).tocsc()
        # B_D = (B D^-1 B^T)^-1 B D^-1 (sparse solve of the block-diagonal system)
        self.BD = sp.csr_matrix(sp.linalg.spsolve(BDB, (self.B @ sp.diags(dinv)).tocsc()))
        self.nU = nU
        # subdomain matrices A^k (dense) and their factors
        self.L_ii, self.fac, self.pins = [], [], []
        for k in range(self.K):
            Kii = np.asarray(dd.kii[k])
            ni = Kii.shape[0]
            Ak = np.block([[Kii, fp.kig[k].toarray()], [fp.agi[k].toarray(), fp.agg[k].toarray()]])
            self.L_ii.append(np.linalg.cholesky(Kii))
            if fp.floating[k]:
                pins = [ni + j for j in choose_pins(fp.z[k], fp.z[k].shape[1])]
                At = Ak.copy()
                At[pins, :] = 0.0
                At[:, pins] = 0.0
                At[pins, pins] = 1.0
            else:
                pins, At = [], Ak
            self.pins.append(pins)
            self.fac.append(sla.cho_factor(At, lower=True))
        # orthonormal kernel bases on Gamma_k (for the projection of S^+)
        self.Q = [np.linalg.qr(fp.z[k])[0] if fp.z[k].shape[1] else None for k in range(self.K)]
        # G = B Z over the stacked kernel bases of the floating subdomains
        zcols = []
        for k in range(self.K):
            for m in range(fp.z[k].shape[1]):
                col = np.zeros(nU)
                col[self.offs[k]:self.offs[k + 1]] = fp.z[k][:, m]
                zcols.append(col)
        self.Z = np.array(zcols).T if zcols else np.zeros((nU, 0))
        self.G = self.B @ self.Z
        self.GtG = self.G.T @ self.G
        self.GtG_fac = sla.cho_factor(self.GtG, lower=True) if self.GtG.size else None

    # -- per subdomain pieces ---------------------------------------------------
    def sl(self, k):
        return slice(self.offs[k], self.offs[k + 1])

    def kii_solve(self, k, v):
        L = self.L_ii[k]
        return sla.solve_triangular(L.T, sla.solve_triangular(L, v, lower=True), lower=False)

    def schur_k(self, k, v):
        """S_k v = A^k_GG v - A^k_GI (A^k_II)^-1 A^k_IG v (eq. subSchurComplement)."""
        fp = self.fp
        return fp.agg[k] @ v - fp.agi[k] @ self.kii_solve(k, fp.kig[k] @ v)

    def project_kernel(self, k, v):
        Q = self.Q[k]
        return v if Q is None else v - Q @ (Q.T @ v)

    def schur_pinv_k(self, k, v):
        """S_k^+ v by the Neumann problem (eq. neumannSubproblem) with the
        pinned factor; the result orthogonal to ker S_k."""
        ni = self.dd.kii[k].shape[0]
        v = self.project_kernel(k, v)
        rhs = np.zeros((ni + v.shape[0],) + v.shape[1:])
        rhs[ni:] = v
        if self.pins[k]:
            rhs[self.pins[k]] = 0.0
        w = sla.cho_solve(self.fac[k], rhs)[ni:]
        return self.project_kernel(k, w)

    # -- operators on U and Lambda -------------------------------------------------
    def S(self, u):
        out = np.empty_like(u)
        for k in range(self.K):
            out[self.sl(k)] = self.schur_k(k, u[self.sl(k)])
        return out

    def S_pinv(self, u):
        out = np.empty_like(u)
        for k in range(self.K):
            out[self.sl(k)] = self.schur_pinv_k(k, u[self.sl(k)])
        return out

    def F(self, lam):
        return self.B @ self.S_pinv(self.B.T @ lam)

    def Minv(self, lam):
        return self.BD @ self.S(self.BD.T @ lam)

    def P(self, lam):
        if self.G.shape[1] == 0:
            return lam
        return lam - self.G @ sla.cho_solve(self.GtG_fac, self.G.T @ lam)

    def forcing(self, b, fG=None):
        """f = (f_k): eq. subForcing per subdomain with the loads f~ of eq.
        bilinear-multi5 (interface part fG per subdomain from
        workloads.feti_loads; interiors b_I^k)."""
        dd, fp = self.dd, self.fp
        b = np.asarray(b, dtype=np.float64).reshape(dd.n_dof, -1)
        f = np.zeros((self.nU, b.shape[1]))
        for k in range(self.K):
            fI = b[dd.i_maps[k]]
            f[self.sl(k)] = fG[k] - fp.agi[k] @ self.kii_solve(k, fI)
        return f

    # -- Algorithm 1 -----------------------------------------------------------------
    def solve(self, b, fG, tol=1e-10, max_it=1000):
        """Returns (u (n_dof x nrhs), iterations per column)."""
        dd = self.dd
        b = np.asarray(b, dtype=np.float64).reshape(dd.n_dof, -1)
        f = self.forcing(b, fG)
        u_all = np.zeros_like(b)
        its = []
        for c in range(b.shape[1]):
            fc = f[:, c]
            d = self.F_rhs(fc)
            e = self.Z.T @ fc
            lam = self.G @ sla.cho_solve(self.GtG_fac, e) if self.G.shape[1] else np.zeros(d.shape)
            r = d - self.F(lam)
            w = self.P(r)
            w0 = np.linalg.norm(w)
            p = None
            wy_old = None
            it = 0
            while np.linalg.norm(w) > tol * w0 and it < max_it:
                y = self.P(self.Minv(w))
                wy = w @ y
                p = y if p is None else y + (wy / wy_old) * p
                q = self.F(p)
                pq = p @ q
                if pq <= 0.0:
                    raise ArithmeticError("p^T F p <= 0")
                a = wy / pq
                lam = lam + a * p
                r = r - a * q
                w = self.P(r)
                wy_old = wy
                it += 1
            its.append(it)
            # eq. forAlpha, eq. forU
            alpha = sla.cho_solve(self.GtG_fac, self.G.T @ (d - self.F(lam))) if self.G.shape[1] else None
            uU = self.S_pinv(fc - self.B.T @ lam)
            if alpha is not None:
                uU = uU - self.Z @ alpha
            u_all[:, c] = self.assemble(b[:, c], uU)
        return u_all, np.array(its)

    def F_rhs(self, f):
        return self.B @ self.S_pinv(f)

    def assemble(self, b, uU):
        """Global solution: interface dofs the mean of their copies, interiors
        by eq. backwardSubstitution from each subdomain's own copy."""
        dd, fp = self.dd, self.fp
        u = np.zeros(dd.n_dof)
        acc = np.zeros(dd.n_gamma)
        for k in range(self.K):
            acc[fp.g_sets[k]] += uU[self.sl(k)]
        u[dd.gamma_map] = acc / self.mult
        for k in range(self.K):
            u[dd.i_maps[k]] = self.kii_solve(k, b[dd.i_maps[k]] - fp.kig[k] @ uU[self.sl(k)])
        return u
