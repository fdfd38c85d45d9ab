"""Seeded synthetic problem generator for the substructuring solver.

This module builds the linear systems the solver is run on: structured P1
meshes of the unit interval / unit square with a Dirichlet collar, the
nonlocal stiffness matrix (assembled in ``nlasm.c``), the overlapping
subdomain decomposition, the algebraic interior/interface split, and the
seeded right-hand sides.  It is shared by the CPU oracle (tests) and by the
GPU path (tests, bench); it contains none of the solver's arithmetic --
no factorisation, no Schur complement products, no Krylov iteration.

Paper passages followed (arXiv:2306.00094):
  * kernels: eqs. scalarkernel, vectorkernel; experiment kernels
    eqs. constantkernel, fractionalkernel, peridynamics;
  * bilinear form and load: eq. bil1 (A(u,v) and F(v));
  * FE grids, free / Dirichlet index sets I and B: section "A discretized weak
    formulation" (the system  A u = f - B g);
  * nonlocal subdivision: Definition nonlocalsubdivision, eq. subRequirement,
    derived sets eq. subdomainDefinitions;
  * construction of the overlapping subdomains by a delta/2 neighbourhood of
    a non-overlapping rectangle decomposition with the exact inf-distance
    criterion: section "Building substructures";
  * interior / interface index sets I_k, G_k and the block split of the
    subdomain stiffness: eqs. subStiffnessMatrix, subStiffnessMatrixSubBlocks.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_nlasm.so")
_lib = None

KER_CONST, KER_FRAC, KER_PD = 0, 1, 2


def build_native(force: bool = True) -> str:
    """Compile the assembler (plain C, OpenMP) into workloads/_nlasm.so."""
    src = os.path.join(_HERE, "nlasm.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp",
                               "-std=c99", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_native(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.nl_assemble_1d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int, dp]
        lib.nl_assemble_1d.restype = ctypes.c_int
        lib.nl_assemble_2d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, dp]
        lib.nl_assemble_2d.restype = ctypes.c_int
        u64p = ctypes.POINTER(ctypes.c_uint64)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.nl_assemble_1d_sub.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_int, u64p, ctypes.c_int, ip, ip, dp]
        lib.nl_assemble_1d_sub.restype = ctypes.c_int
        lib.nl_assemble_2d_sub.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                           u64p, ctypes.c_int, ip, ip, dp]
        lib.nl_assemble_2d_sub.restype = ctypes.c_int
        _lib = lib
    return _lib


def _nthreads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------
# Seeded random numbers: SplitMix64 (Steele, Lea & Flood, 2014).
# --------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """n doubles uniform on [-1, 1): state += golden gamma, mix, top 53 bits."""
    out = np.empty(n, dtype=np.float64)
    state = seed & _M64
    for i in range(n):
        state = (state + 0x9E3779B97F4A7C15) & _M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        z = z ^ (z >> 31)
        out[i] = 2.0 * ((z >> 11) * (1.0 / 9007199254740992.0)) - 1.0
    return out


def splitmix64_uniform_fast(seed: int, n: int) -> np.ndarray:
    """Vectorised SplitMix64 stream, bit-identical to splitmix64_uniform."""
    with np.errstate(over="ignore"):
        idx = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & _M64) + idx * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return 2.0 * ((z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)) - 1.0


# --------------------------------------------------------------------------
# Problem specifications (the paper's experiment shapes, scaled to one GPU).
# --------------------------------------------------------------------------
@dataclass
class Spec:
    name: str
    dim: int
    n: int                 # cells per side inside (0,1)
    delta: float
    kernel: int
    phi: float             # kernel constant
    s: float = 0.0         # fractional order
    cuts: tuple = (4, 1)   # subdomain grid (kx, ky); 1D uses kx strips
    jitter: float = 0.0    # relative width jitter of the cuts
    jitter_seeds: tuple = (0, 0)
    nrhs: int = 1
    seed_base: int = 0
    ncomp: int = 1         # dofs per node

    @property
    def h(self) -> float:
        return 1.0 / self.n

    @property
    def collar(self) -> int:
        return int(math.ceil(self.delta / self.h)) + 1


def spec_1d(n=1024, delta=0.05, strips=4, nrhs=1, seed_base=1000) -> Spec:
    """1D constant kernel 3/(2 delta^3) on |x-y| <= delta (scaled so that the
    nonlocal operator of a quadratic equals -u'')."""
    return Spec("1d-const", 1, n, delta, KER_CONST, 3.0 / (2.0 * delta ** 3),
                cuts=(strips, 1), nrhs=nrhs, seed_base=seed_base)


def spec_2d_const(n=128, delta=0.1, cuts=(4, 4), nrhs=1, seed_base=2000) -> Spec:
    """2D constant kernel 4/(pi delta^4) on the Euclidean ball (barycentre
    pair truncation); the scaling makes the operator of a quadratic -Laplace."""
    return Spec("2d-const", 2, n, delta, KER_CONST, 4.0 / (math.pi * delta ** 4),
                cuts=cuts, nrhs=nrhs, seed_base=seed_base)


def spec_2d_frac(n=96, delta=0.1, s=0.5, cuts=(4, 4), nrhs=8, seed_base=3000) -> Spec:
    """2D fractional-type kernel (2-2s)/(pi delta^(2-2s)) |x-y|^-(2+2s) on the
    Euclidean ball (eq. fractionalkernel), finite horizon delta."""
    return Spec("2d-frac", 2, n, delta, KER_FRAC,
                (2.0 - 2.0 * s) / (math.pi * delta ** (2.0 - 2.0 * s)), s=s,
                cuts=cuts, nrhs=nrhs, seed_base=seed_base)


def spec_2d_pd(n=160, delta=0.05, cuts=(8, 8), jitter=0.3, nrhs=32, seed_base=4000) -> Spec:
    """2D bond-based peridynamics, Phi = 3/delta^3 (x-y)(x)(x-y)/|x-y|^3
    (eq. peridynamics), 2 dofs per node, jittered tensor-grid cuts."""
    return Spec("2d-pd", 2, n, delta, KER_PD, 3.0 / delta ** 3, cuts=cuts,
                jitter=jitter, jitter_seeds=(4000, 4001), nrhs=nrhs,
                seed_base=seed_base, ncomp=2)


SPECS = {
    "cfg1": spec_1d,
    "cfg2": spec_2d_const,
    "cfg3": spec_2d_frac,
    "cfg4": spec_2d_pd,
}


# --------------------------------------------------------------------------
# Assembly
# --------------------------------------------------------------------------
@dataclass
class Assembled:
    spec: Spec
    A: sp.csr_matrix          # free x free (SPD), dofs node-major, comps inner
    Bd: sp.csr_matrix         # free x Dirichlet-node dofs (the coupling to g)
    coords: np.ndarray        # free node coordinates (n_free_nodes x dim)
    dir_coords: np.ndarray    # Dirichlet node coordinates
    window_R: int


def _window_to_csr(spec: Spec, win: np.ndarray, R: int):
    """Turn per-row windows into CSR over (free dofs) x (all nodes' dofs)."""
    n, c = spec.n, spec.collar
    N = n + 2 * c
    W = 2 * R + 1
    nc = spec.ncomp
    if spec.dim == 1:
        nfree = n - 1
        am = c + 1 + np.arange(nfree)
        da = np.arange(-R, R + 1)
        cols_node = am[:, None] + da[None, :]                 # extended node ids
        vals = win.reshape(nfree, W)
        rows = np.repeat(np.arange(nfree), W)
        cols = cols_node.reshape(-1)
        v = vals.reshape(-1)
        nodes_total = N + 1
        # free node id of extended node a (or -1)
        ext_to_free = np.full(nodes_total, -1, dtype=np.int64)
        ext_to_free[c + 1:c + n] = np.arange(nfree)
        coords_all = ((np.arange(nodes_total) - c) / n)[:, None]
    else:
        nfree = (n - 1) * (n - 1)
        ia = np.arange(nfree) % (n - 1)
        ib = np.arange(nfree) // (n - 1)
        am = c + 1 + ia
        bm = c + 1 + ib
        dd = np.arange(-R, R + 1)
        DB, DA = np.meshgrid(dd, dd, indexing="ij")            # window (db, da)
        na = am[:, None] + DA.reshape(-1)[None, :]
        nb = bm[:, None] + DB.reshape(-1)[None, :]
        ext = nb * (N + 1) + na
        nodes_total = (N + 1) * (N + 1)
        ext_to_free = np.full(nodes_total, -1, dtype=np.int64)
        ga, gb = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="xy")
        free_mask = (ga > c) & (ga < c + n) & (gb > c) & (gb < c + n)
        fa = ga[free_mask]
        fb = gb[free_mask]
        ext_to_free[fb * (N + 1) + fa] = (fb - c - 1) * (n - 1) + (fa - c - 1)
        coords_all = np.stack([(ga.reshape(-1) - c) / n, (gb.reshape(-1) - c) / n], axis=1)
        if nc == 1:
            rows = np.repeat(np.arange(nfree), W * W)
            cols = ext.reshape(-1)
            v = win.reshape(-1)
        else:
            # win layout per row node: [rc][window][cc]
            wv = win.reshape(nfree, 2, W * W, 2)
            rows = (2 * np.arange(nfree)[:, None, None, None]
                    + np.arange(2)[None, :, None, None]) * np.ones((1, 1, W * W, 2), dtype=np.int64)
            cols = (2 * ext[:, None, :, None] + np.arange(2)[None, None, None, :]) * np.ones((1, 2, 1, 1), dtype=np.int64)
            rows = rows.reshape(-1)
            cols = cols.reshape(-1)
            v = wv.reshape(-1)
    keep = v != 0.0
    rows, cols, v = rows[keep], cols[keep], v[keep]
    # map columns to free dofs / Dirichlet dofs
    col_node = cols // nc
    col_comp = cols % nc
    free_of = ext_to_free[col_node]
    is_free = free_of >= 0
    A = sp.csr_matrix((v[is_free], (rows[is_free], free_of[is_free] * nc + col_comp[is_free])),
                      shape=(nfree * nc, nfree * nc))
    # Dirichlet nodes: every extended node that is not free, numbered in order
    dir_nodes = np.nonzero(ext_to_free < 0)[0]
    dir_id = np.full(nodes_total, -1, dtype=np.int64)
    dir_id[dir_nodes] = np.arange(dir_nodes.size)
    dn = ~is_free
    Bd = sp.csr_matrix((v[dn], (rows[dn], dir_id[col_node[dn]] * nc + col_comp[dn])),
                       shape=(nfree * nc, dir_nodes.size * nc))
    free_nodes = np.nonzero(ext_to_free >= 0)[0]
    order = np.argsort(ext_to_free[free_nodes])
    coords = coords_all[free_nodes[order]]
    return A, Bd, coords, coords_all[dir_nodes]


def _symmetrise_lower(A: sp.csr_matrix) -> sp.csr_matrix:
    """Mirror the strictly lower triangle onto the upper one so the matrix is
    bitwise symmetric (the row-wise assembly computes both halves with
    different summation orders)."""
    L = sp.tril(A, k=-1, format="csr")
    D = sp.diags(A.diagonal())
    S = (L + L.T + D).tocsr()
    S.sort_indices()
    return S


def window_radius(spec: Spec) -> int:
    """Half width R of the per-row assembly windows."""
    return int(math.ceil(spec.delta / spec.h)) + 2


def assemble_windows(spec: Spec) -> np.ndarray:
    """The per-row assembly windows of a 2D spec (layout of nl_assemble_2d)."""
    assert spec.dim == 2
    lib = _load()
    R = window_radius(spec)
    W = 2 * R + 1
    rowlen = W * W * (4 if spec.kernel == KER_PD else 1)
    win = np.zeros((spec.n - 1) * (spec.n - 1) * rowlen, dtype=np.float64)
    rc = lib.nl_assemble_2d(spec.n, spec.collar, spec.delta, spec.kernel, spec.phi, spec.s, R,
                            _nthreads(), win.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"assembly failed ({rc})")
    return win


def windows_to_matrix(spec: Spec, win: np.ndarray, symmetrise: bool = True) -> sp.csr_matrix:
    """The free-node stiffness matrix of a 2D spec from its assembly windows
    (e.g. the device assembly's), as assemble() forms it."""
    A = _window_to_csr(spec, np.ascontiguousarray(win, dtype=np.float64), window_radius(spec))[0]
    if symmetrise:
        A = _symmetrise_lower(A)
    A.sort_indices()
    return A


def assemble(spec: Spec, symmetrise: bool = True) -> Assembled:
    lib = _load()
    n, c = spec.n, spec.collar
    R = window_radius(spec)
    W = 2 * R + 1
    if spec.dim == 1:
        win = np.zeros((n - 1) * W, dtype=np.float64)
        rc = lib.nl_assemble_1d(n, c, spec.delta, spec.phi, R, _nthreads(),
                                win.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    else:
        win = assemble_windows(spec)
        rc = 0
    if rc != 0:
        raise RuntimeError(f"assembly failed ({rc})")
    A, Bd, coords, dcoords = _window_to_csr(spec, win, R)
    if symmetrise:
        A = _symmetrise_lower(A)
    A.sort_indices()
    Bd.sort_indices()
    return Assembled(spec, A, Bd, coords, dcoords, R)


# --------------------------------------------------------------------------
# Load vectors: b = M f_h with f_h the P1 function of seeded nodal values
# (nodal values zero off the free nodes).  Linear functional F of eq. bil1.
# --------------------------------------------------------------------------
def mass_matrix(spec: Spec) -> sp.csr_matrix:
    n = spec.n
    h = spec.h
    if spec.dim == 1:
        m = n - 1
        main = np.full(m, 4.0 * h / 6.0)
        off = np.full(m - 1, h / 6.0)
        M = sp.diags([off, main, off], [-1, 0, 1], format="csr")
    else:
        # P1 mass on the structured right-triangle mesh, free nodes only
        m = n - 1
        area = 0.5 * h * h
        loc = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
        rows, cols, vals = [], [], []
        # vectorised: cells with corners in free-node index space (-1..m)
        A_, B_ = np.meshgrid(np.arange(-1, m), np.arange(-1, m), indexing="xy")
        A_ = A_.reshape(-1)
        B_ = B_.reshape(-1)
        tri = [((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))]
        for verts in tri:
            va = [A_ + dv[0] for dv in verts]
            vb = [B_ + dv[1] for dv in verts]
            for i in range(3):
                for j in range(3):
                    ok = (va[i] >= 0) & (va[i] < m) & (vb[i] >= 0) & (vb[i] < m) & \
                         (va[j] >= 0) & (va[j] < m) & (vb[j] >= 0) & (vb[j] < m)
                    rows.append((vb[i] * m + va[i])[ok])
                    cols.append((vb[j] * m + va[j])[ok])
                    vals.append(np.full(ok.sum(), loc[i, j]))
        M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(m * m, m * m))
    if spec.ncomp > 1:
        M = sp.kron(M, sp.eye(spec.ncomp), format="csr")
    M.sort_indices()
    return M


def rhs(spec: Spec, nrhs: int | None = None, seed_base: int | None = None) -> np.ndarray:
    """Column-major (n_dof x nrhs) load vectors; column r uses seed base + r."""
    nrhs = spec.nrhs if nrhs is None else nrhs
    seed_base = spec.seed_base if seed_base is None else seed_base
    M = mass_matrix(spec)
    ndof = M.shape[0]
    F = np.empty((ndof, nrhs), dtype=np.float64, order="F")
    for r in range(nrhs):
        F[:, r] = splitmix64_uniform_fast(seed_base + r, ndof)
    return np.asfortranarray(M @ F)


# --------------------------------------------------------------------------
# Nonlocal subdivision (section "Building substructures")
# --------------------------------------------------------------------------
def _cut_positions(n: int, k: int, jitter: float, seed: int) -> np.ndarray:
    """k strips of (0,1) in cell units, widths (1/k)(1+eps_i), eps_i uniform
    in [-jitter, jitter] from SplitMix64, renormalised, snapped to mesh lines."""
    if jitter > 0.0:
        eps = jitter * splitmix64_uniform(seed, k)
        w = (1.0 + eps) / k
        w = w / w.sum()
    else:
        w = np.full(k, 1.0 / k)
    edges = np.concatenate([[0.0], np.cumsum(w)])
    cuts = np.rint(edges * n).astype(np.int64)
    cuts[0], cuts[-1] = 0, n
    if np.any(np.diff(cuts) <= 0):
        raise ValueError("degenerate cut")
    return cuts


def _point_seg_dist2(px, py, ax, ay, bx, by):
    vx, vy = bx - ax, by - ay
    wx, wy = px - ax, py - ay
    L2 = vx * vx + vy * vy
    t = np.clip((wx * vx + wy * vy) / L2, 0.0, 1.0)
    dx, dy = wx - t * vx, wy - t * vy
    return dx * dx + dy * dy


@dataclass
class Partition:
    """Overlapping decomposition and the algebraic interior/interface split."""
    K: int
    interior: list            # per subdomain: free-node ids of I_k (2D: in patch order)
    gamma_nodes: np.ndarray   # free-node ids of the interface (2D: in patch order)
    elem_member: np.ndarray   # (n_interior_elements x K) bool: E in hat-Omega_k
    cuts: tuple               # cut positions (cell units) per axis
    node_free: np.ndarray = None   # (free nodes x K) bool: node of hat-Omega_k


def partition(spec: Spec, rho: float | None = None) -> Partition:
    """hat-Omega_k = tilde-Omega_k plus every element E of (0,1)^d with
    inf dist(E, tilde-Omega_k) <= rho (default delta/2, the exact criterion);
    interface nodes are nodes of elements lying in two or more hat-Omega_k
    (sets of eq. subdomainDefinitions taken as closed element unions)."""
    n = spec.n
    rho = spec.delta / 2.0 if rho is None else rho
    rho_c = rho * n                          # in cell units
    if spec.dim == 1:
        cx = _cut_positions(n, spec.cuts[0], spec.jitter, spec.jitter_seeds[0])
        K = spec.cuts[0]
        e = np.arange(n)                     # element [e, e+1] in cell units
        member = np.zeros((n, K), dtype=bool)
        for k in range(K):
            lo, hi = cx[k], cx[k + 1]
            dist = np.maximum(0, np.maximum(lo - (e + 1), e - hi))
            member[:, k] = dist <= rho_c + 1e-12
        # node a (0..n) belongs to hat-Omega_k if an element of it has a as vertex
        node_in = np.zeros((n + 1, K), dtype=bool)
        node_in[:-1] |= member
        node_in[1:] |= member
        free = np.arange(1, n)
        cnt = node_in[free].sum(axis=1)
        gamma = np.nonzero(cnt >= 2)[0]                  # free-node ids (a-1)
        interior = [np.nonzero((cnt == 1) & node_in[free, k])[0] for k in range(K)]
        return Partition(K, interior, gamma, member, (tuple(cx),), node_in[free])
    # 2D
    kx, ky = spec.cuts
    cx = _cut_positions(n, kx, spec.jitter, spec.jitter_seeds[0])
    cy = _cut_positions(n, ky, spec.jitter, spec.jitter_seeds[1])
    K = kx * ky
    A_, B_ = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    A_ = A_.reshape(-1).astype(np.float64)
    B_ = B_.reshape(-1).astype(np.float64)
    # elements: cell (a,b) with t=0: (a,b),(a+1,b),(a+1,b+1); t=1: (a,b),(a+1,b+1),(a,b+1)
    tv = {0: ((0, 0), (1, 0), (1, 1)), 1: ((0, 0), (1, 1), (0, 1))}
    elems = []
    for t in (0, 1):
        vx = np.stack([A_ + d[0] for d in tv[t]], axis=1)
        vy = np.stack([B_ + d[1] for d in tv[t]], axis=1)
        elems.append((vx, vy))
    # element order: cell-major, t inner -> index 2*cell + t
    vx = np.empty((2 * n * n, 3)); vy = np.empty((2 * n * n, 3))
    vx[0::2], vy[0::2] = elems[0]
    vx[1::2], vy[1::2] = elems[1]
    member = np.zeros((2 * n * n, K), dtype=bool)
    for j in range(ky):
        for i in range(kx):
            k = j * kx + i
            x0, x1, y0, y1 = float(cx[i]), float(cx[i + 1]), float(cy[j]), float(cy[j + 1])
            # triangle vertices -> box
            dxv = np.maximum(0.0, np.maximum(x0 - vx, vx - x1))
            dyv = np.maximum(0.0, np.maximum(y0 - vy, vy - y1))
            d2 = (dxv * dxv + dyv * dyv).min(axis=1)
            # box corners -> triangle edges
            for (px, py) in ((x0, y0), (x1, y0), (x1, y1), (x0, y1)):
                for e0, e1 in ((0, 1), (1, 2), (2, 0)):
                    d2 = np.minimum(d2, _point_seg_dist2(px, py, vx[:, e0], vy[:, e0],
                                                         vx[:, e1], vy[:, e1]))
            # triangles inside the box (distance 0 already), or box corner inside triangle:
            # impossible for mesh-aligned boxes unless the triangle lies inside.
            member[:, k] = d2 <= rho_c * rho_c + 1e-9
    # node membership: node (a,b), a,b in 0..n
    node_in = np.zeros(((n + 1) * (n + 1), K), dtype=bool)
    for v in range(3):
        ids = (vy[:, v].astype(np.int64) * (n + 1) + vx[:, v].astype(np.int64))
        for k in range(K):
            np.logical_or.at(node_in[:, k], ids[member[:, k]], True)
    ga, gb = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    free_mask = ((ga > 0) & (ga < n) & (gb > 0) & (gb < n)).reshape(-1)
    free_ext = np.nonzero(free_mask)[0]                # in (b*(n+1)+a) order == free order
    cnt = node_in[free_ext].sum(axis=1)
    gamma = patch_order(np.nonzero(cnt >= 2)[0], n, spec.ncomp)
    interior = [patch_order(np.nonzero((cnt == 1) & node_in[free_ext, k])[0], n, spec.ncomp)
                for k in range(K)]
    return Partition(K, interior, gamma, member, (tuple(cx), tuple(cy)), node_in[free_ext])


def patch_order(nodes: np.ndarray, n: int, ncomp: int) -> np.ndarray:
    """Free-node ids of a 2D set numbered patch by patch: patches of 2 nodes
    along x and 8 / ncomp along y (16 dofs), patch rows bottom to top, nodes
    row-major inside a patch.  Sixteen consecutive dofs are then a compact
    patch whose nonlocal neighbourhoods nearly coincide, which fills the 16x16
    tiles of the solver's wide-batch products (the ordering of the unknowns is
    the caller's; the system and its solution are the same)."""
    nodes = np.asarray(nodes)
    a, b = nodes % (n - 1), nodes // (n - 1)
    py = 8 // ncomp
    return nodes[np.lexsort((a % 2, b % py, a // 2, b // py))]


# --------------------------------------------------------------------------
# Algebraic split (eq. subStiffnessMatrixSubBlocks with the global matrix)
# --------------------------------------------------------------------------
@dataclass
class DDProblem:
    """Inputs of the solver: per subdomain K_II (dense), K_IG (CSR, local
    interface columns) with its maps, and the global K_GG (CSR)."""
    n_dof: int
    n_gamma: int
    gamma_map: np.ndarray                 # interface index -> global dof
    kgg: sp.csr_matrix                    # n_gamma x n_gamma
    i_maps: list = field(default_factory=list)     # per k: interior local -> global dof
    g_maps: list = field(default_factory=list)     # per k: local interface col -> interface index
    kii: list = field(default_factory=list)        # per k: dense (n_i x n_i) Fortran order
    kig: list = field(default_factory=list)        # per k: CSR (n_i x n_g)

    @property
    def n_sub(self) -> int:
        return len(self.i_maps)


def split(A: sp.csr_matrix, part: Partition, ncomp: int = 1) -> DDProblem:
    """Extract K_II^k = A(I_k, I_k), K_IG^k = A(I_k, G_k), K_GG = A(G, G).

    G_k are the interface dofs coupled to I_k.  Raises if two interiors are
    coupled (the decomposition must be a nonlocal subdivision)."""
    A = A.tocsr()
    n_dof = A.shape[0]

    def dofs(nodes):
        nodes = np.asarray(nodes, dtype=np.int64)
        return (nodes[:, None] * ncomp + np.arange(ncomp)[None, :]).reshape(-1)

    gdofs = dofs(part.gamma_nodes)
    owner = np.full(n_dof, -1, dtype=np.int64)       # -1 interface, else subdomain
    gidx = np.full(n_dof, -1, dtype=np.int64)
    gidx[gdofs] = np.arange(gdofs.size)
    for k, nodes in enumerate(part.interior):
        d = dofs(nodes)
        if np.any(owner[d] != -1):
            raise ValueError("interior sets overlap")
        owner[d] = k
    covered = (owner >= 0) | (gidx >= 0)
    if not np.all(covered):
        raise ValueError("dof neither interior nor interface")
    prob = DDProblem(n_dof=n_dof, n_gamma=gdofs.size, gamma_map=gdofs.astype(np.int32),
                     kgg=A[gdofs][:, gdofs].tocsr())
    prob.kgg.sort_indices()
    for k, nodes in enumerate(part.interior):
        I = dofs(nodes)
        rows = A[I]
        # interior-interior coupling across subdomains must vanish
        rc = rows.tocoo()
        col_owner = owner[rc.col]
        bad = (col_owner >= 0) & (col_owner != k) & (rc.data != 0.0)
        if np.any(bad):
            raise ValueError(f"interior of subdomain {k} couples to another interior")
        kii = rows[:, I].toarray()
        gcols = np.unique(gidx[rc.col[col_owner == -1]])
        gcols = gcols[gcols >= 0]
        kig = rows[:, gdofs[gcols]].tocsr()
        kig.sort_indices()
        prob.i_maps.append(I.astype(np.int32))
        prob.g_maps.append(gcols.astype(np.int32))
        prob.kii.append(np.asfortranarray(kii))
        prob.kig.append(kig)
    return prob


def undecomposed(A: sp.csr_matrix) -> DDProblem:
    """The system with no subdomains: every dof is an interface dof, so
    K_GG = A and the interface Schur complement is A itself.  Solved by the
    substructuring solver this is the diagonally preconditioned CG on the
    whole system that the paper uses as its baseline (section "Considered
    solver strategies")."""
    A = A.tocsr()
    A.sort_indices()
    n = A.shape[0]
    return DDProblem(n_dof=n, n_gamma=n, gamma_map=np.arange(n, dtype=np.int32), kgg=A)


@dataclass
class Workload:
    spec: Spec
    asm: Assembled
    part: Partition
    dd: DDProblem


def build(spec: Spec) -> Workload:
    asm = assemble(spec)
    part = partition(spec)
    dd = split(asm.A, part, spec.ncomp)
    return Workload(spec, asm, part, dd)


def scaled(spec_fn, scale: float, **kw) -> Spec:
    """Problem family member with cells per side scaled by `scale` (delta and
    the subdomain grid fixed)."""
    base = spec_fn(**kw)
    n = max(8, int(round(base.n * scale)))
    kw2 = dict(kw)
    kw2["n"] = n
    return spec_fn(**kw2)


# --------------------------------------------------------------------------
# Subdomain data of the dual method (section "FETI"): for every subdomain k its
# copy Gamma_k of the interface (the interface dofs of hat-Omega_k), the
# subdomain stiffness blocks of eq. subStiffnessMatrix assembled with the
# zeta-weighted form of eq. bilinear-multi1, the floating flag (Gamma^D_k
# empty, remark "floating") and the kernel of the subdomain operator.
# --------------------------------------------------------------------------
@dataclass
class FetiProblem:
    wl: "Workload"
    g_sets: list          # per k: interface indices (dd's numbering) of Gamma_k, increasing
    agg: list             # per k: CSR |G_k| x |G_k|, zeta-weighted A^k_GG
    agi: list             # per k: CSR |G_k| x n_i, A^k_GI of the zeta-weighted assembly
    kig: list             # per k: CSR n_i x |G_k|, A(I_k, Gamma_k) of the global matrix
    floating: list        # per k: True if Gamma^D_k is empty
    z: list               # per k: |G_k| x n_z kernel basis of S_k on Gamma_k (n_z = 0 if not floating)
    member: np.ndarray    # (extended elements x K) bool: E in hat-Omega_k u Gamma^D_k
    zeta_nodes: np.ndarray  # per interface dof: number of copies (zeta(x, x))

    @property
    def dd(self):
        return self.wl.dd


def _ext_membership(spec: Spec, part: Partition) -> np.ndarray:
    """(extended elements x K) membership of hat-Omega_k u Gamma^D_k: elements
    of (0,1)^d from the partition, collar elements within delta of
    tilde-Omega_k (section "Building substructures": Gamma^D_k is the
    interaction domain of tilde-Omega_k)."""
    n, c, K = spec.n, spec.collar, part.K
    N = n + 2 * c
    dc = spec.delta * n                                  # delta in cell units
    if spec.dim == 1:
        member = np.zeros((N, K), dtype=bool)
        member[c:c + n] = part.elem_member
        cx = np.array(part.cuts[0])
        e = np.arange(N) - c                              # element [e, e+1] in cell units
        coll = (e < 0) | (e >= n)
        for k in range(K):
            d = np.maximum(0, np.maximum(cx[k] - (e + 1), e - cx[k + 1]))
            member[coll, k] = d[coll] <= dc + 1e-12
        return member
    cx, cy = np.array(part.cuts[0]), np.array(part.cuts[1])
    kx = len(cx) - 1
    A_, B_ = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    A_ = A_.reshape(-1) - c
    B_ = B_.reshape(-1) - c
    tv = {0: ((0, 0), (1, 0), (1, 1)), 1: ((0, 0), (1, 1), (0, 1))}
    vx = np.empty((2 * N * N, 3)); vy = np.empty((2 * N * N, 3))
    for t in (0, 1):
        vx[t::2] = np.stack([A_ + d[0] for d in tv[t]], axis=1)
        vy[t::2] = np.stack([B_ + d[1] for d in tv[t]], axis=1)
    cell_a = np.repeat(A_, 2)
    cell_b = np.repeat(B_, 2)
    inside = (cell_a >= 0) & (cell_a < n) & (cell_b >= 0) & (cell_b < n)
    member = np.zeros((2 * N * N, K), dtype=bool)
    # elements of (0,1)^2: element 2 (b n + a) + t of the partition
    idx_in = 2 * (cell_b[inside] * n + cell_a[inside]) + np.tile([0, 1], N * N)[inside]
    member[inside] = part.elem_member[idx_in]
    for k in range(K):
        i, j = k % kx, k // kx
        x0, x1, y0, y1 = float(cx[i]), float(cx[i + 1]), float(cy[j]), float(cy[j + 1])
        dxv = np.maximum(0.0, np.maximum(x0 - vx, vx - x1))
        dyv = np.maximum(0.0, np.maximum(y0 - vy, vy - y1))
        d2 = (dxv * dxv + dyv * dyv).min(axis=1)
        for (px, py) in ((x0, y0), (x1, y0), (x1, y1), (x0, y1)):
            for e0, e1 in ((0, 1), (1, 2), (2, 0)):
                d2 = np.minimum(d2, _point_seg_dist2(px, py, vx[:, e0], vy[:, e0], vx[:, e1], vy[:, e1]))
        member[~inside, k] = d2[~inside] <= dc * dc + 1e-9
    return member


def feti_problem(wl: Workload) -> FetiProblem:
    spec, part, dd, A = wl.spec, wl.part, wl.dd, wl.asm.A.tocsr()
    nc, K = spec.ncomp, part.K
    n, c = spec.n, spec.collar
    N = n + 2 * c
    member = _ext_membership(spec, part)
    if K > 64:
        raise ValueError("at most 64 subdomains")
    masks = (member.astype(np.uint64) << np.arange(K, dtype=np.uint64)[None, :]).sum(axis=1,
                                                                                   dtype=np.uint64)
    gidx = np.full(dd.n_dof, -1, dtype=np.int64)
    gidx[dd.gamma_map] = np.arange(dd.n_gamma)
    gnode_set = np.zeros(part.node_free.shape[0], dtype=bool)
    gnode_set[part.gamma_nodes] = True
    # rows: (interface node m of subdomain k) in subdomain order
    rows_node, rows_sub, g_sets = [], [], []
    for k in range(K):
        nodes = np.nonzero(part.node_free[:, k] & gnode_set)[0]
        g_sets.append(np.sort(gidx[(nodes[:, None] * nc + np.arange(nc)[None, :]).reshape(-1)]))
        if spec.dim == 1:
            ext = c + 1 + nodes
        else:
            fa, fb = nodes % (n - 1) + 1, nodes // (n - 1) + 1
            ext = (fb + c) * (N + 1) + (fa + c)
        rows_node.append(ext)
        rows_sub.append(np.full(nodes.size, k))
    rows_node = np.ascontiguousarray(np.concatenate(rows_node), dtype=np.int32)
    rows_sub = np.ascontiguousarray(np.concatenate(rows_sub), dtype=np.int32)
    P = rows_node.size
    R = window_radius(spec)
    Wd = 2 * R + 1
    lib = _load()
    ip = ctypes.POINTER(ctypes.c_int)
    mp = np.ascontiguousarray(masks)
    if spec.dim == 1:
        win = np.zeros(P * Wd)
        rc = lib.nl_assemble_1d_sub(n, c, spec.delta, spec.phi, R, _nthreads(),
                                    mp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), P,
                                    rows_node.ctypes.data_as(ip), rows_sub.ctypes.data_as(ip),
                                    win.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    else:
        rowlen = Wd * Wd * (4 if spec.kernel == KER_PD else 1)
        win = np.zeros(P * rowlen)
        rc = lib.nl_assemble_2d_sub(n, c, spec.delta, spec.kernel, spec.phi, spec.s, R, _nthreads(),
                                    mp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), P,
                                    rows_node.ctypes.data_as(ip), rows_sub.ctypes.data_as(ip),
                                    win.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"subdomain assembly failed ({rc})")
    # windows -> (row dof, column dof) entries over free dofs
    if spec.dim == 1:
        da = np.arange(-R, R + 1)
        col_ext = rows_node[:, None] + da[None, :]
        col_free = col_ext - c - 1
        ok = (col_free >= 0) & (col_free < n - 1)
        r = np.repeat(np.arange(P), Wd).reshape(P, Wd)[ok]
        cfree = col_free[ok]
        v = win.reshape(P, Wd)[ok]
        row_dof = (rows_node - c - 1)[r]
        col_dof = cfree
    else:
        dd_ = np.arange(-R, R + 1)
        DB, DA = np.meshgrid(dd_, dd_, indexing="ij")
        ra, rb = rows_node % (N + 1), rows_node // (N + 1)
        ca_ = ra[:, None] + DA.reshape(-1)[None, :] - c
        cb_ = rb[:, None] + DB.reshape(-1)[None, :] - c
        okn = (ca_ > 0) & (ca_ < n) & (cb_ > 0) & (cb_ < n)
        cfn = (cb_ - 1) * (n - 1) + (ca_ - 1)
        rfn = (rb - c - 1) * (n - 1) + (ra - c - 1)
        if nc == 1:
            r = np.repeat(np.arange(P)[:, None], Wd * Wd, axis=1)[okn]
            v = win.reshape(P, Wd * Wd)[okn]
            row_dof = rfn[r]
            col_dof = cfn[okn]
        else:
            wv = win.reshape(P, 2, Wd * Wd, 2)
            rr, cc, vv, pp = [], [], [], []
            for rcomp in range(2):
                for ccomp in range(2):
                    vals = wv[:, rcomp, :, ccomp][okn]
                    pr = np.repeat(np.arange(P)[:, None], Wd * Wd, axis=1)[okn]
                    rr.append(rfn[pr] * 2 + rcomp)
                    cc.append(cfn[okn] * 2 + ccomp)
                    vv.append(vals)
                    pp.append(pr)
            row_dof = np.concatenate(rr)
            col_dof = np.concatenate(cc)
            v = np.concatenate(vv)
            r = np.concatenate(pp)
    keep = v != 0.0
    row_dof, col_dof, v, r = row_dof[keep], col_dof[keep], v[keep], r[keep]
    sub_of = rows_sub[r]
    owner = np.full(dd.n_dof, -1, dtype=np.int64)
    iloc = np.full(dd.n_dof, -1, dtype=np.int64)
    for k, I in enumerate(dd.i_maps):
        owner[I] = k
        iloc[I] = np.arange(I.size)
    agg, agi, kig, floating, zs = [], [], [], [], []
    zeta_nodes = np.zeros(dd.n_gamma, dtype=np.int64)
    for k in range(K):
        G = g_sets[k]
        zeta_nodes[G] += 1
        gl = np.full(dd.n_gamma, -1, dtype=np.int64)
        gl[G] = np.arange(G.size)
        sel = sub_of == k
        rg = gl[gidx[row_dof[sel]]]
        cg_all = gidx[col_dof[sel]]
        vk = v[sel]
        in_g = cg_all >= 0
        cgl = np.where(in_g, gl[np.maximum(cg_all, 0)], -1)
        okg = in_g & (cgl >= 0)
        if np.any(rg < 0):
            raise AssertionError("row outside Gamma_k")
        agg.append(sp.csr_matrix((vk[okg], (rg[okg], cgl[okg])), shape=(G.size, G.size)))
        # columns in interiors: must be subdomain k's own
        cown = owner[col_dof[sel]]
        oki = (~in_g) & (cown >= 0)
        if np.any(cown[oki] != k):
            raise AssertionError("subdomain row couples to another interior")
        ni = dd.i_maps[k].size
        agi.append(sp.csr_matrix((vk[oki], (rg[oki], iloc[col_dof[sel]][oki])), shape=(G.size, ni)))
        kig.append(A[dd.i_maps[k]][:, dd.gamma_map[G]].tocsr())
        fl = not member[:, k][_collar_elements(spec)].any()
        floating.append(fl)
        if not fl:
            zs.append(np.zeros((G.size, 0)))
        elif nc == 1:
            zs.append(np.ones((G.size, 1)))
        else:
            nodes = dd.gamma_map[G] // 2
            comp = dd.gamma_map[G] % 2
            xy = wl.asm.coords[nodes]
            Z = np.zeros((G.size, 3))
            Z[comp == 0, 0] = 1.0
            Z[comp == 1, 1] = 1.0
            Z[:, 2] = np.where(comp == 0, -xy[:, 1], xy[:, 0])     # rotation (-y, x)
            zs.append(Z)
    for M in agg + agi + kig:
        M.sort_indices()
    return FetiProblem(wl, g_sets, agg, agi, kig, floating, zs, member, zeta_nodes)


def _collar_elements(spec: Spec) -> np.ndarray:
    """Mask of the collar (Dirichlet) elements of the extended mesh."""
    n, c = spec.n, spec.collar
    N = n + 2 * c
    if spec.dim == 1:
        e = np.arange(N) - c
        return (e < 0) | (e >= n)
    A_, B_ = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    a = np.repeat(A_.reshape(-1) - c, 2)
    b = np.repeat(B_.reshape(-1) - c, 2)
    return ~((a >= 0) & (a < n) & (b >= 0) & (b < n))


def feti_loads(fp: FetiProblem, nrhs: int | None = None, seed_base: int | None = None) -> list:
    """Per subdomain the interface part of the load of eq. bilinear-multi5,
    int_{hat-Omega_k} f psi_m zeta(x,x)^-1 dx, for the nodal values of rhs()
    (P1 f_h, zero off the free nodes): per k an array |G_k| x nrhs."""
    wl = fp.wl
    spec, dd = wl.spec, wl.dd
    nrhs = spec.nrhs if nrhs is None else nrhs
    seed_base = spec.seed_base if seed_base is None else seed_base
    nfree = dd.n_dof
    F = np.empty((nfree, nrhs))
    for r in range(nrhs):
        F[:, r] = splitmix64_uniform_fast(seed_base + r, nfree)
    n, c, nc = spec.n, spec.collar, spec.ncomp
    N = n + 2 * c
    member = fp.member
    zeta_e = member.sum(axis=1)
    out = []
    gidx = np.full(dd.n_dof, -1, dtype=np.int64)
    gidx[dd.gamma_map] = np.arange(dd.n_gamma)
    for k in range(len(fp.g_sets)):
        G = fp.g_sets[k]
        gl = np.full(dd.n_gamma, -1, dtype=np.int64)
        gl[G] = np.arange(G.size)
        fk = np.zeros((G.size, nrhs))
        if spec.dim == 1:
            h = spec.h
            loc = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
            for e in np.nonzero(member[:, k] & ~_collar_elements(spec))[0]:
                verts = [e, e + 1]                               # extended node ids
                fr = [v - c - 1 for v in verts]                  # free node ids
                for i in range(2):
                    if not (0 <= fr[i] < n - 1):
                        continue
                    gi = gidx[fr[i]]
                    if gi < 0 or gl[gi] < 0:
                        continue
                    for j in range(2):
                        if 0 <= fr[j] < n - 1:
                            fk[gl[gi]] += loc[i, j] * F[fr[j]] / zeta_e[e]
        else:
            area = 0.5 * spec.h ** 2
            loc = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
            tv = {0: ((0, 0), (1, 0), (1, 1)), 1: ((0, 0), (1, 1), (0, 1))}
            for e in np.nonzero(member[:, k] & ~_collar_elements(spec))[0]:
                cell, t = e // 2, e % 2
                ca, cb = cell % N - c, cell // N - c
                fr = []
                for d in tv[t]:
                    a, b = ca + d[0], cb + d[1]
                    fr.append((b - 1) * (n - 1) + (a - 1) if (0 < a < n and 0 < b < n) else -1)
                for i in range(3):
                    if fr[i] < 0:
                        continue
                    for comp in range(nc):
                        gi = gidx[fr[i] * nc + comp]
                        if gi < 0 or gl[gi] < 0:
                            continue
                        for j in range(3):
                            if fr[j] >= 0:
                                fk[gl[gi]] += loc[i, j] * F[fr[j] * nc + comp] / zeta_e[e]
        out.append(fk)
    return out
