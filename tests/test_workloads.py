"""Pins of the problem generator (assembly, loads, decomposition) against
closed forms, brute force and the invariants the paper states.  CPU only."""
import math

import numpy as np
import pytest
import scipy.integrate as si

import workloads as W


# ------------------------------------------------------------------ helpers --
def ext_nodal(spec, fun, asm):
    """Nodal values of `fun` on the free nodes and on the Dirichlet nodes."""
    if spec.dim == 1:
        xf = asm.coords[:, 0]
        xd = asm.dir_coords[:, 0]
        vf, vd = fun(xf), fun(xd)
    else:
        vf = fun(asm.coords[:, 0], asm.coords[:, 1])
        vd = fun(asm.dir_coords[:, 0], asm.dir_coords[:, 1])
    return np.asarray(vf, float), np.asarray(vd, float)


def apply_full(asm, vf, vd):
    """[A | B] applied to (free, Dirichlet) nodal values: the discrete nonlocal
    operator of the interpolant, tested against the free basis functions."""
    return asm.A @ vf + asm.Bd @ vd


# ------------------------------------------------------------------- seeds --
def test_splitmix64_published_first_output():
    # SplitMix64 (Steele, Lea & Flood 2014) from state 0: first output
    # 0xE220A8397B1DCDAF (reference implementation test value).
    M = (1 << 64) - 1
    z = (0 + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    z ^= z >> 31
    assert z == 0xE220A8397B1DCDAF
    u = W.splitmix64_uniform(0, 1)[0]
    assert u == 2.0 * ((0xE220A8397B1DCDAF >> 11) * 2.0 ** -53) - 1.0


def test_splitmix64_fast_matches_loop():
    for seed in (0, 1, 2000, 4031, 2 ** 63 + 5):
        a = W.splitmix64_uniform(seed, 257)
        b = W.splitmix64_uniform_fast(seed, 257)
        assert np.array_equal(a, b)
        assert a.min() >= -1.0 and a.max() < 1.0


# ------------------------------------------------------------------ 1D pins --
@pytest.mark.parametrize("n,delta", [(32, 1 / 16), (1000, 0.05), (100, 0.07)])
def test_1d_constants_and_linears_in_kernel(n, delta):
    """Row sums vanish and linear functions are in the kernel of [A | B]:
    d_n(x,y) = psi(y) - psi(x) annihilates constants; the symmetric band
    integral of (y - x) vanishes for interior rows."""
    spec = W.spec_1d(n=n, delta=delta)
    asm = W.assemble(spec)
    scale = np.abs(asm.A.diagonal()).max()
    one_f, one_d = ext_nodal(spec, lambda x: np.ones_like(x), asm)
    assert np.abs(apply_full(asm, one_f, one_d)).max() <= 1e-13 * scale
    lf, ldd = ext_nodal(spec, lambda x: x, asm)
    assert np.abs(apply_full(asm, lf, ldd)).max() <= 1e-13 * scale


@pytest.mark.parametrize("n,delta", [(32, 1 / 16), (1000, 0.05), (64, 0.125)])
def test_1d_quadratic_closed_form(n, delta):
    """With gamma = 3/(2 delta^3) on |x-y| <= delta the nonlocal operator of
    x^2 is exactly -2 (strong form with its factor 2), and when 2 delta / h is
    an integer the interpolation error of x^2 is h-periodic with a constant
    band integral, so [A | B] q = -2 h on every free row exactly."""
    spec = W.spec_1d(n=n, delta=delta)
    assert abs(2 * delta * n - round(2 * delta * n)) < 1e-9
    asm = W.assemble(spec)
    qf, qd = ext_nodal(spec, lambda x: x * x, asm)
    got = apply_full(asm, qf, qd)
    assert np.allclose(got, -2.0 / n, rtol=0, atol=1e-11 / n)


def _brute_1d_entry(m_ext, nn_ext, spec):
    """Independent evaluation of A(psi_m, psi_n) for the 1D band kernel by
    adaptive quadrature over every element pair with the band |x-y| <= delta
    as integration limits (no polygon clipping)."""
    h, c, N = spec.h, spec.collar, spec.n + 2 * spec.collar
    gam = spec.phi

    def psi(a, x):
        xa = (a - c) * h
        return max(0.0, 1.0 - abs(x - xa) / h)

    total = 0.0
    support = lambda a: [e for e in (a - 1, a) if 0 <= e < N]
    Es = set(support(m_ext)) | set(support(nn_ext))
    R1 = int(math.ceil(spec.delta / h)) + 1
    for e in range(N):
        for f in range(N):
            if abs(e - f) > R1:
                continue
            if e not in Es and f not in Es:
                continue
            xe, xf = (e - c) * h, (f - c) * h

            def integrand(y, x):
                dm = psi(m_ext, y) - psi(m_ext, x)
                dn = psi(nn_ext, y) - psi(nn_ext, x)
                return dm * dn * gam

            lo = lambda x: max(xf, x - spec.delta)
            hi = lambda x: min(xf + h, x + spec.delta)
            # restrict x to where the band meets F
            xa, xb = max(xe, xf - spec.delta), min(xe + h, xf + h + spec.delta)
            if xb <= xa:
                continue
            val, _ = si.dblquad(integrand, xa, xb, lo, hi, epsabs=1e-15, epsrel=1e-13)
            total += val
    return total


def test_1d_brute_force_entries():
    spec = W.spec_1d(n=16, delta=0.1)
    asm = W.assemble(spec, symmetrise=False)
    c = spec.collar
    A = asm.A.toarray()
    rng = np.random.default_rng(3)
    rows = [0, 5, 14]
    for i in rows:
        m_ext = c + 1 + i
        for j in sorted(set([i, max(0, i - 1), min(14, i + 2)] + list(rng.integers(0, 15, 2)))):
            ref = _brute_1d_entry(m_ext, c + 1 + j, spec)
            assert abs(A[i, j] - ref) <= 1e-12 * abs(A[i, i]), (i, j, A[i, j], ref)


def test_1d_dirichlet_block_brute_force():
    """Coupling to a collar node (the B block) by the same brute force."""
    spec = W.spec_1d(n=16, delta=0.1)
    asm = W.assemble(spec, symmetrise=False)
    c = spec.collar
    # collar node just left of x = 0: extended index c - 1 (Dirichlet id c-1)
    B = asm.Bd.toarray()
    ref = _brute_1d_entry(c + 1, c - 1, spec)
    dir_id = c - 1            # Dirichlet nodes are numbered in extended order
    assert abs(B[0, dir_id] - ref) <= 1e-12 * abs(asm.A[0, 0])


def test_1d_manufactured_quadratic_exact():
    """u = x^2 with Dirichlet data x^2 on the collar and f = -2: the discrete
    solution equals the nodal interpolant (exact quadratic identity)."""
    import oracle
    spec = W.spec_1d(n=64, delta=1 / 16)
    asm = W.assemble(spec)
    qf, qd = ext_nodal(spec, lambda x: x * x, asm)
    # consistent load of the constant f = -2 on the free basis: F(psi_i) = -2 h
    rhs = np.full(qf.size, -2.0 / spec.n)
    u = oracle.monolithic_solve(asm.A, rhs - asm.Bd @ qd)
    assert np.abs(u - qf).max() <= 1e-10


# ------------------------------------------------------------------ 2D pins --
SPECS_2D = [
    W.spec_2d_const(n=24, delta=0.15, cuts=(2, 2)),
    W.spec_2d_frac(n=24, delta=0.15, cuts=(2, 2)),
    W.spec_2d_pd(n=20, delta=0.15, cuts=(2, 2), jitter=0.0),
]


@pytest.mark.parametrize("spec", SPECS_2D, ids=lambda s: s.name)
def test_2d_rowsums(spec):
    """[A | B] 1 = 0 on every free row (d_n of a constant vanishes per
    quadrature term).  Symmetry of the raw assembly is pinned in
    test_assembly_brute_force.py."""
    asm = W.assemble(spec, symmetrise=False)
    A = asm.A
    scale = np.abs(A.diagonal()).max()
    nc = spec.ncomp
    for comp in range(nc):
        def tr(x, y, comp=comp):
            return np.ones_like(x)
        vf, vd = ext_nodal(spec, tr, asm)
        if nc > 1:
            vf2 = np.zeros(vf.size * nc); vf2[comp::nc] = vf
            vd2 = np.zeros(vd.size * nc); vd2[comp::nc] = vd
            vf, vd = vf2, vd2
        assert np.abs(apply_full(asm, vf, vd)).max() <= 1e-12 * scale


def test_2d_pd_rotation_in_kernel():
    """Infinitesimal rotation u = (-x2, x1): (u(y)-u(x)).s = 0 makes every
    quadrature term of the peridynamic form vanish."""
    spec = SPECS_2D[2]
    asm = W.assemble(spec)
    xf, yf = asm.coords[:, 0], asm.coords[:, 1]
    xd, yd = asm.dir_coords[:, 0], asm.dir_coords[:, 1]
    vf = np.stack([-yf, xf], axis=1).ravel()
    vd = np.stack([-yd, xd], axis=1).ravel()
    scale = np.abs(asm.A.diagonal()).max()
    assert np.abs(apply_full(asm, vf, vd)).max() <= 1e-12 * scale


@pytest.mark.parametrize("spec", SPECS_2D, ids=lambda s: s.name)
def test_2d_spd(spec):
    A = W.assemble(spec).A.toarray()
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 1e-10 * ev.max()


def test_2d_quadratic_identity_within_truncation_error():
    """Constant kernel 4/(pi delta^4): the nonlocal operator of a quadratic is
    -Laplace exactly in the continuum; barycentre truncation replaces the ball
    by whole elements, which perturbs its second moment by O(h/delta).  The
    discrete identity [A|B] q = (-Lap q) int psi_i must hold to that order,
    uniformly over the rows of the structured mesh."""
    for n in (16, 32, 64):
        spec = W.spec_2d_const(n=n, delta=0.25, cuts=(1, 1))
        asm = W.assemble(spec)
        qf, qd = ext_nodal(spec, lambda x, y: x * x + 0.5 * y * y, asm)
        got = apply_full(asm, qf, qd)
        want = -3.0 * spec.h ** 2          # -Lap q = -3, int psi_i = h^2
        rel = got / want - 1.0
        assert np.abs(rel).max() <= 0.5 * spec.h / spec.delta
        assert np.ptp(rel) <= 1e-9          # the same stencil on every row


def test_2d_fractional_quadratic_identity_within_truncation_error():
    """Fractional-type kernel (eq. fractionalkernel, s = 1/2, scaled so that
    the nonlocal operator of a quadratic is -Laplace in the continuum): the
    discrete identity [A|B] q = (-Lap q) int psi_i holds to O(h / delta) (the
    barycentre ball, and the singular quadrature of touching pairs), uniformly
    over the rows, and the deviation shrinks under refinement at fixed delta.
    A wrong power of |x - y| or constant would leave an O(1) deviation."""
    devs = []
    for n in (16, 32, 64):
        spec = W.spec_2d_frac(n=n, delta=0.25, cuts=(1, 1))
        asm = W.assemble(spec)
        qf, qd = ext_nodal(spec, lambda x, y: x * x + 0.5 * y * y, asm)
        rel = apply_full(asm, qf, qd) / (-3.0 * spec.h ** 2) - 1.0
        assert np.abs(rel).max() <= 0.5 * spec.h / spec.delta
        assert np.ptp(rel) <= 1e-9
        devs.append(np.abs(rel).max())
    assert devs[2] <= 0.6 * devs[1] <= 0.36 * devs[0]


def test_2d_pd_navier_identity_within_truncation_error():
    """Peridynamic kernel (eq. peridynamics): for the quadratic field
    u = (x1^2, x1 x2) the Navier limit stated with the kernel gives
    -pi/4 Lap u - pi/2 grad div u = (-2 pi, 0); the discrete [A|B] u matches
    (-2 pi, 0) int psi_i to O(h / delta) on every row, converging under
    refinement at fixed delta."""
    devs = []
    for n in (16, 32, 64):
        spec = W.spec_2d_pd(n=n, delta=0.25, cuts=(1, 1), jitter=0.0)
        asm = W.assemble(spec)
        xf, yf = asm.coords[:, 0], asm.coords[:, 1]
        xd, yd = asm.dir_coords[:, 0], asm.dir_coords[:, 1]
        vf = np.stack([xf * xf, xf * yf], axis=1).ravel()
        vd = np.stack([xd * xd, xd * yd], axis=1).ravel()
        got = apply_full(asm, vf, vd).reshape(-1, 2)
        want = np.array([-2.0 * np.pi, 0.0]) * spec.h ** 2
        dev = np.abs(got - want).max() / (2.0 * np.pi * spec.h ** 2)
        assert dev <= 0.5 * spec.h / spec.delta
        devs.append(dev)
    assert devs[2] <= 0.6 * devs[0]


# ------------------------------------------------------------ mass matrix --
def test_mass_matrix_moments_2d():
    """Load b = M f_h (consistent P1 mass on the free nodes): rows of nodes
    away from the boundary integrate the hat function exactly,
    sum_j M_ij = int psi_i = h^2 and sum_j M_ij x_j = x_i h^2 (first moment of a
    symmetric hat); M is symmetric positive definite."""
    spec = W.spec_2d_const(n=12, delta=0.2, cuts=(1, 1))
    M = W.mass_matrix(spec).tocsr()
    m = spec.n - 1
    ia = np.arange(m * m) % m
    ib = np.arange(m * m) // m
    x = (ia + 1) * spec.h
    y = (ib + 1) * spec.h
    inner = (ia > 0) & (ia < m - 1) & (ib > 0) & (ib < m - 1)
    h2 = spec.h ** 2
    assert np.allclose((M @ np.ones(m * m))[inner], h2, rtol=1e-14, atol=0)
    assert np.allclose((M @ x)[inner], x[inner] * h2, rtol=1e-13, atol=0)
    assert np.allclose((M @ y)[inner], y[inner] * h2, rtol=1e-13, atol=0)
    assert abs(M - M.T).max() == 0.0
    assert np.linalg.eigvalsh(M.toarray()).min() > 0
    # vector problems: one copy per component
    Mv = W.mass_matrix(W.spec_2d_pd(n=12, delta=0.2, cuts=(1, 1), jitter=0.0)).tocsr()
    assert abs(Mv[0::2, 0::2] - M).max() == 0.0 and Mv[0::2, 1::2].nnz == 0


def test_mass_matrix_moments_1d():
    spec = W.spec_1d(n=20, delta=0.1)
    M = W.mass_matrix(spec).tocsr()
    x = np.arange(1, spec.n) * spec.h
    inner = slice(1, spec.n - 2)
    assert np.allclose((M @ np.ones(spec.n - 1))[inner], spec.h, rtol=1e-14, atol=0)
    assert np.allclose((M @ x)[inner], x[inner] * spec.h, rtol=1e-13, atol=0)


# --------------------------------------------------------- kernel constants --
def _polar_ball(f, delta, rs=None):
    """int over the Euclidean ball of radius delta of f(s1, s2), polar coordinates."""
    val, _ = si.dblquad(lambda r, t: f(r * np.cos(t), r * np.sin(t)) * r, 0, 2 * np.pi,
                        lambda t: 0.0, lambda t: delta, epsabs=1e-13, epsrel=1e-11)
    return val


@pytest.mark.parametrize("H", [((2, 0), (0, 0)), ((0, 1), (1, 0)), ((1, 0.3), (0.3, 2))])
def test_const_kernel_scaling_gives_minus_laplacian(H):
    """-2 int_B (q(x+s) - q(x)) phi ds = -Lap q for quadratic q, phi = 4/(pi d^4)."""
    delta = 0.1
    phi = W.spec_2d_const(delta=delta).phi
    H = np.array(H, float)
    g = np.array([0.7, -1.3])
    q = lambda s1, s2: g[0] * s1 + g[1] * s2 + 0.5 * (H[0, 0] * s1 * s1 + 2 * H[0, 1] * s1 * s2 + H[1, 1] * s2 * s2)
    Lq = -2.0 * phi * _polar_ball(q, delta)
    assert abs(Lq - (-np.trace(H))) <= 1e-8 * max(1, abs(np.trace(H)))


def test_fractional_kernel_scaling_gives_minus_laplacian():
    """The fractional-type kernel of eq. fractionalkernel with the scaling
    (2-2s)/(pi delta^(2-2s)) reproduces -Lap on quadratics (singular part
    integrable for s < 1)."""
    delta, s = 0.1, 0.5
    phi = W.spec_2d_frac(delta=delta, s=s).phi
    q = lambda s1, s2: 0.5 * (s1 * s1 + 3.0 * s2 * s2)
    f = lambda s1, s2: q(s1, s2) * (s1 * s1 + s2 * s2) ** (-(2 + 2 * s) / 2)
    Lq = -2.0 * phi * _polar_ball(f, delta)
    assert abs(Lq - (-4.0)) <= 1e-7


def test_pd_kernel_gives_navier_operator():
    """Peridynamic kernel 3/delta^3 (x-y)(x)(x-y)/|x-y|^3: for quadratic u the
    operator -2 int Phi(s) (u(x+s)-u(x)) ds equals -pi/4 Lap u - pi/2 grad div u
    (the limit stated with eq. peridynamics), checked on the paper's
    manufactured u = (x2^2, x1^2 x2) at a point, whose f is -pi/2 (1+2x1, x2)."""
    delta = 0.05
    phi = W.spec_2d_pd(delta=delta).phi
    x = np.array([0.3, 0.6])

    def u(p1, p2):
        return np.array([p2 * p2, p1 * p1 * p2])

    out = []
    for comp in range(2):
        def f(s1, s2, comp=comp):
            r = math.hypot(s1, s2)
            if r == 0.0:
                return 0.0
            du = u(x[0] + s1, x[1] + s2) - u(x[0], x[1])
            sv = np.array([s1, s2])
            return phi * sv[comp] * (sv @ du) / r ** 3
        out.append(-2.0 * _polar_ball(f, delta))
    # odd-degree terms integrate to zero over the ball, so the identity is exact
    want = -math.pi / 2 * np.array([1 + 2 * x[0], x[1]])
    assert np.allclose(out, want, rtol=0, atol=1e-8)


# --------------------------------------------------------------- partition --
@pytest.mark.parametrize("spec", [W.spec_1d(n=128, strips=4), W.spec_2d_const(n=32, cuts=(2, 2)),
                                  W.spec_2d_pd(n=40, delta=0.1, cuts=(3, 3), jitter=0.2)],
                         ids=lambda s: s.name)
def test_partition_interiors_decoupled_and_complete(spec):
    wl = W.build(spec)           # split() raises on interior-interior coupling
    A = wl.asm.A.tocsr()
    dd = wl.dd
    owner = np.full(dd.n_dof, -1)
    for k, I in enumerate(dd.i_maps):
        owner[I] = k
    coo = A.tocoo()
    ok = (owner[coo.row] < 0) | (owner[coo.col] < 0) | (owner[coo.row] == owner[coo.col])
    assert ok.all()
    covered = np.zeros(dd.n_dof, int)
    covered[dd.gamma_map] += 1
    for I in dd.i_maps:
        covered[I] += 1
    assert (covered == 1).all()


def test_partition_sizes_match_documented_counts():
    """Sizes of the 1D and 2D constant-kernel problems (free dofs, interface
    dofs, interior range) as stated in the design notes."""
    dd = W.build(W.spec_1d()).dd
    ni = [len(i) for i in dd.i_maps]
    assert (dd.n_dof, dd.n_gamma, min(ni), max(ni), sum(ni)) == (1023, 159, 203, 229, 864)


def test_subdivision_requirement_1d():
    """Every interacting element pair lies in one extended subdomain
    hat-Omega_k u Gamma^D_k (Definition nonlocalsubdivision), with Gamma^D_k the
    collar elements within delta of tilde-Omega_k."""
    spec = W.spec_1d(n=64, delta=0.1, strips=4)
    part = W.partition(spec)
    n, c = spec.n, spec.collar
    h, d = spec.h, spec.delta
    cuts = np.array(part.cuts[0])
    K = part.K
    # element e (extended index) covers [(e-c)h, (e-c+1)h]
    N = n + 2 * c
    member = np.zeros((N, K), bool)
    for k in range(K):
        lo, hi = cuts[k] * h, cuts[k + 1] * h
        for e in range(N):
            a, b = (e - c) * h, (e - c + 1) * h
            inside = 0 <= e - c < n
            if inside:
                member[e, k] = part.elem_member[e - c, k]
            else:
                dist = max(0.0, lo - b, a - hi)
                member[e, k] = dist <= d + 1e-12
    # the interaction region Gamma^D = [-delta, 1 + delta] \\ (0, 1): the mesh pads
    # whole cells beyond it, which take part in no interaction with the domain
    in_region = [max(0.0, -((e - c + 1) * h), (e - c) * h - 1.0) < d - 1e-12 for e in range(N)]
    for e in range(N):
        for f in range(N):
            if not (in_region[e] and in_region[f]):
                continue
            a1, b1 = (e - c) * h, (e - c + 1) * h
            a2, b2 = (f - c) * h, (f - c + 1) * h
            gap = max(0.0, a2 - b1, a1 - b2)
            if gap < d:                     # some points interact
                assert (member[e] & member[f]).any(), (e, f)


def test_zeta_weighted_subdomain_forms_sum_to_A():
    """Sum_k R_k^T A^k R_k = A for the zeta^{-1}-weighted subdomain forms
    (eq. bilinear-multi1 with the counting function of eq. zeta), assembled
    here pair by pair with the brute-force integrator on a tiny 1D mesh."""
    spec = W.spec_1d(n=16, delta=0.1, strips=2)
    part = W.partition(spec)
    n, c, h = spec.n, spec.collar, spec.h
    N = n + 2 * c
    K = part.K
    cuts = np.array(part.cuts[0])
    member = np.zeros((N, K), bool)
    for k in range(K):
        lo, hi = cuts[k] * h, cuts[k + 1] * h
        for e in range(N):
            a, b = (e - c) * h, (e - c + 1) * h
            if 0 <= e - c < n:
                member[e, k] = part.elem_member[e - c, k]
            else:
                member[e, k] = max(0.0, lo - b, a - hi) <= spec.delta + 1e-12
    asm = W.assemble(spec, symmetrise=False)
    A = asm.A.toarray()
    # pair contributions for two free rows, via brute force per element pair
    gam, d = spec.phi, spec.delta

    def psi(a, x):
        return max(0.0, 1.0 - abs(x - (a - c) * h) / h)

    def pair(m, nn, e, f):
        xe, xf = (e - c) * h, (f - c) * h
        xa, xb = max(xe, xf - d), min(xe + h, xf + h + d)
        if xb <= xa:
            return 0.0
        val, _ = si.dblquad(lambda y, x: (psi(m, y) - psi(m, x)) * (psi(nn, y) - psi(nn, x)) * gam,
                            xa, xb, lambda x: max(xf, x - d), lambda x: min(xf + h, x + d),
                            epsabs=1e-15, epsrel=1e-13)
        return val

    for (i, j) in [(6, 7), (7, 9), (3, 3)]:
        m, nn = c + 1 + i, c + 1 + j
        tot = 0.0
        for e in range(N):
            for f in range(N):
                if abs(e - f) > 3:
                    continue
                sup = {m - 1, m, nn - 1, nn}
                if e not in sup and f not in sup:
                    continue
                zeta = (member[e] & member[f]).sum()
                for k in range(K):
                    if member[e, k] and member[f, k]:
                        tot += pair(m, nn, e, f) / zeta
        assert abs(tot - A[i, j]) <= 1e-12 * abs(A[i, i])
