"""Pins of the 2D stiffness assembly (workloads/nlasm.c) against a plain
evaluation of the bilinear form of eq. bil1 written out independently here.

For a free node m the row of A holds, for every node n,
    A(psi_m, psi_n) = sum over ordered element pairs (E, F)
                      int_E int_F (psi_m(y) - psi_m(x)) (psi_n(y) - psi_n(x)) gamma(x, y) dy dx,
with x in E and y in F, the pair kept when the barycentres of E and F are
within delta (the barycentre approximate ball of the section "Approximate
interaction balls", applied per element pair), the integrals by the
7-point degree-5 rule on each triangle, and -- for the fractional kernel of
eq. fractionalkernel on pairs that share a vertex -- the mean of the
(7-point x 6-point) and (6-point x 7-point) product rules.  Kernels:
constant phi (eq. constantkernel), phi |x-y|^-(2+2s) (eq. fractionalkernel)
and the peridynamic tensor phi (x-y)(x-y)^T / |x-y|^3 (eq. peridynamics).

The loop below visits every ordered pair (E, F) with m in E or m in F and
evaluates basis functions from barycentric coordinates; it does not use the
generator's row shortcut (pairs (F, E) folded into (E, F) by a factor).  The
quadrature rules are built from their published closed forms and pinned by
exactness on monomials.  CPU only."""
import math

import numpy as np
import pytest

import workloads as W


# ------------------------------------------------------------ quadrature --
def rule7():
    """Radon's 7-point degree-5 rule on a triangle (barycentric points,
    weights summing to 1)."""
    r = math.sqrt(15.0)
    pts = [(1 / 3, 1 / 3, 1 / 3)]
    wts = [9.0 / 40.0]
    for a, w in (((6 - r) / 21, (155 - r) / 1200), ((6 + r) / 21, (155 + r) / 1200)):
        b = 1 - 2 * a
        for p in ((a, a, b), (a, b, a), (b, a, a)):
            pts.append(p)
            wts.append(w)
    return np.array(pts), np.array(wts)


def rule6():
    """Dunavant's 6-point degree-4 rule (published to 15 digits)."""
    pts, wts = [], []
    for a, w in ((0.445948490915965, 0.223381589678011), (0.091576213509771, 0.109951743655322)):
        b = 1 - 2 * a
        for p in ((a, a, b), (a, b, a), (b, a, a)):
            pts.append(p)
            wts.append(w)
    return np.array(pts), np.array(wts)


@pytest.mark.parametrize("rule,deg,tol", [(rule7, 5, 1e-15), (rule6, 4, 1e-14)])
def test_triangle_rules_exact_on_monomials(rule, deg, tol):
    """Mean of x^i y^j over the unit right triangle is 2 i! j! / (i+j+2)!;
    the rule must reproduce it for every i + j <= deg, and fail at deg + 1."""
    pts, wts = rule()
    x, y = pts[:, 1], pts[:, 2]                     # vertices (0,0), (1,0), (0,1)
    worst = 0.0
    for i in range(deg + 1):
        for j in range(deg + 1 - i):
            exact = 2.0 * math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            worst = max(worst, abs(wts @ (x ** i * y ** j) - exact))
    assert worst <= tol
    over = max(abs(wts @ (x ** i * y ** (deg + 1 - i))
                   - 2.0 * math.factorial(i) * math.factorial(deg + 1 - i) / math.factorial(deg + 3))
               for i in range(deg + 2))
    assert over > 1e-6


# ------------------------------------------------------------------ mesh --
def mesh(spec):
    """Extended structured mesh: nodes (a, b), a, b = 0..N at ((a-c)h, (b-c)h);
    cell (a, b) split into (a,b),(a+1,b),(a+1,b+1) and (a,b),(a+1,b+1),(a,b+1)."""
    n, c = spec.n, spec.collar
    N, h = n + 2 * c, spec.h
    elems = []
    for ca in range(N):
        for cb in range(N):
            elems.append(((ca, cb), (ca + 1, cb), (ca + 1, cb + 1)))
            elems.append(((ca, cb), (ca + 1, cb + 1), (ca, cb + 1)))
    xy = lambda v: np.array([(v[0] - c) * h, (v[1] - c) * h])
    return elems, xy


def brute_row(spec, m):
    """Row of node m (extended coordinates) as {node: value} (scalar kernels)
    or {node: 2x2 block} (peridynamics), by the plain loop over ordered pairs."""
    elems, xy = mesh(spec)
    h, delta, phi = spec.h, spec.delta, spec.phi
    area = 0.5 * h * h
    r7, r6 = rule7(), rule6()
    V = {e: np.array([xy(v) for v in e]) for e in elems}
    bary = {e: V[e].mean(axis=0) for e in elems}
    row = {}
    holds_m = [e for e in elems if m in e]
    pairs = set()
    for E in holds_m:
        for F in elems:
            pairs.add((E, F))
            pairs.add((F, E))
    for E, F in pairs:
        if np.linalg.norm(bary[E] - bary[F]) > delta:
            continue
        touching = bool(set(E) & set(F))
        if spec.kernel == W.KER_FRAC and touching:
            combos = [(r7, r6, 0.5), (r6, r7, 0.5)]
        else:
            combos = [(r7, r7, 1.0)]
        nodes = sorted(set(E) | set(F))
        for (pE, wE), (pF, wF), sc in combos:
            X = pE @ V[E]                                    # points in E
            Y = pF @ V[F]                                    # points in F
            S = X[:, None, :] - Y[None, :, :]                # x - y
            r = np.linalg.norm(S, axis=2)
            wgt = sc * area * area * wE[:, None] * wF[None, :]

            def d(nd):                                       # psi_nd(y) - psi_nd(x)
                py = pF[:, list(F).index(nd)] if nd in F else np.zeros(len(wF))
                px = pE[:, list(E).index(nd)] if nd in E else np.zeros(len(wE))
                return py[None, :] - px[:, None]

            dm = d(m)
            for nd in nodes:
                t = wgt * dm * d(nd)
                if spec.kernel == W.KER_CONST:
                    val = phi * t.sum()
                elif spec.kernel == W.KER_FRAC:
                    val = phi * (t * r ** (-(2.0 + 2.0 * spec.s))).sum()
                else:
                    with np.errstate(divide="ignore", invalid="ignore"):
                        g = np.where(r > 0, phi / r ** 3, 0.0) * t
                    val = np.array([[(g * S[:, :, i] * S[:, :, j]).sum() for j in range(2)]
                                    for i in range(2)])
                row[nd] = row.get(nd, 0.0) + val
    return row


def generator_row(spec, win, m):
    """The same row from the generator's window (free node m)."""
    n, c = spec.n, spec.collar
    R = W.window_radius(spec)
    Wd = 2 * R + 1
    ia, ib = m[0] - c - 1, m[1] - c - 1
    i = ib * (n - 1) + ia
    rowlen = Wd * Wd * (4 if spec.kernel == W.KER_PD else 1)
    w = win[i * rowlen:(i + 1) * rowlen]
    out = {}
    for db in range(-R, R + 1):
        for da in range(-R, R + 1):
            k = (db + R) * Wd + (da + R)
            nd = (m[0] + da, m[1] + db)
            if spec.kernel == W.KER_PD:
                blk = np.array([[w[(0 * Wd * Wd + k) * 2 + 0], w[(0 * Wd * Wd + k) * 2 + 1]],
                                [w[(1 * Wd * Wd + k) * 2 + 0], w[(1 * Wd * Wd + k) * 2 + 1]]])
                if np.any(blk != 0):
                    out[nd] = blk
            elif w[k] != 0.0:
                out[nd] = w[k]
    return out


SPECS = {
    # delta / h = 1.62 and 2.4: no barycentre distance falls on the threshold
    # ((3 delta / h)^2 is not an integer)
    "const": W.spec_2d_const(n=6, delta=0.27, cuts=(1, 1)),
    "frac": W.spec_2d_frac(n=6, delta=0.27, s=0.5, cuts=(1, 1)),
    "frac-s04": W.spec_2d_frac(n=5, delta=0.48, s=0.4, cuts=(1, 1)),
    "pd": W.spec_2d_pd(n=6, delta=0.27, cuts=(1, 1), jitter=0.0),
    # delta / h = 3.6 (the benchmark systems have 8 to 12.8)
    "const-wide": W.spec_2d_const(n=8, delta=0.45, cuts=(1, 1)),
    "frac-wide": W.spec_2d_frac(n=8, delta=0.45, s=0.5, cuts=(1, 1)),
    "pd-wide": W.spec_2d_pd(n=8, delta=0.45, cuts=(1, 1), jitter=0.0),
}


@pytest.mark.parametrize("name", list(SPECS))
def test_generator_rows_equal_plain_pair_loop(name):
    spec = SPECS[name]
    c, n = spec.collar, spec.n
    win = W.assemble_windows(spec)
    # a corner row, a row next to the boundary and a central row
    rows = [(c + 1, c + 1), (c + 2, c + 1), (c + n // 2, c + n // 2)]
    for m in rows:
        ref = brute_row(spec, m)
        got = generator_row(spec, win, m)
        scale = max(np.abs(v).max() for v in ref.values())
        assert set(k for k, v in ref.items() if np.abs(v).max() > 1e-14 * scale) <= set(got), m
        for nd in set(ref) | set(got):
            a = ref.get(nd, 0.0)
            b = got.get(nd, 0.0)
            assert np.abs(np.asarray(a) - np.asarray(b)).max() <= 1e-13 * scale, (m, nd, a, b)


def test_brute_force_detects_a_wrong_fractional_power(monkeypatch):
    """The pin is sharp: the plain loop with a power off by 0.1 disagrees
    with the generator far beyond the gate."""
    spec = SPECS["frac"]
    win = W.assemble_windows(spec)
    m = (spec.collar + 3, spec.collar + 3)
    got = generator_row(spec, win, m)
    wrong = W.spec_2d_frac(n=6, delta=0.27, s=0.55, cuts=(1, 1))
    wrong.phi = spec.phi
    ref = brute_row(wrong, m)
    scale = max(abs(v) for v in ref.values())
    assert max(abs(ref.get(k, 0.0) - got.get(k, 0.0)) for k in ref) > 1e-3 * scale


# --------------------------------------------------------------- symmetry --
@pytest.mark.parametrize("spec", [W.spec_2d_const(n=20, delta=0.15, cuts=(1, 1)),
                                  W.spec_2d_frac(n=20, delta=0.15, cuts=(1, 1)),
                                  W.spec_2d_pd(n=16, delta=0.2, cuts=(1, 1), jitter=0.0)],
                         ids=lambda s: s.name)
def test_2d_raw_assembly_symmetric(spec):
    """The rows are assembled independently (row m sums the pairs touching m),
    so A_raw = A_raw^T holds only up to rounding: |A - A^T| <= 64 eps |A|_max."""
    A = W.windows_to_matrix(spec, W.assemble_windows(spec), symmetrise=False)
    D = (A - A.T).tocoo()
    amax = np.abs(A.data).max()
    assert (np.abs(D.data).max() if D.nnz else 0.0) <= 64 * np.finfo(float).eps * amax
    # the pattern is symmetric as well
    P = (A != 0).astype(int)
    assert (P - P.T).nnz == 0
