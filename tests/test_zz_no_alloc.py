"""The allocation-free Schur product (dd_schur_apply_noalloc, its work vectors
in the library's static device array) against dd_schur_apply on the same
context: two calls in a row, the second on a smaller input (fewer columns,
then a smaller system), each equal to the allocating entry point's result;
work beyond the static array is rejected with DD_EINVAL."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dd():
    import paper_2306_00094_amd as dd
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dd.load_library()
    return dd


def interface_block(n_gamma, nrhs, seed, pad=3):
    """Column-major n_gamma x nrhs block with leading dimension n_gamma + pad
    (torch: nrhs rows of n_gamma + pad), the padding filled with NaN."""
    rng = np.random.default_rng(seed)
    a = np.full((nrhs, n_gamma + pad), np.nan)
    a[:, :n_gamma] = rng.uniform(-1.0, 1.0, (nrhs, n_gamma))
    return torch.from_numpy(a).to("cuda:0")


def both(dd, s, prec, p, nrhs):
    ld = int(p.shape[1])
    q0 = torch.full_like(p, 7.0)
    q1 = torch.full_like(p, -7.0)
    dd.dd_schur_apply(s.ctx, prec, p, q0, nrhs, ld)
    dd.dd_schur_apply_noalloc(s.ctx, prec, p, q1, nrhs, ld)
    return q0[:, :s.n_gamma].cpu().numpy(), q1[:, :s.n_gamma].cpu().numpy(), q1[:, s.n_gamma:].cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_schur_apply_matches_allocating_entry(prec):
    dd = _dd()
    big = workloads.build(workloads.spec_2d_pd(n=40, delta=0.15, cuts=(3, 3), jitter=0.2, nrhs=1))
    small = workloads.build(workloads.spec_1d(n=160, delta=0.05, strips=3, nrhs=1))
    cases = [(big, 8, 1), (big, 3, 2), (small, 2, 3)]      # each call smaller than the one before
    solvers = {}
    try:
        for wl, nrhs, seed in cases:
            key = id(wl)
            if key not in solvers:
                solvers[key] = dd.Solver(wl.dd, max_nrhs=8)
                solvers[key].factor(prec)
            s = solvers[key]
            print(f"case noalloc prec={prec} n_gamma={s.n_gamma} nrhs={nrhs}", flush=True)
            p = interface_block(s.n_gamma, nrhs, seed)
            q0, q1, tail = both(dd, s, prec, p, nrhs)
            scale = np.abs(q0).max()
            assert np.isfinite(q1).all()
            assert np.abs(q1 - q0).max() <= 1e-14 * scale, np.abs(q1 - q0).max() / scale
            assert (tail == -7.0).all()                  # rows past n_gamma untouched
    finally:
        for s in solvers.values():
            s.close()


def test_noalloc_rejects_work_beyond_the_static_array():
    """(2 n_gamma + 2 n_I) * next_pow2(nrhs) doubles must fit in 4 Mi doubles:
    a 40 000-row undecomposed system takes 32 columns, not 64."""
    dd = _dd()
    n = 40000
    A = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    s = dd.Solver(workloads.undecomposed(A), max_nrhs=64)
    try:
        s.factor(dd.DD_FP64)
        print("case noalloc limit", flush=True)
        p = interface_block(n, 64, 5, pad=0)
        q = torch.zeros_like(p)
        with pytest.raises(dd.DDError) as ei:
            dd.dd_schur_apply_noalloc(s.ctx, dd.DD_FP64, p, q, 64, n)
        assert ei.value.status == dd.DD_EINVAL and "static scratch" in str(ei.value)
        p32 = p[:32].contiguous()
        q0, q1, _ = both(dd, s, dd.DD_FP64, p32, 32)
        assert np.abs(q1 - q0).max() <= 1e-14 * np.abs(q0).max()
        # S = A here: the product itself
        ref = (A @ p32.cpu().numpy().T).T
        assert np.abs(q1 - ref).max() <= 1e-13 * np.abs(ref).max()
    finally:
        s.close()
