"""GPU tests of the device assembly (dd_assemble_2d) against the CPU
generator's assembly of the same nonlocal stiffness windows: constant,
fractional (vertex-sharing pairs on the mean of the mixed rules) and
peridynamic kernels at small sizes, and the constant (h = 1/128), fractional
(h = 1/96) and peridynamic (h = 1/160) benchmark systems at full size.

The two sum the same pair integrals in different orders (the device by
rounds of partner triangles per element), so an entry agrees to rounding of
its sum:
each row sums at most 6 elements x (2 ceil(delta/h) + 3)^2 x 2 partners x 49
quadrature products, a few 1e5 terms, so |device - generator| <= 1e-11 of the
largest entry of the row (about 1e5 x 1e-16 with a margin)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "2d-const-32": lambda: workloads.spec_2d_const(n=32, cuts=(2, 2)),
    "2d-frac-28": lambda: workloads.spec_2d_frac(n=28, delta=0.15, cuts=(2, 2)),
    "2d-pd-40": lambda: workloads.spec_2d_pd(n=40, delta=0.1, cuts=(3, 3), jitter=0.2),
    "2d-const-128": lambda: workloads.spec_2d_const(),
    # the fractional and peridynamic benchmark systems at full size
    "2d-frac-96": lambda: workloads.spec_2d_frac(),
    "2d-pd-160": lambda: workloads.spec_2d_pd(),
}


def _dd():
    import paper_2306_00094_amd as dd
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dd.load_library()
    return dd


def device_windows(dd, spec):
    R = workloads.window_radius(spec)
    W = 2 * R + 1
    nc = 4 if spec.kernel == workloads.KER_PD else 1
    win = torch.empty((spec.n - 1) ** 2 * W * W * nc, dtype=torch.float64, device="cuda")
    dd.dd_assemble_2d(spec.n, spec.collar, spec.delta, spec.kernel, spec.phi, spec.s, R, win)
    torch.cuda.synchronize()
    return win.cpu().numpy(), W * W * nc


@pytest.mark.parametrize("name", list(CASES))
def test_device_assembly_matches_generator(name):
    dd = _dd()
    spec = CASES[name]()
    print(f"case assembly {name} n={spec.n} kernel={spec.kernel}", flush=True)
    ref = workloads.assemble_windows(spec)
    got, rowlen = device_windows(dd, spec)
    assert got.shape == ref.shape
    ref = ref.reshape(-1, rowlen)
    got = got.reshape(-1, rowlen)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.all(scale > 0)
    err = (np.abs(got - ref) / scale).max()
    print(f"  max |device - generator| / row max = {err:.2e}", flush=True)
    assert err <= 1e-11
    # the same zero pattern: entries of pairs outside the truncation stay zero
    assert np.array_equal(got == 0.0, ref == 0.0)


@pytest.mark.parametrize("name", ["2d-const-32", "2d-frac-28", "2d-pd-40", "2d-const-128"])
def test_device_assembly_is_bit_reproducible(name):
    """Every window entry is summed in a fixed order: two launches on the same
    arguments give the same bits."""
    dd = _dd()
    spec = CASES[name]()
    print(f"case assembly repeat {name} n={spec.n} kernel={spec.kernel}", flush=True)
    a, _ = device_windows(dd, spec)
    b, _ = device_windows(dd, spec)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_device_assembly_feeds_the_solver():
    """The device windows, turned into the partitioned system by the same host
    code as the generator's, give the generator's solution within the FP64
    gate."""
    dd = _dd()
    import oracle
    spec = CASES["2d-const-32"]()
    print("case assembly feeds solver", flush=True)
    wl = workloads.build(spec)
    got, _ = device_windows(dd, spec)
    A_dev = workloads.windows_to_matrix(spec, got)
    b = workloads.rhs(spec)
    u_gen = oracle.monolithic_solve(wl.asm.A, b)
    u_dev = oracle.monolithic_solve(A_dev, b)
    assert oracle.rel_err(u_dev, u_gen).max() <= 1e-10
