"""The C-ABI library: it loads without a GPU, exports every entry point that
include/dd.h declares (the Python binding uses the same names), and its
host-side validation rejects malformed input.  No device work is started."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dd.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2306_00094_amd as dd
    if not os.path.exists(dd.LIB_PATH):
        from paper_2306_00094_amd import _build
        _build.build()
    return dd, dd.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dd_setup", "dd_factor", "dd_solve", "dd_destroy", "dd_footprint",
                     "dd_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    dd, so = lib
    out = subprocess.run(["nm", "-D", "--defined-only", dd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(so, name)
    assert sorted(dd.EXPORTED) == declared_functions()


def test_default_opts(lib):
    dd, _ = lib
    o = dd.dd_default_opts()
    assert (o.tol, o.max_it, o.precond, o.max_refine, o.inner_tol, o.fp64_fallback,
            o.apply, o.launch, o.check_every, o.verify) == (1e-10, 1000, 1, 8, 0.0, 1, 0, 0, 0, 1)


@pytest.fixture(scope="module")
def small():
    return W.build(W.spec_1d(n=64, strips=2)).dd


def test_footprint_counts_matrices_and_factors(lib, small):
    dd, _ = lib
    b64 = dd.dd_footprint(small, dd.DD_FP64, 1)
    b32 = dd.dd_footprint(small, dd.DD_MIXED, 1)
    kii = sum(k.size for k in small.kii) * 8
    assert b64 >= 3 * kii                          # K_II, factor, inverse
    assert b32 >= kii + 2 * kii // 2
    assert dd.dd_footprint(small, dd.DD_FP64, 64) > b64


def _copy(dd):
    import copy
    return copy.deepcopy(dd)


@pytest.mark.parametrize("breaker,msg", [
    (lambda p: p.i_maps.__setitem__(0, np.concatenate([p.i_maps[0][:-1], p.i_maps[0][:1]])),
     "assigned twice"),
    (lambda p: p.g_maps.__setitem__(0, p.g_maps[0] + p.n_gamma), "g_map entry out of range"),
    (lambda p: p.__setattr__("gamma_map", p.gamma_map[::-1][:-1].copy()), "n_gamma"),
    (lambda p: p.i_maps.__setitem__(1, p.i_maps[1][:-1]), "neither interior nor interface"),
])
def test_setup_rejects_malformed_input(lib, small, breaker, msg):
    dd, _ = lib
    p = _copy(small)
    breaker(p)
    if msg == "n_gamma":
        p.n_gamma = len(p.gamma_map)
        msg = "out of range"
    if msg == "neither interior nor interface":
        p.kii[1] = p.kii[1][:-1, :-1].copy()
        p.kig[1] = p.kig[1][:-1]
    with pytest.raises(dd.DDError) as ei:
        dd.dd_setup(p, stream=0, max_nrhs=1)
    assert ei.value.status == dd.DD_EINVAL
    assert msg in str(ei.value) or "out of range" in str(ei.value)


def test_setup_rejects_bad_batch_width(lib, small):
    dd, _ = lib
    for m in (0, 65):
        with pytest.raises(dd.DDError) as ei:
            dd.dd_setup(small, stream=0, max_nrhs=m)
        assert ei.value.status == dd.DD_EINVAL


def test_assemble_rejects_bad_arguments(lib):
    """Device assembly validates its arguments on the host (no device work):
    unknown kernel, too few cells, a window that misses partners, one wider
    than 128 nodes, window copies beyond 64 KiB per row."""
    dd, L = lib
    fake = ctypes.c_void_p(256)               # never dereferenced: every call fails validation
    cases = [
        ((32, 3, 0.1, 7, 1.0, 0.0, 8), "unknown kernel"),
        ((1, 3, 0.1, 0, 1.0, 0.0, 8), "n < 2"),
        ((32, 3, 0.1, 0, 1.0, 0.0, 5), "misses partners"),      # ceil(0.1 * 32) + 2 = 6
        ((32, 3, 0.1, 0, 1.0, 0.0, 100), "wider than 128"),
        ((64, 3, 0.5, 0, 1.0, 0.0, 34), "64 KiB"),      # delta n = 32: about 3 500 nodes x 4 copies
        ((64, 3, 0.25, 2, 1.0, 0.0, 18), "64 KiB"),     # delta n = 16: about 960 nodes x 3 x 4
    ]
    for args, msg in cases:
        st = L.dd_assemble_2d(*args, fake, None)
        assert st == dd.DD_EINVAL, args
        assert msg in L.dd_last_error(None).decode(), args


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with a message."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_traffic_needs_matching_kernel_source():
    """The stored counter traffic is reported only for the kernel source it was
    measured on."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    import copy
    saved = copy.deepcopy(bench.MEASURED_TRAFFIC)
    try:
        for key, m in saved.items():
            bench.MEASURED_TRAFFIC[key] = dict(m, sha="0" * 16)
            assert bench.measured_traffic(key, m["workload"]) is None
            assert bench.measured_traffic(key, "another workload") is None
            # with the sha of the file as it stands the stored figure is reported
            import hashlib
            src = os.path.join(root, "paper_2306_00094_amd", "csrc", m["src"])
            with open(src, "rb") as f:
                bench.MEASURED_TRAFFIC[key] = dict(m, sha=hashlib.sha256(f.read()).hexdigest()[:16])
            v = bench.measured_traffic(key, m["workload"])
            assert v == 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])
    finally:
        bench.MEASURED_TRAFFIC.clear()
        bench.MEASURED_TRAFFIC.update(saved)
    assert bench.measured_traffic("no such kernel", "cfg4") is None


def test_undecomposed_problem_passes_host_checks(lib):
    """n_sub = 0 (every dof an interface dof, K_GG = A: the paper's baseline
    Jacobi-preconditioned CG on the whole system) is valid input: it has a
    footprint without factor storage, and a gamma_map that is not a
    permutation is still rejected."""
    dd, _ = lib
    A = W.build(W.spec_1d(n=64, strips=2)).asm.A
    und = W.undecomposed(A)
    assert und.n_sub == 0
    nbytes = dd.dd_footprint(und, dd.DD_FP64, 1)
    assert A.nnz * 12 <= nbytes < A.nnz * 12 + 64 * A.shape[0] * 8 + (1 << 20)
    bad = W.undecomposed(A)
    bad.gamma_map = bad.gamma_map.copy()
    bad.gamma_map[0] = 1
    with pytest.raises(dd.DDError) as ei:
        dd.dd_setup(bad, stream=0, max_nrhs=1)
    assert ei.value.status == dd.DD_EINVAL and "not injective" in str(ei.value)


def test_bench_assembly_work_count_brute_force():
    """The element-pair count behind the assembly leg's roofline (one free
    node's interacting pairs times the number of rows) equals a brute-force
    count over every free node, every element holding it and every element
    of the mesh, with the barycentre test written in real coordinates."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec_b = importlib.util.spec_from_file_location("bench_mod2", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec_b)
    spec_b.loader.exec_module(bench)
    for spec in (W.spec_2d_const(n=32, cuts=(2, 2)), W.spec_2d_frac(n=28, delta=0.15, cuts=(2, 2))):
        n, c, h = spec.n, spec.collar, spec.h
        N = n + 2 * c
        # barycentres of all triangles of the mesh (with collar), real coordinates
        a, b = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
        a, b = a.ravel(), b.ravel()
        bary = np.concatenate([np.stack([(3 * a + 2) / 3, (3 * b + 1) / 3], 1),      # lower right
                               np.stack([(3 * a + 1) / 3, (3 * b + 2) / 3], 1)]) * h  # upper left
        total = 0
        for mb in range(c + 1, c + n):
            for ma in range(c + 1, c + n):
                # the six triangles holding node (ma, mb)
                es = [((ma - 1) + 2 / 3, (mb - 1) + 1 / 3), ((ma - 1) + 1 / 3, (mb - 1) + 2 / 3),
                      (ma + 1 / 3, (mb - 1) + 2 / 3), ((ma - 1) + 2 / 3, mb + 1 / 3),
                      (ma + 2 / 3, mb + 1 / 3), (ma + 1 / 3, mb + 2 / 3)]
                for ex, ey in es:
                    d2 = (bary[:, 0] - ex * h) ** 2 + (bary[:, 1] - ey * h) ** 2
                    total += int(np.count_nonzero(d2 <= spec.delta ** 2 * (1 + 1e-12)))
        assert bench.interacting_pairs_per_row(spec) * (n - 1) ** 2 == total
