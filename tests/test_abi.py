"""C-ABI library checks that need no GPU: it loads, exports every entry point
declared in include/lbm.h, and rejects invalid arguments on the host before
any HIP call.  Also checks that the product package never reaches the oracle."""
import ctypes
import math
import os
import re

import pytest

from paper_1105_2904_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    names = _declared()
    assert "lbm_create" in names and "lbm_step" in names and len(names) >= 17
    for n in names:
        assert hasattr(L, n), n


def test_strerror_covers_every_code():
    for code in range(0, -10, -1):
        assert lbm.lbm_strerror(code) != "unknown error"
    assert lbm.lbm_strerror(-99) == "unknown error"


def _rc_workspace(**kw):
    base = dict(lattice=19, nx=16, ny=16, nz=16, tau=0.6, storage="fp32", max_particles=4, max_radius=3.0)
    base.update(kw)
    p = lbm.make_params(**base)
    n = ctypes.c_size_t(0)
    return lbm.lib().lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)), n.value


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), lbm.LBM_EINVAL),
    (dict(tau=float("nan")), lbm.LBM_ENONFINITE),
    (dict(lattice=15), lbm.LBM_EINVAL),
    (dict(lattice=9, nz=2), lbm.LBM_EINVAL),
    (dict(nx=0), lbm.LBM_EINVAL),
    (dict(nx=2048, ny=1024, nz=1024), lbm.LBM_EINVAL),
    (dict(storage=7), lbm.LBM_EINVAL),
    (dict(max_particles=-1), lbm.LBM_EINVAL),
    (dict(max_radius=0.0), lbm.LBM_EINVAL),
    (dict(max_radius=200.0), lbm.LBM_EINVAL),
    (dict(gravity=(0, 0, math.inf)), lbm.LBM_ENONFINITE),
    (dict(walls=8), lbm.LBM_EINVAL),
    (dict(lattice=9, nz=1, walls=4), lbm.LBM_EINVAL),   # no z walls in 2D
    (dict(ny=4, walls=2), lbm.LBM_EINVAL),               # no fluid layer left
    (dict(walls=2, wall_velocity=[0] * 7 + [0.01] + [0] * 10), lbm.LBM_EINVAL),  # normal wall velocity
    (dict(walls=2, wall_velocity=[0] * 6 + [math.nan] + [0] * 11), lbm.LBM_ENONFINITE),
    (dict(nx=1024, ny=1024, nz=1024, storage="fp64"), lbm.LBM_EINVAL),  # a plane above 4 GiB
    (dict(nx=1024, ny=1024, nz=1025, storage="fp32"), lbm.LBM_EINVAL),
])
def test_invalid_parameters_rejected_on_host(kw, code):
    rc, _ = _rc_workspace(**kw)
    assert rc == code


def test_plane_limit_and_aa_layout():
    """Population planes of up to 4 GiB (32-bit offsets): FP32 1024^3 is the
    largest cube.  The AA layout keeps one population array instead of two;
    any other value of the flag is refused."""
    rc, _ = _rc_workspace(nx=1024, ny=1024, nz=1024, storage="fp32", max_particles=0)
    assert rc == 0
    rc2, n2 = _rc_workspace()
    rc1, n1 = _rc_workspace(aa=True)
    assert rc1 == rc2 == 0
    # one FP32 population array less (blocks of 2048 sites: the sites rounded
    # up to whole blocks), one 4-double-per-site staging area more (256-B
    # alignment)
    N = 16 ** 3
    stride = (N + 2047) // 2048 * 2048
    expect = 19 * stride * 4 - 4 * 8 * N
    assert abs((n2 - n1) - expect) <= 512
    p = lbm.make_params(19, 16, 16, 16, tau=0.6, max_particles=4, max_radius=3.0)
    p.aa = 2
    n = ctypes.c_size_t(0)
    assert lbm.lib().lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == lbm.LBM_EINVAL


def test_workspace_size_scales_with_box_and_precision():
    rc32, n32 = _rc_workspace()
    rc64, n64 = _rc_workspace(storage="fp64")
    assert rc32 == rc64 == 0
    # two population buffers dominate: q N sizeof(storage) each
    N = 16 ** 3
    assert n32 >= 2 * 19 * N * 4 and n64 >= 2 * 19 * N * 8
    assert n64 - n32 >= 2 * 19 * N * 4


def test_create_rejects_bad_workspace_without_gpu():
    p = lbm.make_params(19, 16, 16, 16, tau=0.6, max_particles=2, max_radius=3.0)
    need = lbm.lbm_workspace_size(p)
    ctx = ctypes.c_void_p()
    L = lbm.lib()
    assert L.lbm_create(ctypes.byref(p), None, need, None, ctypes.byref(ctx)) == lbm.LBM_EWORKSPACE
    assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(4096 * 1024 + 8), need, None,
                        ctypes.byref(ctx)) == lbm.LBM_EWORKSPACE
    assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(4096 * 1024), need - 1, None,
                        ctypes.byref(ctx)) == lbm.LBM_EWORKSPACE
    bad = lbm.make_params(19, 16, 16, 16, tau=0.4)
    assert L.lbm_create(ctypes.byref(bad), ctypes.c_void_p(4096 * 1024), need, None,
                        ctypes.byref(ctx)) == lbm.LBM_EINVAL


def test_bytes_per_site():
    assert lbm.lbm_bytes_per_site(lbm.make_params(19, 8, 8, 8, storage="fp32")) == 152
    assert lbm.lbm_bytes_per_site(lbm.make_params(19, 8, 8, 8, storage="fp64")) == 304
    assert lbm.lbm_bytes_per_site(lbm.make_params(9, 8, 8, 1, storage="fp32")) == 72


def test_null_context_and_arguments():
    L = lbm.lib()
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_forces(None, None, None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_destroy(None) == lbm.LBM_EINVAL
    assert L.lbm_device_copy(None, None, 16, 1, None) == lbm.LBM_EINVAL
    assert L.lbm_device_copy(None, None, 16, 0, None) == lbm.LBM_EINVAL


def test_product_path_never_uses_the_oracle():
    pkg = os.path.join(ROOT, "paper_1105_2904_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "lbm_oracle" not in text and "ora_" not in text, f


def test_closure_inputs_match_the_oracle_bit_for_bit():
    """The library's closure inputs (host side of the same function the
    closure kernel uses) equal the oracle's, rounded to FP32, for random pairs
    including minimum-image ones."""
    import numpy as np
    import oracle
    rng = np.random.Generator(np.random.PCG64(12))
    for k in range(40):
        L = (int(rng.integers(40, 90)), int(rng.integers(40, 90)))
        ri, rj = rng.uniform(6, 12, 2)
        xi = rng.uniform(0, 1, 2) * L
        ang = rng.uniform(0, 2 * np.pi)
        dist = ri + rj + rng.uniform(0.05, 2.0)
        xj = (xi + dist * np.array([np.cos(ang), np.sin(ang)])) % L
        tau = rng.uniform(0.55, 1.0)
        o = oracle.Oracle(9, L[0], L[1], 1, tau)
        o.add_particles([[xi[0], xi[1], 0], [xj[0], xj[1], 0]], radius=[ri, rj], mass=1.0, inertia=1.0)
        ref = o.closure_inputs(0, 1).astype(np.float32)
        d = xj - xi
        d -= np.array(L) * np.floor(d / np.array(L) + 0.5)
        ours = lbm.closure_inputs(xi, d, ri, rj, tau)[0]
        assert np.array_equal(ours, ref), (k, ours, ref)


def test_bench_measures_one_gpu_only():
    """bench.py refuses a multi-GPU run with a message and exit status 2,
    before it touches a device (the library has one-GPU code only)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_kernel_names_match_the_counter_runs():
    """The sweep kernel names bench.py looks up in the committed HBM counter
    runs are the names those runs list, for every storage and both sweep
    kernels, so that roofline.traffic can only go null when the sources
    change (hash) and not through a naming slip."""
    import importlib.util
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    with open(bench.COUNTERS) as fh:
        c = json.load(fh)
    names = {e[0] for e in c["entries"]}
    for tname in ("float", "_Float16", "bf16s"):
        for width in (0, 256):
            k = bench.sweep_kernel(width, 19, tname, True, "0", 256).replace(",", ", ")
            assert k in names, k
    # the AA pattern's two halves (even and odd steps) are separate kernels;
    # an AA context runs the FP32 context's tuned launch (row or tile kernel)
    for layout in ("1", "2"):
        ks = [bench.sweep_kernel(w, 19, "float", True, layout, 256).replace(",", ", ") for w in (0, 256)]
        assert any(k in names for k in ks), ks
