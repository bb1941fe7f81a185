"""Host-only checks of the C-ABI library: it loads, exports every function
that include/dg.h declares, and validates arguments before touching the GPU.
No compute entry point reaches a kernel launch here: every call below fails
validation first (fake device addresses are never dereferenced)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg.h")


@pytest.fixture(scope="module")
def dg():
    from paper_2006_15698_amd import dg as mod
    return mod


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(dg):
    lib = ctypes.CDLL(dg.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), f"{name} declared in dg.h but not exported"
    # the binding wraps every declared function under the same name
    for name in names:
        assert hasattr(dg, name), f"binding lacks {name}"


def test_create_validates(dg):
    for bad in [(0, 1, 1, 1), (1, -2, 1, 1), (1, 1, 1, 8), (1, 1, 1, -1)]:
        with pytest.raises(dg.DGError):
            dg.dg_create(*bad, 1.4)
    with pytest.raises(dg.DGError):
        dg.dg_create(2, 2, 2, 1, 1.0)
    with pytest.raises(dg.DGError):
        dg.dg_create(2, 2, 2, 1, float("nan"))
    with pytest.raises(dg.DGError):
        dg.dg_create(65536, 65536, 2, 1, 1.4)   # > 2^31 elements


def test_quadrature_matches_library_rule(dg):
    for p in range(8):
        xi, w = dg.dg_quadrature(p)
        xr, wr = np.polynomial.legendre.leggauss(p + 1)
        assert np.max(np.abs(xi - xr)) < 1e-15
        assert np.max(np.abs(w - wr)) < 1e-15


def test_sizes(dg):
    ctx = dg.dg_create(3, 4, 5, 3, 1.4)
    try:
        assert dg.dg_num_dof(ctx) == 60 * 64
        nb = dg.dg_workspace_bytes(ctx)
        assert nb >= 2 * 30 * 16 * 60 * 8   # two face-trace buffers
        assert nb % 256 == 0
    finally:
        dg.dg_destroy(ctx)


def test_argument_errors_before_any_launch(dg):
    lib = dg._lib
    ctx = dg.dg_create(3, 2, 2, 2, 1.4)
    try:
        nd = 5 * dg.dg_num_dof(ctx)
        Q, R = 0x10000000, 0x20000000
        # no workspace yet
        assert lib.dg_rhs(ctx, Q, R) == dg.DG_EWORKSPACE
        assert lib.dg_rk_step(ctx, Q, R, ctypes.c_double(1e-3)) == dg.DG_EWORKSPACE
        # bad workspace
        assert lib.dg_set_workspace(ctx, 0x30000001, 1 << 30) == dg.DG_EINVAL
        assert lib.dg_set_workspace(ctx, 0x30000000, 16) == dg.DG_EWORKSPACE
        assert lib.dg_set_workspace(ctx, None, 1 << 30) == dg.DG_EINVAL
        assert lib.dg_set_workspace(ctx, 0x30000000, dg.dg_workspace_bytes(ctx)) == dg.DG_OK
        # aliasing
        assert lib.dg_rhs(ctx, Q, Q) == dg.DG_EALIAS
        assert lib.dg_rhs(ctx, Q, Q + 8 * (nd - 1)) == dg.DG_EALIAS
        assert lib.dg_rk_step(ctx, Q, Q + 8, ctypes.c_double(1e-3)) == dg.DG_EALIAS
        assert lib.dg_rhs_vjp(ctx, Q, R, Q) == dg.DG_EALIAS
        assert lib.dg_rhs_vjp(ctx, Q, R, R) == dg.DG_EALIAS
        # misaligned (not a multiple of 8 bytes)
        assert lib.dg_rhs(ctx, Q + 4, R) == dg.DG_EINVAL
        assert lib.dg_rk_step(ctx, Q, R + 4, ctypes.c_double(1e-3)) == dg.DG_EINVAL
        assert lib.dg_rhs_vjp(ctx, Q, R + 4, 0x40000000) == dg.DG_EINVAL
        assert lib.dg_rk_stage_vjp(ctx, 1, Q, R, 0x40000004, ctypes.c_double(1e-3)) == dg.DG_EINVAL
        # NULL
        assert lib.dg_rhs(ctx, None, R) == dg.DG_EINVAL
        assert lib.dg_rhs(ctx, Q, None) == dg.DG_EINVAL
        # stage and step ranges, dt
        assert lib.dg_rk_stage(ctx, 5, Q, R, ctypes.c_double(1e-3)) == dg.DG_EINVAL
        assert lib.dg_rk_stage(ctx, -1, Q, R, ctypes.c_double(1e-3)) == dg.DG_EINVAL
        assert lib.dg_rk_stage(ctx, 0, Q, R, ctypes.c_double(float("inf"))) == dg.DG_EINVAL
        assert lib.dg_rk_steps(ctx, Q, R, ctypes.c_double(1e-3), -1) == dg.DG_EINVAL
        assert lib.dg_rk_steps(ctx, Q, R, ctypes.c_double(1e-3), 0) == dg.DG_OK
        # domain and precision
        assert lib.dg_set_domain(ctx, 1.0, 0.0, 1.0) == dg.DG_EINVAL
        assert lib.dg_set_precision(ctx, 7) == dg.DG_EINVAL
        assert "precision" in dg.dg_last_error()
        # NULL context
        assert lib.dg_rhs(None, Q, R) == dg.DG_EINVAL
        assert lib.dg_num_dof(None) == -1
        assert lib.dg_workspace_bytes(None) == 0
    finally:
        dg.dg_destroy(ctx)
    dg.dg_destroy(None)


def test_options_validate_and_read_back(dg):
    ctx = dg.dg_create(4, 3, 2, 3, 1.4)
    try:
        defaults = {k: dg.dg_get_option(ctx, k) for k in dg.OPTION_NAMES}
        assert defaults[dg.DG_OPT_EXCHANGE] == dg.DG_EXCHANGE_NEIGHBOUR
        for key, good, bad in ((dg.DG_OPT_EXCHANGE, dg.DG_EXCHANGE_TRACES, 2),
                               (dg.DG_OPT_ORDER, dg.DG_ORDER_PENCIL, 5),
                               (dg.DG_OPT_PENCIL_X, 7, -1),
                               (dg.DG_OPT_PENCIL_Z, 3, 0)):
            dg.dg_set_option(ctx, key, good)
            assert dg.dg_get_option(ctx, key) == good
            with pytest.raises(dg.DGError):
                dg.dg_set_option(ctx, key, bad)
            assert dg.dg_get_option(ctx, key) == good   # a rejected value changes nothing
        dg.dg_set_option(ctx, dg.DG_OPT_XCD_REMAP, 5)
        assert dg.dg_get_option(ctx, dg.DG_OPT_XCD_REMAP) == 1
        dg.dg_set_option(ctx, dg.DG_OPT_XCD_REMAP, 0)
        assert dg.dg_get_option(ctx, dg.DG_OPT_XCD_REMAP) == 0
        # the viscous stage forms the inviscid rate in its flux launch by default
        assert defaults[dg.DG_OPT_VISC_FUSED] == 1
        dg.dg_set_option(ctx, dg.DG_OPT_VISC_FUSED, 0)
        assert dg.dg_get_option(ctx, dg.DG_OPT_VISC_FUSED) == 0
        dg.dg_set_option(ctx, dg.DG_OPT_VISC_FUSED, 3)
        assert dg.dg_get_option(ctx, dg.DG_OPT_VISC_FUSED) == 1
        with pytest.raises(dg.DGError):
            dg.dg_set_option(ctx, 99, 0)
        with pytest.raises(dg.DGError):
            dg.dg_get_option(ctx, 99)
        assert dg._lib.dg_get_option(ctx, dg.DG_OPT_ORDER, None) == dg.DG_EINVAL
    finally:
        dg.dg_destroy(ctx)


def test_visiting_order_is_a_bijection(tmp_path):
    """The stage kernel's workgroup -> element-block map, compiled for the
    host from the kernel's own header: every element is visited exactly
    once, and a pencil-order block never leaves its x-row, for ragged meshes,
    pencils, blocks and both XCD settings."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "order_map_check")
    src = os.path.join(ROOT, "tests", "order_map_check.cpp")
    cmd = [hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2006_15698_amd", "csrc"), src, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout


def test_paired_line_lane_map(tmp_path):
    """The paired neighbour-line lane map, compiled for the host from the
    kernel's own header: both faces of a direction are covered point by
    point exactly once, and each 16-byte load fetches the line nodes of two
    points that are neighbours in memory inside the element."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "pair_map_check")
    src = os.path.join(ROOT, "tests", "pair_map_check.cpp")
    cmd = [hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2006_15698_amd", "csrc"), src, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout


def test_varp_mesh_tables(dg, tmp_path):
    """The variable-degree builder's tables, checked on the host by a
    program compiled with the builder's own source: geometric neighbours of
    every face, the quarter of every hanging face, every face-flux double
    written once and every element face reading only written doubles, the
    element lists a partition by (degree, size) -- 241 seeded meshes."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "varp_mesh_check")
    libdir = os.path.dirname(dg.LIB_PATH)
    cmd = [hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2006_15698_amd", "csrc"), os.path.join(ROOT, "tests", "varp_mesh_check.cpp"),
           "-o", exe, "-L", libdir, "-ldg", f"-Wl,-rpath,{libdir}"]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout


def test_varp_host_logic(dg):
    """Variable-degree context: degree checks, node offsets (element blocks
    back to back), and workspace checks, all before any device access."""
    lib = dg._lib
    with pytest.raises(dg.DGError, match="degree 8"):
        dg.dg_varp_create(2, 1, 1, [1, 8])
    with pytest.raises(dg.DGError, match="degree -1"):
        dg.dg_varp_create(2, 1, 1, [-1, 0])
    with pytest.raises(dg.DGError):
        dg.dg_varp_create(0, 1, 1, [])
    with pytest.raises(dg.DGError, match="gamma"):
        dg.dg_varp_create(1, 1, 1, [2], gamma=0.9)
    with pytest.raises(dg.DGError, match="lengths"):
        dg.dg_varp_create(1, 1, 1, [2], L=(1.0, -1.0, 1.0))
    deg = np.array([[[0, 1, 7], [2, 3, 4]], [[5, 6, 1], [1, 2, 3]]])   # [nz, ny, nx]
    v = dg.dg_varp_create(3, 2, 2, deg)
    try:
        n3 = (deg.reshape(-1) + 1) ** 3
        off = np.concatenate([[0], np.cumsum(n3)])
        assert dg.dg_varp_num_dof(v) == off[-1]
        assert [dg.dg_varp_offset(v, e) for e in range(13)] == list(off)
        assert dg.dg_varp_offset(v, 13) == -1 and dg.dg_varp_offset(v, -1) == -1
        nb = dg.dg_varp_workspace_bytes(v)
        assert nb >= 5 * off[-1] * 8 and nb % 256 == 0
        Q, R = 0x10000000, 0x20000000
        assert lib.dg_varp_rhs(v, Q, R) == dg.DG_EWORKSPACE
        assert lib.dg_varp_set_workspace(v, 0x10000001, nb) == dg.DG_EINVAL       # misaligned
        assert lib.dg_varp_set_workspace(v, 0x10000000, nb - 256) == dg.DG_EWORKSPACE
        assert lib.dg_varp_rk_steps(v, Q, R, ctypes.c_double(1e-3), 1) == dg.DG_EWORKSPACE
    finally:
        dg.dg_varp_destroy(v)


def test_refined_host_logic(dg):
    """Refined-mesh context: refinement and degree checks, element count
    (a refined cell is eight elements), node offsets in element order, the
    workspace growing with the hanging faces' flux blocks."""
    lib = dg._lib
    with pytest.raises(dg.DGError, match="refinement 2"):
        dg.dg_varp_create_refined(2, 1, 1, [2, 0], [1] * 9)
    with pytest.raises(dg.DGError, match="degree 8"):
        dg.dg_varp_create_refined(2, 1, 1, [1, 0], [1] * 8 + [8])
    with pytest.raises(ValueError, match="degrees for 9 elements"):
        dg.dg_varp_create_refined(2, 1, 1, [1, 0], [1, 1])
    assert lib.dg_varp_create_refined(2, 1, 1, None, (ctypes.c_int * 2)(1, 1), (ctypes.c_double * 3)(1, 1, 1),
                                      ctypes.c_double(1.4)) is None
    ref = np.array([1, 0, 0, 1, 0, 0])   # 3 x 2 x 1 cells
    deg = np.arange(2 * 8 + 4) % 6
    v = dg.dg_varp_create_refined(3, 2, 1, ref, deg)
    u = dg.dg_varp_create(3, 2, 1, [1] * 6)
    try:
        assert dg.dg_varp_num_elements(v) == 20 and dg.dg_varp_num_elements(u) == 6
        off = np.concatenate([[0], np.cumsum((deg + 1) ** 3)])
        assert dg.dg_varp_num_dof(v) == off[-1]
        assert [dg.dg_varp_offset(v, e) for e in range(21)] == list(off)
        nb = dg.dg_varp_workspace_bytes(v)
        assert nb >= 5 * off[-1] * 8 * 2 and nb % 256 == 0
        assert lib.dg_varp_rhs(v, 0x10000000, 0x20000000) == dg.DG_EWORKSPACE
    finally:
        dg.dg_varp_destroy(v)
        dg.dg_varp_destroy(u)
