"""CPU tests of the HIP library's host side: it loads, exports every symbol the
header declares, sizes workspaces, rejects bad arguments before any launch,
and its exact fixed-point helpers agree with 128-bit integer arithmetic."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtforest.h")


@pytest.fixture(scope="module")
def L():
    import paper_1901_05423_amd as rtf
    if not os.path.exists(rtf.LIB_PATH):
        from paper_1901_05423_amd.build import build_library
        build_library()
    return rtf.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rtf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rtf_build", "rtf_build_batched", "rtf_sample", "rtf_sample_batched",
                 "rtf_sample_2d", "rtf_backward", "rtf_quantize_f32", "rtf_check",
                 "rtf_forest_export", "rtf_workspace_bytes", "rtf_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    nm = subprocess.run(["nm", "-D", "--defined-only", L._name], capture_output=True,
                        text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rtf_\w+)", nm))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_binding_covers_the_header():
    import paper_1901_05423_amd as rtf
    assert set(declared_functions()) == set(rtf.SIGNATURES)


def test_workspace_sizes(L):
    a = L.rtf_workspace_bytes(1 << 24, 1 << 24)
    assert a >= 16 * (1 << 24) + 4 * (1 << 24)
    assert a % 256 == 0
    assert L.rtf_workspace_bytes(0, 5) == 0
    assert L.rtf_workspace_bytes(5, 0) == 0
    assert L.rtf_workspace_bytes(1 << 31, 5) == 0
    assert L.rtf_workspace_bytes_batched(3, 2, 10) == 0  # fewer weights than distributions
    assert L.rtf_workspace_bytes_batched(3, 30, 30) > 0
    assert L.rtf_backward_workspace_bytes(2, 100) >= 2 * 8 * 100


def test_argument_errors_before_launch(L):
    import paper_1901_05423_amd as rtf
    desc = rtf.rtf_forest()
    P = ctypes.c_void_p
    fake = P(0x100000)  # never dereferenced: every call below fails validation
    r = L.rtf_build(None, 10, 10, fake, 1 << 20, None, ctypes.byref(desc))
    assert r == rtf.RTF_ERR_INVALID_ARG
    r = L.rtf_build(fake, 0, 10, fake, 1 << 20, None, ctypes.byref(desc))
    assert r == rtf.RTF_ERR_INVALID_ARG
    r = L.rtf_build(fake, 10, 10, P(0x100001), 1 << 20, None, ctypes.byref(desc))
    assert r == rtf.RTF_ERR_INVALID_ARG  # misaligned workspace
    r = L.rtf_build(fake, 1 << 31, 10, fake, 1 << 40, None, ctypes.byref(desc))
    assert r == rtf.RTF_ERR_SIZE
    r = L.rtf_build(fake, 1000, 1000, fake, 64, None, ctypes.byref(desc))
    assert r == rtf.RTF_ERR_WORKSPACE
    # build tiles: 1024 or 2048 elements, anything else refused on the host
    for tile in (0, 512, 1000, 4096, -2048):
        r = L.rtf_build_tiled(fake, 1000, 1000, tile, fake, 1 << 30, None, ctypes.byref(desc))
        assert r == rtf.RTF_ERR_INVALID_ARG, tile
        r = L.rtf_build_batched_tiled(fake, fake, fake, 2, 1000, 1000, tile, fake, 1 << 30, None,
                                      ctypes.byref(desc))
        assert r == rtf.RTF_ERR_INVALID_ARG, tile
    for tile in (1024, 2048):  # a valid tile still meets the workspace check
        r = L.rtf_build_tiled(fake, 1000, 1000, tile, fake, 64, None, ctypes.byref(desc))
        assert r == rtf.RTF_ERR_WORKSPACE
    r = L.rtf_sample(None, fake, 10, fake, None, None)
    assert r == rtf.RTF_ERR_INVALID_ARG
    r = L.rtf_sample(ctypes.byref(desc), fake, 10, fake, None, None)  # empty descriptor
    assert r == rtf.RTF_ERR_INVALID_ARG
    r = L.rtf_quantize_f32(None, None, 1, 10, fake, fake, None, None)
    assert r == rtf.RTF_ERR_INVALID_ARG
    # a well-formed descriptor (never dereferenced) with misaligned pair buffers
    f2 = rtf.rtf_forest(D=2, tile=2048, n_total=10, m_total=10, nodes=0x100000,
                        cells=0x100000, dists=0x100000, status=0x100000)
    r = L.rtf_sample_2d(ctypes.byref(f2), P(0x100008), 4, fake, fake, None)
    assert r == rtf.RTF_ERR_INVALID_ARG  # u2 not 16-byte aligned
    r = L.rtf_sample_2d(ctypes.byref(f2), fake, 4, P(0x100004), fake, None)
    assert r == rtf.RTF_ERR_INVALID_ARG  # out_rc not 8-byte aligned
    r = L.rtf_sample_2d(ctypes.byref(f2), fake, 4, fake, P(0x100008), None)
    assert r == rtf.RTF_ERR_INVALID_ARG  # out_xy not 16-byte aligned
    # the static-scratch backward rejects sizes past its array before any
    # device call
    big = rtf.rtf_forest(D=1, tile=2048, n_total=(1 << 20) + 1, m_total=10, nodes=0x100000,
                         cells=0x100000, dists=0x100000, status=0x100000)
    r = L.rtf_backward_static(ctypes.byref(big), None, None, None, None, 0, fake, fake, None)
    assert r == rtf.RTF_ERR_SIZE
    many = rtf.rtf_forest(D=(1 << 16) + 1, tile=2048, n_total=1 << 20, m_total=1 << 20,
                          nodes=0x100000, cells=0x100000, dists=0x100000, status=0x100000)
    r = L.rtf_backward_static(ctypes.byref(many), fake, None, None, None, 0, fake, fake, None)
    assert r == rtf.RTF_ERR_SIZE
    assert L.rtf_backward_static(None, None, None, None, None, 0, fake, fake, None) == \
        rtf.RTF_ERR_INVALID_ARG
    # import: argument and offset checks happen on the host, before any copy
    f3 = rtf.rtf_forest()
    W = (ctypes.c_uint64 * 2)(5, 7)
    r = L.rtf_forest_import(None, fake, W, None, None, 1, 10, 10, fake, 1 << 20, None,
                            ctypes.byref(f3))
    assert r == rtf.RTF_ERR_INVALID_ARG
    bad_eo = (ctypes.c_int64 * 3)(0, 6, 5)  # not increasing
    co = (ctypes.c_int64 * 3)(0, 5, 10)
    r = L.rtf_forest_import(fake, fake, W, bad_eo, co, 2, 10, 10, fake, 1 << 30, None,
                            ctypes.byref(f3))
    assert r == rtf.RTF_ERR_INVALID_ARG
    r = L.rtf_forest_import(fake, fake, W, None, None, 1, 1000, 1000, fake, 64, None,
                            ctypes.byref(f3))
    assert r == rtf.RTF_ERR_WORKSPACE
    for c in range(7):
        assert L.rtf_status_string(c).decode().startswith("RTF_")


def test_empty_sample_batches_are_no_ops(L):
    """S = 0 is valid: nothing is launched and null buffers are accepted; a
    negative count is an argument error."""
    import paper_1901_05423_amd as rtf
    f2 = rtf.rtf_forest(D=2, tile=2048, n_total=10, m_total=10, nodes=0x100000,
                        cells=0x100000, dists=0x100000, status=0x100000)
    f1 = rtf.rtf_forest(D=1, tile=2048, n_total=10, m_total=10, nodes=0x100000,
                        cells=0x100000, dists=0x100000, status=0x100000)
    P = ctypes.c_void_p
    assert L.rtf_sample(ctypes.byref(f1), None, 0, None, None, None) == rtf.RTF_OK
    assert L.rtf_sample_batched(ctypes.byref(f2), P(0x100000), None, 0, None, None, None) == rtf.RTF_OK
    assert L.rtf_sample_2d(ctypes.byref(f2), None, 0, None, None, None) == rtf.RTF_OK
    assert L.rtf_sample(ctypes.byref(f1), None, -1, None, None, None) == rtf.RTF_ERR_INVALID_ARG


def test_fixed_point_helpers_exact(tmp_path):
    src = os.path.join(ROOT, "tests", "native", "fixed_point_check.hip")
    exe = str(tmp_path / "fixed_point_check")
    subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "include"), "-o", exe, src], check=True,
                   capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout


def test_probe_library_exports_its_header():
    """The measurement probe (librtf_probe.so) exports what include/rtf_probe.h
    declares and rejects bad arguments on the host."""
    import importlib
    b = importlib.import_module("paper_1901_05423_amd.build")
    if not os.path.exists(b.PROBE_LIB):
        b.build_library()
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "rtf_probe.h")).read(),
                  flags=re.S)
    names = sorted(set(re.findall(r"\b(rtf_[a-z0-9_]+)\s*\(", text)))
    assert names == ["rtf_probe_gather"]
    nm = subprocess.run(["nm", "-D", "--defined-only", b.PROBE_LIB], capture_output=True,
                        text=True, check=True).stdout
    assert set(names) <= set(re.findall(r"\bT (rtf_\w+)", nm))
    P = ctypes.CDLL(b.PROBE_LIB)
    f = P.rtf_probe_gather
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    f.argtypes = [vp, i64, vp, i64, vp, i64, i32, vp, vp, vp]
    f.restype = ctypes.c_int
    good = ctypes.c_void_p(256)
    assert f(None, 1, None, 0, good, 1, 1, good, None, None) == 1  # no table
    assert f(good, 0, None, 0, good, 1, 1, good, None, None) == 1  # m < 1
    assert f(good, 1, None, 0, good, 1, 2, good, None, None) == 1  # depth 2 without nodes
    assert f(ctypes.c_void_p(260), 1, None, 0, good, 1, 1, good, None, None) == 1  # misaligned
    assert f(good, 1, None, 0, good, 0, 1, good, None, None) == 0  # nothing to do
