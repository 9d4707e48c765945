"""The C-ABI library loads without a GPU and exports every function include/s7.h declares,
with struct layouts that match the binding."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "s7.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(s7_[a-z_0-9]+)\s*\(", txt)))


def test_header_lists_the_boundary():
    fns = declared_functions()
    for f in ("s7_stencil_apply", "s7_bicgstab_solve", "s7_bicgstab_solve_batched",
              "s7_queue_submit", "s7_queue_poll", "s7_workspace_bytes"):
        assert f in fns


def test_library_exports_every_declared_symbol():
    from paper_2010_03660_amd import binding
    lib = binding.lib()
    for f in declared_functions():
        assert hasattr(lib, f), f
    assert set(declared_functions()) == set(binding.EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    from paper_2010_03660_amd import binding
    src = tmp_path / "sz.c"
    src.write_text('#include "s7.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(s7_options),'
                   ' sizeof(s7_info), sizeof(s7_request), offsetof(s7_info, pass_ms),'
                   ' offsetof(s7_request, rtol), sizeof(s7_dims)); printf("%zu %zu\\n",'
                   ' sizeof(s7_request_2d9), offsetof(s7_request_2d9, rtol)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(binding.Options), C.sizeof(binding.Info), C.sizeof(binding.Request),
            binding.Info.pass_ms.offset, binding.Request.rtol.offset, C.sizeof(binding.Dims),
            C.sizeof(binding.Request2D9), binding.Request2D9.rtol.offset]
    assert got == want


def test_host_side_argument_checks():
    """Calls that fail validation return before touching the GPU."""
    from paper_2010_03660_amd import binding as B
    lib = B.lib()
    assert lib.s7_version() == 0x010000
    o = B.default_options()
    assert o.jacobi == 1
    assert lib.s7_workspace_bytes(B.Dims(0, 4, 4), 0, None) == 0
    assert lib.s7_workspace_bytes(B.Dims(2048, 2048, 1024), 0, None) == 0  # N >= 2^31
    # the largest mesh: N = 2^31 - 2^21 = 2048 * 1024 * 1023, and one column more
    assert lib.s7_workspace_bytes(B.Dims(2048, 1024, 1023), 0, None) > 0
    assert lib.s7_workspace_bytes(B.Dims(2049, 1024, 1023), 0, None) == 0
    assert lib.s7_workspace_bytes(B.Dims(8, 8, 8), 0, None) > 0
    coef = (C.c_void_p * 7)(*([256] * 7))
    info = B.Info()
    bad = [
        (B.Dims(8, 8, 8), -1.0, 10),       # rtol <= 0
        (B.Dims(8, 8, 8), float("nan"), 10),
        (B.Dims(8, 8, 8), 1e-6, -1),       # max_iter < 0
        (B.Dims(0, 8, 8), 1e-6, 10),
    ]
    for d, rtol, mi in bad:
        rc = lib.s7_bicgstab_solve(d, coef, 256, 512, rtol, mi, 0, 1024, 1 << 20, None,
                                   C.byref(info), 0)
        assert rc == B.EINVAL, (d.nx, rtol, mi)
        assert "invalid" in B.last_error()
    # workspace too small, or not 256-byte aligned
    rc = lib.s7_bicgstab_solve(B.Dims(8, 8, 8), coef, 256, 512, 1e-6, 10, 0, 1024, 16, None,
                               C.byref(info), 0)
    assert rc == B.EINVAL and "workspace" in B.last_error()
    rc = lib.s7_bicgstab_solve(B.Dims(8, 8, 8), coef, 256, 512, 1e-6, 10, 0, 1032, 1 << 30, None,
                               C.byref(info), 0)
    assert rc == B.EINVAL
    # u aliasing v
    rc = lib.s7_stencil_apply(B.Dims(8, 8, 8), coef, 4096, 4096, 0)
    assert rc == B.EINVAL


def test_queue_host_side_checks():
    """Queue calls that fail validation return before touching the GPU."""
    from paper_2010_03660_amd import binding as B
    lib = B.lib()
    tb = lib.s7_queue_table_bytes()
    assert tb > 0 and tb % 256 == 0
    q = C.c_void_p()
    assert lib.s7_queue_create(C.byref(q), 0, 1 << 30, None) == B.EINVAL        # no arena
    assert lib.s7_queue_create(C.byref(q), 4096 + 8, 1 << 30, None) == B.EINVAL  # misaligned
    assert lib.s7_queue_create(C.byref(q), 4096, tb, None) == B.EINVAL          # tables only
    assert "arena" in B.last_error()
    assert lib.s7_queue_create(None, 4096, 1 << 30, None) == B.EINVAL
    t = C.c_uint64()
    req = B.Request(B.Dims(8, 8, 8), (C.c_void_p * 7)(*([256] * 7)), 512, 768, 1e-6, 10, 0)
    assert lib.s7_queue_submit(None, C.byref(req), C.byref(t)) == B.EINVAL
    assert lib.s7_queue_poll(None, 1, None) == B.EINVAL
    assert lib.s7_queue_wait(None, 1, None) == B.EINVAL
    assert lib.s7_queue_destroy(None) == B.EINVAL
    req9 = B.Request2D9(8, 8, (C.c_void_p * 9)(*([256] * 9)), 512, 768, 1e-6, 10, 0)
    assert lib.s7_queue_submit_2d9(None, C.byref(req9), C.byref(t)) == B.EINVAL


def test_host_side_argument_checks_2d9():
    """The 2D 9-point calls validate on the host: dims, precision, tolerance, caps,
    workspace size and alignment, aliasing.  The workspace holds 8 (Jacobi) or 9
    coefficient copies, six vectors and the FP32 correction."""
    from paper_2010_03660_amd import binding as B
    lib = B.lib()
    assert lib.s7_workspace_bytes_2d9(0, 4, 0, None) == 0
    assert lib.s7_workspace_bytes_2d9(65536, 32768, 0, None) == 0  # N >= 2^31
    assert lib.s7_workspace_bytes_2d9(8, 8, 7, None) == 0          # no such precision
    n = 1000 * 1000
    f32 = lib.s7_workspace_bytes_2d9(1000, 1000, B.FP32, None)
    b16 = lib.s7_workspace_bytes_2d9(1000, 1000, B.BF16_IR, None)
    assert f32 >= (8 + 6 + 1) * n * 4 and b16 >= (8 + 6) * n * 2 + n * 4 and b16 < f32
    o = B.default_options(jacobi=0)
    assert lib.s7_workspace_bytes_2d9(1000, 1000, B.FP32, C.byref(o)) >= f32 + n * 4
    coef = (C.c_void_p * 9)(*([256] * 9))
    info = B.Info()
    for nx, rtol, mi, prec in ((8, -1.0, 10, 0), (8, float("nan"), 10, 0), (8, 1e-6, -1, 0), (0, 1e-6, 10, 0),
                               (8, 1e-6, 10, 5)):
        rc = lib.s7_bicgstab_solve_2d9(nx, 8, coef, 256, 512, rtol, mi, prec, 1024, 1 << 20, None,
                                       C.byref(info), 0)
        assert rc == B.EINVAL and "invalid" in B.last_error(), (nx, rtol, mi, prec)
    rc = lib.s7_bicgstab_solve_2d9(8, 8, coef, 256, 512, 1e-6, 10, 0, 1024, 16, None, C.byref(info), 0)
    assert rc == B.EINVAL and "workspace" in B.last_error()
    rc = lib.s7_bicgstab_solve_2d9(8, 8, coef, 256, 512, 1e-6, 10, 0, 1032, 1 << 30, None, C.byref(info), 0)
    assert rc == B.EINVAL
    assert lib.s7_stencil9_apply(8, 8, coef, 4096, 4096, 0) == B.EINVAL
    missing = (C.c_void_p * 9)(*([256] * 8 + [None]))
    assert lib.s7_stencil9_apply(8, 8, missing, 4096, 8192, 0) == B.EINVAL
    assert lib.s7_generate_problem_2d9(8, 8, 0, None, None, 4096, 0) == B.EINVAL  # b needs coef and x*


def test_host_side_argument_checks_batched_2d9():
    """The batched 2D call validates every system on the host before any device work,
    and its workspace is the engine tables plus one 2D workspace per mesh."""
    from paper_2010_03660_amd import binding as B
    lib = B.lib()
    nx = (C.c_int32 * 2)(100, 3)
    ny = (C.c_int32 * 2)(37, 1)
    total = lib.s7_batched_workspace_bytes_2d9(2, nx, ny, B.FP32, None)
    one = lib.s7_workspace_bytes_2d9(100, 37, B.FP32, None) + lib.s7_workspace_bytes_2d9(3, 1, B.FP32, None)
    assert total > one
    assert lib.s7_batched_workspace_bytes_2d9(0, nx, ny, B.FP32, None) == 0
    assert lib.s7_batched_workspace_bytes_2d9(2, nx, ny, 9, None) == 0
    bad = (C.c_int32 * 2)(100, 0)
    assert lib.s7_batched_workspace_bytes_2d9(2, bad, ny, B.FP32, None) == 0
    coef = (C.c_void_p * 18)(*([256] * 18))
    bp = (C.c_void_p * 2)(512, 768)
    xp = (C.c_void_p * 2)(1024, 1280)
    rt = (C.c_double * 2)(1e-8, 1e-8)
    mi = (C.c_int32 * 2)(10, 10)
    infos = (B.Info * 2)()

    def call(nx_, coef_=coef, rt_=rt, mi_=mi, ws=4096, wsb=1 << 30, prec=0):
        return lib.s7_bicgstab_solve_batched_2d9(2, nx_, ny, coef_, bp, xp, rt_, mi_, prec, ws, wsb, None,
                                                 infos, 0)
    assert call(bad) == B.EINVAL and "system 1" in B.last_error()
    missing = (C.c_void_p * 18)(*([256] * 17 + [None]))
    assert call(nx, coef_=missing) == B.EINVAL and "system 1" in B.last_error()
    assert call(nx, rt_=(C.c_double * 2)(1e-8, float("nan"))) == B.EINVAL
    assert call(nx, mi_=(C.c_int32 * 2)(-1, 10)) == B.EINVAL and "system 0" in B.last_error()
    assert call(nx, wsb=16) == B.EINVAL and "workspace" in B.last_error()
    assert call(nx, ws=4100) == B.EINVAL  # not 256-byte aligned
    assert call(nx, prec=3) == B.EINVAL


def test_host_side_argument_checks_pipelined():
    from paper_2010_03660_amd import binding as B
    lib = B.lib()
    d = B.Dims(40, 30, 20)
    n = 40 * 30 * 20
    assert lib.s7_workspace_bytes_pipelined(B.Dims(0, 3, 3), None) == 0
    # the classical FP32 workspace plus four vectors (z, w, t, v)
    assert lib.s7_workspace_bytes_pipelined(d, None) >= lib.s7_workspace_bytes(d, B.FP32, None) + 4 * n * 4
    coef = (C.c_void_p * 7)(*([256] * 7))
    info = B.Info()
    rc = lib.s7_bicgstab_solve_pipelined(d, coef, 512, 768, 1e-8, 10, 1024, 16, None, C.byref(info), 0)
    assert rc == B.EINVAL and "workspace" in B.last_error()
    rc = lib.s7_bicgstab_solve_pipelined(d, coef, 512, 768, float("nan"), 10, 1024, 1 << 30, None, C.byref(info), 0)
    assert rc == B.EINVAL
    rc = lib.s7_bicgstab_solve_pipelined(d, coef, 512, 768, 1e-8, 10, 1032, 1 << 30, None, C.byref(info), 0)
    assert rc == B.EINVAL  # workspace not 256-byte aligned


def test_host_side_argument_checks_batched_pipelined():
    """The pipelined batched call validates every system on the host before any device
    work; its workspace is the tables plus, per system, a slice that also holds the
    multi-kernel pipelined workspace (a large system is solved there alone)."""
    from paper_2010_03660_amd import binding as B
    lib = B.lib()
    dims = (B.Dims * 2)(B.Dims(40, 30, 20), B.Dims(3, 1, 2))
    total = lib.s7_batched_workspace_bytes_pipelined(2, dims, None)
    singles = sum(lib.s7_workspace_bytes_pipelined(d, None) for d in (B.Dims(40, 30, 20), B.Dims(3, 1, 2)))
    assert total > singles
    assert lib.s7_batched_workspace_bytes_pipelined(0, dims, None) == 0
    bad = (B.Dims * 2)(B.Dims(40, 30, 20), B.Dims(0, 1, 2))
    assert lib.s7_batched_workspace_bytes_pipelined(2, bad, None) == 0
    coef = (C.c_void_p * 14)(*([256] * 14))
    bp = (C.c_void_p * 2)(512, 768)
    xp = (C.c_void_p * 2)(1024, 1280)
    rt = (C.c_double * 2)(1e-8, 1e-8)
    mi = (C.c_int32 * 2)(10, 10)
    infos = (B.Info * 2)()

    def call(d=dims, coef_=coef, rt_=rt, mi_=mi, ws=4096, wsb=1 << 30):
        return lib.s7_bicgstab_solve_batched_pipelined(2, d, coef_, bp, xp, rt_, mi_, ws, wsb, None, infos, 0)
    assert call(bad) == B.EINVAL and "system 1" in B.last_error()
    missing = (C.c_void_p * 14)(*([256] * 13 + [None]))
    assert call(coef_=missing) == B.EINVAL and "system 1" in B.last_error()
    assert call(rt_=(C.c_double * 2)(float("nan"), 1e-8)) == B.EINVAL and "system 0" in B.last_error()
    assert call(mi_=(C.c_int32 * 2)(10, -1)) == B.EINVAL and "system 1" in B.last_error()
    assert call(wsb=16) == B.EINVAL and "workspace" in B.last_error()
    assert call(ws=4100) == B.EINVAL  # not 256-byte aligned


def test_host_side_argument_checks_p2_designs():
    """The P2 design probe rejects unknown designs and unsupported meshes on the host."""
    from paper_2010_03660_amd import binding as B
    lib = B.lib()
    d = B.Dims(64, 48, 20)
    assert lib.s7_p2_design_part_bytes(0, 0, d) == ((64 * 48 * 20 // 2 + 255) // 256) * 5 * 8
    assert lib.s7_p2_design_part_bytes(3, 8, d) == 2 * 3 * 5 * 8  # two in-plane tiles, three z-blocks
    assert lib.s7_p2_design_part_bytes(9, 0, d) == 0
    assert lib.s7_p2_design_part_bytes(0, 0, B.Dims(0, 4, 4)) == 0
    coef = (C.c_void_p * 6)(*([256] * 6))
    ms = C.c_float()

    def call(kind, param, dims=d, part_bytes=1 << 30, reps=1):
        return lib.s7_p2_design_probe(kind, param, dims, coef, 512, 768, 1024, 0.5, 1280, 1536, part_bytes, reps,
                                      C.byref(ms), 0)
    assert call(4, 0) == B.EINVAL
    assert call(3, 0) == B.EINVAL          # z-march depth must be >= 1
    assert call(1, 2) == B.EINVAL          # tile order: 0 or 1
    assert call(0, 0, dims=B.Dims(36, 8, 4)) == B.EINVAL   # nx not a multiple of 8
    assert call(0, 0, dims=B.Dims(1032, 8, 4)) == B.EINVAL  # nx above 1024
    assert call(0, 0, part_bytes=8) == B.EINVAL and "partial" in B.last_error()
    assert call(0, 0, reps=0) == B.EINVAL
