"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2604_17513_amd import flash as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "flash.h")).read()
    names = set(re.findall(r"^\s*(?:flash_status|const char\s*\*)\s*(flash_\w+)\s*\(", src, re.M))
    return names


def test_library_exports_every_declared_function():
    L = F.lib()
    declared = _declared()
    assert {"flash_create_batch", "flash_set_state", "flash_step", "flash_contacts", "flash_residual"} <= declared
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared <= set(F.EXPORTED)


def test_version_and_kernel_names():
    L = F.lib()
    assert b"gfx950" in L.flash_version()
    names = [L.flash_kernel_name(i).decode() for i in range(9)]
    assert names[:8] == ["detect", "gather", "project", "assemble", "apply", "csp", "correct", "finalize"]
    assert L.flash_kernel_name(99) == b""


def test_invalid_arguments_are_rejected_without_device():
    L = F.lib()
    h = C.c_void_p()
    p = F.flash_params()
    assert L.flash_create_batch(None, 1, C.byref(p), None, C.byref(h)) == F.FLASH_ERR_INVALID_ARG
    assert b"null" in L.flash_last_error()
    d = (F.flash_env_desc * 1)()
    assert L.flash_create_batch(d, 0, C.byref(p), None, C.byref(h)) == F.FLASH_ERR_INVALID_ARG
    p.h = 1.0 / 60
    p.lg_iterations = 0
    p.ncp_tol = 1e-6
    assert L.flash_create_batch(d, 1, C.byref(p), None, C.byref(h)) == F.FLASH_ERR_INVALID_ARG
    p.lg_iterations = 5
    d[0].elem = 7      # neither FLASH_TET nor FLASH_TRI
    d[0].n_vertices = 3
    d[0].n_elements = 1
    assert L.flash_create_batch(d, 1, C.byref(p), None, C.byref(h)) == F.FLASH_ERR_INVALID_ARG
    d[0].elem = 1      # triangles need a thickness
    d[0].thickness = 0.0
    assert L.flash_create_batch(d, 1, C.byref(p), None, C.byref(h)) == F.FLASH_ERR_INVALID_ARG
    assert L.flash_step(None, 1) == F.FLASH_ERR_INVALID_ARG
    assert L.flash_destroy_batch(None) == F.FLASH_ERR_INVALID_ARG
    assert L.flash_residual(None, None, None, None) == F.FLASH_ERR_INVALID_ARG


def test_contact_capacity_beyond_lds_is_rejected_without_device():
    """One workgroup holds an env's contact data in the 160 KB of LDS of a CU (dynamic, plus up
    to 8 KB of static LDS reserved for the kernels' own arrays): 330 contacts fit when the
    contact solve runs in FP64 (FP64 batches, and FP32 batches by default), 814 when an FP32
    batch solves contacts in FP32; one more is rejected at create, before the device is
    touched."""
    L = F.lib()

    def lds(cap, ct_bytes):
        rlds = min(3 * cap, 1536, 480)
        return cap * 3 * 8 + cap * 28 * ct_bytes + rlds * 18 * ct_bytes + cap * 3 * 4 + 64 * 8 + 8192

    assert lds(330, 8) <= 160 * 1024 < lds(331, 8)
    assert lds(814, 4) <= 160 * 1024 < lds(815, 4)
    d = (F.flash_env_desc * 1)()
    d[0].elem = 0
    d[0].n_vertices = 4
    d[0].n_elements = 1
    rest = (C.c_double * 12)(0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 1, 0)
    tet = (C.c_int32 * 4)(0, 1, 2, 3)
    d[0].rest_x = C.cast(rest, type(d[0].rest_x))
    d[0].elements = C.cast(tet, type(d[0].elements))
    d[0].density, d[0].young, d[0].poisson, d[0].mu = 1000.0, 1e5, 0.3, 0.5
    for precision, contact_fp32, limit in ((F.FLASH_FP64, 0, 330), (F.FLASH_FP32, 0, 330), (F.FLASH_FP32, 1, 814)):
        p = F.flash_params()
        p.h, p.lg_iterations, p.ncp_tol, p.contact_margin = 1.0 / 60, 2, 1e-6, 2e-3
        p.precision, p.contact_fp32 = precision, contact_fp32
        p.max_contacts_per_env = limit + 1
        h = C.c_void_p()
        assert L.flash_create_batch(d, 1, C.byref(p), None, C.byref(h)) == F.FLASH_ERR_INVALID_ARG
        assert b"LDS" in L.flash_last_error()
        p.max_contacts_per_env = limit
        st = L.flash_create_batch(d, 1, C.byref(p), None, C.byref(h))
        assert st != F.FLASH_ERR_INVALID_ARG, L.flash_last_error()
        if st == F.FLASH_OK:
            L.flash_destroy_batch(h)
    # the lightweight metric takes capacities beyond LDS (its update then runs from global memory),
    # up to 65536; the exact metric cannot ask for the global-memory update
    p = F.flash_params()
    p.h, p.lg_iterations, p.ncp_tol, p.contact_margin = 1.0 / 60, 2, 1e-6, 2e-3
    h = C.c_void_p()
    for metric, glob, cap, ok in ((F.FLASH_METRIC_LIGHTWEIGHT, 0, 4000, True),
                                  (F.FLASH_METRIC_LIGHTWEIGHT, 1, 65536, True),
                                  (F.FLASH_METRIC_LIGHTWEIGHT, 0, 65537, False),
                                  (F.FLASH_METRIC_EXACT, 1, 100, False),
                                  (F.FLASH_METRIC_LIGHTWEIGHT, 2, 100, False),
                                  (F.FLASH_METRIC_EXACT, 0, 4000, False)):
        p.contact_metric, p.global_contact_solve, p.max_contacts_per_env = metric, glob, cap
        st = L.flash_create_batch(d, 1, C.byref(p), None, C.byref(h))
        assert (st != F.FLASH_ERR_INVALID_ARG) == ok, (metric, glob, cap, L.flash_last_error())
        if st == F.FLASH_OK:
            L.flash_destroy_batch(h)
    # envs per workgroup of the twin products: 0 (automatic) to 8
    p.contact_metric, p.global_contact_solve, p.max_contacts_per_env = F.FLASH_METRIC_LIGHTWEIGHT, 1, 100
    for chunk, ok in ((0, True), (8, True), (9, False), (-1, False)):
        p.twin_chunk = chunk
        st = L.flash_create_batch(d, 1, C.byref(p), None, C.byref(h))
        assert (st != F.FLASH_ERR_INVALID_ARG) == ok, (chunk, L.flash_last_error())
        if st == F.FLASH_OK:
            L.flash_destroy_batch(h)


def test_struct_layouts_match_header_field_order():
    # the ctypes mirrors follow the header's field order; sizes are those of the C structs on LP64
    assert C.sizeof(F.flash_obstacle) == 8 + 8 * (3 + 9 + 3 + 3)
    assert C.sizeof(F.flash_env_desc) == 16 + 16 + 8 * 6
    assert C.sizeof(F.flash_params) == 8 + 24 + 8 + 24 + 16 + 8 + 8 + 8 + 8 + 8
    assert C.sizeof(F.flash_contact) == 16 + 8 * (3 + 3 + 1 + 3 + 3)
    assert C.sizeof(F.flash_env_stats) == 24 + 8


def test_struct_layouts_match_the_header(tmp_path):
    """Every field of the ctypes structures sits at the offset the C header gives it (offsetof
    from a small program compiled against include/flash.h with the host compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [F.flash_env_desc, F.flash_obstacle, F.flash_params, F.flash_contact, F.flash_env_stats,
               F.flash_gripper, F.flash_camera]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "flash.h"', "int main(void) {"]
    expect = []
    for S in structs:
        cname = S.__name__
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        expect.append(C.sizeof(S))
        for fname, _ in S._fields_:
            cfield = "lambda" if fname == "lambda_" else fname
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {cfield}));')
            expect.append(getattr(S, fname).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect
