"""The C-ABI library loads without a GPU and exports every function that
include/mxr.h declares; the binding's struct layouts match the header."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mxr.h")
LIB = os.path.join(ROOT, "paper_2410_08747_amd", "libmxr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(mxr_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libmxr.so not built")
    return ctypes.CDLL(LIB)


def test_header_declares_the_api():
    names = declared_functions()
    # the boundary of the hot path: tracing, the learned proposal (set, box,
    # train from collected rows, apply from the network), the batch and the
    # launch-shape tuners
    for want in ("mxr_abi_version", "mxr_last_error", "mxr_instrument_create", "mxr_instrument_destroy",
                 "mxr_run", "mxr_trace_rays", "mxr_collect", "mxr_proposal_set", "mxr_proposal_box",
                 "mxr_proposal_train", "mxr_proposal_apply", "mxr_batch_create", "mxr_batch_run",
                 "mxr_batch_autotune", "mxr_batch_means", "mxr_autotune_instrument", "mxr_set_launch_shape",
                 "mxr_get_launch_shape"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mxr_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for n in declared_functions():
        getattr(lib, n)


def test_calls_that_need_no_device(lib):
    lib.mxr_abi_version.restype = ctypes.c_uint32
    lib.mxr_last_error.restype = ctypes.c_char_p
    assert lib.mxr_abi_version() == 2
    assert lib.mxr_last_error() is not None
    # validation fails before any device call
    out = ctypes.c_void_p()
    assert lib.mxr_instrument_create(None, ctypes.byref(out)) == -1
    assert b"null" in lib.mxr_last_error()
    assert lib.mxr_run(None, 0, 0, 1, 0, 0, 0, None, 0, None, None) == -1
    lib.mxr_instrument_destroy(None)
    bout = ctypes.c_void_p()
    assert lib.mxr_batch_create(None, 1, None, ctypes.byref(bout)) == -1
    assert lib.mxr_batch_run(None, None) == -1
    lib.mxr_batch_destroy(None)


def test_binding_struct_layout(lib):
    import paper_2410_08747_amd as m  # loads the library; no device call
    desc = m.mxr_component_desc
    # 4 + 4 + 3*8 + 9*8 + 16*8 + 2*8 + 2*8 + 4*4 = 280
    assert ctypes.sizeof(desc) == 280
    assert ctypes.sizeof(m.mxr_tally) == 32
    assert ctypes.sizeof(m.mxr_ray_soa) == 88
    code = r'''
#include <stdio.h>
#include <stddef.h>
#include "mxr.h"
int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(mxr_component_desc), sizeof(mxr_tally), sizeof(mxr_ray_soa), offsetof(mxr_component_desc, data), sizeof(mxr_batch_job), offsetof(mxr_batch_job, tallies), sizeof(mxr_batch_schedule), sizeof(mxr_hits), sizeof(mxr_train_rows), offsetof(mxr_train_rows, floor_frac), sizeof(mxr_launch_shape));return 0;}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src_c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src_c, "w").write(code)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src_c, "-o", exe], check=True)
        sizes = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert sizes[:3] == [280, 32, 88]
    assert sizes[3] == desc.data.offset
    assert sizes[4] == ctypes.sizeof(m.mxr_batch_job) == 160
    assert sizes[5] == m.mxr_batch_job.tallies.offset
    assert sizes[6] == ctypes.sizeof(m.mxr_batch_schedule) == 16
    assert sizes[7] == ctypes.sizeof(m.mxr_hits) == 72
    assert sizes[8] == ctypes.sizeof(m.mxr_train_rows) == 80
    assert sizes[9] == m.mxr_train_rows.floor_frac.offset
    assert sizes[10] == ctypes.sizeof(m.mxr_launch_shape) == 16


def test_every_kernel_stub_finds_its_device_code():
    """The host side launches a kernel through a stub whose mangled name must
    equal the device kernel's: a parameter type spelled differently in the
    two compilation passes (an address space seen only by the device pass)
    builds without error and aborts at the first launch.  Every stub's
    kernel must have its descriptor (<name>.kd) in the library's gfx950
    code objects."""
    if not os.path.exists(LIB):
        pytest.skip("libmxr.so not built")
    out = subprocess.run(["nm", LIB], capture_output=True, text=True, check=True).stdout
    data = open(LIB, "rb").read()
    names = set()
    for line in out.splitlines():
        parts = line.split()
        if len(parts) != 3 or "__device_stub__" not in parts[2]:
            continue
        m = re.match(r"(_ZN12_GLOBAL__N_1|_Z)(\d+)__device_stub__(.*)", parts[2])
        assert m, f"unexpected stub name {parts[2]}"
        names.add(m.group(1) + str(int(m.group(2)) - len("__device_stub__")) + m.group(3))
    assert len(names) > 50
    missing = sorted(n for n in names if (n + ".kd").encode() not in data)
    assert not missing, f"{len(missing)} kernels without device code, e.g. {missing[0]}"
