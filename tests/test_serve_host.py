"""Host-side pieces of the serving layer that need no GPU: the HBM arena's
first-fit allocator (native, checked against a byte-map model under
AddressSanitizer) and argument checks of the server entry points."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_1709_06816_amd as hac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_allocator_matches_model(tmp_path):
    exe = str(tmp_path / "arena_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "paper_1709_06816_amd", "csrc"), "-o", exe,
                    os.path.join(ROOT, "tests", "native", "arena_check.cpp")], check=True)
    res = subprocess.run([exe, "30000"], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                         timeout=300)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stdout[-2000:]


def test_server_entry_points_reject_null():
    lib = hac.load_library()
    h = ctypes.c_void_p()
    assert lib.hac_server_create(None, 1 << 20, 4, 1024, ctypes.byref(h)) == hac.HAC_EINVAL
    assert lib.hac_server_create(None, 1 << 20, 4, 1024, None) == hac.HAC_EINVAL
    t = ctypes.c_uint64()
    assert lib.hac_submit(None, None, 4, 4, 0, ctypes.byref(t)) == hac.HAC_EINVAL
    d = ctypes.c_int32()
    assert lib.hac_poll(None, 0, None, ctypes.byref(d)) == hac.HAC_EINVAL
    assert lib.hac_server_get_stats(None, None) == hac.HAC_EINVAL
    assert lib.hac_server_last_error(None) == b"no server"
    assert lib.hac_server_destroy(None) == hac.HAC_OK
