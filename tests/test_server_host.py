"""Host-side checks of the serving runtime (no GPU): the admission policy
compiled from the library's own header into a CPU test program, and the C
ABI's server entry points present in the built library."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_admission_policy(tmp_path):
    exe = tmp_path / "admission_test"
    src = os.path.join(ROOT, "tests", "cpp", "admission_test.cpp")
    inc = os.path.join(ROOT, "paper_2603_22437_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", inc, src, "-o",
                    str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "all checks passed" in r.stdout


def test_server_symbols_exported():
    import paper_2603_22437_amd as H
    for name in ("hck_server_create", "hck_server_add_tenant", "hck_server_submit",
                 "hck_server_poll", "hck_server_stats_get", "hck_server_destroy",
                 "hck_switch_key_import", "hck_galois_keys_create", "hck_galois_keys_insert"):
        assert hasattr(H.capi, name)
    # the result record's layout matches the C struct (8-byte aligned doubles)
    assert H.ServerResult.t_submit.offset % 8 == 0
    assert H.ServerResult.out_scale.offset == 48
    assert H.ctypes.sizeof(H.ServerResult) == 48 + 32 + 32
