"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The oracle's C core (``oracle/ockks.c``) built with both sanitizers and
  loaded in place of the normal build (``OCKKS_LIB``) while its pins and
  scheme tests run in a child Python process; any out-of-bounds access,
  use after free, overflow of a signed type or misaligned access aborts it.
* The library's host-only client sources (SHAKE-256, samplers, encoder,
  decoder; ``csrc/sampler.cpp``, ``csrc/encoder.cpp``) built with both
  sanitizers into a test program whose outputs must equal the normal build's
  (``libhipckks.so`` through ctypes).
* The serving runtime's admission policy (``csrc/admission.h``) under both
  sanitizers.
"""
import ctypes
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import seeded_inputs as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_22437_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="gcc/g++ not available")


def _libasan() -> str:
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()


def test_oracle_core_under_sanitizers(tmp_path):
    lib = tmp_path / "libockks_san.so"
    subprocess.run(["gcc", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", *SAN, "-o",
                    str(lib), os.path.join(ROOT, "oracle", "ockks.c")], check=True)
    env = dict(os.environ, **SAN_ENV, OCKKS_LIB=str(lib), LD_PRELOAD=_libasan(),
               OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_scheme.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
    assert " passed" in r.stdout


def _parse(out: str) -> dict:
    d = {}
    for line in out.splitlines():
        parts = line.split()
        if not parts or parts[0] == "all":
            continue
        key = parts[0] if parts[0] in ("uniform", "ternary", "gaussian") else tuple(parts[:2])
        d[key] = parts[1:] if isinstance(key, str) else parts[2:]
    return d


def test_host_client_code_under_sanitizers(tmp_path):
    import paper_2603_22437_amd as H

    exe = tmp_path / "host_sanitize_test"
    subprocess.run(["g++", "-std=c++17", "-Wall", *SAN, "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", "cpp", "host_sanitize_test.cpp"),
                    os.path.join(CSRC, "sampler.cpp"), os.path.join(CSRC, "encoder.cpp"),
                    "-o", str(exe)], check=True)
    mods = [int(x) for x in S.params("vital")["q"][:3]]
    r = subprocess.run([str(exe), *map(str, mods)], capture_output=True, text=True,
                       env=dict(os.environ, **SAN_ENV), timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "all checks passed" in r.stdout
    got = _parse(r.stdout)

    # the same calls in the normal build
    for n in (0, 1, 135, 136, 137, 300):
        msg = bytes((i * 7 + 3) & 0xFF for i in range(n))
        out = ctypes.create_string_buffer(200)
        assert H.capi.hck_shake256(msg, n, out, 200) == 0
        assert got[("shake", str(n))][0] == out.raw.hex()
    u = np.zeros(1000, dtype=np.uint64)
    assert H.capi.hck_sample_uniform(b"san", 7, 3, mods[0], u.ctypes.data, 1000) == 0
    assert [int(x) for x in got["uniform"]] == [int(x) for x in u]
    for name, seed in (("ternary", 8), ("gaussian", 9)):
        v = np.zeros(1000, dtype=np.int32)
        fn = getattr(H.capi, f"hck_sample_{name}")
        assert fn(b"san", seed, v.ctypes.data, 1000) == 0
        assert [int(x) for x in got[name]] == [int(x) for x in v]
    # the encoder and decoder are floating-point code compiled by another
    # compiler here (gcc -O1 against hipcc -O3): integer coefficients agree to
    # within one unit of rounding, decoded slots to 1e-12
    lcg = 12345
    for log_n in (4, 8, 12):
        enc = [int(x) for x in got[("encode", str(log_n))]]
        dec = np.array([float(x) for x in got[("decode", str(log_n))]])
        n = 1 << log_n
        assert len(enc) == n and len(dec) == n
        zr, zi = np.zeros(n // 2), np.zeros(n // 2)
        for i in range(n // 2):     # the test program's slot values
            for arr in (zr, zi):
                lcg = (lcg * 6364136223846793005 + 1442695040888963407) % 2 ** 64
                arr[i] = ((lcg >> 11) % 2000001) / 1e6 - 1.0
        c = np.zeros(n, dtype=np.int64)
        assert H.capi.hck_encode_coeffs(log_n, zr.ctypes.data, zi.ctypes.data,
                                        ctypes.c_double(2.0 ** 40), c.ctypes.data) == 0
        assert max(abs(a - int(b)) for a, b in zip(enc, c)) <= 1
        res = np.array([[c % q for c in enc] for q in mods], dtype=np.uint64)
        re = np.zeros(n // 2)
        im = np.zeros(n // 2)
        assert H.capi.hck_decode_residues(log_n, res.ctypes.data,
                                          np.array(mods, dtype=np.uint64).ctypes.data, 3,
                                          ctypes.c_double(2.0 ** 40), re.ctypes.data,
                                          im.ctypes.data) == 0
        np.testing.assert_allclose(np.stack([re, im], 1).reshape(-1), dec, rtol=0, atol=1e-12)
        # and they are the slots that were encoded
        np.testing.assert_allclose(re, zr, rtol=0, atol=1e-9)
        np.testing.assert_allclose(im, zi, rtol=0, atol=1e-9)


def test_admission_policy_under_sanitizers(tmp_path):
    exe = tmp_path / "admission_test_san"
    subprocess.run(["g++", "-std=c++17", "-Wall", "-Werror", *SAN, "-I", CSRC,
                    os.path.join(ROOT, "tests", "cpp", "admission_test.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True,
                       env=dict(os.environ, **SAN_ENV), timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "all checks passed" in r.stdout
