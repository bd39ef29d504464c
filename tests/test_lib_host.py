"""Host-side checks of the HIP library (no GPU needed).

* the shared library loads and exports every function hipckks.h declares;
* its SHAKE-256 matches Python's hashlib (FIPS 202);
* its samplers draw exactly the oracle's values from the same seeds;
* its encoder/decoder agree with the oracle's canonical embedding.
"""
import hashlib
import os
import re

import numpy as np
import pytest

import oracle as O
import seeded_inputs as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_2603_22437_amd as H
    return H


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hipckks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hck_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) > 50
    for name in names:
        assert hasattr(lib.capi, name), name
        assert name in lib.SIGNATURES, f"binding lacks {name}"
    # and the binding declares nothing the header does not
    assert set(lib.SIGNATURES) <= set(names) | {
        "hck_shake256", "hck_sample_uniform", "hck_sample_ternary", "hck_sample_gaussian",
        "hck_encode_coeffs", "hck_decode_residues"}


def test_host_utilities_are_declared():
    names = declared_functions()
    for extra in ["hck_shake256", "hck_sample_uniform", "hck_sample_ternary",
                  "hck_sample_gaussian", "hck_encode_coeffs", "hck_decode_residues"]:
        assert extra in names


@pytest.mark.parametrize("mlen", [0, 1, 7, 135, 136, 137, 300])
@pytest.mark.parametrize("olen", [1, 32, 136, 137, 1000])
def test_shake256_matches_hashlib(lib, mlen, olen):
    msg = bytes((i * 37 + 11) % 256 for i in range(mlen))
    assert lib.shake256(msg, olen) == hashlib.shake_256(msg).digest(olen)


@pytest.mark.parametrize("name", ["tiny", "vital"])
def test_samplers_match_oracle(lib, name):
    prm = S.params(name)
    n = 4096
    mods = prm["q"][:3] + prm["p"][:1]
    ref = O.sample_uniform("gk/5/a/1", 9, mods, n)
    for t, q in enumerate(mods):
        assert np.array_equal(lib.sample_uniform("gk/5/a/1", 9, t, q, n), ref[t])
    assert np.array_equal(lib.sample_ternary("sk", 3, n), O.sample_ternary("sk", 3, n))
    assert np.array_equal(lib.sample_gaussian("enc_e", 4, 1 << 16),
                          O.sample_gaussian("enc_e", 4, 1 << 16))


@pytest.mark.parametrize("log_n,scale", [(12, 2.0 ** 25), (12, 2.0 ** 40), (16, 2.0 ** 50)])
def test_encoder_matches_oracle(lib, log_n, scale):
    n = 1 << log_n
    z = S.uniform_slots(n // 2, 5, complex_=True)
    mine = lib.encode_coeffs(log_n, z, scale)
    ref = np.array(O.encode_int(z, n, scale), dtype=np.int64)
    # two fp64 FFTs of length N round differently: allow a few units at 2^50
    tol = max(1, int(scale * 2.0 ** -48))
    assert np.max(np.abs(mine - ref)) <= tol
    # decoding integer residues: the library's CRT + FFT vs the oracle's
    prm = S.params("vital")
    mods = prm["q"][:3]
    res = O.ints_to_residues([int(x) for x in ref], mods)
    got = lib.decode_residues(log_n, res, mods, scale)
    want = O.decode_ints(O.crt_centered(res, mods), n, scale)
    assert np.max(np.abs(got - want)) < 1e-9
    # coefficient rounding (|err| <= 1/2 each) moves a slot by about sqrt(N/12)/scale
    assert np.max(np.abs(got - z)) < 8 * np.sqrt(n) / scale
