"""The interchange form on the CPU: the oracle's writer against the
library's header parser and prime hash (host-only entry points), and
malformed blobs refused by both."""
import numpy as np
import pytest

import oracle as O
import seeded_inputs as S
from oracle import interchange as OI

H = pytest.importorskip("paper_2603_22437_amd")


def test_fnv1a_known_answers():
    # the published FNV-1a 64 test vectors for "" and "a"
    assert OI.fnv1a64(b"") == 0xCBF29CE484222325
    assert OI.fnv1a64(b"a") == 0xAF63DC4C8601EC8C


@pytest.mark.parametrize("name", ["tiny", "mix15", "vital", "gesture"])
def test_prime_hash_matches_library(name):
    prm = S.params(name)
    assert H.params_hash(prm) == OI.params_hash(O.Oracle(prm))


def test_prime_hash_tells_parameter_sets_apart():
    hs = {H.params_hash(S.params_with_dnum("mix15", d)) for d in (2, 3, 4, 6)}
    assert len(hs) == 4
    prm = S.params("mix15")
    swapped = dict(prm, q=[prm["q"][1], prm["q"][0]] + prm["q"][2:])
    assert H.params_hash(swapped) != H.params_hash(prm)


def test_oracle_blobs_parse_in_library():
    prm = S.params("tiny")
    o = O.Oracle(prm)
    res = S.uniform_residues(o.qmods(1), o.n, 5, count=3)
    ct = O.Ciphertext(res, 1, 2.0 ** 25)
    blob = OI.serialize_ciphertext(o, ct)
    h = H.blob_parse(blob)
    assert (h["magic"], h["kind"], h["log_n"], h["num_q"], h["num_p"], h["dnum"], h["level"],
            h["polys"], h["rows"], h["scale"], h["words"]) == (
        b"HCKCKKS1", 1, 12, 3, 1, 3, 1, 3, 2, 2.0 ** 25, 3 * 2 * 4096)
    assert h["prime_hash"] == H.params_hash(prm)
    back = OI.deserialize_ciphertext(o, blob)
    assert np.array_equal(back.polys, res) and back.level == 1 and back.scale == 2.0 ** 25
    key = S.uniform_residues((o.q + o.p) * 2 * o.dnum, o.n, 6)[0].reshape(
        o.dnum, 2, o.L + o.K, o.n)
    kb = OI.serialize_switch_key(o, key)
    hk = H.blob_parse(kb)
    assert (hk["kind"], hk["polys"], hk["rows"], hk["level"]) == (2, 6, 4, 2)
    assert np.array_equal(OI.deserialize_switch_key(o, kb), key)


def test_malformed_blobs_are_refused():
    prm = S.params("tiny")
    o = O.Oracle(prm)
    ct = O.Ciphertext(S.uniform_residues(o.qmods(2), o.n, 7, count=2), 2, 1.0)
    blob = OI.serialize_ciphertext(o, ct)
    bad = [b"XXXXXXXX" + blob[8:],               # magic
           blob[:-8],                            # truncated
           blob + b"\0" * 8,                     # trailing bytes
           blob[:8] + (3).to_bytes(4, "little") + blob[12:],      # kind
           blob[:28] + (3).to_bytes(4, "little") + blob[32:],     # level beyond the chain
           blob[:32] + (4).to_bytes(4, "little") + blob[36:]]     # size 4
    for b in bad:
        with pytest.raises(H.HckError):
            H.blob_parse(b)
    with pytest.raises(ValueError):
        OI.deserialize_ciphertext(o, blob[:-8])
    other = O.Oracle(S.params_with_dnum("tiny", 1))
    with pytest.raises(ValueError):
        OI.deserialize_ciphertext(other, blob)
