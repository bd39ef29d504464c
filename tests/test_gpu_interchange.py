"""The interchange form through the library (N = 2^15, L = 12): blobs the
library writes equal the oracle's byte for byte, blobs the oracle writes
import to the same residues, a deserialized key works like the original, and
blobs of another parameter set or kind are refused."""
import numpy as np
import pytest

import oracle as O
import seeded_inputs as S
from oracle import interchange as OI

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_2603_22437_amd")


def test_blobs_match_oracle_and_round_trip():
    prm = S.params("mix15")
    o = O.Oracle(prm)
    ctx = H.Context.from_params(prm)
    for level, size in ((o.L - 1, 2), (4, 3), (0, 2)):
        res = S.uniform_residues(o.qmods(level), o.n, 800 + level, count=size)
        ct = ctx.ciphertext_import(res, level, 2.0 ** 45)
        blob = ctx.serialize(ct)
        assert blob == OI.serialize_ciphertext(o, O.Ciphertext(res, level, 2.0 ** 45))
        back = ctx.ciphertext_deserialize(blob)
        got, lvl, sc = ctx.ciphertext_export(back)
        assert np.array_equal(got, res) and lvl == level and sc == 2.0 ** 45
    sk, s_o = ctx.keygen_secret(1), o.keygen_secret(1)
    rlk = ctx.keygen_relin(sk, 7)
    kblob = ctx.serialize(rlk)
    assert kblob == OI.serialize_switch_key(o, o.keygen_relin(s_o, 7))
    rlk2 = ctx.switch_key_deserialize(kblob)
    x = S.uniform_residues(o.qmods(6), o.n, 850, count=3)
    t = ctx.ciphertext_import(x, 6, 2.0 ** 40)
    a = ctx.ciphertext_export(ctx.relinearize(t, rlk))[0]
    b = ctx.ciphertext_export(ctx.relinearize(t, rlk2))[0]
    assert np.array_equal(a, b)


def test_foreign_blobs_are_refused():
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    other = O.Oracle(S.params_with_dnum("mix15", 4))
    res = S.uniform_residues(other.qmods(3), other.n, 860, count=2)
    blob = OI.serialize_ciphertext(other, O.Ciphertext(res, 3, 1.0))
    with pytest.raises(H.HckError) as e:
        ctx.ciphertext_deserialize(blob)
    assert e.value.code == -7              # HCK_EPARAMS
    o = O.Oracle(prm)
    good = OI.serialize_ciphertext(o, O.Ciphertext(S.uniform_residues(o.qmods(3), o.n, 861,
                                                                      count=2), 3, 1.0))
    with pytest.raises(H.HckError):        # a ciphertext is not a key
        ctx.switch_key_deserialize(good)
    w = np.frombuffer(good, dtype=np.uint8).copy()
    w[64:72] = 0xFF                        # a residue above its prime
    with pytest.raises(H.HckError):
        ctx.ciphertext_deserialize(w.tobytes())
