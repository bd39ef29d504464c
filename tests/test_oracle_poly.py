"""Pins of the oracle's constant encoding and polynomial evaluation
(reading A28) against closed forms: the decoded result of sum_k c_k x^k
equals numpy's polynomial in every slot, for dense, sparse and negative
coefficients and the degrees whose power trees differ (powers of two and
not), and the evaluation uses exactly ceil(log2 d) + 1 levels."""
import numpy as np
import pytest

import oracle as O
import seeded_inputs as S


@pytest.fixture(scope="module")
def deep():
    prm = S.params("deep12")
    o = O.Oracle(prm)
    s = o.keygen_secret(1)
    rlk = o.keygen_relin(s, 7)
    x = S.uniform_slots(o.n_slots, 3)
    ct = o.encrypt_sk(s, o.encode(x, prm["scale"], o.L - 1), 11)
    return o, s, rlk, x, ct


def test_encode_const_decodes_to_the_constant():
    prm = S.params("deep12")
    o = O.Oracle(prm)
    for v in (0.75, -1.5, 3e-4):
        pt = o.encode_const(v, prm["scale"], 4)
        np.testing.assert_allclose(o.decode(pt), v, rtol=0, atol=2 ** -45)
        assert pt.res[:, 1:].max() == 0     # one nonzero coefficient


@pytest.mark.parametrize("coeffs", [
    [0.3, -0.7],                                  # degree 1
    [0.0, 0.0, 1.0],                              # x^2 alone
    [0.1, 0.5, -0.25, 0.125],                     # degree 3 (x^3 = x^2 x)
    [0.0, 1.0, 0.0, -1 / 6, 0.0, 1 / 120, 0.0, -1 / 5040],   # sine, odd terms only
    list(np.random.default_rng(5).uniform(-1, 1, 16)),      # degree 15, dense
])
def test_poly_eval_matches_numpy(deep, coeffs):
    o, s, rlk, x, ct = deep
    out = o.poly_eval(ct, coeffs, rlk)
    d = len(coeffs) - 1
    assert out.level == ct.level - ((d - 1).bit_length() + 1)
    assert abs(out.scale / ct.scale - 1) < 2 ** -30
    want = np.polynomial.polynomial.polyval(x, coeffs)
    got = o.decode(o.decrypt(s, out)).real
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-6)


def test_poly_eval_errors(deep):
    o, s, rlk, x, ct = deep
    with pytest.raises(ValueError):
        o.poly_eval(ct, [1.0], rlk)                # no term of degree >= 1
    with pytest.raises(ValueError):
        o.poly_eval(o.drop_level(ct, 2), [0.0, 0.0, 0.0, 0.0, 1.0], rlk)   # depth 3 > level 2
