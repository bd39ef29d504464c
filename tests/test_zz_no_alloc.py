"""hck_rotate_noalloc: the rotation that allocates nothing (its key switch
runs in the library's static scratch array) against hck_rotate, bit for bit,
through the C ABI, on two calls in a row (the second with a smaller input),
with an output aliasing its input, and its error paths."""
import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_2603_22437_amd")


def _rand_ct(ctx, prm, level, seed):
    res = S.uniform_residues(prm["q"][: level + 1], prm["n"], seed, count=2)
    return ctx.ciphertext_import(res, level, 2.0 ** 40)


def _export(ctx, ct):
    res, level, scale = ctx.ciphertext_export(ct)
    return res, level, scale


@pytest.mark.parametrize("name", ["vital", "mix15"])
def test_noalloc_rotation_matches_rotate(name):
    prm = S.params(name)
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    gks = ctx.keygen_rotation(sk, [1, 5], 5)
    top = len(prm["q"]) - 1
    need = ctx.rotate_noalloc_scratch()
    L, K = len(prm["q"]), len(prm["p"])
    rows = 4 * L + (prm["dnum"] + 2) * (L + K)     # one key-switch slot and a copy of c0
    assert need == rows * prm["n"] * 8
    assert need <= H.capi.hck_rotate_noalloc_scratch(None)
    out = _rand_ct(ctx, prm, top, 40)      # holds storage for two polynomials
    for call, (level, step) in enumerate([(top, 1), (3, 5)]):
        print(f"case {name}: call {call} level {level} step {step}", flush=True)
        a = _rand_ct(ctx, prm, level, 50 + call)
        want = _export(ctx, ctx.rotate(a, step, gks))
        ctx.rotate_noalloc(a, step, gks, out)
        got = _export(ctx, out)
        assert got[1] == want[1] and got[2] == want[2]
        assert np.array_equal(got[0], want[0]), f"call {call}"
    # output aliasing its input, then a step that only copies
    a = _rand_ct(ctx, prm, 7, 60)
    want = _export(ctx, ctx.rotate(a, 5, gks))
    ctx.rotate_noalloc(a, 5, gks, a)
    assert np.array_equal(_export(ctx, a)[0], want[0])
    ctx.rotate_noalloc(a, prm["n"] // 2, gks, out)
    assert np.array_equal(_export(ctx, out)[0], want[0])


def test_noalloc_rotation_errors():
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    gks = ctx.keygen_rotation(sk, [1], 5)
    a = _rand_ct(ctx, prm, 5, 70)
    with pytest.raises(H.HckError):        # a fresh handle holds no storage
        ctx.rotate_noalloc(a, 1, gks, ctx.ciphertext())
    out = _rand_ct(ctx, prm, 5, 71)
    with pytest.raises(H.HckError):        # no key for step 2
        ctx.rotate_noalloc(a, 2, gks, out)
    # still usable after the errors
    want = _export(ctx, ctx.rotate(a, 1, gks))[0]
    assert np.array_equal(_export(ctx, ctx.rotate_noalloc(a, 1, gks, out))[0], want)


def test_noalloc_rotation_refuses_contexts_beyond_the_array():
    """N = 2^17 with 20 + 7 moduli needs 215 MiB of scratch: refused before
    any device work."""
    two_n = 2 << 17
    taken = set()
    q = S._primes_near(60, two_n, 1, taken, False) + S._primes_near(50, two_n, 19, taken, True)
    p = S._primes_near(60, two_n, 7, taken, False)
    ctx = H.Context(17, q, p, 3)
    assert ctx.rotate_noalloc_scratch() > H.capi.hck_rotate_noalloc_scratch(None)
    prm = dict(q=q, n=1 << 17)
    a = _rand_ct(ctx, prm, 0, 80)
    out = _rand_ct(ctx, prm, 0, 81)
    with pytest.raises(H.HckError, match="MiB"):
        ctx.rotate_noalloc(a, 1, None, out)
