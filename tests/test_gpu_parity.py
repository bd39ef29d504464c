"""GPU <-> oracle parity through the C ABI (MI355X).

Every test feeds the same seeded inputs to the HIP library and to the CPU
oracle and requires bit-identical residues (coefficient domain, fully
reduced).  Inputs are either uniform residue arrays from ``seeded_inputs`` or
objects both sides derive from the same seeds (keys, encryptions).  Ring
sizes: N = 2^12 (L = 3, K = 1), N = 2^15 (L = 12, K = 4), the benchmark's
N = 2^16, L = 24, K = 8 and the gesture shape N = 2^16, L = 30, K = 10 (ten
60-bit special primes, where the basis-conversion sums come closest to their
2^64 bound), all with dnum = 3; levels from the top down to 0 exercise ragged
last digits.
"""
import numpy as np
import pytest

import oracle as O
import seeded_inputs as S

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_2603_22437_amd")


class Pair:
    """A GPU context and an oracle over one parameter set, with one secret."""

    def __init__(self, name, prm=None):
        self.prm = S.params(name) if prm is None else prm
        self.ctx = H.Context.from_params(self.prm)
        self.o = O.Oracle(self.prm)
        self.s_o = self.o.keygen_secret(1)
        self.sk = self.ctx.keygen_secret(1)
        self.gk_cache = {}

    def galois(self, steps):
        """GPU Galois keys and the oracle's, for the rotation steps."""
        els = sorted({self.o.galois_element(k) for k in steps if k % self.o.n_slots})
        missing = [g for g in els if g not in self.gk_cache]
        for g in missing:
            self.gk_cache[g] = self.o.keygen_galois(self.s_o, g, 5)
        gks = self.ctx.keygen_galois(self.sk, els, 5)
        return gks, {g: self.gk_cache[g] for g in els}

    def rand_ct(self, level, seed, size=2):
        res = S.uniform_residues(self.o.qmods(level), self.o.n, seed, count=size)
        ct_o = O.Ciphertext(res, level, 2.0 ** 40)
        ct_g = self.ctx.ciphertext_import(res, level, 2.0 ** 40)
        return ct_g, ct_o

    def export(self, ct):
        return self.ctx.ciphertext_export(ct)[0]


_pairs = {}


def pair(name):
    if name not in _pairs:
        _pairs[name] = Pair(name)
    return _pairs[name]


CONFIGS = ["tiny", "mix15", "vital", "gesture"]


@pytest.mark.parametrize("name", CONFIGS)
def test_import_export_roundtrip(name):
    p = pair(name)
    ct, ct_o = p.rand_ct(p.o.L - 1, 100)
    assert np.array_equal(p.export(ct), ct_o.polys)


@pytest.mark.parametrize("name", CONFIGS)
def test_poly_product_via_mul_plain(name):
    """NTT -> pointwise -> INTT on the GPU equals the oracle's negacyclic product."""
    p = pair(name)
    level = p.o.L - 1
    ct, ct_o = p.rand_ct(level, 101)
    ptres = S.uniform_residues(p.o.qmods(level), p.o.n, 102)[0]
    pt = p.ctx.plaintext_import(ptres, level, 3.0)
    got = p.export(p.ctx.mul_plain(ct, pt))
    want = p.o.mul_plain(ct_o, O.Plaintext(ptres, level, 3.0)).polys
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", CONFIGS)
def test_keys_match_oracle(name):
    p = pair(name)
    o = p.o
    pk = p.ctx.public_key_export(p.ctx.keygen_public(p.sk, 2))
    assert np.array_equal(pk, o.keygen_public(p.s_o, 2))
    g = o.galois_element(3)
    gks, gko = p.galois([3])
    assert np.array_equal(p.ctx.galois_keys_export(gks, g), gko[g])
    rlk = p.ctx.switch_key_export(p.ctx.keygen_relin(p.sk, 7))
    assert np.array_equal(rlk, o.keygen_relin(p.s_o, 7))


@pytest.mark.parametrize("name", CONFIGS)
def test_encrypt_matches_oracle(name):
    p = pair(name)
    o = p.o
    level = o.L - 1
    res = S.uniform_residues(o.qmods(level), o.n, 103)[0]
    pt = p.ctx.plaintext_import(res, level, 2.0 ** 30)
    got = p.export(p.ctx.encrypt_sk(p.sk, pt, 10))
    want = o.encrypt_sk(p.s_o, O.Plaintext(res, level, 2.0 ** 30), 10).polys
    assert np.array_equal(got, want)
    pk = p.ctx.keygen_public(p.sk, 2)
    got = p.export(p.ctx.encrypt_pk(pk, pt, 11))
    want = o.encrypt_pk(o.keygen_public(p.s_o, 2), O.Plaintext(res, level, 2.0 ** 30), 11).polys
    assert np.array_equal(got, want)
    # decryption: c0 + c1 s
    ct, ct_o = p.rand_ct(level, 104)
    dec, lvl, _ = p.ctx.plaintext_export(p.ctx.decrypt(p.sk, ct))
    assert np.array_equal(dec, o.decrypt(p.s_o, ct_o).res)


def _levels(o):
    return sorted({o.L - 1, (o.L - 1) // 2, o.alpha, 0})


@pytest.mark.parametrize("name", CONFIGS)
def test_keyswitch_matches_oracle(name):
    """Raw hybrid key switching of polynomial 0 with the relinearization key."""
    p = pair(name)
    o = p.o
    rlk = p.ctx.keygen_relin(p.sk, 7)
    rlk_o = o.keygen_relin(p.s_o, 7)
    for level in _levels(o):
        ct, ct_o = p.rand_ct(level, 200 + level)
        got = p.export(p.ctx.keyswitch(ct, rlk))
        u0, u1 = o.keyswitch(ct_o.polys[0], level, rlk_o)
        assert np.array_equal(got[0], u0), f"level {level} u0"
        assert np.array_equal(got[1], u1), f"level {level} u1"


@pytest.mark.parametrize("name", CONFIGS)
def test_rotation_matches_oracle(name):
    p = pair(name)
    o = p.o
    steps = [1, -1, 5, o.n_slots // 2 + 3]
    gks, gko = p.galois(steps)
    for level in _levels(o):
        ct, ct_o = p.rand_ct(level, 300 + level)
        for k in (steps if level == o.L - 1 else steps[:1]):
            got = p.export(p.ctx.rotate(ct, k, gks))
            want = o.rotate(ct_o, k, gko).polys
            assert np.array_equal(got, want), f"level {level} step {k}"


@pytest.mark.parametrize("name", ["tiny", "mix15"])
def test_conjugation_matches_oracle(name):
    p = pair(name)
    o = p.o
    g = 2 * o.n - 1
    gks = p.ctx.keygen_galois(p.sk, [g], 6)
    ct, ct_o = p.rand_ct(o.L - 1, 400)
    got = p.export(p.ctx.apply_galois(ct, g, gks))
    want = o.apply_galois(ct_o, g, o.keygen_galois(p.s_o, g, 6)).polys
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", CONFIGS)
def test_tensor_relin_rescale_match_oracle(name):
    p = pair(name)
    o = p.o
    level = o.L - 1
    a, a_o = p.rand_ct(level, 500)
    b, b_o = p.rand_ct(level, 501)
    t = p.ctx.mul(a, b)
    t_o = o.tensor(a_o, b_o)
    assert np.array_equal(p.export(t), t_o.polys)
    rlk = p.ctx.keygen_relin(p.sk, 7)
    r = p.ctx.relinearize(t, rlk)
    r_o = o.relinearize(t_o, o.keygen_relin(p.s_o, 7))
    assert np.array_equal(p.export(r), r_o.polys)
    for lv in [level, 1]:
        c, c_o = p.rand_ct(lv, 510 + lv)
        rs = p.ctx.rescale(c)
        rs_o = o.rescale(c_o)
        assert rs.level == lv - 1
        assert np.array_equal(p.export(rs), rs_o.polys), f"rescale at level {lv}"
    # a 3-part rescale
    t3 = p.ctx.rescale(t)
    assert np.array_equal(p.export(t3), o.rescale(t_o).polys)


@pytest.mark.parametrize("name", ["tiny", "vital", "gesture"])
def test_elementwise_match_oracle(name):
    p = pair(name)
    o = p.o
    level = o.L - 2
    a, a_o = p.rand_ct(level, 600)
    b, b_o = p.rand_ct(level, 601)
    assert np.array_equal(p.export(p.ctx.add(a, b)), o.add(a_o, b_o).polys)
    assert np.array_equal(p.export(p.ctx.sub(a, b)), o.sub(a_o, b_o).polys)
    ptres = S.uniform_residues(o.qmods(level), o.n, 602)[0]
    pt = p.ctx.plaintext_import(ptres, level, 2.0 ** 40)
    assert np.array_equal(p.export(p.ctx.add_plain(a, pt)),
                          o.add_plain(a_o, O.Plaintext(ptres, level, 2.0 ** 40)).polys)
    d = p.ctx.drop_level(a, 1)
    assert np.array_equal(p.export(d), o.drop_level(a_o, 1).polys)
    # in-place (out aliases an input)
    c, c_o = p.rand_ct(level, 603)
    p.ctx.add(c, b, out=c)
    assert np.array_equal(p.export(c), o.add(c_o, b_o).polys)


@pytest.mark.parametrize("name,n_diag,n1", [("tiny", 127, 16), ("mix15", 9, 4)])
def test_linear_transform_matches_oracle(name, n_diag, n1):
    """BSGS over integer diagonal plaintexts imported identically on both sides."""
    p = pair(name)
    o = p.o
    level = o.L - 1
    half = n_diag // 2
    offsets = list(range(-half, n_diag - half))
    res = {k: S.uniform_residues(o.qmods(level), o.n, 700 + i)[0]
           for i, k in enumerate(offsets)}
    lt = p.ctx.lt_create_from_residues(res, n1, level, float(o.q[level]))
    lt_o = o.lt_from_plaintexts({k: O.Plaintext(r, level, float(o.q[level]))
                                 for k, r in res.items()}, n1, level, float(o.q[level]))
    steps = p.ctx.lt_required_steps(lt)
    assert steps == o.lt_required_steps(lt_o)
    gks, gko = p.galois(steps)
    ct, ct_o = p.rand_ct(level, 710)
    got = p.export(p.ctx.lt_apply(lt, ct, gks))
    want = o.lt_apply(lt_o, ct_o, gko).polys
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", ["tiny", "vital"])
def test_rotate_many_matches_single_rotations(name):
    """Batched key switching (one key stream for several ciphertexts) gives the
    oracle's residues for every member, including an output aliasing its input
    and more members than one batch holds."""
    p = pair(name)
    o = p.o
    gks, gko = p.galois([3])
    level = o.L - 1 if name == "tiny" else o.L // 2
    cts = [p.rand_ct(level, 1000 + i) for i in range(10)]
    outs = [p.ctx.ciphertext() for _ in range(9)] + [cts[9][0]]   # last one in place
    p.ctx.rotate_many([c for c, _ in cts], 3, gks, outs)
    for (c, c_o), out in zip(cts, outs):
        assert np.array_equal(p.export(out), o.rotate(c_o, 3, gko).polys)


@pytest.mark.parametrize("name", CONFIGS)
def test_rotate_steps_matches_single_rotations(name):
    """Rotations by different steps switched together (each batch member with
    its own key) give the oracle's residues, including a zero step (a copy), an
    in-place member and more members than one batch holds."""
    p = pair(name)
    o = p.o
    steps = ([1, 3, 0, 5, 1, -2, 3, 5, 1, 7] if name in ("tiny", "mix15")
             else [1, 3, 0, 1, 3, 1, 3, 1, 3, 1])
    gks, gko = p.galois(steps)
    level = o.L - 1 if name != "mix15" else o.L // 2
    cts = [p.rand_ct(level, 1100 + i) for i in range(len(steps))]
    outs = [p.ctx.ciphertext() for _ in range(len(steps) - 1)] + [cts[-1][0]]
    p.ctx.rotate_steps([c for c, _ in cts], steps, gks, outs)
    for (c, c_o), k, out in zip(cts, steps, outs):
        assert np.array_equal(p.export(out), o.rotate(c_o, k, gko).polys), k


@pytest.mark.parametrize("name,d,n1", [("tiny", 16, 4), ("mix15", 6, 3)])
def test_lt_eval_complex_dft_matches_oracle(name, d, n1):
    """The complex DFT form d_re = C v_re - S v_im, d_im = S v_re + C v_im with
    shared baby steps and combined giant rotations."""
    p = pair(name)
    o = p.o
    level = o.L - 1
    offs = list(range(-(d - 1), d))
    mats = {}
    for m, seed in (("C", 1100), ("S", 1200)):
        res = {k: S.uniform_residues(o.qmods(level), o.n, seed + i)[0] for i, k in enumerate(offs)}
        qs = float(o.q[level])
        mats[m] = (p.ctx.lt_create_from_residues(res, n1, level, qs),
                   o.lt_from_plaintexts({k: O.Plaintext(r, level, qs) for k, r in res.items()},
                                        n1, level, qs))
    steps = sorted(set(p.ctx.lt_required_steps(mats["C"][0])))
    gks, gko = p.galois(steps)
    v_re, v_re_o = p.rand_ct(level, 1300)
    v_im, v_im_o = p.rand_ct(level, 1301)
    terms = [("C", 0, 0, 1), ("S", 1, 0, -1), ("S", 0, 1, 1), ("C", 1, 1, 1)]
    got = p.ctx.lt_eval([v_re, v_im], [(mats[m][0], i, j, s) for m, i, j, s in terms], gks)
    want = o.lt_eval([v_re_o, v_im_o], [(mats[m][1], i, j, s) for m, i, j, s in terms], gko, 2)
    for g, w in zip(got, want):
        assert np.array_equal(p.export(g), w.polys)
    # hoisted baby steps
    goth = p.ctx.lt_eval([v_re, v_im], [(mats[m][0], i, j, s) for m, i, j, s in terms], gks,
                         hoist=True)
    wanth = o.lt_eval([v_re_o, v_im_o], [(mats[m][1], i, j, s) for m, i, j, s in terms], gko, 2,
                      hoist=True)
    for g_, w in zip(goth, wanth):
        assert np.array_equal(p.export(g_), w.polys)
    # giant rotations sharing one ModDown per output, with and without
    # hoisted baby steps
    for hb in (False, True):
        gotg = p.ctx.lt_eval([v_re, v_im], [(mats[m][0], i, j, s) for m, i, j, s in terms], gks,
                             hoist=hb, hoist_giant=True)
        wantg = o.lt_eval([v_re_o, v_im_o], [(mats[m][1], i, j, s) for m, i, j, s in terms],
                          gko, 2, hoist=hb, hoist_giant=True)
        for g_, w in zip(gotg, wantg):
            assert np.array_equal(p.export(g_), w.polys), f"hoist={hb}"
    # outputs aliasing inputs
    gota = p.ctx.lt_eval([v_re, v_im], [(mats[m][0], i, j, s) for m, i, j, s in terms], gks,
                         outputs=[v_re, v_im], hoist=True, hoist_giant=True)
    want_hh = o.lt_eval([v_re_o, v_im_o], [(mats[m][1], i, j, s) for m, i, j, s in terms], gko,
                        2, hoist=True, hoist_giant=True)
    assert np.array_equal(p.export(gota[0]), want_hh[0].polys)
    assert np.array_equal(p.export(gota[1]), want_hh[1].polys)
    v_re = p.ctx.ciphertext_import(v_re_o.polys, level, v_re_o.scale)
    v_im = p.ctx.ciphertext_import(v_im_o.polys, level, v_im_o.scale)
    # outputs aliasing inputs
    got2 = p.ctx.lt_eval([v_re, v_im], [(mats[m][0], i, j, s) for m, i, j, s in terms], gks,
                         outputs=[v_im, v_re])
    assert np.array_equal(p.export(got2[0]), want[0].polys)
    assert np.array_equal(p.export(got2[1]), want[1].polys)


@pytest.mark.parametrize("name", ["tiny", "mix15", "vital", "gesture"])
def test_hoisted_rotations_match_oracle(name):
    p = pair(name)
    o = p.o
    steps = [1, 5, -1, o.n_slots // 2 + 3, 0]
    gks, gko = p.galois(steps)
    for level in sorted({o.L - 1, o.alpha - 1, 0}):
        ct, ct_o = p.rand_ct(level, 1400 + level)
        got = p.ctx.rotate_hoisted(ct, steps, gks)
        want = o.rotate_hoisted(ct_o, steps, gko)
        for k, g_, w in zip(steps, got, want):
            assert np.array_equal(p.export(g_), w.polys), f"level {level} step {k}"
    # an output aliasing the input
    ct, ct_o = p.rand_ct(o.L - 1, 1450)
    outs = p.ctx.rotate_hoisted(ct, [5, 1], gks, outs=[p.ctx.ciphertext(), ct])
    want = o.rotate_hoisted(ct_o, [5, 1], gko)
    assert np.array_equal(p.export(outs[0]), want[0].polys)
    assert np.array_equal(p.export(outs[1]), want[1].polys)


def test_error_paths():
    p = pair("tiny")
    o = p.o
    ct, _ = p.rand_ct(o.L - 1, 800)
    gks, _ = p.galois([1])
    with pytest.raises(H.HckError) as e:
        p.ctx.rotate(ct, 2, gks)
    assert e.value.code == H.HCK_ENOKEY
    low, _ = p.rand_ct(0, 801)
    with pytest.raises(H.HckError) as e:
        p.ctx.rescale(low)
    assert e.value.code == H.HCK_ELEVEL
    with pytest.raises(H.HckError) as e:
        p.ctx.add(ct, low)
    assert e.value.code == H.HCK_ELEVEL
    other = p.ctx.ciphertext_import(S.uniform_residues(o.qmods(o.L - 1), o.n, 802, 2),
                                    o.L - 1, 2.0 ** 41)
    with pytest.raises(H.HckError) as e:
        p.ctx.add(ct, other)
    assert e.value.code == H.HCK_ESCALE
    bad = S.uniform_residues(o.qmods(0), o.n, 803, 2)
    bad[0, 0, 0] = o.q[0]
    with pytest.raises(H.HckError) as e:
        p.ctx.ciphertext_import(bad, 0, 1.0)
    assert e.value.code == H.HCK_EINVAL
    prm = dict(p.prm)
    with pytest.raises(H.HckError) as e:
        H.Context(12, [prm["q"][0] + 2] + prm["q"][1:], prm["p"], 3)
    assert e.value.code == H.HCK_EPARAMS
    with pytest.raises(H.HckError) as e:
        H.Context(12, prm["q"], prm["p"], 5)   # dnum > L
    assert e.value.code == H.HCK_EPARAMS
    # rotation by a multiple of N/2 slots is a copy and needs no key
    z = p.ctx.rotate(ct, o.n_slots, gks)
    assert np.array_equal(p.export(z), p.export(ct))


def test_tiny_config_decoded_end_to_end():
    """The tiny workload with the GPU's own encoder: encrypt 2048 slots,
    (I_32 (x) M64) x by BSGS, rescale, square + relinearize; decoded result
    within 1e-3 of plaintext math (and of the oracle's decoded result)."""
    from test_oracle_scheme import block_diag_diagonals
    p = pair("tiny")
    o, ctx = p.o, p.ctx
    x = S.uniform_slots(o.n_slots, 0)
    m = S.uniform_matrix(64, 64, 0, 0.125)
    diags = block_diag_diagonals(m, 32)
    lt = ctx.lt_create(diags, 16, 2)
    steps = ctx.lt_required_steps(lt)
    gks = ctx.keygen_rotation(p.sk, steps, 5)
    rlk = ctx.keygen_relin(p.sk, 7)
    ct = ctx.encrypt_sk(p.sk, ctx.encode(x, 2.0 ** 25, 2), 10)
    y = ctx.rescale(ctx.lt_apply(lt, ct, gks))
    sq = ctx.relinearize(ctx.mul(y, y), rlk)
    lin = np.kron(np.eye(32), m) @ x
    assert np.max(np.abs(ctx.decode(ctx.decrypt(p.sk, y)).real - lin)) < 1e-3
    got = ctx.decode(ctx.decrypt(p.sk, sq)).real
    assert np.max(np.abs(got - lin ** 2)) < 1e-3


@pytest.mark.parametrize("name", ["edge11", "edge17"])
def test_edge_rings_match_oracle(name):
    """The smallest (N = 2^11) and largest (N = 2^17) supported rings: NTT
    product, key switching at the top level and level 0 (ragged digits with
    dnum = 2 and 3), rotation, tensor + relinearize + rescale, all bit-exact."""
    p = pair(name)
    o = p.o
    top = o.L - 1
    # negacyclic product through the evaluation domain
    a = S.uniform_residues(o.qmods(top), o.n, 5)[0]
    b = S.uniform_residues(o.qmods(top), o.n, 6)[0]
    ct = p.ctx.ciphertext_import(np.stack([a, a]), top, 1.0)
    pt = p.ctx.plaintext_import(b, top, 1.0)
    got = p.export(p.ctx.mul_plain(ct, pt))
    assert np.array_equal(got[0], O.poly_mul(a, b, o.log_n, o.qmods(top)))
    gks, gko = p.galois([1, -3])
    rlk = p.ctx.keygen_relin(p.sk, 7)
    rlk_o = o.keygen_relin(p.s_o, 7)
    for level in sorted({top, 0}):
        c, c_o = p.rand_ct(level, 1500 + level)
        for k in (1, -3):
            assert np.array_equal(p.export(p.ctx.rotate(c, k, gks)),
                                  o.rotate(c_o, k, gko).polys), (level, k)
        if level > 0:
            d, d_o = p.rand_ct(level, 1600 + level)
            got = p.export(p.ctx.rescale(p.ctx.relinearize(p.ctx.mul(c, d), rlk)))
            want = o.rescale(o.relinearize(o.tensor(c_o, d_o), rlk_o)).polys
            assert np.array_equal(got, want), level


def test_empty_batches():
    """Batched calls with no members do nothing and succeed."""
    p = pair("tiny")
    gks, _ = p.galois([1])
    assert p.ctx.rotate_many([], 1, gks, []) == []
    assert p.ctx.rotate_steps([], [], gks, []) == []
    c, _ = p.rand_ct(p.o.L - 1, 1700)
    assert p.ctx.rotate_hoisted(c, [], gks) == []


@pytest.mark.parametrize("name", CONFIGS)
def test_relinearize_many_matches_oracle(name):
    """Relinearizations switched together in batches (one relinearization key
    stream) give the oracle's residues for every member, including an
    in-place member and more members than one batch holds."""
    p = pair(name)
    o = p.o
    level = o.L - 1 if name == "tiny" else o.L // 2
    rlk = p.ctx.keygen_relin(p.sk, 7)
    rlk_o = o.keygen_relin(p.s_o, 7)
    cts = [p.rand_ct(level, 1800 + i, size=3)
           for i in range(10 if name in ("tiny", "mix15") else 9)]
    outs = [p.ctx.ciphertext() for _ in range(len(cts) - 1)] + [cts[-1][0]]
    p.ctx.relinearize_many([c for c, _ in cts], rlk, outs)
    for (c, c_o), out in zip(cts, outs):
        assert np.array_equal(p.export(out), o.relinearize(c_o, rlk_o).polys)


@pytest.mark.slow
def test_lt_eval_full_size_bench_shape():
    """The benchmark's linear-transform launch at full size (N = 2^16, L = 24,
    n1 = 20, complex four-term evaluation over shared inputs, hoisted baby
    steps and one ModDown per output): 2 x 61 diagonals over 4 giant groups
    instead of 2 x 399 (which the oracle would take many minutes to multiply),
    same kernels and launch shapes, bit-exact."""
    p = pair("vital")
    o = p.o
    level = o.L - 1
    offs = list(range(-30, 31))
    mats = {}
    qs = float(o.q[level])
    for m, seed in (("C", 2100), ("S", 2200)):
        res = {k: S.uniform_residues(o.qmods(level), o.n, seed + i)[0] for i, k in enumerate(offs)}
        mats[m] = (p.ctx.lt_create_from_residues(res, 20, level, qs),
                   o.lt_from_plaintexts({k: O.Plaintext(r, level, qs) for k, r in res.items()},
                                        20, level, qs))
    steps = sorted(set(p.ctx.lt_required_steps(mats["C"][0])))
    gks, gko = p.galois(steps)
    v_re, v_re_o = p.rand_ct(level, 2300)
    v_im, v_im_o = p.rand_ct(level, 2301)
    terms = [("C", 0, 0, 1), ("S", 1, 0, -1), ("S", 0, 1, 1), ("C", 1, 1, 1)]
    got = p.ctx.lt_eval([v_re, v_im], [(mats[m][0], i, j, s) for m, i, j, s in terms], gks,
                        hoist=True, hoist_giant=True)
    want = o.lt_eval([v_re_o, v_im_o], [(mats[m][1], i, j, s) for m, i, j, s in terms], gko, 2,
                     hoist=True, hoist_giant=True)
    for g_, w in zip(got, want):
        assert np.array_equal(p.export(g_), w.polys)


def test_bench_step_decodes_at_full_size():
    """The benchmark step itself (2 x 399 cached diagonals of the windowed
    200-point DFT, n1 = 20, then |.|^2) decodes to |W z|^2 of the synthetic
    window within 1e-3 (a property that holds at any size)."""
    prm = S.params("vital")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    frames, bins, n1 = 200, 64, 20
    z = S.vital_window(1000, frames, bins)
    n_slots = ctx.n_slots
    v = np.zeros(n_slots, dtype=np.complex128)
    v[: frames * bins] = z.T.reshape(-1)
    top = len(prm["q"]) - 1
    ct_re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], top), 100)
    ct_im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], top), 101)
    w = S.windowed_dft_matrix(frames)

    def block_diagonals(mat):
        out = {}
        k = np.arange(frames)
        for off in range(-(frames - 1), frames):
            col = k + off
            ok = (col >= 0) & (col < frames)
            vals = np.where(ok, mat[k, np.clip(col, 0, frames - 1)], 0.0)
            vec = np.zeros(n_slots)
            vec[: bins * frames] = np.tile(vals, bins)
            if np.any(vec):
                out[off] = vec
        return out

    lt_c = ctx.lt_create(block_diagonals(w.real), n1, top)
    lt_s = ctx.lt_create(block_diagonals(w.imag), n1, top)
    steps = sorted(set(ctx.lt_required_steps(lt_c)) | set(ctx.lt_required_steps(lt_s)))
    gks = ctx.keygen_rotation(sk, steps, 5)
    rlk = ctx.keygen_relin(sk, 7)
    d_re, d_im = ctx.lt_eval([ct_re, ct_im], [(lt_c, 0, 0, 1), (lt_s, 1, 0, -1),
                                              (lt_s, 0, 1, 1), (lt_c, 1, 1, 1)], gks,
                             hoist=True, hoist_giant=True)
    d_re, d_im = ctx.rescale(d_re), ctx.rescale(d_im)
    pw = ctx.rescale(ctx.relinearize(ctx.add(ctx.mul(d_re, d_re), ctx.mul(d_im, d_im)), rlk))
    got = ctx.decode(ctx.decrypt(sk, pw)).real[: frames * bins].reshape(bins, frames)
    ref = np.abs(w @ z).T ** 2
    assert np.max(np.abs(got - ref)) < 1e-3


def test_torch_allocator_hook():
    """hck_set_allocator with torch's caching allocator: the context's buffers
    come from torch (its counter rises while they live and falls after
    close), results equal the default allocator's bit for bit, and the hook
    cannot be swapped while buffers of the current allocator are alive."""
    import torch
    prm = S.params("tiny")
    z = np.random.default_rng(3).uniform(-1, 1, 1 << (prm["log_n"] - 1))

    def run(ctx):
        sk = ctx.keygen_secret(1)
        gks = ctx.keygen_rotation(sk, [1, 5], 2)
        rlk = ctx.keygen_relin(sk, 3)
        ct = ctx.encrypt_sk(sk, ctx.encode(z, prm["scale"], len(prm["q"]) - 1), 4)
        r = ctx.rotate(ctx.relinearize(ctx.mul(ct, ct), rlk), 5, gks)
        return ctx.ciphertext_export(r)[0]

    ref_ctx = H.Context.from_params(prm)
    ref = run(ref_ctx)
    ref_ctx.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    ctx = H.Context.from_params(prm)
    ctx.use_torch_allocator()
    sk = ctx.keygen_secret(9)
    assert torch.cuda.memory_allocated() > before
    with pytest.raises(H.HckError):   # buffers of the hook are alive
        ctx.use_default_allocator()
    del sk
    got = run(ctx)
    assert np.array_equal(got, ref)
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_autotune_keyswitch_keeps_results_exact():
    """The key-switch autotuner picks a batch size per level within the launch
    limits, and batched rotations give the same residues under the built-in
    rule, the tuned sizes and one key switch per launch."""
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    gks = ctx.keygen_rotation(sk, [3], 2)
    top = len(prm["q"]) - 1
    cts = [ctx.encrypt_sk(sk, ctx.encode(np.random.default_rng(k).uniform(-1, 1, ctx.n_slots),
                                         prm["scale"], 5), 10 + k) for k in range(19)]

    def rotated():
        return [ctx.ciphertext_export(c)[0] for c in ctx.rotate_many(cts, 3, gks)]

    ref = rotated()
    rule = {l: ctx.keyswitch_batch_limit(l) for l in (0, 5, top)}
    tuned = ctx.autotune_keyswitch([0, 5, top], count=16)
    for l, (cap, us) in tuned.items():
        assert 1 <= cap <= 32 and us > 0
        assert ctx.keyswitch_batch_limit(l) == cap
    assert all(np.array_equal(a, b) for a, b in zip(ref, rotated()))
    ctx.set_keyswitch_cap(5, 1)
    assert ctx.keyswitch_batch_limit(5) == 1
    assert all(np.array_equal(a, b) for a, b in zip(ref, rotated()))
    ctx.set_keyswitch_cap(5, 0)
    assert ctx.keyswitch_batch_limit(5) == rule[5]
    with pytest.raises(H.HckError):
        ctx.set_keyswitch_cap(top + 1, 4)


@pytest.mark.parametrize("coeffs", [
    [0.3, -0.7],
    [0.1, 0.5, -0.25, 0.125],
    [0.0, 1.0, 0.0, -1 / 6, 0.0, 1 / 120, 0.0, -1 / 5040],
    list(np.random.default_rng(5).uniform(-1, 1, 16)),
])
def test_poly_eval_matches_oracle(coeffs):
    """hck_poly_eval bit-exact against the oracle's polynomial evaluation on
    one encrypted input (N = 2^12, L = 8), and decoded against numpy."""
    p = pair("deep12")
    o = p.o
    x = S.uniform_slots(o.n_slots, 3)
    ct_o = o.encrypt_sk(p.s_o, o.encode(x, p.prm["scale"], o.L - 1), 11)
    ct = p.ctx.ciphertext_import(ct_o.polys, ct_o.level, ct_o.scale)
    rlk = p.ctx.keygen_relin(p.sk, 7)
    want = o.poly_eval(ct_o, coeffs, o.keygen_relin(p.s_o, 7))
    got = p.ctx.poly_eval(ct, coeffs, rlk)
    assert got.level == want.level and got.scale == want.scale
    assert np.array_equal(p.export(got), want.polys)
    dec = p.ctx.decode(p.ctx.decrypt(p.sk, got)).real
    np.testing.assert_allclose(dec, np.polynomial.polynomial.polyval(x, coeffs), rtol=0,
                               atol=1e-6)


def test_encode_const_and_poly_eval_errors():
    p = pair("deep12")
    pt = p.ctx.encode_const(-1.25, 2.0 ** 40, 3)
    res, lvl, sc = p.ctx.plaintext_export(pt)
    assert np.array_equal(res, p.o.encode_const(-1.25, 2.0 ** 40, 3).res)
    rlk = p.ctx.keygen_relin(p.sk, 7)
    ct, _ = p.rand_ct(2, 520)
    with pytest.raises(H.HckError):       # depth 3 above level 2
        p.ctx.poly_eval(ct, [0, 0, 0, 0, 1.0], rlk)
    with pytest.raises(H.HckError):       # nothing of degree >= 1
        p.ctx.poly_eval(ct, [1.0, 0.0], rlk)
    with pytest.raises(H.HckError):
        p.ctx.poly_eval(ct, [0.0, 1.0], rlk, out=ct)


@pytest.mark.parametrize("dnum", [2, 4, 6])
def test_other_digit_counts_match_oracle(dnum):
    """The parameter sets the dnum autotuner chooses among (N = 2^15, L = 12
    with 2, 4 or 6 digits and K = 6, 3, 2 special primes): key switching at
    every level class and a rotation, bit-exact."""
    p = Pair(f"mix15/dnum{dnum}", S.params_with_dnum("mix15", dnum))
    o = p.o
    rlk = p.ctx.keygen_relin(p.sk, 7)
    rlk_o = o.keygen_relin(p.s_o, 7)
    for level in _levels(o):
        ct, ct_o = p.rand_ct(level, 700 + level)
        got = p.export(p.ctx.keyswitch(ct, rlk))
        u0, u1 = o.keyswitch(ct_o.polys[0], level, rlk_o)
        assert np.array_equal(got[0], u0) and np.array_equal(got[1], u1), level
    gks, gko = p.galois([5])
    ct, ct_o = p.rand_ct(o.L - 1, 710)
    assert np.array_equal(p.export(p.ctx.rotate(ct, 5, gks)), o.rotate(ct_o, 5, gko).polys)


@pytest.mark.parametrize("name", ["tiny", "mix15"])
def test_wide_special_primes_match_oracle(name):
    """Special primes just below 2^61, where the basis conversions take their
    whole-word path (the 30-bit one needs every modulus below 2^60): key
    switching at every level class, a batch of rotations large enough for
    paired conversion launches, and a rescale, bit-exact."""
    p = Pair(f"{name}/p61", S.params_wide_special(name))
    o = p.o
    assert min(o.p) >= 1 << 60 and max(o.p) < 1 << 61
    rlk = p.ctx.keygen_relin(p.sk, 7)
    rlk_o = o.keygen_relin(p.s_o, 7)
    for level in _levels(o):
        ct, ct_o = p.rand_ct(level, 760 + level)
        got = p.export(p.ctx.keyswitch(ct, rlk))
        u0, u1 = o.keyswitch(ct_o.polys[0], level, rlk_o)
        assert np.array_equal(got[0], u0) and np.array_equal(got[1], u1), level
    steps = [1, 3, 5, 7, -1, -3, 2, 4, 6, 9, 11, 13, 1, 3, 5, 7]
    gks, gko = p.galois(steps)
    cts = [p.rand_ct(o.L - 1, 780 + i) for i in range(len(steps))]
    outs = [p.ctx.ciphertext() for _ in steps]
    p.ctx.rotate_steps([c for c, _ in cts], steps, gks, outs)
    for (c, c_o), k, out in zip(cts, steps, outs):
        assert np.array_equal(p.export(out), o.rotate(c_o, k, gko).polys), k
    ct, ct_o = p.rand_ct(o.L - 1, 799)
    assert np.array_equal(p.export(p.ctx.rescale(ct)), o.rescale(ct_o).polys)


def test_autotune_dnum():
    """The dnum autotuner times each candidate's key switch and reports its
    key size; the best is the fastest."""
    dnums = (2, 3, 4, 6)
    cands = [S.params_with_dnum("mix15", d) for d in dnums]
    r = H.autotune_dnum(cands, level=11, count=8)
    assert len(r["us_per_switch"]) == len(dnums) and min(r["us_per_switch"]) > 0
    for d, c, kb in zip(dnums, cands, r["key_bytes"]):
        assert kb == 8 * d * 2 * (len(c["q"]) + len(c["p"])) * c["n"]
    assert r["best"] == int(np.argmin(r["us_per_switch"]))
    bad = dict(cands[1], q=list(reversed(cands[1]["q"])))
    with pytest.raises(H.HckError):
        H.autotune_dnum([cands[0], bad], level=11)


@pytest.mark.parametrize("name", ["tiny", "mix15", "vital"])
def test_ntt_splits_match_oracle(name):
    """The full transforms on every split the NTT tuner can choose (the
    default 2^ceil(log N / 2) x 2^floor(log N / 2) and one step either side):
    imports (forward NTT), exports (inverse NTT), products and encryption
    bit-exact against the oracle; the tuner keeps one of the candidates."""
    p = pair(name)
    o = p.o
    a0 = (p.prm["log_n"] + 1) // 2
    tried = []
    try:
        for a in (a0 - 1, a0 + 1, a0):
            try:
                p.ctx.set_ntt_split(a)
            except H.HckError:
                continue
            tried.append(a)
            assert p.ctx.ntt_split() == a
            level = o.L - 1
            ct, ct_o = p.rand_ct(level, 130 + a)
            assert np.array_equal(p.export(ct), ct_o.polys), a
            ptres = S.uniform_residues(o.qmods(level), o.n, 140 + a)[0]
            pt = p.ctx.plaintext_import(ptres, level, 3.0)
            got = p.export(p.ctx.mul_plain(ct, pt))
            assert np.array_equal(got, o.mul_plain(ct_o, O.Plaintext(ptres, level, 3.0)).polys), a
            enc = p.export(p.ctx.encrypt_sk(p.sk, pt, 12))
            assert np.array_equal(enc, o.encrypt_sk(p.s_o, O.Plaintext(ptres, level, 3.0),
                                                    12).polys), a
        assert len(tried) == 3
        tuned = p.ctx.autotune_ntt(rows=32)
        assert set(tuned["splits"]) == set(tried) and min(tuned["splits"].values()) > 0
        assert p.ctx.ntt_split() == tuned["chosen"] in tried
        with pytest.raises(H.HckError):
            p.ctx.set_ntt_split(a0 + 2)
    finally:
        p.ctx.set_ntt_split(0)
