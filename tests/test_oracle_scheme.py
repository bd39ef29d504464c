"""Scheme-level checks of the CPU oracle on the tiny ring (N = 2^12).

Decrypted and decoded results are compared with plaintext arithmetic on the
same seeded slots (the paper's plaintext pipeline comparison, section 5.1
baselines), and key switching with the exact noise bound of hybrid key
switching.  None of these reuse an oracle formula as its own reference.
"""
import math

import numpy as np
import pytest

import oracle as O
import seeded_inputs as S


@pytest.fixture(scope="module")
def tiny():
    o = O.Oracle(S.params("tiny"))
    s = o.keygen_secret(1)
    return o, s


def centred(res, mods):
    return O.crt_centered(res, mods)


def test_encrypt_decrypt_sk_and_pk(tiny):
    o, s = tiny
    z = S.uniform_slots(o.n_slots, 0)
    pt = o.encode(z, 2.0 ** 25, 2)
    ct = o.encrypt_sk(s, pt, 10)
    assert np.max(np.abs(o.decode(o.decrypt(s, ct)) - z)) < 1e-4
    pk = o.keygen_public(s, 2)
    ct2 = o.encrypt_pk(pk, pt, 11)
    # public-key noise at N = 2^12, scale 2^25 (reading A10): a few 1e-3
    assert np.max(np.abs(o.decode(o.decrypt(s, ct2)) - z)) < 1e-2
    # the public key is an encryption of zero: b + a s is small
    e = centred(O.poly_add(pk[0], O.poly_mul(pk[1], O.embed_small(s, o.log_n, o.q),
                                             o.log_n, o.q), o.log_n, o.q), o.q)
    assert max(abs(x) for x in e) <= 19


def ks_error_bound(o, level):
    """|u0 + u1 s - d s'| bound of hybrid key switching: per digit the key
    error times the extended digit, divided by P, plus the ModDown floor
    error (K + K N for the s term, rounding ModDown)."""
    big_p = math.prod(o.p)
    alpha = o.alpha
    qj = max(math.prod(o.q[j * alpha: min((j + 1) * alpha, level + 1)])
             for j in range(o.dnum) if j * alpha <= level)
    return o.dnum * o.n * alpha * qj * 19 / big_p + o.K * (1 + o.n) + 1


@pytest.mark.parametrize("level", [2, 1, 0])
def test_keyswitch_noise_bound(tiny, level):
    o, s = tiny
    mods = o.qmods(level)
    g = o.galois_element(3)
    gk = o.keygen_galois(s, g, 5)
    d = S.uniform_residues(mods, o.n, seed=21)[0]
    u0, u1 = o.keyswitch(d, level, gk)
    s_r = O.embed_small(s, o.log_n, mods)
    s_g = O.automorphism(s_r, g, o.log_n, mods)
    err = O.poly_sub(O.poly_add(u0, O.poly_mul(u1, s_r, o.log_n, mods), o.log_n, mods),
                     O.poly_mul(d, s_g, o.log_n, mods), o.log_n, mods)
    e = centred(err, mods)
    assert max(abs(x) for x in e) < ks_error_bound(o, level)


def test_wide_special_primes_parameter_set():
    """The sets of the whole-word basis-conversion parity test: the chain of
    the named set with special primes in [2^60, 2^61), = 1 mod 2N, prime,
    distinct from the chain and summing below 2^64 (the library's bound on
    the conversion sums)."""
    for name in ("tiny", "mix15"):
        prm, base = S.params_wide_special(name), S.params(name)
        assert prm["q"] == base["q"] and len(prm["p"]) == len(base["p"])
        for p in prm["p"]:
            assert (1 << 60) <= p < (1 << 61) and p % (2 * prm["n"]) == 1 and S.is_prime(p)
        assert not set(prm["p"]) & set(prm["q"]) and sum(prm["p"]) < 1 << 64


@pytest.mark.parametrize("level", [2, 0])
def test_keyswitch_noise_bound_wide_special_primes(level):
    """Hybrid key switching with a 61-bit special prime stays within the same
    exact noise bound (key noise over P, plus the ModDown rounding)."""
    o = O.Oracle(S.params_wide_special("tiny"))
    s = o.keygen_secret(1)
    mods = o.qmods(level)
    g = o.galois_element(3)
    gk = o.keygen_galois(s, g, 5)
    d = S.uniform_residues(mods, o.n, seed=23)[0]
    u0, u1 = o.keyswitch(d, level, gk)
    s_r = O.embed_small(s, o.log_n, mods)
    s_g = O.automorphism(s_r, g, o.log_n, mods)
    err = O.poly_sub(O.poly_add(u0, O.poly_mul(u1, s_r, o.log_n, mods), o.log_n, mods),
                     O.poly_mul(d, s_g, o.log_n, mods), o.log_n, mods)
    assert max(abs(x) for x in centred(err, mods)) < ks_error_bound(o, level)


def test_keyswitch_wrong_key_is_not_small(tiny):
    """The bound above is meaningful: a key for another element fails it."""
    o, s = tiny
    mods = o.qmods(2)
    gk = o.keygen_galois(s, o.galois_element(5), 5)
    d = S.uniform_residues(mods, o.n, seed=21)[0]
    u0, u1 = o.keyswitch(d, 2, gk)
    s_r = O.embed_small(s, o.log_n, mods)
    s_g = O.automorphism(s_r, o.galois_element(3), o.log_n, mods)
    err = O.poly_sub(O.poly_add(u0, O.poly_mul(u1, s_r, o.log_n, mods), o.log_n, mods),
                     O.poly_mul(d, s_g, o.log_n, mods), o.log_n, mods)
    assert max(abs(x) for x in centred(err, mods)) > 1000 * ks_error_bound(o, 2)


@pytest.fixture(scope="module")
def tiny_ct(tiny):
    o, s = tiny
    z = S.uniform_slots(o.n_slots, 0)
    ct = o.encrypt_sk(s, o.encode(z, 2.0 ** 25, 2), 10)
    return z, ct


@pytest.mark.parametrize("step", [1, 5, -3, 1000])
def test_rotation_decodes_to_left_roll(tiny, tiny_ct, step):
    o, s = tiny
    z, ct = tiny_ct
    g = o.galois_element(step)
    gks = {g: o.keygen_galois(s, g, 5)}
    r = o.rotate(ct, step, gks)
    assert np.max(np.abs(o.decode(o.decrypt(s, r)).real - np.roll(z, -step))) < 1e-3


def test_rotation_composition_and_order(tiny, tiny_ct):
    o, s = tiny
    z, ct = tiny_ct
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5) for k in (2, 3, 5)}
    ab = o.rotate(o.rotate(ct, 2, gks), 3, gks)
    c = o.rotate(ct, 5, gks)
    da, dc = o.decode(o.decrypt(s, ab)).real, o.decode(o.decrypt(s, c)).real
    assert np.max(np.abs(da - dc)) < 1e-3
    # 5 has order N/2 modulo 2N: a rotation by N/2 slots is the identity element
    assert pow(5, o.n_slots, 2 * o.n) == 1
    same = o.rotate(ct, o.n_slots, gks)
    assert np.array_equal(same.polys, ct.polys)


def test_conjugation(tiny):
    o, s = tiny
    z = S.uniform_slots(o.n_slots, 3, complex_=True)
    ct = o.encrypt_sk(s, o.encode(z, 2.0 ** 25, 2), 12)
    g = 2 * o.n - 1
    r = o.apply_galois(ct, g, o.keygen_galois(s, g, 6))
    assert np.max(np.abs(o.decode(o.decrypt(s, r)) - np.conj(z))) < 1e-3


def test_multiply_relinearize_rescale(tiny):
    o, s = tiny
    z1 = S.uniform_slots(o.n_slots, 4)
    z2 = S.uniform_slots(o.n_slots, 5)
    # inputs at scale 2^30 (~ q): after one rescale by a 30-bit prime the
    # scale is ~2^30 again, so rounding noise stays far below 1e-3
    c1 = o.encrypt_sk(s, o.encode(z1, 2.0 ** 30, 2), 13)
    c2 = o.encrypt_sk(s, o.encode(z2, 2.0 ** 30, 2), 14)
    t = o.tensor(c1, c2)
    assert t.polys.shape[0] == 3
    # three-part decryption c0 + c1 s + c2 s^2
    assert np.max(np.abs(o.decode(o.decrypt(s, t)).real - z1 * z2)) < 1e-3
    r = o.relinearize(t, o.keygen_relin(s, 7))
    assert np.max(np.abs(o.decode(o.decrypt(s, r)).real - z1 * z2)) < 1e-3
    rs = o.rescale(r)
    assert rs.level == 1 and rs.scale == pytest.approx(2.0 ** 60 / o.q[2])
    assert np.max(np.abs(o.decode(o.decrypt(s, rs)).real - z1 * z2)) < 1e-3
    with pytest.raises(ValueError):
        o.rescale(o.rescale(rs))


def test_add_sub_plain_ops(tiny, tiny_ct):
    o, s = tiny
    z, ct = tiny_ct
    w = S.uniform_slots(o.n_slots, 6)
    pw = o.encode(w, 2.0 ** 25, 2)
    assert np.max(np.abs(o.decode(o.decrypt(s, o.add_plain(ct, pw))).real - (z + w))) < 1e-4
    c2 = o.encrypt_sk(s, pw, 15)
    assert np.max(np.abs(o.decode(o.decrypt(s, o.sub(ct, c2))).real - (z - w))) < 1e-4
    m = o.mul_plain(ct, o.encode(w, float(o.q[2]), 2))
    m = o.rescale(m)
    assert np.max(np.abs(o.decode(o.decrypt(s, m)).real - z * w)) < 1e-3
    with pytest.raises(ValueError):
        o.add(ct, o.drop_level(c2, 1))


def block_diag_diagonals(m, blocks):
    """Generalized diagonals of I_blocks (x) M: diag_k[j] = A[j][(j+k) mod n]."""
    d = m.shape[0]
    n = d * blocks
    out = {}
    for k in range(-(d - 1), d):
        v = np.zeros(n)
        for j in range(n):
            col = (j + k) % n
            if col // d == j // d:
                v[j] = m[j % d, col % d]
        if np.any(v):
            out[k] = v
    return out


def test_bsgs_tiny_config_end_to_end(tiny):
    """The tiny benchmark workload (reading A19): x uniform[-1,1] in 2048
    slots, y = (I_32 (x) M64) x by BSGS (n1 = 16), rescale, y^2 with
    relinearization; decoded result within 1e-3 of plaintext math."""
    o, s = tiny
    x = S.uniform_slots(o.n_slots, 0)
    m = S.uniform_matrix(64, 64, 0, 0.125)
    diags = block_diag_diagonals(m, 32)
    assert len(diags) == 127
    lt = o.lt_create(diags, 16, 2)
    steps = o.lt_required_steps(lt)
    assert len(steps) == 15 + 7
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5) for k in steps}
    ct = o.encrypt_sk(s, o.encode(x, 2.0 ** 25, 2), 10)
    y = o.rescale(o.lt_apply(lt, ct, gks))
    ref = np.kron(np.eye(32), m) @ x
    assert np.max(np.abs(o.decode(o.decrypt(s, y)).real - ref)) < 1e-3
    sq = o.relinearize(o.tensor(y, y), o.keygen_relin(s, 7))
    assert np.max(np.abs(o.decode(o.decrypt(s, sq)).real - ref ** 2)) < 1e-3


def test_bsgs_equals_naive_diagonal_method(tiny):
    """BSGS and the plain diagonal method sum_k diag_k * Rot(x, k) decode alike."""
    o, s = tiny
    x = S.uniform_slots(o.n_slots, 8)
    m = S.uniform_matrix(8, 8, 1, 0.3)
    diags = block_diag_diagonals(m, o.n_slots // 8)
    lt = o.lt_create(diags, 4, 2)
    steps = set(o.lt_required_steps(lt)) | set(diags)
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5) for k in steps}
    ct = o.encrypt_sk(s, o.encode(x, 2.0 ** 25, 2), 10)
    bsgs = o.decode(o.decrypt(s, o.rescale(o.lt_apply(lt, ct, gks)))).real
    naive = None
    for k, v in diags.items():
        term = o.mul_plain(o.rotate(ct, k, gks), o.encode(v, float(o.q[2]), 2))
        naive = term if naive is None else o.add(naive, term)
    naive = o.decode(o.decrypt(s, o.rescale(naive))).real
    assert np.max(np.abs(bsgs - naive)) < 1e-3
    assert np.max(np.abs(bsgs - np.kron(np.eye(o.n_slots // 8), m) @ x)) < 1e-3


def test_lt_eval_complex_dft_decodes(tiny):
    """Sums of transforms with shared baby steps and combined giant rotations
    (the complex DFT form of Eq. dft_re) decode to the plaintext result."""
    o, s = tiny
    d, n1, level = 8, 4, 2
    c = S.uniform_matrix(d, d, 1, 0.2)
    sm = S.uniform_matrix(d, d, 2, 0.2)
    lc = o.lt_create(block_diag_diagonals(c, o.n_slots // d), n1, level)
    ls = o.lt_create(block_diag_diagonals(sm, o.n_slots // d), n1, level)
    steps = set(o.lt_required_steps(lc)) | set(o.lt_required_steps(ls))
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5) for k in steps}
    xr, xi = S.uniform_slots(o.n_slots, 3), S.uniform_slots(o.n_slots, 4)
    cr = o.encrypt_sk(s, o.encode(xr, 2.0 ** 25, level), 10)
    ci = o.encrypt_sk(s, o.encode(xi, 2.0 ** 25, level), 11)
    out = o.lt_eval([cr, ci], [(lc, 0, 0, 1), (ls, 1, 0, -1), (ls, 0, 1, 1), (lc, 1, 1, 1)],
                    gks, 2)
    eye = np.eye(o.n_slots // d)
    re = np.kron(eye, c) @ xr - np.kron(eye, sm) @ xi
    im = np.kron(eye, sm) @ xr + np.kron(eye, c) @ xi
    assert np.max(np.abs(o.decode(o.decrypt(s, o.rescale(out[0]))).real - re)) < 1e-3
    assert np.max(np.abs(o.decode(o.decrypt(s, o.rescale(out[1]))).real - im)) < 1e-3


def test_hoisted_rotations_decode_and_differ(tiny, tiny_ct):
    """Hoisted rotations (one ModUp for several steps) decode to the rolled
    slots like plain rotations, with different but valid residues."""
    o, s = tiny
    z, ct = tiny_ct
    steps = [1, 2, 7, -5]
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5) for k in steps}
    outs = o.rotate_hoisted(ct, steps, gks)
    for k, r in zip(steps, outs):
        assert np.max(np.abs(o.decode(o.decrypt(s, r)).real - np.roll(z, -k))) < 1e-3
    plain = o.rotate(ct, 1, gks)
    assert not np.array_equal(plain.polys, outs[0].polys)


def test_keyswitch_split_equals_whole(tiny):
    """ModUp followed by the extended-basis inner product and ModDown is the
    key switch (same residues)."""
    o, s = tiny
    rlk = o.keygen_relin(s, 7)
    for level in (2, 0):
        d = S.uniform_residues(o.qmods(level), o.n, 31)[0]
        u0, u1 = o.keyswitch(d, level, rlk)
        v0, v1 = o.keyswitch_ext(o.modup(d, level), level, rlk)
        assert np.array_equal(u0, v0) and np.array_equal(u1, v1)


def test_inner_product_then_moddown_is_keyswitch_ext(tiny):
    """The extended-basis inner product followed by ModDown of each
    accumulator gives the key switch's residues."""
    o, s = tiny
    rlk = o.keygen_relin(s, 7)
    level = 2
    ext = o.modup(S.uniform_residues(o.qmods(level), o.n, 32)[0], level)
    a0, a1 = o.ks_inner(ext, level, rlk)
    assert a0.shape == (level + 1 + o.K, o.n)
    u0, u1 = o.keyswitch_ext(ext, level, rlk)
    assert np.array_equal(o.moddown(a0, level), u0)
    assert np.array_equal(o.moddown(a1, level), u1)


def test_giant_sum_of_one_rotation_is_the_rotation(tiny, tiny_ct):
    """With a single rotated part the shared ModDown is that rotation's own
    ModDown: same residues as rotate(), also next to an unrotated part."""
    o, s = tiny
    z, ct = tiny_ct
    g = o.galois_element(5)
    gks = {g: o.keygen_galois(s, g, 5)}
    assert np.array_equal(o.giant_sum([(5, ct)], gks).polys, o.rotate(ct, 5, gks).polys)
    other = o.encrypt_sk(s, o.encode(S.uniform_slots(o.n_slots, 9), 2.0 ** 25, 2), 12)
    want = o.add(other, o.rotate(ct, 5, gks))
    assert np.array_equal(o.giant_sum([(0, other), (5, ct)], gks).polys, want.polys)


def test_giant_sum_decodes_and_differs(tiny):
    """Several rotations sharing one ModDown decode to the sum of the rolled
    slots (within the noise of one key switch per part) and differ in their
    residues from the sum of separate rotations."""
    o, s = tiny
    steps = [0, 1, 6, -11, 300]
    zs = [S.uniform_slots(o.n_slots, 40 + i) for i in range(len(steps))]
    cts = [o.encrypt_sk(s, o.encode(z, 2.0 ** 25, 2), 20 + i) for i, z in enumerate(zs)]
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5)
           for k in steps if k}
    got = o.giant_sum(list(zip(steps, cts)), gks)
    want = sum(np.roll(z, -k) for z, k in zip(zs, steps))
    assert np.max(np.abs(o.decode(o.decrypt(s, got)).real - want)) < 1e-3
    plain = cts[0]
    for k, c in zip(steps[1:], cts[1:]):
        plain = o.add(plain, o.rotate(c, k, gks))
    assert not np.array_equal(plain.polys, got.polys)


def test_lt_eval_with_shared_giant_moddown_decodes(tiny):
    """The complex DFT of Eq. dft_re with hoisted baby steps and one ModDown
    per output for the giant steps decodes to the plaintext result."""
    o, s = tiny
    d, n1, level = 8, 4, 2
    c = S.uniform_matrix(d, d, 1, 0.2)
    sm = S.uniform_matrix(d, d, 2, 0.2)
    lc = o.lt_create(block_diag_diagonals(c, o.n_slots // d), n1, level)
    ls = o.lt_create(block_diag_diagonals(sm, o.n_slots // d), n1, level)
    steps = set(o.lt_required_steps(lc)) | set(o.lt_required_steps(ls))
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5) for k in steps}
    xr, xi = S.uniform_slots(o.n_slots, 3), S.uniform_slots(o.n_slots, 4)
    cr = o.encrypt_sk(s, o.encode(xr, 2.0 ** 25, level), 10)
    ci = o.encrypt_sk(s, o.encode(xi, 2.0 ** 25, level), 11)
    out = o.lt_eval([cr, ci], [(lc, 0, 0, 1), (ls, 1, 0, -1), (ls, 0, 1, 1), (lc, 1, 1, 1)],
                    gks, 2, hoist=True, hoist_giant=True)
    eye = np.eye(o.n_slots // d)
    re = np.kron(eye, c) @ xr - np.kron(eye, sm) @ xi
    im = np.kron(eye, sm) @ xr + np.kron(eye, c) @ xi
    assert np.max(np.abs(o.decode(o.decrypt(s, o.rescale(out[0]))).real - re)) < 1e-3
    assert np.max(np.abs(o.decode(o.decrypt(s, o.rescale(out[1]))).real - im)) < 1e-3
