"""Pins of the CPU oracle against definitions it does not itself use.

Each test checks one oracle function against something independent of it:
Python big-integer arithmetic, a direct (Horner / O(N^2)) evaluation of a
definition, an exact integer identity, a FIPS 202 known answer, or the sizes
printed in the paper's Table 6.  A dropped term, a wrong sign, a swapped
operand or an off-by-one index in the oracle fails one of these.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import seeded_inputs as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def py_ints(a):
    return [int(x) for x in np.asarray(a).ravel()]


# ---------------------------------------------------------------------------
# scalar modular arithmetic
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("q", [S.params("tiny")["q"][0], S.params("vital")["q"][0],
                               S.params("vital")["q"][5], (1 << 61) - 1])
def test_mulmod_edges_vs_python(q):
    rng = np.random.default_rng(1)
    vals = [0, 1, 2, q - 1, q - 2, q // 2, (q + 1) // 2] + [int(x) for x in rng.integers(0, q, 50)]
    for a in vals:
        for b in vals[:12]:
            assert O.mulmod(a, b, q) == a * b % q
    assert O._load().ock_powmod(3, q - 1, q) == pow(3, q - 1, q)
    for a in vals[1:]:
        assert O._load().ock_invmod(a, q) * a % q == 1 or a % q == 0


@pytest.mark.parametrize("name", ["tiny", "mix15", "vital"])
def test_root_2n_is_primitive(name):
    prm = S.params(name)
    n = prm["n"]
    for q in prm["q"][:3] + prm["p"][:1]:
        psi = O.root_2n(q, n)
        assert pow(psi, n, q) == q - 1          # psi^N = -1
        assert pow(psi, 2 * n, q) == 1          # order divides 2N, hence exactly 2N


# ---------------------------------------------------------------------------
# NTT
# ---------------------------------------------------------------------------

def horner(coeffs, x, q):
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * x + c) % q
    return acc


@pytest.mark.parametrize("log_n", [1, 3, 5, 7])
def test_ntt_is_evaluation_at_odd_powers(log_n):
    """out[k] = a(psi^(2k+1)), checked by Horner evaluation with Python ints."""
    n = 1 << log_n
    q = S.params("tiny")["q"][1]
    # a prime that is 1 mod 2n for every tested n (tiny primes are 1 mod 2^13)
    a = S.uniform_residues([q], n, seed=3)[0, 0]
    psi = O.root_2n(q, n)
    out = O.ntt(a, log_n, q)
    ai = py_ints(a)
    for k in range(n):
        assert int(out[k]) == horner(ai, pow(psi, 2 * k + 1, q), q)


def schoolbook_py(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                out[i + j] += a[i] * b[j]
            else:
                out[i + j - n] -= a[i] * b[j]
    return [x % q for x in out]


@pytest.mark.parametrize("name,log_n", [("tiny", 4), ("tiny", 6), ("vital", 5), ("vital", 6)])
def test_ntt_product_matches_python_schoolbook(name, log_n):
    prm = S.params(name)
    mods = prm["q"][:2] + prm["p"][:1]
    n = 1 << log_n
    a = S.uniform_residues(mods, n, seed=4)[0]
    b = S.uniform_residues(mods, n, seed=5)[0]
    prod = O.poly_mul(a, b, log_n, mods)
    for t, q in enumerate(mods):
        assert py_ints(prod[t]) == schoolbook_py(py_ints(a[t]), py_ints(b[t]), q)
        assert py_ints(O.poly_mul_schoolbook(a[t], b[t], log_n, q)) == py_ints(prod[t])


def test_ntt_product_large_ring_vs_c_schoolbook():
    prm = S.params("tiny")
    q = prm["q"][0]
    a = S.uniform_residues([q], 4096, seed=6)[0, 0]
    b = S.uniform_residues([q], 4096, seed=7)[0, 0]
    assert np.array_equal(O.poly_mul(a[None], b[None], 12, [q])[0],
                          O.poly_mul_schoolbook(a, b, 12, q))


@pytest.mark.parametrize("name", ["tiny", "mix15"])
def test_intt_inverts_ntt_and_monomial_closed_form(name):
    prm = S.params(name)
    log_n, n = prm["log_n"], prm["n"]
    q = prm["q"][-1]
    a = S.uniform_residues([q], n, seed=8)[0, 0]
    assert np.array_equal(O.intt(O.ntt(a, log_n, q), log_n, q), a)
    # NTT(X^k)[j] = psi^((2j+1)k)
    k = 37
    mono = np.zeros(n, dtype=np.uint64)
    mono[k] = 1
    psi = O.root_2n(q, n)
    out = O.ntt(mono, log_n, q)
    for j in [0, 1, 2, n // 2, n - 1]:
        assert int(out[j]) == pow(psi, (2 * j + 1) * k, q)


# ---------------------------------------------------------------------------
# automorphism
# ---------------------------------------------------------------------------

def test_automorphism_definition_and_homomorphism():
    prm = S.params("tiny")
    log_n, n, mods = 5, 32, prm["q"][:2]
    a = S.uniform_residues(mods, n, seed=9)[0]
    b = S.uniform_residues(mods, n, seed=10)[0]
    for g in [5, 25, 2 * n - 1, 3]:
        out = O.automorphism(a, g, log_n, mods)
        for t, q in enumerate(mods):
            ref = [0] * n
            for i in range(n):
                e = i * g % (2 * n)
                # X^(i g) = -X^(i g - N) when i g mod 2N >= N
                if e < n:
                    ref[e] = int(a[t, i])
                else:
                    ref[e - n] = (-int(a[t, i])) % q
            assert py_ints(out[t]) == ref
        # ring homomorphism: phi(a b) = phi(a) phi(b)
        lhs = O.automorphism(O.poly_mul(a, b, log_n, mods), g, log_n, mods)
        rhs = O.poly_mul(O.automorphism(a, g, log_n, mods),
                         O.automorphism(b, g, log_n, mods), log_n, mods)
        assert np.array_equal(lhs, rhs)
    # composition: phi_g o phi_h = phi_(g h mod 2N)
    lhs = O.automorphism(O.automorphism(a, 5, log_n, mods), 25, log_n, mods)
    assert np.array_equal(lhs, O.automorphism(a, 125 % (2 * n), log_n, mods))


def test_automorphism_permutes_evaluations():
    """phi_g(a)(psi^(2k+1)) = a(psi^((2k+1) g))."""
    prm = S.params("tiny")
    log_n, n, q = 6, 64, prm["q"][2]
    a = S.uniform_residues([q], n, seed=11)[0]
    psi = O.root_2n(q, n)
    g = 5 ** 7 % (2 * n)
    out = O.automorphism(a, g, log_n, [q])
    for k in range(0, n, 5):
        x = pow(psi, 2 * k + 1, q)
        assert horner(py_ints(out[0]), x, q) == horner(py_ints(a[0]), pow(x, g, q), q)


# ---------------------------------------------------------------------------
# basis conversion, ModDown, rescale: exact integer identities
# ---------------------------------------------------------------------------

def crt_py(res_cols, mods):
    big = math.prod(mods)
    acc = 0
    for r, q in zip(res_cols, mods):
        hat = big // q
        acc += r * pow(hat % q, -1, q) * hat
    return acc % big


@pytest.mark.parametrize("name,ns", [("vital", 8), ("vital", 3), ("tiny", 1), ("gesture", 10)])
def test_bconv_exact_identity(name, ns):
    """BConv(x) = x + u B mod t with integer u in [0, ns)."""
    prm = S.params(name)
    log_n, n = 4, 16
    allm = prm["q"] + prm["p"]
    src, dst = allm[:ns], allm[ns:ns + 5]
    x = S.uniform_residues(src, n, seed=12)[0]
    out = O.bconv(x, src, dst, log_n)
    big_b = math.prod(src)
    for c in range(n):
        xv = crt_py([int(x[i, c]) for i in range(ns)], src)
        us = set()
        for t, m in enumerate(dst):
            diff = (int(out[t, c]) - xv) % m
            cand = [u for u in range(ns) if (u * big_b - diff) % m == 0]
            assert len(cand) == 1
            us.add(cand[0])
        assert len(us) == 1  # the same u for every target


def test_moddown_exact_identity():
    """ModDown(u) = round(u / P) - v mod q_i with one integer v in [0, K)."""
    prm = S.params("vital")
    log_n, n = 4, 16
    q, p = prm["q"][:4], prm["p"][:3]
    u = S.uniform_residues(q + p, n, seed=13)[0]
    out = O.moddown(u, q, p, log_n)
    big_p = math.prod(p)
    big_q = math.prod(q)
    for c in range(n):
        uv = crt_py([int(u[i, c]) for i in range(len(q) + len(p))], q + p)
        ov = crt_py([int(out[i, c]) for i in range(len(q))], q)
        nearest = (2 * uv + big_p) // (2 * big_p)      # P odd: no ties
        vs = [v for v in range(len(p)) if (nearest - v - ov) % big_q == 0]
        assert len(vs) == 1


def test_rescale_rounds_to_nearest():
    """rescale(c) = round(c / q_l) for the centred integer c mod Q_l."""
    prm = S.params("mix15")
    log_n, n = 4, 16
    level = 3
    q = prm["q"][: level + 1]
    c = S.uniform_residues(q, n, seed=14)[0]
    out = O.rescale_poly(c, prm["q"], level, log_n)
    big_q = math.prod(q)
    ql = q[level]
    for k in range(n):
        cv = crt_py([int(c[i, k]) for i in range(level + 1)], q)
        if cv > big_q // 2:
            cv -= big_q
        # nearest integer to cv / ql (ql odd: no ties)
        r = (2 * cv + ql) // (2 * ql)
        ov = crt_py([int(out[i, k]) for i in range(level)], q[:level])
        assert (ov - r) % math.prod(q[:level]) == 0


# ---------------------------------------------------------------------------
# sampler
# ---------------------------------------------------------------------------

def test_shake256_known_answer():
    """FIPS 202 SHAKE256 of the empty message (first 32 bytes)."""
    import hashlib
    assert hashlib.shake_256(b"").hexdigest(32) == \
        "46b9dd2b0ba88d13233b3feb743eeb243fcd52ea62b81b82b50c27646ed5762f"


def test_samplers_distribution():
    n = 1 << 16
    t = O.sample_ternary("sk", 1, n)
    assert set(np.unique(t)) <= {-1, 0, 1}
    counts = [np.sum(t == v) for v in (-1, 0, 1)]
    assert all(abs(c - n / 3) < 5 * math.sqrt(n * 2 / 9) for c in counts)
    e = O.sample_gaussian("pk_e", 1, n)
    assert np.abs(e).max() <= 19
    assert abs(e.mean()) < 5 * 3.2 / math.sqrt(n)
    assert abs(e.std() - 3.2) < 0.05
    q = S.params("vital")["q"][3]
    u = O.sample_uniform("pk_a", 1, [q], n)[0]
    assert int(u.max()) < q
    assert abs(float(u.mean()) / q - 0.5) < 0.01


def test_gaussian_cdt_against_float_probabilities():
    cdt = O.gaussian_cdt()
    rho = [math.exp(-k * k / (2 * 3.2 ** 2)) for k in range(20)]
    mass = [rho[0]] + [2 * r for r in rho[1:]]
    tot = sum(mass)
    acc = 0.0
    for k in range(19):
        acc += mass[k]
        assert abs(cdt[k] / 2 ** 63 - acc / tot) < 1e-12
    assert cdt == sorted(cdt) and cdt[-1] == 1 << 63


def test_sampler_streams_are_prefix_stable():
    q = S.params("tiny")["q"][0]
    a = O.sample_uniform("x", 7, [q, q], 1000)
    b = O.sample_uniform("x", 7, [q, q], 3000)
    assert np.array_equal(a, b[:, :1000])
    assert not np.array_equal(a[0], a[1])   # streams differ by limb index


# ---------------------------------------------------------------------------
# encoding
# ---------------------------------------------------------------------------

def test_encode_matches_canonical_embedding_definition():
    """m(zeta^(5^j)) = z_j by direct O(N^2) evaluation, zeta = exp(i pi / N)."""
    n = 64
    z = S.uniform_slots(n // 2, 1, complex_=True)
    m = O.encode_real(z, n, 1.0)
    zeta = np.exp(1j * np.pi / n)
    for j in range(n // 2):
        root = zeta ** pow(5, j, 2 * n)
        val = sum(m[i] * root ** i for i in range(n))
        assert abs(val - z[j]) < 1e-12
    # real coefficients, and decode inverts encode
    assert np.allclose(O.decode_ints(O.encode_int(z, n, 2.0 ** 40), n, 2.0 ** 40), z, atol=1e-10)


def test_crt_centered_roundtrip():
    prm = S.params("mix15")
    mods = prm["q"][:5]
    vals = [0, 1, -1, 2 ** 200, -(2 ** 250) + 17, 123456789]
    res = O.ints_to_residues(vals, mods)
    assert O.crt_centered(res, mods) == vals


# ---------------------------------------------------------------------------
# sizes of the paper's Table 6
# ---------------------------------------------------------------------------

def test_sizes_match_table6():
    """Table 6 sizes from the oracle's own objects.

    A ciphertext is [2][L][N] words and a switching key [dnum][2][L+K][N]
    words (dnum = 3, K = ceil(L/3)).  The oracle builds both on a 2^5 ring
    with the paper's limb counts; scaled to N = 2^15 (the sizes are linear in
    N) they must reproduce the printed MB/GB figures."""
    g = json.load(open(os.path.join(GOLDEN, "table6_sizes.json")))
    n_paper = 1 << g["ring_log_n"]
    base = S.params("gesture")          # primes = 1 mod 2^17, hence mod 2^6
    for name in ("vital", "gesture"):
        row = g[name]
        L = row["limbs"]
        K = -(-L // 3)
        prm = dict(log_n=5, n=32, q=base["q"][:L], p=base["p"][:K], dnum=3, scale=2.0 ** 30)
        o = O.Oracle(prm)
        s = o.keygen_secret(1)
        ct = o.encrypt_sk(s, o.encode(np.zeros(16), 2.0 ** 30, L - 1), 2)
        pk = o.keygen_public(s, 3)
        rlk = o.keygen_relin(s, 4)
        f = n_paper / 32
        assert ct.polys.nbytes * f / 2 ** 20 == pytest.approx(row["ct_MB"], abs=0.05)
        assert pk.nbytes * f / 2 ** 20 == pytest.approx(row["pk_MB"], abs=0.05)
        assert rlk.nbytes * f / 2 ** 20 == pytest.approx(row["relin_MB"], abs=0.05)
        for gk in row["galois"]:
            gkey = o.keygen_galois(s, 5, 6)
            assert gk["keys"] * gkey.nbytes * f / 2 ** 30 == pytest.approx(gk["GB"], abs=0.05)
