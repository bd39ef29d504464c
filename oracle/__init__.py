"""CPU oracle for RNS-CKKS evaluation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_2603_22437_amd``) and never imports it; the
only module both sides use is ``seeded_inputs`` (parameters and seeded random
data, no scheme arithmetic).

What it computes.  The paper builds every encrypted kernel from the CKKS
operations listed in its primer (section 3.2): KeyGen producing sk, pk, a
relinearization key and one Galois key per rotation amount; encoding of up to
N/2 slots; slot-wise addition; slot-wise multiplication that consumes one
level; and the cyclic slot rotation Rot(Enc(a), k).  Its DFT, FIR and FC
kernels apply plaintext matrices to ciphertexts with the Halevi-Shoup diagonal
method under baby-step/giant-step scheduling (section 3.3, Kernel 3, Eq.
dft_re; Appendix D.1).  The paper leaves the scheme's internals to its backend
libraries, so this oracle writes them out from the textbook definitions of
RNS-CKKS with hybrid key switching; every reading taken where the paper is
silent is listed in the design document (readings A1-A23):

* ring Z_Q[X]/(X^N+1) in RNS form, residues per prime, coefficient domain;
* canonical-embedding encoding with slot j at the root zeta^(5^j mod 2N),
  zeta = exp(i pi / N), coefficients rounded half away from zero (A11);
* secret ternary, errors discrete Gaussian sigma = 3.2 cut at 19 (A7, A8),
  all randomness from SHAKE-256 streams (A9);
* hybrid key switching with dnum contiguous digits, fast basis conversion
  without correction and ModDown with rounding (A6, A14, A15);
* Rot(ct, k) = automorphism X -> X^(5^k) then key switching (A12, A13);
* rescale by the last prime with a centred lift (A16); exact scale tracking
  (A17); BSGS with generalized diagonals and pre-rotated plaintexts (A18).

The C core (``ockks.c``) does the ring arithmetic; this module draws the
randomness, encodes and decodes, and composes the operations.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OCKKS_LIB names another build of ockks.c (the sanitizer test loads one built
# with AddressSanitizer and UndefinedBehaviorSanitizer)
_LIB_PATH = os.environ.get("OCKKS_LIB") or os.path.join(_HERE, "libockks.so")
_lib = None

u64p = ctypes.POINTER(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # test infrastructure: build the oracle's C on demand
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    U, I = ctypes.c_uint64, ctypes.c_uint32
    P = ctypes.c_void_p
    sig = {
        "ock_mulmod": ([U, U, U], U), "ock_powmod": ([U, U, U], U),
        "ock_invmod": ([U, U], U), "ock_root_2n": ([U, U], U),
        "ock_ntt": ([P, I, U], None), "ock_intt": ([P, I, U], None),
        "ock_poly_mul": ([P, P, P, I, P, I], None),
        "ock_poly_mul_schoolbook": ([P, P, P, I, U], None),
        "ock_add": ([P, P, P, I, P, I], None), "ock_sub": ([P, P, P, I, P, I], None),
        "ock_embed_small": ([P, P, I, P, I], None),
        "ock_automorphism": ([P, P, I, P, I, U], None),
        "ock_bconv": ([P, P, I, P, P, I, I], None),
        "ock_moddown": ([P, P, P, I, P, I, I], None),
        "ock_keyswitch": ([P, I, P, P, I, P, I, I, I, P, P], None),
        "ock_modup": ([P, I, P, I, P, I, I, I, P], I),
        "ock_keyswitch_ext": ([P, I, I, P, P, I, P, I, I, P, P], None),
        "ock_ks_inner": ([P, I, I, P, P, I, P, I, I, P, P], None),
        "ock_rescale": ([P, P, P, I, I], None),
        "ock_num_threads": ([], ctypes.c_int),
        "ock_set_num_threads": ([ctypes.c_int], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _u64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


def num_threads() -> int:
    return _load().ock_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's limb loops from now on."""
    _load().ock_set_num_threads(n)


# ---------------------------------------------------------------------------
# C core wrappers (residue arrays, coefficient form, [limb][N])
# ---------------------------------------------------------------------------

def mulmod(a: int, b: int, q: int) -> int:
    return _load().ock_mulmod(a, b, q)


def root_2n(q: int, n: int) -> int:
    return _load().ock_root_2n(q, n)


def ntt(a: np.ndarray, log_n: int, q: int) -> np.ndarray:
    """out[k] = a(psi^(2k+1)), psi = ``root_2n(q, N)``."""
    out = _u64(a).copy()
    _load().ock_ntt(_ptr(out), log_n, q)
    return out


def intt(a: np.ndarray, log_n: int, q: int) -> np.ndarray:
    out = _u64(a).copy()
    _load().ock_intt(_ptr(out), log_n, q)
    return out


def poly_mul(a, b, log_n: int, mods) -> np.ndarray:
    a, b = _u64(a), _u64(b)
    mods = _u64(mods)
    out = np.empty_like(a)
    _load().ock_poly_mul(_ptr(a), _ptr(b), _ptr(out), log_n, _ptr(mods), len(mods))
    return out


def poly_mul_schoolbook(a, b, log_n: int, q: int) -> np.ndarray:
    a, b = _u64(a), _u64(b)
    out = np.empty_like(a)
    _load().ock_poly_mul_schoolbook(_ptr(a), _ptr(b), _ptr(out), log_n, q)
    return out


def poly_add(a, b, log_n: int, mods) -> np.ndarray:
    a, b, mods = _u64(a), _u64(b), _u64(mods)
    out = np.empty_like(a)
    _load().ock_add(_ptr(a), _ptr(b), _ptr(out), log_n, _ptr(mods), len(mods))
    return out


def poly_sub(a, b, log_n: int, mods) -> np.ndarray:
    a, b, mods = _u64(a), _u64(b), _u64(mods)
    out = np.empty_like(a)
    _load().ock_sub(_ptr(a), _ptr(b), _ptr(out), log_n, _ptr(mods), len(mods))
    return out


def embed_small(v, log_n: int, mods) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(v, dtype=np.int64))
    mods = _u64(mods)
    out = np.empty((len(mods), 1 << log_n), dtype=np.uint64)
    _load().ock_embed_small(_ptr(v), _ptr(out), log_n, _ptr(mods), len(mods))
    return out


def automorphism(a, g: int, log_n: int, mods) -> np.ndarray:
    a, mods = _u64(a), _u64(mods)
    out = np.empty_like(a)
    _load().ock_automorphism(_ptr(a), _ptr(out), log_n, _ptr(mods), len(mods), g)
    return out


def bconv(x, src, dst, log_n: int) -> np.ndarray:
    x, src, dst = _u64(x), _u64(src), _u64(dst)
    out = np.empty((len(dst), 1 << log_n), dtype=np.uint64)
    _load().ock_bconv(_ptr(x), _ptr(src), len(src), _ptr(out), _ptr(dst), len(dst), log_n)
    return out


def moddown(u, q, p, log_n: int) -> np.ndarray:
    u, q, p = _u64(u), _u64(q), _u64(p)
    out = np.empty((len(q), 1 << log_n), dtype=np.uint64)
    _load().ock_moddown(_ptr(u), _ptr(out), _ptr(q), len(q), _ptr(p), len(p), log_n)
    return out


def rescale_poly(c, q_chain, level: int, log_n: int) -> np.ndarray:
    c, qc = _u64(c), _u64(q_chain)
    out = np.empty((level, 1 << log_n), dtype=np.uint64)
    _load().ock_rescale(_ptr(c), _ptr(out), _ptr(qc), level, log_n)
    return out


# ---------------------------------------------------------------------------
# Randomness: SHAKE-256 streams (reading A9)
# ---------------------------------------------------------------------------

SIGMA = 3.2
GAUSS_TAIL = 19  # floor(6 sigma)


def shake_stream(tag: str, seed: int, index: int, nbytes: int) -> bytes:
    """SHAKE-256("hipckks/" || tag || "/" || le64(seed) || le32(index)), nbytes long."""
    msg = b"hipckks/" + tag.encode() + b"/" + int(seed).to_bytes(8, "little") \
        + int(index).to_bytes(4, "little")
    return hashlib.shake_256(msg).digest(nbytes)


def sample_uniform(tag: str, seed: int, mods, n: int) -> np.ndarray:
    """Row t uniform in [0, mods[t]): 64-bit little-endian words of stream t,
    masked to bitlen(q), kept when below q, first n kept."""
    out = np.empty((len(mods), n), dtype=np.uint64)
    for t, q in enumerate(mods):
        q = int(q)
        mask = np.uint64((1 << q.bit_length()) - 1)
        nbytes = 8 * (2 * n + 64)
        while True:
            w = np.frombuffer(shake_stream(tag, seed, t, nbytes), dtype="<u8") & mask
            keep = w[w < np.uint64(q)]
            if len(keep) >= n:
                out[t] = keep[:n]
                break
            nbytes *= 2
    return out


def sample_ternary(tag: str, seed: int, n: int) -> np.ndarray:
    """Bytes of stream 0, value 255 rejected, b mod 3 -> (0, +1, -1)."""
    nbytes = 2 * n + 64
    while True:
        b = np.frombuffer(shake_stream(tag, seed, 0, nbytes), dtype=np.uint8)
        b = b[b != 255][:n]
        if len(b) == n:
            break
        nbytes *= 2
    v = (b % 3).astype(np.int64)
    v[v == 2] = -1
    return v


def gaussian_cdt() -> list[int]:
    """Thresholds T[k] = floor(2^63 * Pr(|e| <= k)) of the discrete Gaussian
    rho(x) = exp(-x^2 / (2 sigma^2)) on [-19, 19] (reading A8), computed with
    50-digit arithmetic; T[19] = 2^63."""
    import mpmath
    mpmath.mp.dps = 50
    s2 = 2 * mpmath.mpf(SIGMA) ** 2
    rho = [mpmath.e ** (-(mpmath.mpf(k) ** 2) / s2) for k in range(GAUSS_TAIL + 1)]
    mass = [rho[0]] + [2 * r for r in rho[1:]]
    total = sum(mass)
    out, acc = [], mpmath.mpf(0)
    for k in range(GAUSS_TAIL):
        acc += mass[k]
        out.append(int(mpmath.floor(acc / total * mpmath.mpf(2) ** 63)))
    out.append(1 << 63)
    return out


_CDT = None


def sample_gaussian(tag: str, seed: int, n: int) -> np.ndarray:
    """64-bit words of stream 0: u = w >> 1 picks the magnitude (first k with
    u < T[k]); bit 0 is the sign (ignored for magnitude 0)."""
    global _CDT
    if _CDT is None:
        _CDT = np.array(gaussian_cdt(), dtype=np.uint64)
    w = np.frombuffer(shake_stream(tag, seed, 0, 8 * n), dtype="<u8")
    u = w >> np.uint64(1)
    mag = np.searchsorted(_CDT, u, side="right").astype(np.int64)
    neg = (w & np.uint64(1)).astype(bool) & (mag != 0)
    return np.where(neg, -mag, mag)


# ---------------------------------------------------------------------------
# Encoding (canonical embedding) and CRT
# ---------------------------------------------------------------------------

def slot_roots(n_ring: int) -> np.ndarray:
    """Index k (root zeta^(2k+1)) of slot j: (5^j mod 2N - 1) / 2."""
    two_n = 2 * n_ring
    e = np.empty(n_ring // 2, dtype=np.int64)
    acc = 1
    for j in range(n_ring // 2):
        e[j] = acc
        acc = acc * 5 % two_n
    return (e - 1) // 2


def _round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def encode_real(z, n_ring: int, scale: float) -> np.ndarray:
    """Real coefficients m with m(zeta^(5^j)) = z_j, zeta = exp(i pi/N), before
    scaling (fp64).  Evaluations at all odd powers E[k] = m(zeta^(2k+1)) are
    E = N * ifft(m_i zeta^i); slot j fills E at (5^j - 1)/2 and its conjugate
    at (2N - 5^j - 1)/2, then m_i = zeta^-i fft(E)_i / N."""
    n_slots = n_ring // 2
    z = np.asarray(z, dtype=np.complex128)
    assert z.shape == (n_slots,)
    k = slot_roots(n_ring)
    e = np.zeros(n_ring, dtype=np.complex128)
    e[k] = z
    e[n_ring - 1 - k] = np.conj(z)
    i = np.arange(n_ring)
    zeta_pow = np.exp(1j * np.pi * i / n_ring)
    m = np.fft.fft(e) / n_ring / zeta_pow
    return m.real * scale


def encode_int(z, n_ring: int, scale: float) -> list[int]:
    """Integer plaintext coefficients round(scale * m_i) (half away from zero)."""
    return [int(v) for v in _round_half_away(encode_real(z, n_ring, scale))]


def ints_to_residues(coeffs, mods) -> np.ndarray:
    c = np.array([int(v) for v in coeffs], dtype=object)
    out = np.empty((len(mods), len(c)), dtype=np.uint64)
    for t, q in enumerate(mods):
        out[t] = np.array([int(v) % int(q) for v in c], dtype=np.uint64)
    return out


def crt_centered(res: np.ndarray, mods) -> list[int]:
    """Centred integers x in (-Q/2, Q/2] with x = res[t] mod mods[t] (Garner-free
    textbook CRT with Python integers)."""
    mods = [int(q) for q in mods]
    big_q = math.prod(mods)
    acc = np.zeros(res.shape[1], dtype=object)
    for t, q in enumerate(mods):
        hat = big_q // q
        inv = pow(hat % q, -1, q)
        y = (res[t].astype(object) * inv) % q
        acc = acc + y * hat
    acc = acc % big_q
    half = big_q // 2
    return [int(v) - big_q if v > half else int(v) for v in acc]


def decode_ints(coeffs, n_ring: int, scale: float) -> np.ndarray:
    """Slots z_j = m(zeta^(5^j)) / scale from integer coefficients."""
    m = np.array([float(c) for c in coeffs], dtype=np.float64) / scale
    i = np.arange(n_ring)
    zeta_pow = np.exp(1j * np.pi * i / n_ring)
    e = n_ring * np.fft.ifft(m * zeta_pow)
    return e[slot_roots(n_ring)]


# ---------------------------------------------------------------------------
# The scheme
# ---------------------------------------------------------------------------

@dataclass
class Ciphertext:
    polys: np.ndarray          # uint64 [k][level+1][N], coefficient form
    level: int
    scale: float


@dataclass
class Plaintext:
    res: np.ndarray            # uint64 [level+1][N], coefficient form
    level: int
    scale: float


@dataclass
class LinearTransform:
    """Pre-rotated, encoded diagonals grouped for BSGS (reading A18)."""
    n1: int
    level: int
    scale: float
    groups: dict = field(default_factory=dict)   # g -> list of (b, Plaintext)


class Oracle:
    """RNS-CKKS over the parameter set ``prm`` (see ``seeded_inputs.params``)."""

    def __init__(self, prm: dict):
        self.prm = prm
        self.log_n = prm["log_n"]
        self.n = 1 << self.log_n
        self.q = [int(x) for x in prm["q"]]
        self.p = [int(x) for x in prm["p"]]
        self.L = len(self.q)
        self.K = len(self.p)
        self.dnum = prm["dnum"]
        self.alpha = -(-self.L // self.dnum)
        self.n_slots = self.n // 2
        for m in self.q + self.p:
            if m % (2 * self.n) != 1 or m >= 1 << 61:
                raise ValueError(f"modulus {m} is not an NTT prime below 2^61")

    # --- moduli -----------------------------------------------------------
    def qmods(self, level: int) -> list[int]:
        return self.q[: level + 1]

    def full_mods(self) -> list[int]:
        return self.q + self.p

    # --- keys -------------------------------------------------------------
    def keygen_secret(self, seed: int) -> np.ndarray:
        return sample_ternary("sk", seed, self.n)

    def keygen_public(self, s: np.ndarray, seed: int) -> np.ndarray:
        mods = self.q
        a = sample_uniform("pk_a", seed, mods, self.n)
        e = embed_small(sample_gaussian("pk_e", seed, self.n), self.log_n, mods)
        s_r = embed_small(s, self.log_n, mods)
        b = poly_add(poly_sub(np.zeros_like(a), poly_mul(a, s_r, self.log_n, mods),
                              self.log_n, mods), e, self.log_n, mods)
        return np.stack([b, a])

    def switch_key(self, s: np.ndarray, s_prime: np.ndarray, tag: str, seed: int) -> np.ndarray:
        """swk_j = (-a_j s + e_j + [limb in D_j] (P mod q_i) s', a_j) on all
        L+K limbs; ``s_prime`` is given as residues [L+K][N]."""
        mods = self.full_mods()
        s_r = embed_small(s, self.log_n, mods)
        big_p = math.prod(self.p)
        out = np.empty((self.dnum, 2, self.L + self.K, self.n), dtype=np.uint64)
        for j in range(self.dnum):
            a = sample_uniform(f"{tag}/a/{j}", seed, mods, self.n)
            e = embed_small(sample_gaussian(f"{tag}/e/{j}", seed, self.n), self.log_n, mods)
            b = poly_add(poly_sub(np.zeros_like(a), poly_mul(a, s_r, self.log_n, mods),
                                  self.log_n, mods), e, self.log_n, mods)
            for i in range(j * self.alpha, min((j + 1) * self.alpha, self.L)):
                qi = self.q[i]
                pm = big_p % qi
                term = (s_prime[i].astype(object) * pm) % qi
                b[i] = ((b[i].astype(object) + term) % qi).astype(np.uint64)
            out[j, 0] = b
            out[j, 1] = a
        return out

    def keygen_relin(self, s: np.ndarray, seed: int) -> np.ndarray:
        mods = self.full_mods()
        s_r = embed_small(s, self.log_n, mods)
        s2 = poly_mul(s_r, s_r, self.log_n, mods)
        return self.switch_key(s, s2, "rlk", seed)

    def galois_element(self, step: int) -> int:
        return pow(5, step % self.n_slots, 2 * self.n)

    def keygen_galois(self, s: np.ndarray, g: int, seed: int) -> np.ndarray:
        mods = self.full_mods()
        s_g = automorphism(embed_small(s, self.log_n, mods), g, self.log_n, mods)
        return self.switch_key(s, s_g, f"gk/{g}", seed)

    # --- plaintexts ----------------------------------------------------------
    def encode(self, z, scale: float, level: int) -> Plaintext:
        coeffs = encode_int(z, self.n, scale)
        return Plaintext(ints_to_residues(coeffs, self.qmods(level)), level, scale)

    def plaintext_from_ints(self, coeffs, level: int, scale: float) -> Plaintext:
        return Plaintext(ints_to_residues(coeffs, self.qmods(level)), level, scale)

    def decode(self, pt: Plaintext) -> np.ndarray:
        return decode_ints(crt_centered(pt.res, self.qmods(pt.level)), self.n, pt.scale)

    # --- encryption ------------------------------------------------------------
    def encrypt_sk(self, s: np.ndarray, pt: Plaintext, seed: int) -> Ciphertext:
        mods = self.qmods(pt.level)
        a = sample_uniform("enc_a", seed, mods, self.n)
        e = embed_small(sample_gaussian("enc_e", seed, self.n), self.log_n, mods)
        s_r = embed_small(s, self.log_n, mods)
        c0 = poly_sub(poly_add(e, pt.res, self.log_n, mods),
                      poly_mul(a, s_r, self.log_n, mods), self.log_n, mods)
        return Ciphertext(np.stack([c0, a]), pt.level, pt.scale)

    def encrypt_pk(self, pk: np.ndarray, pt: Plaintext, seed: int) -> Ciphertext:
        mods = self.qmods(pt.level)
        nl = pt.level + 1
        v = embed_small(sample_ternary("enc_v", seed, self.n), self.log_n, mods)
        e0 = embed_small(sample_gaussian("enc_e0", seed, self.n), self.log_n, mods)
        e1 = embed_small(sample_gaussian("enc_e1", seed, self.n), self.log_n, mods)
        c0 = poly_add(poly_add(poly_mul(v, pk[0, :nl], self.log_n, mods), e0, self.log_n, mods),
                      pt.res, self.log_n, mods)
        c1 = poly_add(poly_mul(v, pk[1, :nl], self.log_n, mods), e1, self.log_n, mods)
        return Ciphertext(np.stack([c0, c1]), pt.level, pt.scale)

    def decrypt(self, s: np.ndarray, ct: Ciphertext) -> Plaintext:
        """m = c0 + c1 s (+ c2 s^2 for a three-part ciphertext)."""
        mods = self.qmods(ct.level)
        s_r = embed_small(s, self.log_n, mods)
        m = ct.polys[0].copy()
        s_pow = s_r
        for k in range(1, ct.polys.shape[0]):
            m = poly_add(m, poly_mul(ct.polys[k], s_pow, self.log_n, mods), self.log_n, mods)
            s_pow = poly_mul(s_pow, s_r, self.log_n, mods)
        return Plaintext(m, ct.level, ct.scale)

    # --- evaluation --------------------------------------------------------------
    def _check_pair(self, a: Ciphertext, b: Ciphertext):
        if a.level != b.level:
            raise ValueError("level mismatch")
        if abs(a.scale - b.scale) > 2.0 ** -30 * max(a.scale, b.scale):
            raise ValueError("scale mismatch")

    def add(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        self._check_pair(a, b)
        mods = self.qmods(a.level)
        return Ciphertext(np.stack([poly_add(x, y, self.log_n, mods)
                                    for x, y in zip(a.polys, b.polys)]), a.level, a.scale)

    def sub(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        self._check_pair(a, b)
        mods = self.qmods(a.level)
        return Ciphertext(np.stack([poly_sub(x, y, self.log_n, mods)
                                    for x, y in zip(a.polys, b.polys)]), a.level, a.scale)

    def add_plain(self, a: Ciphertext, pt: Plaintext) -> Ciphertext:
        if a.level != pt.level:
            raise ValueError("level mismatch")
        mods = self.qmods(a.level)
        polys = a.polys.copy()
        polys[0] = poly_add(polys[0], pt.res, self.log_n, mods)
        return Ciphertext(polys, a.level, a.scale)

    def mul_plain(self, a: Ciphertext, pt: Plaintext) -> Ciphertext:
        if a.level != pt.level:
            raise ValueError("level mismatch")
        mods = self.qmods(a.level)
        return Ciphertext(np.stack([poly_mul(x, pt.res, self.log_n, mods) for x in a.polys]),
                          a.level, a.scale * pt.scale)

    def drop_level(self, a: Ciphertext, level: int) -> Ciphertext:
        if level > a.level:
            raise ValueError("cannot raise the level")
        return Ciphertext(a.polys[:, : level + 1].copy(), level, a.scale)

    def tensor(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        """(a0 b0, a0 b1 + a1 b0, a1 b1)."""
        if a.level != b.level:
            raise ValueError("level mismatch")
        mods = self.qmods(a.level)
        m = lambda x, y: poly_mul(x, y, self.log_n, mods)
        d0 = m(a.polys[0], b.polys[0])
        d1 = poly_add(m(a.polys[0], b.polys[1]), m(a.polys[1], b.polys[0]), self.log_n, mods)
        d2 = m(a.polys[1], b.polys[1])
        return Ciphertext(np.stack([d0, d1, d2]), a.level, a.scale * b.scale)

    def keyswitch(self, d: np.ndarray, level: int, swk: np.ndarray):
        out0 = np.empty((level + 1, self.n), dtype=np.uint64)
        out1 = np.empty_like(out0)
        d = _u64(d)
        swk = _u64(swk)
        q, p = _u64(self.q), _u64(self.p)
        _load().ock_keyswitch(_ptr(d), level, _ptr(swk), _ptr(q), self.L, _ptr(p), self.K,
                              self.dnum, self.log_n, _ptr(out0), _ptr(out1))
        return out0, out1

    def modup(self, d: np.ndarray, level: int) -> np.ndarray:
        """Extended digits [digits][level+1+K][N] of d (coefficient form)."""
        ne = level + 1 + self.K
        ext = np.empty((self.dnum, ne, self.n), dtype=np.uint64)
        q, p = _u64(self.q), _u64(self.p)
        digits = _load().ock_modup(_ptr(_u64(d)), level, _ptr(q), self.L, _ptr(p), self.K,
                                   self.dnum, self.log_n, _ptr(ext))
        return np.ascontiguousarray(ext[:digits])

    def keyswitch_ext(self, ext: np.ndarray, level: int, swk: np.ndarray):
        out0 = np.empty((level + 1, self.n), dtype=np.uint64)
        out1 = np.empty_like(out0)
        q, p = _u64(self.q), _u64(self.p)
        ext = _u64(ext)
        _load().ock_keyswitch_ext(_ptr(ext), ext.shape[0], level, _ptr(_u64(swk)), _ptr(q),
                                  self.L, _ptr(p), self.K, self.log_n, _ptr(out0), _ptr(out1))
        return out0, out1

    def ks_inner(self, ext: np.ndarray, level: int, swk: np.ndarray):
        """Key inner product of extended digits in Q_level u P, without
        ModDown: (acc0, acc1), each [level+1+K][N] (q limbs, then P limbs)."""
        ne = level + 1 + self.K
        acc0 = np.empty((ne, self.n), dtype=np.uint64)
        acc1 = np.empty_like(acc0)
        q, p = _u64(self.q), _u64(self.p)
        ext = _u64(ext)
        _load().ock_ks_inner(_ptr(ext), ext.shape[0], level, _ptr(_u64(swk)), _ptr(q), self.L,
                             _ptr(p), self.K, self.log_n, _ptr(acc0), _ptr(acc1))
        return acc0, acc1

    def moddown(self, acc: np.ndarray, level: int) -> np.ndarray:
        """ModDown (with rounding, A15) of a [level+1+K][N] polynomial to Q_level."""
        return moddown(acc, self.qmods(level), self.p, self.log_n)

    def rotate_hoisted(self, c: Ciphertext, steps: list, gks: dict) -> list:
        """Rotations of one ciphertext by several steps sharing one ModUp
        (reading A13): the extended digits of c1 are computed once; for each
        step the automorphism X -> X^g is applied to every extended limb
        before the key inner product and ModDown, and phi_g(c0) is added.
        Valid key switches, with residues that differ from rotate()."""
        ext = self.modup(c.polys[1], c.level)
        ne_mods = self.qmods(c.level) + self.p
        mods = self.qmods(c.level)
        out = []
        for k in steps:
            if k % self.n_slots == 0:
                out.append(Ciphertext(c.polys.copy(), c.level, c.scale))
                continue
            g = self.galois_element(k)
            if g not in gks:
                raise KeyError(f"no Galois key for element {g}")
            ext_g = np.stack([automorphism(e, g, self.log_n, ne_mods) for e in ext])
            u0, u1 = self.keyswitch_ext(ext_g, c.level, gks[g])
            c0 = automorphism(c.polys[0], g, self.log_n, mods)
            out.append(Ciphertext(np.stack([poly_add(c0, u0, self.log_n, mods), u1]),
                                  c.level, c.scale))
        return out

    def relinearize(self, c: Ciphertext, rlk: np.ndarray) -> Ciphertext:
        mods = self.qmods(c.level)
        u0, u1 = self.keyswitch(c.polys[2], c.level, rlk)
        return Ciphertext(np.stack([poly_add(c.polys[0], u0, self.log_n, mods),
                                    poly_add(c.polys[1], u1, self.log_n, mods)]),
                          c.level, c.scale)

    def apply_galois(self, c: Ciphertext, g: int, gk: np.ndarray) -> Ciphertext:
        """(phi_g(c0), 0) + KS(phi_g(c1), gk_g): automorphism first (A13)."""
        mods = self.qmods(c.level)
        c0 = automorphism(c.polys[0], g, self.log_n, mods)
        c1 = automorphism(c.polys[1], g, self.log_n, mods)
        u0, u1 = self.keyswitch(c1, c.level, gk)
        return Ciphertext(np.stack([poly_add(c0, u0, self.log_n, mods), u1]), c.level, c.scale)

    def rotate(self, c: Ciphertext, step: int, gks: dict) -> Ciphertext:
        """Left rotation of the slots by ``step`` (A12); ``gks`` maps Galois
        element -> switching key."""
        if step % self.n_slots == 0:
            return Ciphertext(c.polys.copy(), c.level, c.scale)
        g = self.galois_element(step)
        if g not in gks:
            raise KeyError(f"no Galois key for element {g}")
        return self.apply_galois(c, g, gks[g])

    def rescale(self, c: Ciphertext) -> Ciphertext:
        if c.level == 0:
            raise ValueError("no level left to rescale")
        polys = np.stack([rescale_poly(x, self.q, c.level, self.log_n) for x in c.polys])
        return Ciphertext(polys, c.level - 1, c.scale / self.q[c.level])

    # --- constants and polynomials (reading A28) --------------------------------
    def encode_const(self, value: float, scale: float, level: int) -> Plaintext:
        """The constant slot vector `value` at `scale`: its only nonzero
        coefficient is m_0 = round(value * scale), half away from zero (a
        constant has that single coefficient in the inverse canonical
        embedding)."""
        c = [0] * self.n
        c[0] = int(_round_half_away(np.array([value * scale]))[0])
        return self.plaintext_from_ints(c, level, scale)

    def poly_eval(self, x: Ciphertext, coeffs, rlk) -> Ciphertext:
        """sum_k coeffs[k] x^k, slot-wise (reading A28).

        Powers: x^(2^j) by repeated squaring; any other x^k as x^a x^(k-a) with
        a the largest power of two below k, the factor on the higher level
        dropped to the other's level; every product relinearized and rescaled,
        so x^k sits at level l - ceil(log2 k).  Terms: each x^k with a nonzero
        coefficient, dropped to level l_f + 1 (l_f = l - ceil(log2 d) - 1),
        times the constant coeffs[k] encoded at scale s q_(l_f+1) / scale(x^k)
        (s: the input's scale), rescaled to level l_f; the terms are added in
        increasing k, then coeffs[0] at the sum's scale."""
        d = len(coeffs) - 1
        if d < 1 or not any(coeffs[1:]):
            raise ValueError("need a nonzero coefficient of degree >= 1")
        depth = (d - 1).bit_length() + 1
        if x.level < depth:
            raise ValueError("not enough levels for this degree")
        pw = {1: x}
        for k in range(2, d + 1):
            a = 1 << ((k - 1).bit_length() - 1)     # largest power of two below k
            u, v = pw[a], pw[k - a]
            lv = min(u.level, v.level)
            u, v = self.drop_level(u, lv), self.drop_level(v, lv)
            pw[k] = self.rescale(self.relinearize(self.tensor(u, v), rlk))
        lf = x.level - depth
        acc = None
        for k in range(1, d + 1):
            if coeffs[k] == 0:
                continue
            t = self.drop_level(pw[k], lf + 1)
            pt = self.encode_const(coeffs[k], x.scale * self.q[lf + 1] / t.scale, lf + 1)
            term = self.rescale(self.mul_plain(t, pt))
            acc = term if acc is None else self.add(acc, term)
        if coeffs[0] != 0:
            acc = self.add_plain(acc, self.encode_const(coeffs[0], acc.scale, lf))
        return acc

    # --- baby-step/giant-step linear transform (reading A18) ---------------------
    @staticmethod
    def bsgs_split(offset: int, n1: int):
        g = offset // n1
        return g, offset - g * n1

    def lt_create(self, diags: dict, n1: int, level: int, scale: float | None = None
                  ) -> LinearTransform:
        """``diags``: offset k -> generalized diagonal diag_k[j] = A[j][(j+k) mod n].
        Diagonal k = g n1 + b is stored pre-rotated by -g n1 and encoded at
        ``scale`` (default q_level)."""
        scale = float(self.q[level]) if scale is None else scale
        lt = LinearTransform(n1, level, scale)
        for k, vec in sorted(diags.items()):
            g, b = self.bsgs_split(k, n1)
            shifted = np.roll(np.asarray(vec), g * n1)   # v'[j] = v[(j - g n1) mod n]
            lt.groups.setdefault(g, []).append((b, self.encode(shifted, scale, level)))
        return lt

    def lt_from_plaintexts(self, pts: dict, n1: int, level: int, scale: float) -> LinearTransform:
        """Same transform from already encoded, pre-rotated diagonals (offset -> Plaintext)."""
        lt = LinearTransform(n1, level, scale)
        for k, pt in sorted(pts.items()):
            g, b = self.bsgs_split(k, n1)
            lt.groups.setdefault(g, []).append((b, pt))
        return lt

    def lt_required_steps(self, lt: LinearTransform) -> list[int]:
        steps = set()
        for g, items in lt.groups.items():
            if g != 0:
                steps.add(g * lt.n1)
            for b, _ in items:
                if b != 0:
                    steps.add(b)
        return sorted(steps)

    def lt_eval(self, inputs: list, terms: list, gks: dict, n_out: int,
                hoist: bool = False, hoist_giant: bool = False) -> list:
        """Sums of transforms over shared inputs (the complex DFT of Eq. dft_re
        is C v_re - S v_im and S v_re + C v_im): terms are (transform, input
        index, output index, sign).  For every output and giant index g the
        inner sum runs over the terms' baby-step products, and is rotated once
        by g n1: out_o = sum_g Rot(sum_t sign_t sum_b pt_{t,g,b} Rot(x_t, b), g n1).
        With hoist the baby rotations of an input are hoisted rotations.  With
        hoist_giant an output's giant rotations share one ModDown: their key
        inner products are summed in Q u P and reduced once (giant_sum)."""
        n1 = terms[0][0].n1
        need = {}
        for lt, i, _o, _s in terms:
            for items in lt.groups.values():
                for b, _ in items:
                    need.setdefault(i, set()).add(b)
        babies = {}
        for i, bs in need.items():
            bs = sorted(bs)
            if hoist:
                rotated = self.rotate_hoisted(inputs[i], [b for b in bs if b != 0], gks)
                it = iter(rotated)
                for b in bs:
                    babies[(i, b)] = inputs[i] if b == 0 else next(it)
            else:
                for b in bs:
                    babies[(i, b)] = inputs[i] if b == 0 else self.rotate(inputs[i], b, gks)
        giants = sorted({g for lt, _i, _o, _s in terms for g in lt.groups})
        parts = [[] for _ in range(n_out)]   # (g, inner sum) per output
        for g in giants:
            inner = [None] * n_out
            for lt, i, o, sign in terms:
                for b, pt in lt.groups.get(g, []):
                    term = self.mul_plain(babies[(i, b)], pt)
                    if inner[o] is None:
                        inner[o] = term if sign > 0 else self.sub(
                            Ciphertext(np.zeros_like(term.polys), term.level, term.scale), term)
                    else:
                        inner[o] = self.add(inner[o], term) if sign > 0 else self.sub(inner[o], term)
            for o in range(n_out):
                if inner[o] is not None:
                    parts[o].append((g * n1, inner[o]))
        out = []
        for o in range(n_out):
            if hoist_giant:
                out.append(self.giant_sum(parts[o], gks))
                continue
            acc = None
            for step, u in parts[o]:
                r = u if step == 0 else self.rotate(u, step, gks)
                acc = r if acc is None else self.add(acc, r)
            out.append(acc)
        return out

    def giant_sum(self, parts: list, gks: dict) -> Ciphertext:
        """sum_k Rot(u_k, step_k) with one ModDown for all the key switches
        (the giant-step half of double hoisting): for each rotated part the
        automorphism phi_g is applied to u_k, phi_g(c1) is extended (ModUp)
        and multiplied by gk_g in Q u P; the products of all parts are added
        in Q u P and ModDown runs once per polynomial; the phi_g(c0) (and the
        unrotated parts) are added in Q.  Valid rotations whose residues
        differ from a sum of rotate() results."""
        level, scale = parts[0][1].level, parts[0][1].scale
        mods = self.qmods(level)
        ne_mods = mods + self.p
        c0 = np.zeros((level + 1, self.n), dtype=np.uint64)
        c1 = np.zeros_like(c0)
        pq0 = pq1 = None
        for step, u in parts:
            if step % self.n_slots == 0:
                c0 = poly_add(c0, u.polys[0], self.log_n, mods)
                c1 = poly_add(c1, u.polys[1], self.log_n, mods)
                continue
            g = self.galois_element(step)
            if g not in gks:
                raise KeyError(f"no Galois key for element {g}")
            c0 = poly_add(c0, automorphism(u.polys[0], g, self.log_n, mods), self.log_n, mods)
            ext = self.modup(automorphism(u.polys[1], g, self.log_n, mods), level)
            a0, a1 = self.ks_inner(ext, level, gks[g])
            pq0 = a0 if pq0 is None else poly_add(pq0, a0, self.log_n, ne_mods)
            pq1 = a1 if pq1 is None else poly_add(pq1, a1, self.log_n, ne_mods)
        if pq0 is not None:
            c0 = poly_add(c0, self.moddown(pq0, level), self.log_n, mods)
            c1 = poly_add(c1, self.moddown(pq1, level), self.log_n, mods)
        return Ciphertext(np.stack([c0, c1]), level, scale)

    def lt_apply(self, lt: LinearTransform, c: Ciphertext, gks: dict) -> Ciphertext:
        """y = sum_g Rot(sum_b pt_{g,b} * Rot(c, b), g n1); no rescale."""
        if c.level != lt.level:
            raise ValueError("level mismatch")
        babies = {0: c}
        for items in lt.groups.values():
            for b, _ in items:
                if b not in babies:
                    babies[b] = self.rotate(c, b, gks)
        out = None
        for g in sorted(lt.groups):
            inner = None
            for b, pt in lt.groups[g]:
                term = self.mul_plain(babies[b], pt)
                inner = term if inner is None else self.add(inner, term)
            if g != 0:
                inner = self.rotate(inner, g * lt.n1, gks)
            out = inner if out is None else self.add(out, inner)
        return out
