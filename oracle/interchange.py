"""Interchange form of ciphertexts and switching keys, oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Written from the
format's definition, sharing no code with the library's reader and writer:
a 64-byte little-endian header

    magic "HCKCKKS1" | kind u32 (1 ciphertext, 2 switching key) | log_n u32 |
    L u32 | K u32 | dnum u32 | level u32 | polys u32 | rows u32 |
    scale f64 | prime hash u64 | words u64

then the residues as little-endian u64 words, coefficient domain, in the
export layout: ciphertexts [size][level+1][N], switching keys
[dnum][2][L+K][N] (keys carry level L-1 and scale 0).  The prime hash is the
64-bit FNV-1a hash of the q primes then the special primes, each as 8
little-endian bytes.  The paper's client sends its evaluation keys once, at
enrollment, and the cloud keeps them (section 5.4); windows travel as
ciphertexts.
"""
from __future__ import annotations

import struct

import numpy as np

from . import Ciphertext, Oracle

MAGIC = b"HCKCKKS1"
KIND_CIPHERTEXT, KIND_SWITCH_KEY = 1, 2
_HEAD = struct.Struct("<8s8Id2Q")
assert _HEAD.size == 64

FNV_OFFSET, FNV_PRIME = 0xCBF29CE484222325, 0x100000001B3


def fnv1a64(data: bytes) -> int:
    """64-bit FNV-1a of a byte string (Fowler, Noll and Vo)."""
    h = FNV_OFFSET
    for b in data:
        h = ((h ^ b) * FNV_PRIME) % (1 << 64)
    return h


def params_hash(o: Oracle) -> int:
    return fnv1a64(b"".join(int(m).to_bytes(8, "little") for m in o.q + o.p))


def _blob(o: Oracle, kind: int, level: int, polys: int, rows: int, scale: float,
          words: np.ndarray) -> bytes:
    w = np.ascontiguousarray(words, dtype="<u8").reshape(-1)
    assert w.size == polys * rows * o.n
    head = _HEAD.pack(MAGIC, kind, o.log_n, o.L, o.K, o.dnum, level, polys, rows, scale,
                      params_hash(o), w.size)
    return head + w.tobytes()


def serialize_ciphertext(o: Oracle, ct: Ciphertext) -> bytes:
    k = ct.polys.shape[0]
    return _blob(o, KIND_CIPHERTEXT, ct.level, k, ct.level + 1, ct.scale, ct.polys)


def serialize_switch_key(o: Oracle, key: np.ndarray) -> bytes:
    return _blob(o, KIND_SWITCH_KEY, o.L - 1, 2 * o.dnum, o.L + o.K, 0.0, key)


def _read(o: Oracle, blob: bytes, kind: int):
    if len(blob) < _HEAD.size:
        raise ValueError("blob shorter than its header")
    (magic, k, log_n, L, K, dnum, level, polys, rows, scale, h,
     words) = _HEAD.unpack_from(blob)
    if magic != MAGIC:
        raise ValueError("not an interchange blob")
    if k != kind:
        raise ValueError("blob holds another kind of object")
    if (log_n, L, K, dnum) != (o.log_n, o.L, o.K, o.dnum) or h != params_hash(o):
        raise ValueError("blob made under another parameter set")
    if words != polys * rows * o.n or len(blob) != _HEAD.size + 8 * words:
        raise ValueError("blob size inconsistent with its header")
    w = np.frombuffer(blob, dtype="<u8", offset=_HEAD.size).astype(np.uint64)
    return w.reshape(polys, rows, o.n), level, scale


def deserialize_ciphertext(o: Oracle, blob: bytes) -> Ciphertext:
    w, level, scale = _read(o, blob, KIND_CIPHERTEXT)
    if w.shape[1] != level + 1:
        raise ValueError("rows do not match the level")
    return Ciphertext(w.copy(), level, scale)


def deserialize_switch_key(o: Oracle, blob: bytes) -> np.ndarray:
    w, _, _ = _read(o, blob, KIND_SWITCH_KEY)
    return w.reshape(o.dnum, 2, o.L + o.K, o.n).copy()
