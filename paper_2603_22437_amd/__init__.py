"""Python binding of libhipckks, the MI355X (gfx950) RNS-CKKS evaluation library.

Argument marshalling only: every homomorphic operation runs in the HIP
library's kernels.  The raw C entry points are available under their C names
(``capi.hck_add`` ...); ``Context`` and the handle classes wrap them.  There is
no fallback: importing this package without the built library raises.

Build the library first: ``python paper_2603_22437_amd/build.py``.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhipckks.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2603_22437_amd/build.py`")

# torch ships its own HIP runtime.  Loading torch first makes the library bind
# to that same runtime, so that one runtime serves both in the process: torch
# then sees the GPU, and torch's streams and allocator are usable here.
# Loaded the other way round, a second HIP runtime would come up beside the
# library's, and torch would find no GPU.
try:
    import torch  # noqa: F401
except ImportError:
    pass

capi = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_U32, _U64, _I32, _D, _SZ, _I = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_size_t, ctypes.c_int)
_PU32 = ctypes.POINTER(ctypes.c_uint32)
_PD = ctypes.POINTER(ctypes.c_double)


# allocator hook types of hck_set_allocator
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Params(ctypes.Structure):
    _fields_ = [("log_n", _U32), ("num_q", _U32), ("num_p", _U32), ("dnum", _U32),
                ("q", ctypes.POINTER(ctypes.c_uint64)), ("p", ctypes.POINTER(ctypes.c_uint64))]


class BlobHeader(ctypes.Structure):
    """hck_blob_header: the 64-byte header of the interchange form."""
    _fields_ = [("magic", ctypes.c_char * 8), ("kind", _U32), ("log_n", _U32), ("num_q", _U32),
                ("num_p", _U32), ("dnum", _U32), ("level", _U32), ("polys", _U32),
                ("rows", _U32), ("scale", _D), ("prime_hash", _U64), ("words", _U64)]


def params_hash(prm: dict) -> int:
    """FNV-1a prime hash of a parameter set (hck_params_hash; host only)."""
    q, p = _u64(prm["q"]), _u64(prm["p"])
    par = _Params(prm["log_n"], len(q), len(p), prm["dnum"],
                  q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                  p.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    h = ctypes.c_uint64()
    _check(capi.hck_params_hash(ctypes.byref(par), ctypes.byref(h)))
    return h.value


def blob_parse(blob: bytes) -> dict:
    """The checked header of a blob (hck_blob_parse; host only)."""
    h = BlobHeader()
    _check(capi.hck_blob_parse(blob, len(blob), ctypes.byref(h)))
    return {f: getattr(h, f) for f, _ in BlobHeader._fields_}


class TraceRecord(ctypes.Structure):
    """hck_trace_record: one kernel launch, allocation or release."""
    _fields_ = [("name", ctypes.c_char * 32), ("grid", _U32 * 3), ("bytes", _D),
                ("mulmods", _D)]


# C signature table: name -> (argtypes, restype).  Every symbol of hipckks.h.
SIGNATURES = {
    "hck_context_create": ([ctypes.POINTER(_Params), _I, _P, _PP], _I),
    "hck_context_destroy": ([_P], _I),
    "hck_context_set_stream": ([_P, _P], _I),
    "hck_set_allocator": ([_P, ALLOC_FN, FREE_FN, _P], _I),
    "hck_synchronize": ([_P], _I),
    "hck_last_error": ([], ctypes.c_char_p),
    "hck_galois_element": ([_P, _I32], _U32),
    "hck_keygen_secret": ([_P, _U64, _PP], _I),
    "hck_secret_key_import": ([_P, _P, _PP], _I),
    "hck_secret_key_destroy": ([_P], _I),
    "hck_keygen_public": ([_P, _P, _U64, _PP], _I),
    "hck_public_key_export": ([_P, _P, _P, _SZ], _I),
    "hck_public_key_destroy": ([_P], _I),
    "hck_keygen_relin": ([_P, _P, _U64, _PP], _I),
    "hck_switch_key_export": ([_P, _P, _P, _SZ], _I),
    "hck_switch_key_destroy": ([_P], _I),
    "hck_keygen_galois": ([_P, _P, _P, _U32, _U64, _PP], _I),
    "hck_keygen_rotation": ([_P, _P, _P, _U32, _U64, _PP], _I),
    "hck_galois_keys_export": ([_P, _P, _U32, _P, _SZ], _I),
    "hck_galois_keys_count": ([_P, _PU32], _I),
    "hck_galois_keys_destroy": ([_P], _I),
    "hck_encode": ([_P, _P, _P, _U32, _D, _U32, _PP], _I),
    "hck_plaintext_import": ([_P, _P, _U32, _D, _PP], _I),
    "hck_plaintext_export": ([_P, _P, _P, _SZ, _PU32, _PD], _I),
    "hck_decode": ([_P, _P, _P, _P, _U32], _I),
    "hck_plaintext_destroy": ([_P], _I),
    "hck_ciphertext_create": ([_P, _PP], _I),
    "hck_ciphertext_import": ([_P, _P, _U32, _U32, _D, _PP], _I),
    "hck_ciphertext_export": ([_P, _P, _P, _SZ, _PU32, _PU32, _PD], _I),
    "hck_ciphertext_info": ([_P, _PU32, _PU32, _PD], _I),
    "hck_ciphertext_destroy": ([_P], _I),
    "hck_encrypt_sk": ([_P, _P, _P, _U64, _P], _I),
    "hck_encrypt_pk": ([_P, _P, _P, _U64, _P], _I),
    "hck_decrypt": ([_P, _P, _P, _PP], _I),
    "hck_add": ([_P, _P, _P, _P], _I),
    "hck_sub": ([_P, _P, _P, _P], _I),
    "hck_add_plain": ([_P, _P, _P, _P], _I),
    "hck_mul_plain": ([_P, _P, _P, _P], _I),
    "hck_drop_level": ([_P, _P, _U32, _P], _I),
    "hck_mul": ([_P, _P, _P, _P], _I),
    "hck_relinearize": ([_P, _P, _P, _P], _I),
    "hck_rescale": ([_P, _P, _P], _I),
    "hck_rotate": ([_P, _P, _I32, _P, _P], _I),
    "hck_rotate_noalloc": ([_P, _P, _I32, _P, _P], _I),
    "hck_rotate_noalloc_scratch": ([_P], _SZ),
    "hck_apply_galois": ([_P, _P, _U32, _P, _P], _I),
    "hck_rotate_many": ([_P, _P, _U32, _I32, _P, _P], _I),
    "hck_rotate_steps": ([_P, _P, _P, _U32, _P, _P], _I),
    "hck_relinearize_many": ([_P, _P, _U32, _P, _P], _I),
    "hck_vital_required_steps": ([_P, _P, _P, _U32, _PU32], _I),
    "hck_vital_eval": ([_P, _P, _P, _P, _P, _P, _P], _I),
    "hck_vital_eval_many": ([_P, _P, _P, _P, _U32, _P, _P, _P], _I),
    "hck_gesture_required_steps": ([_P, _P, _P, _U32, _PU32], _I),
    "hck_gesture_eval": ([_P, _P, _P, _P, _P, _P, _P], _I),
    "hck_vital_eval_taps": ([_P, _P, _P, _P, _P, _P, _P, _P], _I),
    "hck_gesture_eval_taps": ([_P, _P, _P, _P, _P, _P, _P, _P], _I),
    "hck_gesture_eval_frames": ([_P, _P, _P, _P, _U32, _P, _P, _P], _I),
    "hck_gesture_cnn_required_steps": ([_P, _P, _P, _U32, _PU32], _I),
    "hck_gesture_cnn_eval": ([_P, _P, _P, _P, _P, _P, _P, _P], _I),
    "hck_measure_mulmod_rate": ([_P, _PD], _I),
    "hck_lt_eval": ([_P, _P, _U32, _P, _P, _P, _P, _U32, _P, _P, _U32, _U32], _I),
    "hck_rotate_hoisted": ([_P, _P, _P, _U32, _P, _P], _I),
    "hck_keyswitch": ([_P, _P, _P, _P], _I),
    "hck_lt_create": ([_P, _P, _P, _P, _U32, _U32, _U32, _D, _U32, _PP], _I),
    "hck_lt_create_from_residues": ([_P, _P, _P, _U32, _U32, _D, _U32, _PP], _I),
    "hck_lt_required_steps": ([_P, _P, _U32, _PU32], _I),
    "hck_lt_apply": ([_P, _P, _P, _P, _P], _I),
    "hck_lt_destroy": ([_P], _I),
    "hck_timing_enable": ([_P, _I], _I),
    "hck_timing_reset": ([_P], _I),
    "hck_timing_read": ([_P, ctypes.c_char_p, _PD, ctypes.POINTER(ctypes.c_uint64), _PD, _PD], _I),
    "hck_timing_names": ([_P, ctypes.c_char_p, _SZ], _I),
    "hck_graph_begin": ([_P, _U32], _I),
    "hck_graph_end": ([_P, _U32, _PP], _I),
    "hck_graph_launch": ([_P], _I),
    "hck_graph_info": ([_P, _PU32, ctypes.POINTER(_SZ)], _I),
    "hck_graph_destroy": ([_P], _I),
    "hck_autotune_dnum": ([_P, _U32, _I, _P, _U32, _U32, _P, _P, _PU32], _I),
    "hck_params_hash": ([ctypes.POINTER(_Params), ctypes.POINTER(_U64)], _I),
    "hck_blob_parse": ([_P, _SZ, _P], _I),
    "hck_ciphertext_serialize": ([_P, _P, _P, _SZ, ctypes.POINTER(_SZ)], _I),
    "hck_switch_key_serialize": ([_P, _P, _P, _SZ, ctypes.POINTER(_SZ)], _I),
    "hck_ciphertext_deserialize": ([_P, _P, _SZ, _PP], _I),
    "hck_switch_key_deserialize": ([_P, _P, _SZ, _PP], _I),
    "hck_vital_frames_required_steps": ([_P, _P, _P, _U32, _PU32], _I),
    "hck_vital_eval_frames": ([_P, _P, _P, _P, _U32, _P, _P, _P], _I),
    "hck_autotune_ntt": ([_P, _U32, _P, _P, _U32, _PU32, _P], _I),
    "hck_set_ntt_split": ([_P, _I32], _I),
    "hck_ntt_split": ([_P, _P], _I),
    "hck_trace_enable": ([_P, _I], _I),
    "hck_trace_read": ([_P, _P, _SZ, ctypes.POINTER(_SZ)], _I),
    "hck_shake256": ([_P, _SZ, _P, _SZ], _I),
    "hck_sample_uniform": ([ctypes.c_char_p, _U64, _U32, _U64, _P, _SZ], _I),
    "hck_sample_ternary": ([ctypes.c_char_p, _U64, _P, _SZ], _I),
    "hck_sample_gaussian": ([ctypes.c_char_p, _U64, _P, _SZ], _I),
    "hck_encode_coeffs": ([_U32, _P, _P, _D, _P], _I),
    "hck_decode_residues": ([_U32, _P, _P, _U32, _D, _P, _P], _I),
    "hck_switch_key_import": ([_P, _P, _SZ, _PP], _I),
    "hck_encode_const": ([_P, _D, _D, _U32, _PP], _I),
    "hck_poly_eval": ([_P, _P, _P, _U32, _P, _P], _I),
    "hck_autotune_keyswitch": ([_P, _P, _U32, _U32, _P, _P], _I),
    "hck_set_keyswitch_cap": ([_P, _U32, _U32], _I),
    "hck_keyswitch_batch_limit": ([_P, _U32, _PU32], _I),
    "hck_galois_keys_create": ([_P, _PP], _I),
    "hck_galois_keys_insert": ([_P, _U32, _P], _I),
    "hck_server_create": ([_P, _P, _PP], _I),
    "hck_server_add_tenant": ([_P, _U32, _U32, _P, _P, _P, _U32, _P], _I),
    "hck_server_submit": ([_P, _U64, _U32, _P, _P, _U32, _D, _P, _SZ], _I),
    "hck_server_poll": ([_P, _U32, _P, _U32, _PU32], _I),
    "hck_server_stats_get": ([_P, _P], _I),
    "hck_server_destroy": ([_P], _I),
}

for _name, (_args, _res) in SIGNATURES.items():
    _fn = getattr(capi, _name)
    _fn.argtypes = _args
    _fn.restype = _res
    globals()[_name] = _fn

HCK_OK, HCK_EINVAL, HCK_ENOMEM, HCK_EDEVICE, HCK_ELEVEL, HCK_ESCALE, HCK_ENOKEY, HCK_EPARAMS = \
    0, -1, -2, -3, -4, -5, -6, -7


class HckError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hipckks error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != 0:
        raise HckError(rc, capi.hck_last_error().decode())


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


# ---------------------------------------------------------------------------
# host utilities (no device)
# ---------------------------------------------------------------------------

def shake256(msg: bytes, outlen: int) -> bytes:
    out = ctypes.create_string_buffer(outlen)
    buf = ctypes.create_string_buffer(msg, len(msg))
    _check(capi.hck_shake256(buf, len(msg), out, outlen))
    return out.raw


def sample_uniform(tag: str, seed: int, index: int, q: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _check(capi.hck_sample_uniform(tag.encode(), seed, index, q, _ptr(out), n))
    return out


def sample_ternary(tag: str, seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _check(capi.hck_sample_ternary(tag.encode(), seed, _ptr(out), n))
    return out


def sample_gaussian(tag: str, seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _check(capi.hck_sample_gaussian(tag.encode(), seed, _ptr(out), n))
    return out


def encode_coeffs(log_n: int, z, scale: float) -> np.ndarray:
    z = np.asarray(z)
    re = np.ascontiguousarray(z.real, dtype=np.float64)
    im = np.ascontiguousarray(z.imag, dtype=np.float64) if np.iscomplexobj(z) else None
    out = np.empty(1 << log_n, dtype=np.int64)
    _check(capi.hck_encode_coeffs(log_n, _ptr(re), _ptr(im) if im is not None else None,
                                  scale, _ptr(out)))
    return out


def decode_residues(log_n: int, res: np.ndarray, mods, scale: float) -> np.ndarray:
    res = _u64(res)
    mods = _u64(mods)
    re = np.empty((1 << log_n) // 2)
    im = np.empty_like(re)
    _check(capi.hck_decode_residues(log_n, _ptr(res), _ptr(mods), len(mods), scale,
                                    _ptr(re), _ptr(im)))
    return re + 1j * im


# ---------------------------------------------------------------------------
# handles
# ---------------------------------------------------------------------------

class _Handle:
    """A library object.  It is freed by close() or, at the latest, when it
    is garbage-collected or the interpreter exits (weakref.finalize, which
    also runs the handles' finalizers before the older context's).  The C
    side makes any order safe: destroying a context releases the device
    memory of every handle still alive, whose own destroy call then frees
    only its host record."""
    _destroy = None

    def __init__(self, ctx, h):
        self.ctx = ctx          # keeps the context alive
        self.h = h
        self._fin = weakref.finalize(self, type(self)._destroy, h) if h else None

    def close(self):
        if self._fin is not None:
            self._fin()
            self._fin = None
        self.h = None

    def _disown(self):
        """The library took ownership of the object (e.g. a key inserted
        into a key set): forget it without destroying it."""
        if self._fin is not None:
            self._fin.detach()
            self._fin = None
        self.h = None

    @property
    def _as_parameter_(self):
        return self.h


class SecretKey(_Handle):
    _destroy = staticmethod(lambda h: capi.hck_secret_key_destroy(h))


class PublicKey(_Handle):
    _destroy = staticmethod(lambda h: capi.hck_public_key_destroy(h))


class SwitchKey(_Handle):
    _destroy = staticmethod(lambda h: capi.hck_switch_key_destroy(h))


class GaloisKeys(_Handle):
    _destroy = staticmethod(lambda h: capi.hck_galois_keys_destroy(h))

    def __len__(self):
        n = ctypes.c_uint32()
        _check(capi.hck_galois_keys_count(self.h, ctypes.byref(n)))
        return n.value


class Plaintext(_Handle):
    _destroy = staticmethod(lambda h: capi.hck_plaintext_destroy(h))


class Ciphertext(_Handle):
    _destroy = staticmethod(lambda h: capi.hck_ciphertext_destroy(h))

    def info(self):
        s, l, sc = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_double()
        _check(capi.hck_ciphertext_info(self.h, ctypes.byref(s), ctypes.byref(l),
                                        ctypes.byref(sc)))
        return s.value, l.value, sc.value

    @property
    def size(self):
        return self.info()[0]

    @property
    def level(self):
        return self.info()[1]

    @property
    def scale(self):
        return self.info()[2]


class LinearTransform(_Handle):
    _destroy = staticmethod(lambda h: capi.hck_lt_destroy(h))


class VitalPlan(ctypes.Structure):
    """hck_vital_plan: layout of one vital-sign window and its public operands."""
    _fields_ = [("frames", ctypes.c_uint32), ("bins", ctypes.c_uint32),
                ("taylor_order", ctypes.c_uint32), ("lanes_resp", ctypes.c_uint32),
                ("lanes_hr", ctypes.c_uint32)] + [
        (name, ctypes.c_void_p) for name in (
            "bin_index", "bin_mask", "fir_resp", "fir_hr", "third", "dft_re_resp",
            "dft_im_resp", "dft_re_hr", "dft_im_hr", "freq", "mask")] + [
        ("mag_degree", ctypes.c_uint32), ("mag_coeffs", ctypes.c_void_p),
        ("gamma", ctypes.c_uint32), ("phase_power", ctypes.c_uint32)]

    OPERANDS = ("bin_index", "bin_mask", "fir_resp", "fir_hr", "third", "dft_re_resp",
                "dft_im_resp", "dft_re_hr", "dft_im_hr", "freq", "mask")
    OUTPUTS = ("num_bin", "den_bin", "num_rates", "den_rates")

    @classmethod
    def build(cls, frames, bins, taylor_order, lanes_resp, lanes_hr, operands: dict,
              mag_coeffs=None, gamma: int = 2, phase_power: int = 2):
        """operands: name -> Plaintext / LinearTransform handle (kept alive by
        the plan object); mag_coeffs: the magnitude option's polynomial;
        gamma: the soft-attention exponent (2 or 4); phase_power: K4's mask
        exponent P_phi (2 .. 5)."""
        plan = cls(frames, bins, taylor_order, lanes_resp, lanes_hr)
        plan.gamma = gamma
        plan.phase_power = phase_power
        plan._keep = dict(operands)
        for name in cls.OPERANDS:
            h = operands.get(name)
            setattr(plan, name, h.h if h is not None else None)
        if mag_coeffs is not None and len(mag_coeffs) > 1:
            c = np.ascontiguousarray(np.asarray(mag_coeffs, dtype=np.float64))
            plan._mag = c
            plan.mag_degree = len(c) - 1
            plan.mag_coeffs = c.ctypes.data
        return plan


class GesturePlan(ctypes.Structure):
    """hck_gesture_plan: layout of one gesture window and its public operands."""
    OPERANDS = ("dft_c", "dft_s", "fc1", "fc2", "fc3", "notch", "bias1", "bias2", "bias3")
    _fields_ = [("frames", ctypes.c_uint32), ("bins", ctypes.c_uint32),
                ("chirps", ctypes.c_uint32), ("hidden1", ctypes.c_uint32)] + [
        (name, ctypes.c_void_p) for name in OPERANDS]

    @classmethod
    def build(cls, frames, bins, chirps, hidden1, operands: dict):
        plan = cls(frames, bins, chirps, hidden1)
        plan._keep = dict(operands)
        for name in cls.OPERANDS:
            h = operands.get(name)
            setattr(plan, name, h.h if h is not None else None)
        return plan


class GestureCnnPlan(ctypes.Structure):
    """hck_gesture_cnn_plan: layout of one gesture window, the CNN's shape and
    its public operands."""
    OPERANDS = ("dft_c", "dft_s", "notch", "conv1", "conv2", "dense1", "dense2", "bias1",
                "bias2")
    _fields_ = [(name, ctypes.c_uint32) for name in
                ("frames", "bins", "chirps", "c1", "c2", "hidden", "classes")] + [
        (name, ctypes.c_void_p) for name in OPERANDS] + [
        ("act_degree", ctypes.c_uint32), ("act_coeffs", ctypes.POINTER(ctypes.c_double))]

    @classmethod
    def build(cls, shape: dict, operands: dict, act_coeffs):
        plan = cls(*[int(shape[k]) for k in
                     ("frames", "bins", "chirps", "c1", "c2", "hidden", "classes")])
        plan._keep = dict(operands)
        for name in cls.OPERANDS:
            h = operands.get(name)
            setattr(plan, name, h.h if h is not None else None)
        coeffs = np.ascontiguousarray(act_coeffs, dtype=np.float64)
        plan._coeffs = coeffs
        plan.act_degree = len(coeffs) - 1
        plan.act_coeffs = coeffs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return plan


def _destroy_context(h, hooks_keep):
    capi.hck_context_destroy(h)
    hooks_keep.clear()


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream   # torch.cuda.Stream


def autotune_dnum(candidates: list, level: int, count: int = 16, device: int = 0,
                  stream=None) -> dict:
    """Times key switching for parameter sets that differ only in dnum and
    their special primes (hck_autotune_dnum).  candidates: parameter dicts
    (``seeded_inputs.params`` form).  Returns {"best": index, "us_per_switch":
    [...], "key_bytes": [...]}."""
    n = len(candidates)
    keep = [(_u64(c["q"]), _u64(c["p"])) for c in candidates]
    arr = (_Params * n)(*[_Params(c["log_n"], len(q), len(p), c["dnum"],
                                  q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  p.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
                          for c, (q, p) in zip(candidates, keep)])
    us = np.zeros(n, dtype=np.float64)
    kb = np.zeros(n, dtype=np.float64)
    best = ctypes.c_uint32()
    _check(capi.hck_autotune_dnum(arr, n, device, _stream_handle(stream), level, count, _ptr(us),
                                  _ptr(kb), ctypes.byref(best)))
    return {"best": best.value, "us_per_switch": us.tolist(), "key_bytes": kb.tolist()}


class Graph:
    """Evaluation calls on one or more contexts recorded into HIP graphs, one
    per context on its stream, replayed together (hck_graph_*).  Use
    ``capture``::

        with H.Graph.capture([ctx16, ctx15]) as g:
            ctx16.vital_eval(...)      # recorded, not run
            ctx15.gesture_eval(...)
        g.launch()                     # replays every recorded call

    Every context needs a stream of its own (``Context.set_stream``), and the
    recorded calls must have run once before (no allocation while
    recording)."""

    def __init__(self, ctxs):
        self.ctxs = list(ctxs)        # keeps the contexts alive
        self.h = None
        self._fin = None

    @classmethod
    def capture(cls, ctxs):
        return _GraphCapture(cls(ctxs))

    def launch(self):
        _check(capi.hck_graph_launch(self.h))

    def info(self) -> dict:
        c, n = ctypes.c_uint32(), ctypes.c_size_t()
        _check(capi.hck_graph_info(self.h, ctypes.byref(c), ctypes.byref(n)))
        return dict(contexts=c.value, nodes=n.value)

    def close(self):
        if self._fin is not None:
            self._fin()
            self._fin = None
        self.h = None


class _GraphCapture:
    def __init__(self, g: Graph):
        self.g = g
        self.arr = (ctypes.c_void_p * len(g.ctxs))(*[c.h for c in g.ctxs])

    def __enter__(self) -> Graph:
        _check(capi.hck_graph_begin(self.arr, len(self.g.ctxs)))
        return self.g

    def __exit__(self, exc_type, exc, tb):
        h = ctypes.c_void_p()
        rc = capi.hck_graph_end(self.arr, len(self.g.ctxs), ctypes.byref(h))
        if exc_type is not None:
            if rc == 0:
                capi.hck_graph_destroy(h.value)
            return False
        _check(rc)
        self.g.h = h.value
        self.g._fin = weakref.finalize(self.g, capi.hck_graph_destroy, h.value)
        return False


class Context:
    """One parameter set on one device and stream (hck_context)."""

    def __init__(self, log_n: int, q, p, dnum: int, device: int = 0, stream=None):
        self._q = _u64(q)
        self._p = _u64(p)
        prm = _Params(log_n, len(self._q), len(self._p), dnum,
                      self._q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                      self._p.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        h = ctypes.c_void_p()
        _check(capi.hck_context_create(ctypes.byref(prm), device, _stream_handle(stream),
                                       ctypes.byref(h)))
        self.h = h.value
        # the finalizer holds the allocator hooks (use_torch_allocator) alive
        # until the context is destroyed: its destroy call still frees
        # through them
        self._hooks_keep = []
        self._fin = weakref.finalize(self, _destroy_context, self.h, self._hooks_keep)
        self.log_n, self.n, self.dnum = log_n, 1 << log_n, dnum
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        self.L, self.K = len(self.q), len(self.p)
        self.n_slots = self.n // 2
        self.device = device
        self._alloc_hooks = None

    @classmethod
    def from_params(cls, prm: dict, device: int = 0, stream=None):
        return cls(prm["log_n"], prm["q"], prm["p"], prm["dnum"], device, stream)

    def close(self):
        """Destroys the context.  Handles still alive lose their device
        memory and can no longer be used (calls with them fail); closing
        them afterwards is harmless."""
        fin = getattr(self, "_fin", None)
        if fin is not None:
            fin()
            self._fin = None
        self.h = None

    @property
    def _as_parameter_(self):
        return self.h

    def _new(self, fn, *args, cls):
        h = ctypes.c_void_p()
        _check(fn(self.h, *args, ctypes.byref(h)))
        return cls(self, h.value)

    def set_stream(self, stream):
        _check(capi.hck_context_set_stream(self.h, _stream_handle(stream)))

    def use_torch_allocator(self):
        """Routes the context's device buffers through torch's caching
        allocator (hck_set_allocator), on the context's stream.  Call it right
        after creation; close() the context before torch shuts down."""
        import torch
        dev = self.device

        def alloc(size, stream, user):
            try:
                return torch.cuda.caching_allocator_alloc(size, dev, stream or 0)
            except Exception:       # out of memory: the library reports HCK_ENOMEM
                return None

        def free(ptr, stream, user):
            torch.cuda.caching_allocator_delete(ptr)

        hooks = (ALLOC_FN(alloc), FREE_FN(free))
        _check(capi.hck_set_allocator(self.h, hooks[0], hooks[1], None))
        self._alloc_hooks = hooks   # the C side calls them until close()
        self._hooks_keep.append(hooks)

    def use_default_allocator(self):
        _check(capi.hck_set_allocator(self.h, ALLOC_FN(), FREE_FN(), None))
        self._alloc_hooks = None

    def synchronize(self):
        _check(capi.hck_synchronize(self.h))

    def galois_element(self, step: int) -> int:
        return capi.hck_galois_element(self.h, step)

    # --- keys ---
    def keygen_secret(self, seed: int) -> SecretKey:
        return self._new(capi.hck_keygen_secret, seed, cls=SecretKey)

    def secret_key_import(self, coeffs) -> SecretKey:
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.int8))
        return self._new(capi.hck_secret_key_import, _ptr(c), cls=SecretKey)

    def keygen_public(self, sk, seed: int) -> PublicKey:
        return self._new(capi.hck_keygen_public, sk, seed, cls=PublicKey)

    def public_key_export(self, pk) -> np.ndarray:
        out = np.empty((2, self.L, self.n), dtype=np.uint64)
        _check(capi.hck_public_key_export(self.h, pk, _ptr(out), out.size))
        return out

    def keygen_relin(self, sk, seed: int) -> SwitchKey:
        return self._new(capi.hck_keygen_relin, sk, seed, cls=SwitchKey)

    def switch_key_export(self, swk) -> np.ndarray:
        out = np.empty((self.dnum, 2, self.L + self.K, self.n), dtype=np.uint64)
        _check(capi.hck_switch_key_export(self.h, swk, _ptr(out), out.size))
        return out

    def switch_key_import(self, words) -> SwitchKey:
        w = _u64(words).reshape(-1)
        return self._new(capi.hck_switch_key_import, _ptr(w), w.size, cls=SwitchKey)

    def galois_keys_from_words(self, keys: dict) -> GaloisKeys:
        """A Galois key set from exported words: {element: words}."""
        gks = self._new(capi.hck_galois_keys_create, cls=GaloisKeys)
        for g, words in keys.items():
            swk = self.switch_key_import(words)
            _check(capi.hck_galois_keys_insert(gks.h, int(g), swk.h))
            swk._disown()    # owned by the set now
        return gks

    def keygen_galois(self, sk, elements, seed: int) -> GaloisKeys:
        e = np.ascontiguousarray(np.asarray(elements, dtype=np.uint32))
        return self._new(capi.hck_keygen_galois, sk, _ptr(e), len(e), seed, cls=GaloisKeys)

    def keygen_rotation(self, sk, steps, seed: int) -> GaloisKeys:
        s = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
        return self._new(capi.hck_keygen_rotation, sk, _ptr(s), len(s), seed, cls=GaloisKeys)

    def galois_keys_export(self, gks, element: int) -> np.ndarray:
        out = np.empty((self.dnum, 2, self.L + self.K, self.n), dtype=np.uint64)
        _check(capi.hck_galois_keys_export(self.h, gks, element, _ptr(out), out.size))
        return out

    # --- plaintexts ---
    def encode(self, z, scale: float, level: int) -> Plaintext:
        z = np.asarray(z)
        re = np.ascontiguousarray(z.real, dtype=np.float64)
        im = np.ascontiguousarray(z.imag, dtype=np.float64) if np.iscomplexobj(z) else None
        return self._new(capi.hck_encode, _ptr(re), _ptr(im) if im is not None else None,
                         len(re), scale, level, cls=Plaintext)

    def encode_const(self, value: float, scale: float, level: int) -> Plaintext:
        return self._new(capi.hck_encode_const, float(value), float(scale), level, cls=Plaintext)

    def poly_eval(self, x, coeffs, rlk, out=None):
        """sum_k coeffs[k] x^k slot-wise (hck_poly_eval)."""
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
        out = self._out(out)
        _check(capi.hck_poly_eval(self.h, x, _ptr(c), len(c) - 1, rlk, out))
        return out

    def plaintext_import(self, res, level: int, scale: float) -> Plaintext:
        r = _u64(res)
        return self._new(capi.hck_plaintext_import, _ptr(r), level, scale, cls=Plaintext)

    def plaintext_export(self, pt):
        lvl, sc = ctypes.c_uint32(), ctypes.c_double()
        out = np.empty((self.L, self.n), dtype=np.uint64)
        _check(capi.hck_plaintext_export(self.h, pt, _ptr(out), out.size, ctypes.byref(lvl),
                                         ctypes.byref(sc)))
        return out[: lvl.value + 1].copy(), lvl.value, sc.value

    def decode(self, pt) -> np.ndarray:
        re = np.empty(self.n_slots)
        im = np.empty(self.n_slots)
        _check(capi.hck_decode(self.h, pt, _ptr(re), _ptr(im), self.n_slots))
        return re + 1j * im

    # --- ciphertexts ---
    def ciphertext(self) -> Ciphertext:
        return self._new(capi.hck_ciphertext_create, cls=Ciphertext)

    def ciphertext_import(self, res, level: int, scale: float) -> Ciphertext:
        r = _u64(res)
        return self._new(capi.hck_ciphertext_import, _ptr(r), r.shape[0], level, scale,
                         cls=Ciphertext)

    def serialize(self, obj) -> bytes:
        """The interchange blob of a Ciphertext or SwitchKey."""
        fn = (capi.hck_ciphertext_serialize if isinstance(obj, Ciphertext)
              else capi.hck_switch_key_serialize)
        n = ctypes.c_size_t()
        _check(fn(self.h, obj, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(fn(self.h, obj, buf, n.value, ctypes.byref(n)))
        return buf.raw[: n.value]

    def ciphertext_deserialize(self, blob: bytes) -> Ciphertext:
        return self._new(capi.hck_ciphertext_deserialize, blob, len(blob), cls=Ciphertext)

    def switch_key_deserialize(self, blob: bytes) -> SwitchKey:
        return self._new(capi.hck_switch_key_deserialize, blob, len(blob), cls=SwitchKey)

    def ciphertext_export(self, ct):
        size, lvl, sc = ct.info()
        out = np.empty((size, lvl + 1, self.n), dtype=np.uint64)
        _check(capi.hck_ciphertext_export(self.h, ct, _ptr(out), out.size, None, None, None))
        return out, lvl, sc

    def _out(self, out):
        return self.ciphertext() if out is None else out

    def encrypt_sk(self, sk, pt, seed: int, out=None) -> Ciphertext:
        out = self._out(out)
        _check(capi.hck_encrypt_sk(self.h, sk, pt, seed, out))
        return out

    def encrypt_pk(self, pk, pt, seed: int, out=None) -> Ciphertext:
        out = self._out(out)
        _check(capi.hck_encrypt_pk(self.h, pk, pt, seed, out))
        return out

    def decrypt(self, sk, ct) -> Plaintext:
        return self._new(capi.hck_decrypt, sk, ct, cls=Plaintext)

    # --- evaluation ---
    def _binary(self, fn, a, b, out):
        out = self._out(out)
        _check(fn(self.h, a, b, out))
        return out

    def add(self, a, b, out=None):
        return self._binary(capi.hck_add, a, b, out)

    def sub(self, a, b, out=None):
        return self._binary(capi.hck_sub, a, b, out)

    def add_plain(self, a, pt, out=None):
        return self._binary(capi.hck_add_plain, a, pt, out)

    def mul_plain(self, a, pt, out=None):
        return self._binary(capi.hck_mul_plain, a, pt, out)

    def mul(self, a, b, out=None):
        return self._binary(capi.hck_mul, a, b, out)

    def relinearize(self, a, rlk, out=None):
        return self._binary(capi.hck_relinearize, a, rlk, out)

    def keyswitch(self, a, swk, out=None):
        return self._binary(capi.hck_keyswitch, a, swk, out)

    def drop_level(self, a, level: int, out=None):
        out = self._out(out)
        _check(capi.hck_drop_level(self.h, a, level, out))
        return out

    def rescale(self, a, out=None):
        out = self._out(out)
        _check(capi.hck_rescale(self.h, a, out))
        return out

    def rotate(self, a, step: int, gks, out=None):
        out = self._out(out)
        _check(capi.hck_rotate(self.h, a, step, gks, out))
        return out

    def rotate_noalloc(self, a, step: int, gks, out):
        """hck_rotate without allocation (the library's static scratch
        array): `out` must already hold two polynomials (an earlier result
        or import).  Calls on one GPU must not overlap in time."""
        _check(capi.hck_rotate_noalloc(self.h, a, step, gks, out))
        return out

    def rotate_noalloc_scratch(self) -> int:
        """Bytes of the static array a no-allocation rotation needs here."""
        return int(capi.hck_rotate_noalloc_scratch(self.h))

    def rotate_many(self, cts, step: int, gks, outs=None):
        outs = [self.ciphertext() for _ in cts] if outs is None else outs
        a = (ctypes.c_void_p * len(cts))(*[c.h for c in cts])
        o = (ctypes.c_void_p * len(outs))(*[c.h for c in outs])
        _check(capi.hck_rotate_many(self.h, a, len(cts), step, gks, o))
        return outs

    def relinearize_many(self, cts, rlk, outs=None):
        """Relinearizations of several 3-part ciphertexts of one level,
        key-switched together in batches."""
        outs = [self.ciphertext() for _ in cts] if outs is None else outs
        a = (ctypes.c_void_p * len(cts))(*[c.h for c in cts])
        o = (ctypes.c_void_p * len(outs))(*[c.h for c in outs])
        _check(capi.hck_relinearize_many(self.h, a, len(cts), rlk, o))
        return outs

    def rotate_steps(self, cts, steps, gks, outs=None):
        """a[i] rotated by steps[i], key-switched together in batches."""
        if len(steps) != len(cts):
            raise ValueError("one step per ciphertext")
        outs = [self.ciphertext() for _ in cts] if outs is None else outs
        a = (ctypes.c_void_p * len(cts))(*[c.h for c in cts])
        o = (ctypes.c_void_p * len(outs))(*[c.h for c in outs])
        st = (ctypes.c_int32 * len(steps))(*steps)
        _check(capi.hck_rotate_steps(self.h, a, st, len(cts), gks, o))
        return outs

    def apply_galois(self, a, element: int, gks, out=None):
        out = self._out(out)
        _check(capi.hck_apply_galois(self.h, a, element, gks, out))
        return out

    # --- linear transforms ---
    def lt_create(self, diags: dict, baby_step: int, level: int, pt_scale: float = 0.0
                  ) -> LinearTransform:
        offs = np.array(sorted(diags), dtype=np.int32)
        mat = np.stack([np.asarray(diags[k]) for k in offs])
        re = np.ascontiguousarray(mat.real, dtype=np.float64)
        im = np.ascontiguousarray(mat.imag, dtype=np.float64) if np.iscomplexobj(mat) else None
        return self._new(capi.hck_lt_create, _ptr(re), _ptr(im) if im is not None else None,
                         _ptr(offs), len(offs), self.n_slots, baby_step, pt_scale, level,
                         cls=LinearTransform)

    def lt_create_from_residues(self, res: dict, baby_step: int, level: int,
                                pt_scale: float) -> LinearTransform:
        offs = np.array(sorted(res), dtype=np.int32)
        r = _u64(np.stack([res[int(k)] for k in offs]))
        return self._new(capi.hck_lt_create_from_residues, _ptr(r), _ptr(offs), len(offs),
                         baby_step, pt_scale, level, cls=LinearTransform)

    def lt_required_steps(self, lt) -> list[int]:
        n = ctypes.c_uint32()
        _check(capi.hck_lt_required_steps(lt, None, 0, ctypes.byref(n)))
        out = np.empty(n.value, dtype=np.int32)
        _check(capi.hck_lt_required_steps(lt, _ptr(out), n.value, ctypes.byref(n)))
        return [int(x) for x in out]

    def lt_apply(self, lt, a, gks, out=None):
        out = self._out(out)
        _check(capi.hck_lt_apply(self.h, lt, a, gks, out))
        return out

    def rotate_hoisted(self, a, steps, gks, outs=None):
        outs = [self.ciphertext() for _ in steps] if outs is None else outs
        s = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
        o = (ctypes.c_void_p * len(outs))(*[c.h for c in outs])
        _check(capi.hck_rotate_hoisted(self.h, a, _ptr(s), len(s), gks, o))
        return outs

    def lt_eval(self, inputs, terms, gks, outputs=None, n_out=None, hoist=False,
                hoist_giant=False):
        """terms: list of (transform, input index, output index, sign +-1);
        returns the outputs out[o] = sum sign * lt(inputs[i]); with hoist the
        baby rotations of each input share one ModUp, with hoist_giant the
        giant rotations of each output share one ModDown."""
        if outputs is None:
            n_out = n_out if n_out is not None else 1 + max(t[2] for t in terms)
            outputs = [self.ciphertext() for _ in range(n_out)]
        ins = (ctypes.c_void_p * len(inputs))(*[c.h for c in inputs])
        lts = (ctypes.c_void_p * len(terms))(*[t[0].h for t in terms])
        ti = np.array([t[1] for t in terms], dtype=np.uint32)
        to = np.array([t[2] for t in terms], dtype=np.uint32)
        ts = np.array([t[3] for t in terms], dtype=np.int32)
        outs = (ctypes.c_void_p * len(outputs))(*[c.h for c in outputs])
        _check(capi.hck_lt_eval(self.h, ins, len(inputs), lts, _ptr(ti), _ptr(to), _ptr(ts),
                                len(terms), gks, outs, len(outputs),
                                (1 if hoist else 0) | (2 if hoist_giant else 0)))
        return outputs

    # --- vital-sign pipeline ---
    def vital_required_steps(self, plan: VitalPlan) -> list:
        n = ctypes.c_uint32()
        _check(capi.hck_vital_required_steps(self.h, ctypes.addressof(plan), None, 0,
                                             ctypes.byref(n)))
        buf = (ctypes.c_int32 * max(1, n.value))()
        _check(capi.hck_vital_required_steps(self.h, ctypes.addressof(plan), buf, n.value,
                                             ctypes.byref(n)))
        return list(buf[: n.value])

    def vital_eval(self, plan: VitalPlan, re, im, gks, rlk, outputs=None):
        """The four outputs num_bin, den_bin (slot 0) and num_rates,
        den_rates (respiration in slot 0, heart rate in slot
        vital.lane_group(...))."""
        outputs = [self.ciphertext() for _ in range(4)] if outputs is None else outputs
        outs = (ctypes.c_void_p * 4)(*[c.h for c in outputs])
        _check(capi.hck_vital_eval(self.h, ctypes.addressof(plan), re, im, gks, rlk, outs))
        return outputs

    VITAL_TAPS = ("K1 p", "K1 energy", "K2 attention", "K4 I", "K4 Q", "K5 If resp",
                  "K5 Qf resp", "K5 If hr", "K5 Qf hr", "K7 dphi resp", "K7 dphi hr",
                  "K3 Re X", "K3 Im X", "K1 spectrum power", "K2 sharpened")

    def vital_eval_taps(self, plan: VitalPlan, re, im, gks, rlk):
        """(outputs, taps): hck_vital_eval's four outputs and the kernels'
        intermediate ciphertexts, in the order of VITAL_TAPS."""
        outputs = [self.ciphertext() for _ in range(4)]
        taps = [self.ciphertext() for _ in self.VITAL_TAPS]
        outs = (ctypes.c_void_p * 4)(*[c.h for c in outputs])
        tp = (ctypes.c_void_p * len(taps))(*[c.h for c in taps])
        _check(capi.hck_vital_eval_taps(self.h, ctypes.addressof(plan), re, im, gks, rlk, outs,
                                        tp))
        return outputs, taps

    def vital_frames_required_steps(self, plan: VitalPlan) -> list[int]:
        n = ctypes.c_uint32()
        _check(capi.hck_vital_frames_required_steps(self.h, ctypes.addressof(plan), None, 0,
                                                    ctypes.byref(n)))
        buf = (ctypes.c_int32 * max(1, n.value))()
        _check(capi.hck_vital_frames_required_steps(self.h, ctypes.addressof(plan), buf, n.value,
                                                    ctypes.byref(n)))
        return list(buf[: n.value])

    def vital_eval_frames(self, plan: VitalPlan, res, ims, gks, rlk, outputs=None):
        """The pipeline on per-frame packing: res[t], ims[t] hold frame t's
        range bins in slots 0 .. R-1; the four outputs as vital_eval."""
        f = len(res)
        if len(ims) != f:
            raise ValueError("one imaginary ciphertext per frame")
        outputs = [self.ciphertext() for _ in range(4)] if outputs is None else outputs
        a = (ctypes.c_void_p * f)(*[c.h for c in res])
        b = (ctypes.c_void_p * f)(*[c.h for c in ims])
        o = (ctypes.c_void_p * 4)(*[c.h for c in outputs])
        _check(capi.hck_vital_eval_frames(self.h, ctypes.addressof(plan), a, b, f, gks, rlk, o))
        return outputs

    def vital_eval_many(self, plan: VitalPlan, res, ims, gks, rlk, outputs=None):
        """Several windows together; returns one list of 4 outputs per window."""
        n = len(res)
        if len(ims) != n:
            raise ValueError("one imaginary ciphertext per window")
        outputs = ([self.ciphertext() for _ in range(4 * n)] if outputs is None
                   else [c for w in outputs for c in w])
        a = (ctypes.c_void_p * n)(*[c.h for c in res])
        b = (ctypes.c_void_p * n)(*[c.h for c in ims])
        o = (ctypes.c_void_p * (4 * n))(*[c.h for c in outputs])
        _check(capi.hck_vital_eval_many(self.h, ctypes.addressof(plan), a, b, n, gks, rlk, o))
        return [outputs[4 * k: 4 * k + 4] for k in range(n)]

    # --- gesture-classification pipeline ---
    def gesture_required_steps(self, plan: GesturePlan) -> list:
        n = ctypes.c_uint32()
        _check(capi.hck_gesture_required_steps(self.h, ctypes.addressof(plan), None, 0,
                                               ctypes.byref(n)))
        buf = (ctypes.c_int32 * max(1, n.value))()
        _check(capi.hck_gesture_required_steps(self.h, ctypes.addressof(plan), buf, n.value,
                                               ctypes.byref(n)))
        return list(buf[: n.value])

    def gesture_eval(self, plan: GesturePlan, re, im, gks, rlk, out=None):
        """The logits ciphertext (slots 0 .. classes-1)."""
        out = self._out(out)
        _check(capi.hck_gesture_eval(self.h, ctypes.addressof(plan), re, im, gks, rlk, out))
        return out

    def gesture_eval_frames(self, plan: GesturePlan, res, ims, gks, rlk, out=None):
        """The logits from per-frame packing: res[f], ims[f] hold frame f in
        slots r D + c (zeros elsewhere)."""
        n = len(res)
        if len(ims) != n:
            raise ValueError("one imaginary ciphertext per frame")
        out = self._out(out)
        a = (ctypes.c_void_p * max(1, n))(*[c.h for c in res])
        b = (ctypes.c_void_p * max(1, n))(*[c.h for c in ims])
        _check(capi.hck_gesture_eval_frames(self.h, ctypes.addressof(plan), a, b, n, gks, rlk,
                                            out))
        return out

    def gesture_cnn_required_steps(self, plan: GestureCnnPlan) -> list[int]:
        n = ctypes.c_uint32()
        _check(capi.hck_gesture_cnn_required_steps(self.h, ctypes.addressof(plan), None, 0,
                                                   ctypes.byref(n)))
        buf = (ctypes.c_int32 * max(1, n.value))()
        _check(capi.hck_gesture_cnn_required_steps(self.h, ctypes.addressof(plan), buf, n.value,
                                                   ctypes.byref(n)))
        return list(buf[: n.value])

    GESTURE_CNN_TAPS = ("feature", "conv1 + act", "conv2 + act", "dense1 + act")

    def gesture_cnn_eval(self, plan: GestureCnnPlan, re, im, gks, rlk, out=None, taps=False):
        """The CNN variant's logits (slots 0 .. classes-1); with taps=True,
        (logits, [feature, conv1 + act, conv2 + act, dense1 + act])."""
        out = self._out(out)
        if taps:
            ts = [self.ciphertext() for _ in self.GESTURE_CNN_TAPS]
            arr = (ctypes.c_void_p * len(ts))(*[t.h for t in ts])
            _check(capi.hck_gesture_cnn_eval(self.h, ctypes.addressof(plan), re, im, gks, rlk,
                                             out, arr))
            return out, ts
        _check(capi.hck_gesture_cnn_eval(self.h, ctypes.addressof(plan), re, im, gks, rlk, out,
                                         None))
        return out

    GESTURE_TAPS = ("K3 d_re", "K3 d_im", "K1 power", "K6 notch", "K2 P^4", "K2 feature",
                    "FC1", "FC2")

    def gesture_eval_taps(self, plan: GesturePlan, re, im, gks, rlk):
        """(logits, taps): hck_gesture_eval's output and the stages'
        intermediate ciphertexts, in the order of GESTURE_TAPS."""
        out = self.ciphertext()
        taps = [self.ciphertext() for _ in self.GESTURE_TAPS]
        tp = (ctypes.c_void_p * len(taps))(*[c.h for c in taps])
        _check(capi.hck_gesture_eval_taps(self.h, ctypes.addressof(plan), re, im, gks, rlk,
                                          out, tp))
        return out, taps

    def autotune_keyswitch(self, levels=None, count: int = 32) -> dict:
        """Times key-switch batch sizes at each level (all by default) and
        keeps the fastest; returns {level: (batch size, microseconds per key
        switch)}."""
        lv = np.ascontiguousarray(np.asarray(range(self.L) if levels is None else levels,
                                             dtype=np.uint32))
        caps = np.zeros(len(lv), dtype=np.uint32)
        us = np.zeros(len(lv), dtype=np.float64)
        _check(capi.hck_autotune_keyswitch(self.h, _ptr(lv), len(lv), count, _ptr(caps),
                                           _ptr(us)))
        return {int(l): (int(c), float(u)) for l, c, u in zip(lv, caps, us)}

    def autotune_ntt(self, rows: int = 64) -> dict:
        """Times the candidate NTT splits of the full transforms and keeps the
        fastest; returns {"splits": {log2 R1: us per row}, "chosen": log2 R1}."""
        sp = np.zeros(3, dtype=np.int32)
        us = np.zeros(3, dtype=np.float64)
        n = ctypes.c_uint32()
        ch = ctypes.c_int32()
        _check(capi.hck_autotune_ntt(self.h, rows, _ptr(sp), _ptr(us), 3, ctypes.byref(n),
                                     ctypes.byref(ch)))
        return {"splits": {int(a): float(u) for a, u in zip(sp[:n.value], us[:n.value])},
                "chosen": ch.value}

    def set_ntt_split(self, log_r1: int):
        _check(capi.hck_set_ntt_split(self.h, log_r1))

    def ntt_split(self) -> int:
        v = ctypes.c_int32()
        _check(capi.hck_ntt_split(self.h, ctypes.byref(v)))
        return v.value

    def set_keyswitch_cap(self, level: int, cap: int):
        _check(capi.hck_set_keyswitch_cap(self.h, level, cap))

    def keyswitch_batch_limit(self, level: int) -> int:
        c = ctypes.c_uint32()
        _check(capi.hck_keyswitch_batch_limit(self.h, level, ctypes.byref(c)))
        return c.value

    def measure_mulmod_rate(self) -> float:
        """Sustained 64-bit Shoup modular products per second on this device (T/s)."""
        r = ctypes.c_double()
        _check(capi.hck_measure_mulmod_rate(self.h, ctypes.byref(r)))
        return r.value

    # --- kernel timing ---
    def timing(self, on: bool):
        _check(capi.hck_timing_enable(self.h, 1 if on else 0))

    def timing_reset(self):
        _check(capi.hck_timing_reset(self.h))

    def timing_read(self, name: str) -> dict:
        """Summed duration (ms), launches, algorithmic bytes and modular
        multiplications of one kernel since the last reset."""
        ms, cnt, by, mm = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_double(), ctypes.c_double()
        _check(capi.hck_timing_read(self.h, name.encode(), ctypes.byref(ms), ctypes.byref(cnt),
                                    ctypes.byref(by), ctypes.byref(mm)))
        return dict(ms=ms.value, launches=cnt.value, bytes=by.value, mulmods=mm.value)

    def timing_names(self) -> list[str]:
        buf = ctypes.create_string_buffer(4096)
        _check(capi.hck_timing_names(self.h, buf, 4096))
        return [x for x in buf.value.decode().split(",") if x]

    # --- launch trace (data obliviousness) ---
    def trace(self, on: bool):
        """Starts (clearing the log) or stops the launch trace."""
        _check(capi.hck_trace_enable(self.h, 1 if on else 0))

    def trace_read(self) -> list[tuple]:
        """The trace records in issue order: (name, (gx, gy, gz), bytes, mulmods)."""
        n = ctypes.c_size_t()
        _check(capi.hck_trace_read(self.h, None, 0, ctypes.byref(n)))
        recs = (TraceRecord * max(1, n.value))()
        _check(capi.hck_trace_read(self.h, recs, n.value, ctypes.byref(n)))
        return [(r.name.decode(), tuple(r.grid), r.bytes, r.mulmods) for r in recs[:n.value]]


# --- serving runtime -----------------------------------------------------

SERVE_VITAL, SERVE_GESTURE = 1, 2


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", _U64), ("max_batch", _U32), ("max_inflight", _U32)]


class ServerResult(ctypes.Structure):
    _fields_ = [("request", _U64), ("status", _I32), ("tenant", _U32), ("n_out", _U32),
                ("batch", _U32), ("key_load", _U32), ("out_level", _U32 * 4),
                ("out_scale", _D * 4),
                ("t_submit", _D), ("t_admit", _D), ("t_launch", _D), ("t_done", _D)]


class ServerStats(ctypes.Structure):
    _fields_ = [(name, _U64) for name in (
        "budget", "resident_bytes", "tenants", "submitted", "completed", "failed", "pending",
        "batches", "windows", "key_loads", "evictions", "key_bytes_loaded")]


class Server:
    """hck_server: continuous batching of encrypted windows from many tenants.
    While it exists, the context belongs to its worker thread: use only the
    server's methods until close()."""

    def __init__(self, ctx: Context, hbm_budget: int, max_batch: int = 8,
                 max_inflight: int = 16):
        self.ctx = ctx
        cfg = ServerConfig(hbm_budget, max_batch, max_inflight)
        h = ctypes.c_void_p()
        _check(capi.hck_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h.value
        self._fin = weakref.finalize(self, capi.hck_server_destroy, self.h)
        self._keep = {}         # tenants' plans and key words
        self._out = {}          # request -> output buffer

    def add_tenant(self, tenant: int, kind: int, plan, steps, gk_words, rlk_words):
        """gk_words[i]: exported words of the key of steps[i] (kept alive, and
        read again whenever the tenant's keys are loaded)."""
        st = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
        gk = [w if isinstance(w, np.ndarray) else np.asarray(w) for w in gk_words]
        for w in gk + [rlk_words]:
            if w.dtype != np.uint64 or not w.flags["C_CONTIGUOUS"]:
                raise ValueError("key words must be C-contiguous uint64 arrays")
        ptrs = (ctypes.c_void_p * max(1, len(gk)))(*[w.ctypes.data for w in gk])
        _check(capi.hck_server_add_tenant(self.h, tenant, kind, ctypes.addressof(plan),
                                          _ptr(st), ptrs, len(gk), rlk_words.ctypes.data))
        self._keep[tenant] = (kind, plan, st, gk, rlk_words, ptrs)

    def submit(self, request: int, tenant: int, re_words, im_words, level: int, scale: float):
        re = _u64(re_words)
        im = _u64(im_words)
        n_out = 1 if self._keep.get(tenant, (SERVE_VITAL,))[0] == SERVE_GESTURE else 4
        out = np.empty(n_out * 2 * self.ctx.L * self.ctx.n, dtype=np.uint64)
        rc = capi.hck_server_submit(self.h, request, tenant, _ptr(re), _ptr(im), level, scale,
                                    _ptr(out), out.size)
        _check(rc)
        self._out[request] = out    # the server writes it when the request completes

    def poll(self, timeout_ms: int = 0, cap: int = 64) -> list:
        """Completed requests: dicts with the result record and 'outputs', the
        output ciphertexts' words ([2][level+1][N] each)."""
        buf = (ServerResult * cap)()
        n = ctypes.c_uint32()
        _check(capi.hck_server_poll(self.h, timeout_ms, buf, cap, ctypes.byref(n)))
        done = []
        for r in buf[: n.value]:
            words = self._out.pop(r.request)
            outs, off = [], 0
            if r.status == 0:
                for i in range(r.n_out):
                    size = 2 * (r.out_level[i] + 1) * self.ctx.n
                    outs.append(words[off: off + size].reshape(2, r.out_level[i] + 1,
                                                               self.ctx.n).copy())
                    off += size
            done.append({"request": r.request, "status": r.status, "tenant": r.tenant,
                         "batch": r.batch, "key_load": bool(r.key_load),
                         "levels": list(r.out_level[: r.n_out]),
                         "scales": list(r.out_scale[: r.n_out]), "t_submit": r.t_submit,
                         "t_admit": r.t_admit, "t_launch": r.t_launch, "t_done": r.t_done,
                         "outputs": outs})
        return done

    def stats(self) -> dict:
        st = ServerStats()
        _check(capi.hck_server_stats_get(self.h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if self._fin is not None:
            self._fin()
            self._fin = None
        self.h = None
