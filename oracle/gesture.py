"""The paper's encrypted gesture-classification pipeline (section 3.3.3,
example pipelines: K3 -> K1 -> K2 + K6, frame accumulation, then
FC1 -> x^2 -> FC2 -> x^2 -> FC3; the depth accounting of Table 1) composed
from the oracle's ciphertext operations.

TEST INFRASTRUCTURE ONLY: this module is the reference the GPU pipeline is
checked against.  Nothing in the product path imports it.

Slot layout: frame t, range bin r and chirp c sit in slot (t R + r) D + c,
F frames, zero beyond; T2 is the power of two >= F and T2 R D = N/2 (the
frame sum then leaves the accumulated map in every block of R D slots).
Stages and the level each ends at (input level l0):

  K3  Doppler DFT of every (frame, range) block of D chirps: d_re = C v_re -
      S v_im, d_im = S v_re + C v_im with C + jS = I (x) W_D (Eq. dft_re,
      windowed fftshifted DFT; BSGS, hoisted baby steps, one ModDown per
      output; l0-1)
  K1  P = d_re^2 + d_im^2 (l0-2)
  K6  notch: P m with m = 0 on the notch Doppler bins (l0-3)
  K2  w = P^4 (gamma = 4, two squarings; l0-5); feature = P w (l0-6)
      frame accumulation: rotations R D, 2 R D, ... (depth 0)
  FC1 y = W1 x + b1 (x: the R D features, cyclic in every block): the H1
      diagonals diag_k[j] = W1[j mod H1][(j + k) mod RD] (j < RD) over
      offsets 0..H1-1, then a sum of the RD / H1 blocks of H1 slots by
      rotations H1, 2 H1, ...; square (l0-7, l0-8)
  FC2 y = W2 h + b2 by the rectangular generalized diagonals
      diag_d[i] = W2[i][i + d]; square (l0-9, l0-10)
  FC3 logits = W3 h + b3 (l0-11), in slots 0 .. classes-1.
"""
from __future__ import annotations

import numpy as np

from . import Ciphertext, Oracle

DEPTH = 11


def _pow2_at_least(x: int) -> int:
    p = 1
    while p < x:
        p *= 2
    return p


def check_layout(cfg: dict, n_slots: int):
    f, r, d = cfg["frames"], cfg["bins"], cfg["chirps"]
    h1 = cfg["weights"][0].shape[0]
    if _pow2_at_least(f) * r * d != n_slots:
        raise ValueError("pow2(frames) x bins x chirps must fill the slots")
    if (r * d) % h1 or (r * d // h1) & (r * d // h1 - 1):
        raise ValueError("FC1 outputs must divide the feature count by a power of two")


def _rect_diagonals(w: np.ndarray, n_slots: int) -> dict:
    """Generalized diagonals diag_d[i] = W[i][i + d] of a rows x cols block at
    slot 0 (zero elsewhere), offsets -(rows-1) .. cols-1."""
    rows, cols = w.shape
    out = {}
    for d in range(-(rows - 1), cols):
        v = np.zeros(n_slots)
        for i in range(rows):
            if 0 <= i + d < cols:
                v[i] = w[i, i + d]
        if np.any(v):
            out[d % n_slots] = v
    return out


def operand_vectors(cfg: dict, n_slots: int) -> dict:
    """Real slot vectors / diagonal dicts of every public operand."""
    check_layout(cfg, n_slots)
    r, d = cfg["bins"], cfg["chirps"]
    rd = r * d
    n = np.arange(d)
    win = np.asarray(cfg["window"])
    sig = (n + d // 2) % d
    wmat = win[None, :] * np.exp(-2j * np.pi * np.outer(sig, n) / d) / win.sum()
    v = {}
    for part, mat in (("dft_c", wmat.real), ("dft_s", wmat.imag)):
        diags = {}
        for k in range(-(d - 1), d):
            blk = np.zeros(d)
            for i in range(d):
                if 0 <= i + k < d:
                    blk[i] = mat[i, i + k]
            if np.any(blk):
                diags[k % n_slots] = np.tile(blk, n_slots // d)
        v[part] = diags
    mask = np.ones(n_slots)
    for b in cfg["notch"]:
        mask[b::d] = 0.0
    v["notch"] = mask
    w1, w2, w3 = cfg["weights"]
    h1 = w1.shape[0]
    fc1 = {}
    j = np.arange(rd)
    for k in range(h1):
        vec = np.zeros(n_slots)
        vec[:rd] = w1[j % h1, (j + k) % rd]
        fc1[k] = vec
    v["fc1"] = fc1
    v["fc2"] = _rect_diagonals(w2, n_slots)
    v["fc3"] = _rect_diagonals(w3, n_slots)
    for i, b in enumerate(cfg["biases"]):
        vec = np.zeros(n_slots)
        vec[: len(b)] = b
        v[f"bias{i + 1}"] = vec
    return v


def levels(level0: int) -> dict:
    return {"dft": level0, "notch": level0 - 2, "fc1": level0 - 6, "fc2": level0 - 8,
            "fc3": level0 - 10, "out": level0 - 11}


BABY = {"dft_c": 8, "dft_s": 8, "fc1": 8, "fc2": 10, "fc3": 6}


def bias_scales(o: Oracle, level0: int, scale0: float) -> list:
    """Scale of the ciphertext each bias is added to, following the scale
    arithmetic of the operations in order (products multiply scales, rescale
    divides by the dropped prime; plaintext factors are encoded at q_level)."""
    q = o.q
    s = scale0 * float(q[level0]) / float(q[level0])        # K3
    s = s * s / float(q[level0 - 1])                       # K1
    s = s * float(q[level0 - 2]) / float(q[level0 - 2])    # K6
    s2 = s * s / float(q[level0 - 3])                      # P^2
    s4 = s2 * s2 / float(q[level0 - 4])                    # P^4
    s = s * s4 / float(q[level0 - 5])                      # P w
    out = []
    s = s * float(q[level0 - 6]) / float(q[level0 - 6])    # FC1
    out.append(s)
    s = s * s / float(q[level0 - 7])                       # square
    s = s * float(q[level0 - 8]) / float(q[level0 - 8])    # FC2
    out.append(s)
    s = s * s / float(q[level0 - 9])                       # square
    s = s * float(q[level0 - 10]) / float(q[level0 - 10])  # FC3
    out.append(s)
    return out


def encode_operands(o: Oracle, cfg: dict, level0: int, scale0: float,
                    vecs: dict | None = None) -> dict:
    vecs = operand_vectors(cfg, o.n_slots) if vecs is None else vecs
    lv = levels(level0)
    ops = {}
    for name, lvl in (("dft_c", lv["dft"]), ("dft_s", lv["dft"]), ("fc1", lv["fc1"]),
                      ("fc2", lv["fc2"]), ("fc3", lv["fc3"])):
        ops[name] = o.lt_create(vecs[name], BABY[name], lvl)
    ops["notch"] = o.encode(vecs["notch"], float(o.q[lv["notch"]]), lv["notch"])
    for i, (s, lvl) in enumerate(zip(bias_scales(o, level0, scale0),
                                     (lv["fc1"] - 1, lv["fc2"] - 1, lv["fc3"] - 1))):
        ops[f"bias{i + 1}"] = o.encode(vecs[f"bias{i + 1}"], s, lvl)
    return ops


def required_steps(o: Oracle, cfg: dict, ops: dict) -> list:
    r, d = cfg["bins"], cfg["chirps"]
    rd = r * d
    t2 = _pow2_at_least(cfg["frames"])
    h1 = cfg["weights"][0].shape[0]
    steps = {rd * (1 << i) for i in range(t2.bit_length() - 1)}
    steps |= {h1 * (1 << i) for i in range((rd // h1).bit_length() - 1)}
    for name in ("dft_c", "dft_s", "fc1", "fc2", "fc3"):
        steps |= set(o.lt_required_steps(ops[name]))
    return sorted(steps)


def _mul(o, a, b, rlk):
    return o.rescale(o.relinearize(o.tensor(a, b), rlk))


def _front_end(o: Oracle, ops: dict, re: Ciphertext, im: Ciphertext, gks: dict,
               rlk) -> Ciphertext:
    """K3 -> K1 -> K6 -> K2 on one ciphertext pair: the feature P P^4 of
    every frame block it holds."""
    terms = [(ops["dft_c"], 0, 0, 1), (ops["dft_s"], 1, 0, -1), (ops["dft_s"], 0, 1, 1),
             (ops["dft_c"], 1, 1, 1)]
    d_re, d_im = (o.rescale(c) for c in o.lt_eval([re, im], terms, gks, 2, hoist=True,
                                                   hoist_giant=True))
    p = o.rescale(o.relinearize(o.add(o.tensor(d_re, d_re), o.tensor(d_im, d_im)), rlk))
    p = o.rescale(o.mul_plain(p, ops["notch"]))
    p2 = _mul(o, p, p, rlk)
    p4 = _mul(o, p2, p2, rlk)
    return _mul(o, o.drop_level(p, p4.level), p4, rlk)


def _spread(o: Oracle, cfg: dict, feat: Ciphertext, gks: dict) -> Ciphertext:
    """Adds the blocks of R D slots cyclically (rotations R D, 2 R D, ...): each
    block ends with the sum of all blocks."""
    rd = cfg["bins"] * cfg["chirps"]
    s = rd
    while s < o.n_slots:
        feat = o.add(feat, o.rotate(feat, s, gks))
        s *= 2
    return feat


def _fc_tail(o: Oracle, cfg: dict, ops: dict, feat: Ciphertext, gks: dict, rlk) -> Ciphertext:
    """FC1 -> x^2 -> FC2 -> x^2 -> FC3 on the features present in every block."""
    rd = cfg["bins"] * cfg["chirps"]
    h1 = cfg["weights"][0].shape[0]
    y = o.rescale(o.lt_eval([feat], [(ops["fc1"], 0, 0, 1)], gks, 1, hoist=True,
                            hoist_giant=True)[0])
    s = h1
    while s < rd:
        y = o.add(y, o.rotate(y, s, gks))
        s *= 2
    y = o.add_plain(y, ops["bias1"])
    h = _mul(o, y, y, rlk)
    y = o.rescale(o.lt_eval([h], [(ops["fc2"], 0, 0, 1)], gks, 1, hoist=True,
                            hoist_giant=True)[0])
    y = o.add_plain(y, ops["bias2"])
    h = _mul(o, y, y, rlk)
    y = o.rescale(o.lt_eval([h], [(ops["fc3"], 0, 0, 1)], gks, 1, hoist=True,
                            hoist_giant=True)[0])
    return o.add_plain(y, ops["bias3"])


def evaluate(o: Oracle, cfg: dict, ops: dict, re: Ciphertext, im: Ciphertext, gks: dict,
             rlk) -> Ciphertext:
    """Batched packing: all frames in one ciphertext pair; the frame sum is
    the block spreading itself (pow2(F) R D = N/2)."""
    check_layout(cfg, o.n_slots)
    feat = _front_end(o, ops, re, im, gks, rlk)
    return _fc_tail(o, cfg, ops, _spread(o, cfg, feat, gks), gks, rlk)


def evaluate_frames(o: Oracle, cfg: dict, ops: dict, res: list, ims: list, gks: dict,
                    rlk) -> Ciphertext:
    """Per-frame packing (section 3.3.2, one ciphertext pair per frame, frame
    f in slots r D + c): the front end on every pair, the features added in
    frame order, then spread to every block of R D slots for the FC network."""
    if not res or len(res) != len(ims):
        raise ValueError("one real and one imaginary ciphertext per frame")
    feat = None
    for re, im in zip(res, ims):
        f = _front_end(o, ops, re, im, gks, rlk)
        feat = f if feat is None else o.add(feat, f)
    return _fc_tail(o, cfg, ops, _spread(o, cfg, feat, gks), gks, rlk)


def plain(cfg: dict, x: np.ndarray) -> np.ndarray:
    """The same circuit on plaintext numbers (x: [frames][bins][chirps]
    complex): the logits."""
    d = cfg["chirps"]
    n = np.arange(d)
    win = np.asarray(cfg["window"])
    sig = (n + d // 2) % d
    wmat = win[None, :] * np.exp(-2j * np.pi * np.outer(sig, n) / d) / win.sum()
    spec = np.einsum("kn,frn->frk", wmat, x)
    p = np.abs(spec) ** 2
    mask = np.ones(d)
    mask[list(cfg["notch"])] = 0.0
    p = p * mask
    feat = (p * p ** 4).sum(axis=0).reshape(-1)
    w1, w2, w3 = cfg["weights"]
    b1, b2, b3 = cfg["biases"]
    h = (w1 @ feat + b1) ** 2
    h = (w2 @ h + b2) ** 2
    return w3 @ h + b3


def encrypt_window(o: Oracle, s, x: np.ndarray, level: int, scale: float, seed: int):
    v = np.zeros(o.n_slots, dtype=np.complex128)
    v[: x.size] = x.reshape(-1)
    return (o.encrypt_sk(s, o.encode(v.real, scale, level), seed),
            o.encrypt_sk(s, o.encode(v.imag, scale, level), seed + 1))


def encrypt_frames(o: Oracle, s, x: np.ndarray, level: int, scale: float, seed: int):
    """Per-frame packing of x [frames][bins][chirps]: frame f's real and
    imaginary parts in slots r D + c of their own ciphertexts (seeds
    seed + 2f, seed + 2f + 1)."""
    res, ims = [], []
    for f in range(x.shape[0]):
        v = np.zeros(o.n_slots, dtype=np.complex128)
        v[: x[f].size] = x[f].reshape(-1)
        res.append(o.encrypt_sk(s, o.encode(v.real, scale, level), seed + 2 * f))
        ims.append(o.encrypt_sk(s, o.encode(v.imag, scale, level), seed + 2 * f + 1))
    return res, ims
