"""The gesture classifier's CNN variant composed from the oracle's
ciphertext operations: the front end of the paper's gesture pipeline
(section 3.3.3: K3 Doppler DFT -> K1 power -> K6 notch -> K2 soft attention,
frame accumulation), then two 3 x 3 convolutions with stride 2 and zero
padding, 2 x 2 average pooling and two dense layers, with a degree-3
polynomial activation after both convolutions and the first dense layer.

TEST INFRASTRUCTURE ONLY: this module is the reference the GPU pipeline is
checked against.  Nothing in the product path imports it.

Packing (N/2 slots, B = N/2 / (R D) blocks of R D slots; feature (r, c) of a
block at slot r D + c).  After the frame accumulation every block holds the
R x D feature map.
  conv1  block b computes output channel b mod C1 at the positions (r, c),
         both even, of the stride-2 output grid: the generalized diagonal of
         offset dy D + dx carries w1[b mod C1][dy][dx] where (r + dy, c + dx)
         lies inside the map, zero elsewhere (9 diagonals, baby step D).
  act    slot-wise degree-3 polynomial (Oracle.poly_eval).
  conv2  block b computes channel o = b mod C2 at positions (r, c), both
         multiples of 4, from input channel (b + delta) mod C1 of block
         b + delta: offset delta R D + 2 (dy D + dx), delta < C1 (9 C1
         diagonals, baby step R D: the baby rotations shift inside the map,
         the giant ones move channels between blocks).
  act
  dense1 the pooling folded into W1: W''[u][o R D + r D + c] = W1[u][o, i, j]
         / 4 for r = 4 (2i + a), c = 4 (2j + b), a, b < 2.  The hybrid
         diagonal method over the period C2 R D of the replicated channels:
         diag_k[j] = W''[j mod H][(j + k) mod C2 R D] for j < C2 R D, k < H,
         then rotations H, 2H, ..., C2 R D / 2 sum the sub-blocks: y[u] in
         slot u.  Plus bias1.
  act
  dense2 logits = W2 y + b2 by the rectangular diagonals of W2 (slots 0 .. classes-1).
Levels (input level l0, degree-3 activations of 3 levels each): feature
l0-6, conv1 l0-7, act l0-10, conv2 l0-11, act l0-14, dense1 l0-15, act l0-18,
dense2 l0-19.
"""
from __future__ import annotations

import numpy as np

from . import Oracle
from .gesture import _front_end, _rect_diagonals, _spread, operand_vectors as _fe_vectors

BABY_DENSE1 = 8
BABY_DENSE2 = 10


def _blocks(cfg: dict, n_slots: int) -> int:
    return n_slots // (cfg["bins"] * cfg["chirps"])


def check_layout(cfg: dict, n_slots: int):
    r, d = cfg["bins"], cfg["chirps"]
    c1, c2 = cfg["conv1"].shape[0], cfg["conv2"].shape[0]
    h = cfg["dense1"].shape[0]
    t2 = 1 << max(0, (cfg["frames"] - 1).bit_length())
    if t2 * r * d != n_slots:
        raise ValueError("pow2(frames) x bins x chirps must fill the slots")
    if r % 8 or d % 8:
        raise ValueError("bins and chirps must be multiples of 8")
    b = _blocks(cfg, n_slots)
    if b % c1 or b % c2:
        raise ValueError("the block count must be a multiple of both channel counts")
    period = c2 * r * d
    if period % h or (period // h) & (period // h - 1):
        raise ValueError("c2 bins chirps / hidden must be a power of two")


def operand_vectors(cfg: dict, n_slots: int) -> dict:
    """Public operands as real slot vectors (front end as the FC pipeline's)
    and diagonal dicts offset -> vector."""
    check_layout(cfg, n_slots)
    r_, d_ = cfg["bins"], cfg["chirps"]
    rd = r_ * d_
    fe = _fe_vectors(_fc_shaped(cfg), n_slots)
    v = {k: fe[k] for k in ("dft_c", "dft_s", "notch")}
    slots = np.arange(n_slots)
    blk, pos = slots // rd, slots % rd
    row, col = pos // d_, pos % d_
    w1, w2 = cfg["conv1"], cfg["conv2"]
    c1, c2 = w1.shape[0], w2.shape[0]
    conv1 = {}
    on1 = (row % 2 == 0) & (col % 2 == 0)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            inside = (row + dy >= 0) & (row + dy < r_) & (col + dx >= 0) & (col + dx < d_)
            vec = np.where(on1 & inside, w1[blk % c1, dy + 1, dx + 1], 0.0)
            if np.any(vec):
                conv1[(dy * d_ + dx) % n_slots] = vec
    v["conv1"] = conv1
    conv2 = {}
    on2 = (row % 4 == 0) & (col % 4 == 0)
    for delta in range(c1):
        cin = (blk + delta) % c1
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                inside = ((row + 2 * dy >= 0) & (row + 2 * dy < r_) &
                          (col + 2 * dx >= 0) & (col + 2 * dx < d_))
                vec = np.where(on2 & inside, w2[blk % c2, cin, dy + 1, dx + 1], 0.0)
                if np.any(vec):
                    conv2[(delta * rd + 2 * (dy * d_ + dx)) % n_slots] = vec
    v["conv2"] = conv2
    # dense1 with the 2 x 2 average pooling folded in, over one period of
    # c2 blocks
    wd1 = cfg["dense1"]
    h = wd1.shape[0]
    period = c2 * rd
    ph, pw = r_ // 8, d_ // 8
    wfull = np.zeros((h, period))
    for o in range(c2):
        for i in range(ph):
            for j in range(pw):
                col_w = wd1[:, (o * ph + i) * pw + j] / 4.0
                for a in (0, 1):
                    for b in (0, 1):
                        m = o * rd + 4 * (2 * i + a) * d_ + 4 * (2 * j + b)
                        wfull[:, m] = col_w
    jj = np.arange(period)
    dense1 = {}
    for k in range(h):
        vec = np.zeros(n_slots)
        vec[:period] = wfull[jj % h, (jj + k) % period]
        if np.any(vec):
            dense1[k] = vec
    v["dense1"] = dense1
    v["dense2"] = _rect_diagonals(cfg["dense2"], n_slots)
    for name in ("bias1", "bias2"):
        vec = np.zeros(n_slots)
        vec[: len(cfg[name])] = cfg[name]
        v[name] = vec
    return v


def _fc_shaped(cfg: dict) -> dict:
    """The FC pipeline's configuration fields the front end reads (its FC
    weights only satisfy the layout check)."""
    rd = cfg["bins"] * cfg["chirps"]
    return dict(frames=cfg["frames"], bins=cfg["bins"], chirps=cfg["chirps"],
                window=cfg["window"], notch=cfg["notch"],
                weights=[np.zeros((rd, rd)), np.zeros((1, rd)), np.zeros((1, 1))],
                biases=[np.zeros(rd), np.zeros(1), np.zeros(1)])


def act_depth(coeffs) -> int:
    """Levels one activation consumes (Oracle.poly_eval: ceil(log2 d) + 1)."""
    return (len(coeffs) - 2).bit_length() + 1


def levels(level0: int, coeffs) -> dict:
    """Level of each stage's input (its plaintext operands' level)."""
    a = act_depth(coeffs)
    return {"dft": level0, "notch": level0 - 2, "conv1": level0 - 6,
            "conv2": level0 - 7 - a, "dense1": level0 - 8 - 2 * a,
            "bias1": level0 - 9 - 2 * a, "dense2": level0 - 9 - 3 * a,
            "bias2": level0 - 10 - 3 * a, "out": level0 - 10 - 3 * a}


def baby_steps(cfg: dict) -> dict:
    return {"conv1": cfg["chirps"], "conv2": cfg["bins"] * cfg["chirps"],
            "dense1": BABY_DENSE1, "dense2": BABY_DENSE2}


def bias_scales(o: Oracle, level0: int, scale0: float, coeffs) -> list:
    """Scale of the ciphertext each bias is added to, by the scale arithmetic
    of the operations in order (plaintext factors at scale q_level; a
    polynomial's result carries its first nonzero term's scale)."""
    q = [float(v) for v in o.q]
    lv = levels(level0, coeffs)
    s = scale0 * q[level0] / q[level0]                       # K3
    s = s * s / q[level0 - 1]                                # K1
    s = s * q[level0 - 2] / q[level0 - 2]                    # K6
    s2 = s * s / q[level0 - 3]
    s4 = s2 * s2 / q[level0 - 4]
    s = s * s4 / q[level0 - 5]                               # feature, level l0-6

    def lt(s, lvl):
        return s * q[lvl] / q[lvl]

    def act(s, lvl):
        # powers x^k at level lvl - ceil(log2 k): x^a x^(k-a), a the largest
        # power of two below k, rescaled by the prime of their common level
        d = len(coeffs) - 1
        lf = lvl - act_depth(coeffs)
        ps = {1: (s, lvl)}
        for k in range(2, d + 1):
            a = 1 << ((k - 1).bit_length() - 1)
            (sa, la), (sb, lb) = ps[a], ps[k - a]
            lm = min(la, lb)
            ps[k] = (sa * sb / q[lm], lm - 1)
        k = min(i for i in range(1, d + 1) if coeffs[i] != 0)
        sk = ps[k][0]
        return sk * (s * q[lf + 1] / sk) / q[lf + 1]

    s = act(lt(s, lv["conv1"]), lv["conv1"] - 1)
    s = act(lt(s, lv["conv2"]), lv["conv2"] - 1)
    s = lt(s, lv["dense1"])
    out = [s]
    s = lt(act(s, lv["bias1"]), lv["dense2"])
    out.append(s)
    return out


def encode_operands(o: Oracle, cfg: dict, level0: int, scale0: float,
                    vecs: dict | None = None) -> dict:
    vecs = operand_vectors(cfg, o.n_slots) if vecs is None else vecs
    lv = levels(level0, cfg["act"])
    bs = baby_steps(cfg)
    ops = {"dft_c": o.lt_create(vecs["dft_c"], 8, lv["dft"]),
           "dft_s": o.lt_create(vecs["dft_s"], 8, lv["dft"]),
           "notch": o.encode(vecs["notch"], float(o.q[lv["notch"]]), lv["notch"])}
    for name in ("conv1", "conv2", "dense1", "dense2"):
        ops[name] = o.lt_create(vecs[name], bs[name], lv[name])
    for i, s in enumerate(bias_scales(o, level0, scale0, cfg["act"])):
        name = f"bias{i + 1}"
        ops[name] = o.encode(vecs[name], s, lv[name])
    return ops


def required_steps(o: Oracle, cfg: dict, ops: dict) -> list:
    rd = cfg["bins"] * cfg["chirps"]
    t2 = 1 << max(0, (cfg["frames"] - 1).bit_length())
    period = cfg["conv2"].shape[0] * rd
    h = cfg["dense1"].shape[0]
    steps = {rd * (1 << i) for i in range(t2.bit_length() - 1)}
    steps |= {h * (1 << i) for i in range((period // h).bit_length() - 1)}
    for name in ("dft_c", "dft_s", "conv1", "conv2", "dense1", "dense2"):
        steps |= set(o.lt_required_steps(ops[name]))
    return sorted(steps)


def _lt(o: Oracle, lt, x, gks):
    return o.rescale(o.lt_eval([x], [(lt, 0, 0, 1)], gks, 1, hoist=True, hoist_giant=True)[0])


def evaluate(o: Oracle, cfg: dict, ops: dict, re, im, gks: dict, rlk, taps: list | None = None):
    """The CNN classifier on one window (batched packing): the logits in
    slots 0 .. classes-1.  taps (a list) receives the intermediates: the
    accumulated feature map, conv1 + act, conv2 + act, dense1 + bias + act."""
    check_layout(cfg, o.n_slots)
    act = cfg["act"]
    rd = cfg["bins"] * cfg["chirps"]
    period = cfg["conv2"].shape[0] * rd
    h = cfg["dense1"].shape[0]
    tap = taps.append if taps is not None else (lambda c: None)
    feat = _spread(o, cfg, _front_end(o, ops, re, im, gks, rlk), gks)
    tap(feat)
    x = o.poly_eval(_lt(o, ops["conv1"], feat, gks), act, rlk)
    tap(x)
    x = o.poly_eval(_lt(o, ops["conv2"], x, gks), act, rlk)
    tap(x)
    y = _lt(o, ops["dense1"], x, gks)
    s = h
    while s < period:
        y = o.add(y, o.rotate(y, s, gks))
        s *= 2
    y = o.poly_eval(o.add_plain(y, ops["bias1"]), act, rlk)
    tap(y)
    return o.add_plain(_lt(o, ops["dense2"], y, gks), ops["bias2"])


def _act(coeffs, x):
    return sum(c * x ** k for k, c in enumerate(coeffs))


def plain_stages(cfg: dict, x: np.ndarray) -> dict:
    """The same network on plaintext numbers by its definition (direct
    convolution loops; x: [frames][bins][chirps] complex): the feature map
    [bins][chirps], a1 [c1][bins/2][chirps/2], a2 [c2][bins/4][chirps/4], a3
    [hidden] and the logits."""
    d = cfg["chirps"]
    n = np.arange(d)
    win = np.asarray(cfg["window"])
    sig = (n + d // 2) % d
    wmat = win[None, :] * np.exp(-2j * np.pi * np.outer(sig, n) / d) / win.sum()
    p = np.abs(np.einsum("kn,frn->frk", wmat, x)) ** 2
    mask = np.ones(d)
    mask[list(cfg["notch"])] = 0.0
    p = p * mask
    feat = (p * p ** 4).sum(axis=0)

    def conv(img, w):                                   # img [cin][H][W], w [cout][cin][3][3]
        cin, hh, ww = img.shape
        out = np.zeros((w.shape[0], hh // 2, ww // 2))
        for o_ in range(w.shape[0]):
            for i in range(hh // 2):
                for j in range(ww // 2):
                    acc = 0.0
                    for c in range(cin):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                y_, x_ = 2 * i + dy, 2 * j + dx
                                if 0 <= y_ < hh and 0 <= x_ < ww:
                                    acc += w[o_, c, dy + 1, dx + 1] * img[c, y_, x_]
                    out[o_, i, j] = acc
        return out

    act = cfg["act"]
    a1 = _act(act, conv(feat[None], cfg["conv1"][:, None]))
    a2 = _act(act, conv(a1, cfg["conv2"]))
    c2, hh, ww = a2.shape
    pooled = a2.reshape(c2, hh // 2, 2, ww // 2, 2).mean(axis=(2, 4))
    a3 = _act(act, cfg["dense1"] @ pooled.reshape(-1) + cfg["bias1"])
    return {"feature": feat, "a1": a1, "a2": a2, "a3": a3,
            "logits": cfg["dense2"] @ a3 + cfg["bias2"]}


def plain(cfg: dict, x: np.ndarray) -> np.ndarray:
    return plain_stages(cfg, x)["logits"]


def stage_slots(cfg: dict, n_slots: int, stages: dict) -> list:
    """plain_stages' values at the slots where the taps of evaluate() hold
    them: a list (per tap) of (slot indices, values)."""
    r_, d_ = cfg["bins"], cfg["chirps"]
    rd = r_ * d_
    blocks = n_slots // rd
    out = []
    idx = np.arange(rd)
    out.append((idx, stages["feature"].reshape(-1)))
    for name, stride in (("a1", 2), ("a2", 4)):
        a = stages[name]
        c = a.shape[0]
        sl, va = [], []
        for b in range(blocks):
            for i in range(a.shape[1]):
                for j in range(a.shape[2]):
                    sl.append(b * rd + stride * i * d_ + stride * j)
                    va.append(a[b % c, i, j])
        out.append((np.array(sl), np.array(va)))
    out.append((np.arange(len(stages["a3"])), stages["a3"]))
    return out
