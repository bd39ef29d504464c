"""Public operands of the gesture-classification pipeline
(hck_gesture_eval): the Doppler DFT's block-diagonal transforms, the notch
mask, and the FC layers' diagonals and biases for F frames x R range bins x
D chirps packed (t R + r) D + c, encoded with this library's encoder.

This is plaintext setup (the pipeline's public weights, section 3.3.3);
every homomorphic step runs in the library.
"""
import numpy as np

DEPTH = 11
BABY = {"dft_c": 8, "dft_s": 8, "fc1": 8, "fc2": 10, "fc3": 6}


def _shifted_dft(d: int, window) -> np.ndarray:
    n = np.arange(d)
    w = np.asarray(window, dtype=np.float64)
    rows = (n + d // 2) % d          # fftshift of the output bins
    return w[None, :] * np.exp(-2j * np.pi * np.outer(rows, n) / d) / w.sum()


def _diagonals(mat: np.ndarray, n_slots: int, tile: bool) -> dict:
    """Generalized diagonals diag_k[i] = M[i][i + k] of a rows x cols matrix
    at slot 0; with tile, repeated over every block of `rows` slots (a
    block-diagonal I (x) M over all slots)."""
    rows, cols = mat.shape
    i = np.arange(rows)
    out = {}
    for k in range(-(rows - 1), cols):
        ok = (i + k >= 0) & (i + k < cols)
        if not ok.any():
            continue
        blk = np.where(ok, mat[i, np.clip(i + k, 0, cols - 1)], 0.0)
        if not blk.any():
            continue
        vec = np.tile(blk, n_slots // rows) if tile else np.concatenate(
            [blk, np.zeros(n_slots - rows)])
        out[k % n_slots] = vec
    return out


def operand_vectors(cfg: dict, n_slots: int) -> dict:
    F, R, D = cfg["frames"], cfg["bins"], cfg["chirps"]
    RD = R * D
    if (1 << max(0, (F - 1).bit_length())) * RD != n_slots:
        raise ValueError("pow2(frames) x bins x chirps must equal the slot count")
    w1, w2, w3 = (np.asarray(w, dtype=np.float64) for w in cfg["weights"])
    H1 = w1.shape[0]
    dft = _shifted_dft(D, cfg["window"])
    out = {"dft_c": _diagonals(dft.real, n_slots, True),
           "dft_s": _diagonals(dft.imag, n_slots, True)}
    notch = np.ones(n_slots)
    for b in cfg["notch"]:
        notch[b::D] = 0.0
    out["notch"] = notch
    # FC1 over the cyclic feature vector: diag_k[j] = W1[j mod H1][(j + k) mod RD]
    j = np.arange(RD)
    out["fc1"] = {k: np.concatenate([w1[j % H1, (j + k) % RD], np.zeros(n_slots - RD)])
                  for k in range(H1)}
    out["fc2"] = _diagonals(w2, n_slots, False)
    out["fc3"] = _diagonals(w3, n_slots, False)
    for idx, b in enumerate(cfg["biases"], start=1):
        v = np.zeros(n_slots)
        v[: len(b)] = b
        out[f"bias{idx}"] = v
    return out


def scales_at_biases(q, level0: int, scale0: float) -> list:
    """Scale of the ciphertext at each bias addition, from the operations'
    scale arithmetic in order (plaintext factors encoded at q_level)."""
    q = [float(x) for x in q]

    def pt_rescale(s, lvl):
        return s * q[lvl] / q[lvl]

    def square_rescale(s, lvl):
        return s * s / q[lvl]

    s = pt_rescale(scale0, level0)                 # Doppler DFT
    s = square_rescale(s, level0 - 1)              # |.|^2
    s = pt_rescale(s, level0 - 2)                  # notch
    s2 = square_rescale(s, level0 - 3)
    s4 = square_rescale(s2, level0 - 4)
    s = s * s4 / q[level0 - 5]                     # P w
    out = []
    for k, lvl in enumerate((level0 - 6, level0 - 8, level0 - 10)):
        s = pt_rescale(s, lvl)
        out.append(s)
        if k < 2:
            s = square_rescale(s, lvl - 1)
    return out


def encode_plan(ctx, cfg: dict, level0: int, scale0: float, vectors: dict | None = None):
    from . import GesturePlan
    vec = operand_vectors(cfg, ctx.n // 2) if vectors is None else vectors
    q = ctx.q
    lv = {"dft_c": level0, "dft_s": level0, "fc1": level0 - 6, "fc2": level0 - 8,
          "fc3": level0 - 10}
    ops = {name: ctx.lt_create(vec[name], BABY[name], lvl) for name, lvl in lv.items()}
    ops["notch"] = ctx.encode(vec["notch"], float(q[level0 - 2]), level0 - 2)
    for idx, s in enumerate(scales_at_biases(q, level0, scale0), start=1):
        lvl = lv[f"fc{idx}"] - 1
        ops[f"bias{idx}"] = ctx.encode(vec[f"bias{idx}"], s, lvl)
    return GesturePlan.build(cfg["frames"], cfg["bins"], cfg["chirps"],
                             np.asarray(cfg["weights"][0]).shape[0], ops)


def plain_stages(cfg: dict, x: np.ndarray, n_slots: int) -> list:
    """Plaintext execution of the pipeline, the reference of the per-kernel
    encryption noise (section 5.2, Table 3).  For each tap of
    hck_gesture_eval_taps, then the logits: (slot indices, values) where the
    encrypted result holds them."""
    F, R, D = cfg["frames"], cfg["bins"], cfg["chirps"]
    if (1 << max(0, (F - 1).bit_length())) * R * D != n_slots:
        raise ValueError("pow2(frames) x bins x chirps must equal the slot count")
    dft = _shifted_dft(D, cfg["window"])
    spec = np.einsum("kn,frn->frk", dft, np.asarray(x))
    slots = np.arange(F * R * D)
    power = np.abs(spec) ** 2
    mask = np.ones(D)
    mask[list(cfg["notch"])] = 0.0
    notched = power * mask
    p4 = notched ** 4
    feat = (notched * p4).sum(axis=0).reshape(-1)
    w1, w2, w3 = (np.asarray(w, dtype=np.float64) for w in cfg["weights"])
    b1, b2, b3 = (np.asarray(b, dtype=np.float64) for b in cfg["biases"])
    y1 = w1 @ feat + b1
    y2 = w2 @ y1 ** 2 + b2
    y3 = w3 @ y2 ** 2 + b3
    return [(slots, spec.real.reshape(-1)), (slots, spec.imag.reshape(-1)),
            (slots, power.reshape(-1)), (slots, notched.reshape(-1)), (slots, p4.reshape(-1)),
            (np.arange(R * D), feat), (np.arange(len(y1)), y1), (np.arange(len(y2)), y2),
            (np.arange(len(y3)), y3)]


def pack_frames(x: np.ndarray, n_slots: int) -> list:
    """Per-frame packing of x [frames][bins][chirps] (complex): one slot
    vector per frame with range bin r, chirp c in slot r D + c and zeros
    elsewhere, the input layout of Context.gesture_eval_frames."""
    out = []
    for f in range(x.shape[0]):
        v = np.zeros(n_slots, dtype=np.complex128)
        v[: x[f].size] = x[f].reshape(-1)
        out.append(v)
    return out


# ---- the CNN variant (hck_gesture_cnn_eval) -------------------------------

CNN_BABY = {"dft_c": 8, "dft_s": 8, "dense1": 8, "dense2": 10}


def cnn_act_depth(coeffs) -> int:
    """Levels one activation consumes: ceil(log2 degree) + 1."""
    return int(np.ceil(np.log2(max(1, len(coeffs) - 1)))) + 1


def cnn_levels(level0: int, coeffs) -> dict:
    a = cnn_act_depth(coeffs)
    return {"dft_c": level0, "dft_s": level0, "notch": level0 - 2, "conv1": level0 - 6,
            "conv2": level0 - 7 - a, "dense1": level0 - 8 - 2 * a, "bias1": level0 - 9 - 2 * a,
            "dense2": level0 - 9 - 3 * a, "bias2": level0 - 10 - 3 * a}


def cnn_operand_vectors(cfg: dict, n_slots: int) -> dict:
    """Public operands of the CNN variant as slot vectors: the front end's
    (Doppler DFT diagonals, notch mask) and the generalized diagonals of the
    two convolutions and two dense layers, biases at slot 0."""
    F, R, D = cfg["frames"], cfg["bins"], cfg["chirps"]
    RD = R * D
    if (1 << max(0, (F - 1).bit_length())) * RD != n_slots:
        raise ValueError("pow2(frames) x bins x chirps must equal the slot count")
    k1 = np.asarray(cfg["conv1"], dtype=np.float64)          # [c1][3][3]
    k2 = np.asarray(cfg["conv2"], dtype=np.float64)          # [c2][c1][3][3]
    d1 = np.asarray(cfg["dense1"], dtype=np.float64)
    C1, C2, H = k1.shape[0], k2.shape[0], d1.shape[0]
    dft = _shifted_dft(D, cfg["window"])
    out = {"dft_c": _diagonals(dft.real, n_slots, True),
           "dft_s": _diagonals(dft.imag, n_slots, True)}
    notch = np.ones(n_slots)
    for b in cfg["notch"]:
        notch[b::D] = 0.0
    out["notch"] = notch
    s = np.arange(n_slots)
    block, r, c = s // RD, (s % RD) // D, s % D

    def inside(dr, dc):
        return (r + dr >= 0) & (r + dr < R) & (c + dc >= 0) & (c + dc < D)

    # conv1: block b -> channel b mod C1 at even (r, c)
    even = (r % 2 == 0) & (c % 2 == 0)
    conv1 = {}
    for ky in range(3):
        for kx in range(3):
            dr, dc = ky - 1, kx - 1
            vec = k1[block % C1, ky, kx] * (even & inside(dr, dc))
            if vec.any():
                conv1[(dr * D + dc) % n_slots] = vec
    out["conv1"] = conv1
    # conv2: block b -> channel b mod C2 at (r, c) multiples of 4, reading
    # channel (b + delta) mod C1 from block b + delta, neighbours 2 apart
    quad = (r % 4 == 0) & (c % 4 == 0)
    conv2 = {}
    for delta in range(C1):
        src = (block + delta) % C1
        for ky in range(3):
            for kx in range(3):
                dr, dc = 2 * (ky - 1), 2 * (kx - 1)
                vec = k2[block % C2, src, ky, kx] * (quad & inside(dr, dc))
                if vec.any():
                    conv2[(delta * RD + dr * D + dc) % n_slots] = vec
    out["conv2"] = conv2
    # dense1: W1 over the 2 x 2 pooled conv2 map, as one row per hidden unit
    # over the slots of one period of C2 blocks (pooling weights 1/4)
    period = C2 * RD
    ph, pw = R // 8, D // 8
    ps = np.arange(period)
    pb, pr, pc = ps // RD, (ps % RD) // D, ps % D
    used = (pr % 4 == 0) & (pc % 4 == 0)
    feat_index = (pb * ph + pr // 8) * pw + pc // 8
    row_w = np.where(used[None, :], d1[:, np.where(used, feat_index, 0)] / 4.0, 0.0)
    dense1 = {}
    for k in range(H):
        vec = np.zeros(n_slots)
        vec[:period] = row_w[ps % H, (ps + k) % period]
        if vec.any():
            dense1[k] = vec
    out["dense1"] = dense1
    out["dense2"] = _diagonals(np.asarray(cfg["dense2"], dtype=np.float64), n_slots, False)
    for name in ("bias1", "bias2"):
        v = np.zeros(n_slots)
        b = np.asarray(cfg[name], dtype=np.float64)
        v[: b.size] = b
        out[name] = v
    return out


def cnn_scales_at_biases(q, level0: int, scale0: float, coeffs) -> list:
    """Scale of the ciphertext at each bias addition of the CNN variant, from
    the operations' scale arithmetic in order; an activation (hck_poly_eval)
    returns its first nonzero term's scale."""
    q = [float(x) for x in q]
    lv = cnn_levels(level0, coeffs)
    deg = len(coeffs) - 1
    a = cnn_act_depth(coeffs)

    def after_lt(s, lvl):
        return s * q[lvl] / q[lvl]

    def after_act(s, lvl):
        pw = {1: (s, lvl)}
        for k in range(2, deg + 1):
            hi = 1 << (k - 1).bit_length() - 1
            (s1, l1), (s2, l2) = pw[hi], pw[k - hi]
            m = min(l1, l2)
            pw[k] = (s1 * s2 / q[m], m - 1)
        first = next(k for k in range(1, deg + 1) if coeffs[k] != 0)
        sk = pw[first][0]
        lf = lvl - a
        return sk * (s * q[lf + 1] / sk) / q[lf + 1]

    s = after_lt(scale0, level0)                              # Doppler DFT
    s = s * s / q[level0 - 1]                                 # |.|^2
    s = after_lt(s, level0 - 2)                               # notch
    s2 = s * s / q[level0 - 3]
    s4 = s2 * s2 / q[level0 - 4]
    s = s * s4 / q[level0 - 5]                                # feature
    s = after_act(after_lt(s, lv["conv1"]), lv["conv1"] - 1)
    s = after_act(after_lt(s, lv["conv2"]), lv["conv2"] - 1)
    s = after_lt(s, lv["dense1"])
    first = s
    s = after_lt(after_act(s, lv["bias1"]), lv["dense2"])
    return [first, s]


def encode_cnn_plan(ctx, cfg: dict, level0: int, scale0: float, vectors: dict | None = None):
    from . import GestureCnnPlan
    vec = cnn_operand_vectors(cfg, ctx.n // 2) if vectors is None else vectors
    lv = cnn_levels(level0, cfg["act"])
    baby = dict(CNN_BABY, conv1=cfg["chirps"], conv2=cfg["bins"] * cfg["chirps"])
    ops = {name: ctx.lt_create(vec[name], baby[name], lv[name])
           for name in ("dft_c", "dft_s", "conv1", "conv2", "dense1", "dense2")}
    ops["notch"] = ctx.encode(vec["notch"], float(ctx.q[lv["notch"]]), lv["notch"])
    for name, s in zip(("bias1", "bias2"), cnn_scales_at_biases(ctx.q, level0, scale0,
                                                               cfg["act"])):
        ops[name] = ctx.encode(vec[name], s, lv[name])
    return GestureCnnPlan.build(cnn_shape(cfg), ops, cfg["act"])


def cnn_shape(cfg: dict) -> dict:
    return dict(frames=cfg["frames"], bins=cfg["bins"], chirps=cfg["chirps"],
                c1=np.shape(cfg["conv1"])[0], c2=np.shape(cfg["conv2"])[0],
                hidden=np.shape(cfg["dense1"])[0], classes=np.shape(cfg["dense2"])[0])


def cnn_plain(cfg: dict, x: np.ndarray) -> np.ndarray:
    """The CNN on plaintext numbers (x: [frames][bins][chirps] complex): the
    logits, for checking decoded results."""
    D = cfg["chirps"]
    spec = np.einsum("kn,frn->frk", _shifted_dft(D, cfg["window"]), np.asarray(x))
    p = np.abs(spec) ** 2
    p[:, :, list(cfg["notch"])] = 0.0
    feat = (p ** 5).sum(axis=0)
    act = lambda v: np.polynomial.polynomial.polyval(v, cfg["act"])

    def conv(img, k):                       # img [cin][H][W], k [cout][cin][3][3]
        cin, h, w = img.shape
        pad = np.zeros((cin, h + 2, w + 2))
        pad[:, 1:-1, 1:-1] = img
        out = np.zeros((k.shape[0], h // 2, w // 2))
        for ky in range(3):
            for kx in range(3):
                win = pad[:, ky:ky + h:2, kx:kx + w:2]          # [cin][h/2][w/2]
                out += np.einsum("oc,cij->oij", k[:, :, ky, kx], win)
        return out

    a1 = act(conv(feat[None], np.asarray(cfg["conv1"])[:, None]))
    a2 = act(conv(a1, np.asarray(cfg["conv2"])))
    c2, h, w = a2.shape
    pooled = a2.reshape(c2, h // 2, 2, w // 2, 2).mean(axis=(2, 4)).reshape(-1)
    a3 = act(np.asarray(cfg["dense1"]) @ pooled + np.asarray(cfg["bias1"]))
    return np.asarray(cfg["dense2"]) @ a3 + np.asarray(cfg["bias2"])
