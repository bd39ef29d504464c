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
