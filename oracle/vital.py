"""The paper's encrypted vital-sign pipeline (section 3.3.3, example
pipelines: K1 -> K2 -> K4 -> K5 -> K7 -> K3 -> K1 -> K2; depth budget of
Table 1) composed from the oracle's ciphertext operations.

TEST INFRASTRUCTURE ONLY: this module is the reference the GPU pipeline is
checked against.  Nothing in the product path imports it.

Slot layout (frame-major, the batched packing of section 3.3.1): frame t and
range bin r sit in slot t R + r, F frames x R bins, zero elsewhere; T2 is the
power of two >= F with T2 R <= N/2.  The stages and the level each ends at
(input level l0):

  K1  p = Re^2 + Im^2 (l0-1); E_r = sum_t p[t, r] by rotations R, 2R, ...
      on a copy of p dropped to level BIN_LEVEL (the bin branch needs only
      two more levels, plus one of headroom at its end, so its rotations run
      on few limbs).  With the magnitude option (cfg["mag_coeffs"], reading
      A29) the bin branch sums the polynomial magnitude poly(p) ~ |z|
      (Oracle.poly_eval) instead of p
  K2  w = E^gamma by log2(gamma) squarings (level 2; gamma = cfg["gamma"],
      2 by default, 4 for sharper selection, Eq. soft_power_weight);
      num_r = sum_r r w_r / F^2, den_r = sum_r w_r / F^2 (index and mask
      plaintexts, rotations 1 .. R/2; level 1)
  K4  m = p^P_phi (Eq. phase_mask; P_phi = cfg["phase_power"], 2 .. 5):
      p^2 (l0-2), p^3 = p^2 p and p^4 = p^2 p^2 (l0-3), p^5 = p^4 p (l0-4);
      I[t] = sum_r m Re, Q[t] = sum_r m Im, left in slot t R (one level
      below m: l0-3 for P_phi = 2, and every later stage as many levels
      lower as m is)
  K5  per band b: If_b = T_b I, Qf_b = T_b Q with the zero-padded Toeplitz
      matrix of the band's taps, T_b[t][t+k] = h_b[k] (BSGS over offsets
      k R with hoisted baby steps and one ModDown per output; l0-4)
  K7  y = Qf[t] If[t-1] - If[t] Qf[t-1], x = If[t] If[t-1] + Qf[t] Qf[t-1]
      (t-1 by a rotation of -R; l0-5); third order: dphi = y x^2 - y^3 / 3
      (l0-7), first order: dphi = y
  K3  the bands' DFT bins sit in two lane groups of G lanes (G the power of
      two >= both bin counts; slot t R + c): respiration in lanes 0 .. G-1,
      heart rate in lanes G .. 2G-1.  Each band's dphi is copied into its
      lanes by rotations -1, -2, ..., multiplied by g w[t] cos(2 pi k t / F)
      / sum w and by -g w[t] sin(...) / sum w (g: the folded DFT gain); the
      two bands' products are added (disjoint lanes) and summed over t by
      rotations R, 2R, ... (one chain for the real, one for the imaginary
      part)
  K1  P = Re X^2 + Im X^2
  K2  S = P^gamma; num = sum_c a f_c S_c, den = sum_c a S_c over each lane
      group (f_c the bin frequency in beats per minute, a the band's public
      factor from the configuration's rate_gain; rotations 1 .. G/2)

Outputs: num_bin, den_bin (value in slot 0; the target bin r^ = num / den),
num_rates, den_rates (respiration in slot 0, heart rate in slot G; rate in
BPM = num / den): the client's scalar divisions of section 3.3.4.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import Ciphertext, Oracle, Plaintext

OUTPUTS = ("num_bin", "den_bin", "num_rates", "den_rates")

# level of the energy sums of the bin branch (K1 -> K2) for gamma = 2: its
# outputs end at level 1 (bin_level adds a level per further squaring)
BIN_LEVEL = 3


def log2_gamma(cfg: dict) -> int:
    g = cfg.get("gamma", 2)
    if g not in (2, 4):
        raise ValueError("gamma must be 2 or 4")
    return g.bit_length() - 1


def phase_extra(cfg: dict) -> int:
    """Levels the mask p^P_phi takes beyond p^2."""
    e = cfg.get("phase_power", 2)
    if e not in (2, 3, 4, 5):
        raise ValueError("P_phi must be 2 .. 5")
    return {2: 0, 3: 1, 4: 1, 5: 2}[e]


def bin_level(cfg: dict) -> int:
    """Level of the bin branch's energy sums: w = E^gamma lands on level 2."""
    return 2 + log2_gamma(cfg)


def _pow2_at_least(x: int) -> int:
    p = 1
    while p < x:
        p *= 2
    return p


@dataclass
class Layout:
    frames: int
    bins: int
    t2: int          # frames rounded up to a power of two
    n_slots: int
    group: int       # lanes per band group (power of two)
    lanes: dict      # band -> first lane, count
    copies: dict     # band -> lanes its dphi is copied into (power of two)


def layout(cfg: dict, n_slots: int) -> Layout:
    f, r = cfg["frames"], cfg["bins"]
    t2 = _pow2_at_least(f)
    if r & (r - 1) or t2 * r > n_slots:
        raise ValueError("bins must be a power of two and T2 R <= N/2")
    nr, nh = len(cfg["k_resp"]), len(cfg["k_hr"])
    g = _pow2_at_least(max(nr, nh))
    if 2 * g > r:
        raise ValueError("two lane groups do not fit the range bins")
    return Layout(f, r, t2, n_slots, g, {"resp": (0, nr), "hr": (g, nh)},
                  {"resp": _pow2_at_least(nr), "hr": _pow2_at_least(g + nh)})


def _gain(cfg: dict, band: str) -> float:
    """Public factor a of one band's rate average (per band, or one number
    for both; 1 if absent)."""
    g = cfg.get("rate_gain", 1.0)
    return float(g[band] if isinstance(g, dict) else g)


def operand_vectors(cfg: dict, n_slots: int) -> dict:
    """Real slot vectors of every public plaintext operand, and the FIR
    transforms' generalized diagonals (offset -> vector)."""
    lay = layout(cfg, n_slots)
    f, r = lay.frames, lay.bins
    v = {}
    idx = np.zeros(n_slots)
    idx[:r] = np.arange(r) / f ** 2
    v["bin_index"] = idx
    msk = np.zeros(n_slots)
    msk[:r] = 1.0 / f ** 2
    v["bin_mask"] = msk
    for band in ("resp", "hr"):
        h = np.asarray(cfg[f"taps_{band}"])
        half = (len(h) - 1) // 2
        diags = {}
        for k in range(-half, half + 1):
            d = np.zeros(n_slots)
            for t in range(f):
                if 0 <= t + k < f:
                    d[t * r] = h[k + half]
            if np.any(d):
                diags[(k * r) % n_slots] = d
        v[f"fir_{band}"] = diags
    v["third"] = np.full(n_slots, 1.0 / 3.0)
    w = np.asarray(cfg["window"])
    ws = w.sum() / cfg["dft_gain"]
    t = np.arange(f)
    fr = np.zeros(n_slots)
    mk = np.zeros(n_slots)
    for band in ("resp", "hr"):
        c0, nb = lay.lanes[band]
        re = np.zeros(n_slots)
        im = np.zeros(n_slots)
        for i, k in enumerate(cfg[f"k_{band}"]):
            c = c0 + i
            re[t * r + c] = w * np.cos(2 * np.pi * k * t / f) / ws
            im[t * r + c] = -w * np.sin(2 * np.pi * k * t / f) / ws
            fr[c] = 60.0 * k * cfg["fps"] / f * _gain(cfg, band)
            mk[c] = _gain(cfg, band)
        v[f"dft_re_{band}"] = re
        v[f"dft_im_{band}"] = im
    v["freq"] = fr
    v["mask"] = mk
    return v


def levels(cfg: dict, level0: int) -> dict:
    """Level of each operand for inputs at level0."""
    e = phase_extra(cfg)
    phi = level0 - (7 if cfg["taylor_order"] == 3 else 5) - e
    sharp = phi - 2 - log2_gamma(cfg)          # S = P^gamma
    return {"bin_index": 2, "bin_mask": 2, "fir": level0 - 3 - e,
            "third": level0 - 5 - e, "dft": phi, "freq": sharp, "out": sharp - 1}


def fir_baby_step(cfg: dict, n_slots: int | None = None) -> int:
    """Baby step of the FIR transforms in slots.  The Toeplitz backend (the
    default): n1 frames of R slots, the n1 with the fewest rotations for the
    evaluation's 2 inputs and 4 outputs, i.e. 2 (n1 - 1) baby steps plus 4
    per nonzero giant step over the offsets -h .. h (smallest n1 on ties).
    The rotation backend (cfg["fir_backend"] == "rotation", section 3.3's
    alternative): n1 = N/2 slots, so every tap is its own (hoisted) rotation
    of the input and there is no giant step."""
    if cfg.get("fir_backend", "toeplitz") == "rotation":
        if n_slots is None:
            raise ValueError("the rotation backend needs the slot count")
        return n_slots
    h = (len(cfg["taps_resp"]) - 1) // 2
    best, best_n1 = None, 1
    for n1 in range(1, 2 * h + 2):
        giants = h // n1 - (-h // n1)          # nonzero giants among floor(k / n1)
        cost = 2 * (n1 - 1) + 4 * giants
        if best is None or cost < best:
            best, best_n1 = cost, n1
    return cfg["bins"] * best_n1


def encode_operands(o: Oracle, cfg: dict, level0: int, vecs: dict | None = None) -> dict:
    """Plaintexts (at q_level scale) and FIR transforms for inputs at level0."""
    vecs = operand_vectors(cfg, o.n_slots) if vecs is None else vecs
    lv = levels(cfg, level0)
    enc = lambda name, lvl: o.encode(vecs[name], float(o.q[lvl]), lvl)
    ops = {"bin_index": enc("bin_index", lv["bin_index"]),
           "bin_mask": enc("bin_mask", lv["bin_mask"]),
           "third": enc("third", lv["third"])}
    n1 = fir_baby_step(cfg, o.n_slots)
    for band in ("resp", "hr"):
        ops[f"fir_{band}"] = o.lt_create(vecs[f"fir_{band}"], n1, lv["fir"])
        for part in ("dft_re", "dft_im"):
            ops[f"{part}_{band}"] = enc(f"{part}_{band}", lv["dft"])
    for part in ("freq", "mask"):
        ops[part] = enc(part, lv["freq"])
    return ops


def required_steps(o: Oracle, cfg: dict, ops: dict) -> list:
    lay = layout(cfg, o.n_slots)
    r = lay.bins
    steps = {r * (1 << i) for i in range(lay.t2.bit_length() - 1)}
    steps |= {1 << i for i in range(r.bit_length() - 1)}
    steps.add(-r)
    steps |= {-(1 << i) for i in range(lay.copies["hr"].bit_length() - 1)}
    for band in ("resp", "hr"):
        steps |= set(o.lt_required_steps(ops[f"fir_{band}"]))
    return sorted(steps)


def _square_sum(o: Oracle, a: Ciphertext, b: Ciphertext, rlk) -> Ciphertext:
    """a^2 + b^2, relinearized and rescaled."""
    return o.rescale(o.relinearize(o.add(o.tensor(a, a), o.tensor(b, b)), rlk))


def _mul(o: Oracle, a: Ciphertext, b: Ciphertext, rlk) -> Ciphertext:
    return o.rescale(o.relinearize(o.tensor(a, b), rlk))


def _rotsum(o: Oracle, c: Ciphertext, step: int, count: int, gks) -> Ciphertext:
    """c + Rot(c, step) + ... over `count` (a power of two) shifts, by doubling."""
    s = step
    while s < step * count:
        c = o.add(c, o.rotate(c, s, gks))
        s *= 2
    return c


def evaluate(o: Oracle, cfg: dict, ops: dict, re: Ciphertext, im: Ciphertext, gks: dict,
             rlk) -> dict:
    lay = layout(cfg, o.n_slots)
    r, t2 = lay.bins, lay.t2
    out = {}
    # K1: energy per bin (of the power, or of the polynomial magnitude),
    # summed on few limbs
    p = _square_sum(o, re, im, rlk)
    src = o.poly_eval(p, cfg["mag_coeffs"], rlk) if cfg.get("mag_coeffs") else p
    e = _rotsum(o, o.drop_level(src, bin_level(cfg)), r, t2, gks)
    # K2: soft power attention over bins, w = E^gamma by squarings
    _bin_outputs(o, cfg, ops, e, rlk, gks, out)
    # K4: soft I/Q with the mask p^P_phi
    i_t, q_t = _soft_iq(o, cfg, p, re, im, rlk, gks)
    _tail(o, cfg, ops, lay, i_t, q_t, gks, rlk, out)
    return out


def _mask(o: Oracle, cfg: dict, p: Ciphertext, rlk) -> Ciphertext:
    """K4's mask p^P_phi: p^2, then p^3 = p^2 p, p^4 = p^2 p^2, p^5 = p^4 p."""
    e = cfg.get("phase_power", 2)
    m = _mul(o, p, p, rlk)
    if e >= 4:
        m = _mul(o, m, m, rlk)
    if e in (3, 5):
        m = _mul(o, m, o.drop_level(p, m.level), rlk)
    return m


def _soft_iq(o: Oracle, cfg: dict, p, re, im, rlk, gks):
    """K4: I = sum_r m Re, Q = sum_r m Im, by rotations 1 .. R/2."""
    r = cfg["bins"]
    m = _mask(o, cfg, p, rlk)
    re2, im2 = o.drop_level(re, m.level), o.drop_level(im, m.level)
    return (_rotsum(o, _mul(o, m, re2, rlk), 1, r, gks),
            _rotsum(o, _mul(o, m, im2, rlk), 1, r, gks))


def _bin_outputs(o: Oracle, cfg: dict, ops: dict, e: Ciphertext, rlk, gks, out: dict):
    """K2 over bins on the energy sums: w = E^gamma, num_bin, den_bin."""
    w = e
    for _ in range(log2_gamma(cfg)):
        w = _mul(o, w, w, rlk)
    r = cfg["bins"]
    out["num_bin"] = _rotsum(o, o.rescale(o.mul_plain(w, ops["bin_index"])), 1, r, gks)
    out["den_bin"] = _rotsum(o, o.rescale(o.mul_plain(w, ops["bin_mask"])), 1, r, gks)


def evaluate_frames(o: Oracle, cfg: dict, ops: dict, res: list, ims: list, gks: dict,
                    rlk) -> dict:
    """The pipeline on per-frame packing (section 3.3.2): res[t], ims[t] hold
    frame t's R range bins in slots 0 .. R-1.  K1 per frame; E = the sum of
    the frames' copies at the bin branch's level (additions in frame order);
    K4 per frame (I_t, Q_t in slot 0); then the frames' I_t and Q_t go to slot
    t R of one ciphertext each by a tree: at step j (shift 2^j R) every other
    entry, rotated by -shift, is added to its left neighbour; K5 -> K2 as in
    evaluate()."""
    lay = layout(cfg, o.n_slots)
    if len(res) != lay.frames or len(ims) != lay.frames:
        raise ValueError("one ciphertext pair per frame")
    out = {}
    ps = [_square_sum(o, a, b, rlk) for a, b in zip(res, ims)]
    srcs = [o.poly_eval(p, cfg["mag_coeffs"], rlk) if cfg.get("mag_coeffs") else p for p in ps]
    e = o.drop_level(srcs[0], bin_level(cfg))
    for src in srcs[1:]:
        e = o.add(e, o.drop_level(src, bin_level(cfg)))
    _bin_outputs(o, cfg, ops, e, rlk, gks, out)
    cur = [_soft_iq(o, cfg, p, a, b, rlk, gks) for p, a, b in zip(ps, res, ims)]
    shift = lay.bins
    while len(cur) > 1:
        nxt = []
        for i in range(0, len(cur), 2):
            if i + 1 < len(cur):
                (a_i, a_q), (b_i, b_q) = cur[i], cur[i + 1]
                nxt.append((o.add(a_i, o.rotate(b_i, -shift, gks)),
                            o.add(a_q, o.rotate(b_q, -shift, gks))))
            else:
                nxt.append(cur[i])
        cur = nxt
        shift *= 2
    i_t, q_t = cur[0]
    _tail(o, cfg, ops, lay, i_t, q_t, gks, rlk, out)
    return out


def frames_required_steps(o: Oracle, cfg: dict, ops: dict) -> list:
    """Galois steps of the per-frame packing: the batched pipeline's and
    -R, -2R, ..., -(T2/2) R."""
    lay = layout(cfg, o.n_slots)
    extra = {-(lay.bins << j) for j in range(lay.t2.bit_length() - 1)}
    return sorted(set(required_steps(o, cfg, ops)) | extra)


def encrypt_frames(o: Oracle, s, z: np.ndarray, level: int, scale: float, seed: int):
    """Per-frame packing: frame t's bins in slots 0 .. R-1 of its own pair
    (encryption seeds seed + 2t, seed + 2t + 1)."""
    pairs = []
    for t, row in enumerate(np.asarray(z)):
        v = np.zeros(o.n_slots, dtype=np.complex128)
        v[: row.size] = row
        pairs.append((o.encrypt_sk(s, o.encode(v.real, scale, level), seed + 2 * t),
                      o.encrypt_sk(s, o.encode(v.imag, scale, level), seed + 2 * t + 1)))
    return [a for a, _ in pairs], [b for _, b in pairs]


def _tail(o: Oracle, cfg: dict, ops: dict, lay: Layout, i_t: Ciphertext, q_t: Ciphertext,
          gks: dict, rlk, out: dict):
    """K5 -> K7 -> K3 -> K1 -> K2 on the phase series I, Q (slot t R)."""
    r, t2 = lay.bins, lay.t2
    # K5: FIR into the two bands
    terms = [(ops["fir_resp"], 0, 0, 1), (ops["fir_resp"], 1, 1, 1),
             (ops["fir_hr"], 0, 2, 1), (ops["fir_hr"], 1, 3, 1)]
    filt = [o.rescale(c) for c in o.lt_eval([i_t, q_t], terms, gks, 4, hoist=True,
                                                hoist_giant=True)]
    # K7 and K3 per band; the bands' DFT products are added before the sum
    # over frames
    x_re = x_im = None
    for band, (fi, fq) in (("resp", (filt[0], filt[1])), ("hr", (filt[2], filt[3]))):
        fi1, fq1 = o.rotate(fi, -r, gks), o.rotate(fq, -r, gks)
        y = o.rescale(o.relinearize(o.sub(o.tensor(fq, fi1), o.tensor(fi, fq1)), rlk))
        if cfg["taylor_order"] == 3:
            x = o.rescale(o.relinearize(o.add(o.tensor(fi, fi1), o.tensor(fq, fq1)), rlk))
            x2 = _mul(o, x, x, rlk)
            a = _mul(o, o.drop_level(y, x2.level), x2, rlk)
            y2 = _mul(o, y, y, rlk)
            yc = o.rescale(o.mul_plain(y, ops["third"]))
            dphi = o.sub(a, _mul(o, yc, y2, rlk))
        else:
            dphi = y
        rep = dphi
        s = 1
        while s < lay.copies[band]:
            rep = o.add(rep, o.rotate(rep, -s, gks))
            s *= 2
        xr = o.rescale(o.mul_plain(rep, ops[f"dft_re_{band}"]))
        xi = o.rescale(o.mul_plain(rep, ops[f"dft_im_{band}"]))
        x_re = xr if x_re is None else o.add(x_re, xr)
        x_im = xi if x_im is None else o.add(x_im, xi)
    x_re = _rotsum(o, x_re, r, t2, gks)
    x_im = _rotsum(o, x_im, r, t2, gks)
    # K1 on the spectrum, K2: sharpening and weighted frequency averages
    pw = _square_sum(o, x_re, x_im, rlk)
    sh = pw
    for _ in range(log2_gamma(cfg)):
        sh = _mul(o, sh, sh, rlk)
    out["num_rates"] = _rotsum(o, o.rescale(o.mul_plain(sh, ops["freq"])), 1, lay.group, gks)
    out["den_rates"] = _rotsum(o, o.rescale(o.mul_plain(sh, ops["mask"])), 1, lay.group, gks)


def plain(cfg: dict, z: np.ndarray) -> dict:
    """The same circuit on plaintext numbers (z: [frames][bins] complex): the
    'mmFHE on plaintext' comparison of section 5.1."""
    f, r = cfg["frames"], cfg["bins"]
    re, im = z.real, z.imag
    p = re ** 2 + im ** 2
    if cfg.get("mag_coeffs"):
        e = np.polynomial.polynomial.polyval(p, cfg["mag_coeffs"]).sum(axis=0)
    else:
        e = p.sum(axis=0)
    w = e ** cfg.get("gamma", 2)
    out = {"num_bin": float(np.sum(np.arange(r) * w) / f ** 2),
           "den_bin": float(np.sum(w) / f ** 2)}
    m = p ** cfg.get("phase_power", 2)
    i_t = (m * re).sum(axis=1)
    q_t = (m * im).sum(axis=1)
    win = np.asarray(cfg["window"])
    t = np.arange(f)
    spec = {}
    for band in ("resp", "hr"):
        h = np.asarray(cfg[f"taps_{band}"])
        half = (len(h) - 1) // 2

        def fir(x):
            y = np.zeros(f)
            for k in range(-half, half + 1):
                lo, hi = max(0, -k), min(f, f - k)
                y[lo:hi] += h[k + half] * x[lo + k:hi + k]
            return y

        fi, fq = fir(i_t), fir(q_t)
        fi1 = np.concatenate([[0.0], fi[:-1]])
        fq1 = np.concatenate([[0.0], fq[:-1]])
        y = fq * fi1 - fi * fq1
        if cfg["taylor_order"] == 3:
            x = fi * fi1 + fq * fq1
            dphi = y * x ** 2 - y ** 3 / 3
        else:
            dphi = y
        ks = np.asarray(cfg[f"k_{band}"])
        ws = win.sum() / cfg["dft_gain"]
        xr = np.array([np.sum(win * np.cos(2 * np.pi * k * t / f) * dphi) for k in ks]) / ws
        xi = np.array([-np.sum(win * np.sin(2 * np.pi * k * t / f) * dphi) for k in ks]) / ws
        s = (xr ** 2 + xi ** 2) ** cfg.get("gamma", 2)
        fk = 60.0 * ks * cfg["fps"] / f
        g = _gain(cfg, band)
        out[f"num_{band}"] = float(g * np.sum(fk * s))
        out[f"den_{band}"] = float(g * np.sum(s))
    return out


def plain_slots(cfg: dict, z: np.ndarray, n_slots: int) -> dict:
    """plain() arranged as the outputs' decoded slots: output name -> {slot:
    value}."""
    lay = layout(cfg, n_slots)
    v = plain(cfg, z)
    return {"num_bin": {0: v["num_bin"]}, "den_bin": {0: v["den_bin"]},
            "num_rates": {0: v["num_resp"], lay.group: v["num_hr"]},
            "den_rates": {0: v["den_resp"], lay.group: v["den_hr"]}}


def encrypt_window(o: Oracle, s, z: np.ndarray, level: int, scale: float, seed: int):
    """Re and Im of a [frames][bins] window packed frame-major (slot t R + r)."""
    v = np.zeros(o.n_slots, dtype=np.complex128)
    v[: z.size] = z.reshape(-1)
    return (o.encrypt_sk(s, o.encode(v.real, scale, level), seed),
            o.encrypt_sk(s, o.encode(v.imag, scale, level), seed + 1))
