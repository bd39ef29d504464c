"""Public operands of the vital-sign pipeline (hck_vital_eval): the slot
vectors of the masks, index and frequency weights, the FIR transforms'
diagonals and the DFT weights for a window of F frames x R bins packed
frame-major (slot t R + r), encoded with this library's encoder.

This is plaintext setup (the pipeline's public weights, section 3.3.3);
every homomorphic step runs in the library.
"""
import numpy as np


def _next_pow2(x: int) -> int:
    return 1 << max(0, (int(x) - 1).bit_length())


# level of the bin branch's energy sums (K1 -> K2) for gamma = 2; one more per
# further squaring, so that its plaintexts sit at level 2 and its outputs end
# at level 1
BIN_LEVEL = 3


def phase_extra(phase_power: int = 2) -> int:
    """Levels K4's mask p^P_phi takes beyond p^2 (p^3 = p^2 p, p^4 = (p^2)^2,
    p^5 = (p^2)^2 p)."""
    return {2: 0, 3: 1, 4: 1, 5: 2}[phase_power]


def plan_levels(taylor_order: int, level0: int, gamma: int = 2, phase_power: int = 2) -> dict:
    """Level at which each operand is applied, for inputs at level0."""
    e = phase_extra(phase_power)
    dft = level0 - (7 if taylor_order == 3 else 5) - e
    squarings = {2: 1, 4: 2}[gamma]
    return dict(bins=2, fir=level0 - 3 - e, third=level0 - 5 - e, dft=dft,
                freq=dft - 2 - squarings)


def operand_vectors(cfg: dict, n_slots: int) -> dict:
    """name -> real slot vector (FIR transforms: offset -> diagonal vector)."""
    F, R = cfg["frames"], cfg["bins"]
    if _next_pow2(F) * R > n_slots:
        raise ValueError("window does not fit the slots")
    if 2 * lane_group(cfg) > R:
        raise ValueError("the two DFT lane groups do not fit the range bins")
    frames = np.arange(F)
    out = {}
    zero = lambda: np.zeros(n_slots)
    out["bin_index"], out["bin_mask"] = zero(), zero()
    out["bin_index"][:R] = np.arange(R, dtype=np.float64) / (F * F)
    out["bin_mask"][:R] = 1.0 / (F * F)
    for band in ("resp", "hr"):
        taps = np.asarray(cfg["taps_" + band], dtype=np.float64)
        h = len(taps) // 2
        diags = {}
        for k in range(-h, h + 1):
            rows = frames[(frames + k >= 0) & (frames + k < F)]
            if rows.size == 0:
                continue
            d = zero()
            d[rows * R] = taps[k + h]
            diags[(k * R) % n_slots] = d
        out["fir_" + band] = diags
    out["third"] = np.full(n_slots, 1.0 / 3.0)
    win = np.asarray(cfg["window"], dtype=np.float64)
    norm = cfg["dft_gain"] / win.sum()
    group = lane_group(cfg)
    lane0 = {"resp": 0, "hr": group}
    out["freq"], out["mask"] = zero(), zero()
    for band in ("resp", "hr"):
        vr, vi = zero(), zero()
        for lane, k in enumerate(cfg["k_" + band], start=lane0[band]):
            ang = 2.0 * np.pi * k * frames / F
            vr[frames * R + lane] = norm * win * np.cos(ang)
            vi[frames * R + lane] = -norm * win * np.sin(ang)
            out["freq"][lane] = 60.0 * k * cfg["fps"] / F * band_gain(cfg, band)
            out["mask"][lane] = band_gain(cfg, band)
        out["dft_re_" + band], out["dft_im_" + band] = vr, vi
    return out


def band_gain(cfg: dict, band: str) -> float:
    """The public factor of a band's rate average (1 when the configuration
    has none; a number applies to both bands)."""
    g = cfg.get("rate_gain", 1.0)
    return float(g[band] if isinstance(g, dict) else g)


def lane_group(cfg: dict) -> int:
    """Lanes per band group: respiration's DFT bins from lane 0, heart rate's
    from this lane, of every frame's R slots (the rates' output slots)."""
    return _next_pow2(max(len(cfg["k_resp"]), len(cfg["k_hr"])))


def fir_baby_step(cfg: dict, n_slots: int | None = None) -> int:
    """Baby step of the FIR transforms in slots (offsets are multiples of R).
    Toeplitz backend (default): the number of frames that needs the fewest
    rotations for the evaluation's 2 inputs (baby steps, hoisted) and 4
    outputs (giant steps).  Rotation backend (cfg["fir_backend"] ==
    "rotation"): all N/2 slots, every tap a hoisted rotation of the input."""
    if cfg.get("fir_backend", "toeplitz") == "rotation":
        if n_slots is None:
            raise ValueError("the rotation backend needs the slot count")
        return n_slots
    half = len(cfg["taps_resp"]) // 2
    costs = []
    for frames in range(1, 2 * half + 2):
        lo, hi = -half // frames, half // frames     # giant indices floor(k / frames)
        costs.append((2 * (frames - 1) + 4 * (hi - lo), frames))
    return cfg["bins"] * min(costs)[1]


def encode_plan(ctx, cfg: dict, level0: int, vectors: dict | None = None):
    """A VitalPlan with every operand encoded by the library at the level it
    is applied, at scale q_level (a product then keeps the ciphertext scale)."""
    from . import VitalPlan
    vec = operand_vectors(cfg, ctx.n // 2) if vectors is None else vectors
    lv = plan_levels(cfg["taylor_order"], level0, cfg.get("gamma", 2),
                     cfg.get("phase_power", 2))
    q = ctx.q

    def pt(name, level):
        return ctx.encode(vec[name], float(q[level]), level)

    ops = {"bin_index": pt("bin_index", lv["bins"]), "bin_mask": pt("bin_mask", lv["bins"]),
           "third": pt("third", lv["third"])}
    n1 = fir_baby_step(cfg, ctx.n_slots)
    for band in ("resp", "hr"):
        ops["fir_" + band] = ctx.lt_create(vec["fir_" + band], n1, lv["fir"])
        for name in ("dft_re_", "dft_im_"):
            ops[name + band] = pt(name + band, lv["dft"])
    for name in ("freq", "mask"):
        ops[name] = pt(name, lv["freq"])
    return VitalPlan.build(cfg["frames"], cfg["bins"], cfg["taylor_order"], len(cfg["k_resp"]),
                           len(cfg["k_hr"]), ops, cfg.get("mag_coeffs"), cfg.get("gamma", 2),
                           cfg.get("phase_power", 2))


def plain_stages(cfg: dict, z: np.ndarray, n_slots: int) -> list:
    """Plaintext execution of the pipeline, the reference of the per-kernel
    encryption noise (section 5.2, Table 3).  For each tap of
    hck_vital_eval_taps, then each of the four outputs: (slot indices,
    values) where the encrypted result holds them."""
    F, R = cfg["frames"], cfg["bins"]
    if _next_pow2(F) * R > n_slots or 2 * lane_group(cfg) > R:
        raise ValueError("window does not fit the slots")
    G = lane_group(cfg)
    re, im = np.asarray(z).real, np.asarray(z).imag
    t = np.arange(F)
    frame0 = t * R
    p = re ** 2 + im ** 2
    # the bin estimate sums the power, or with the magnitude option the
    # polynomial magnitude of the power
    mag = np.polynomial.polynomial.polyval(p, cfg["mag_coeffs"]) if cfg.get("mag_coeffs") else p
    e = mag.sum(axis=0)
    gamma = cfg.get("gamma", 2)
    w = e ** gamma
    m = p ** cfg.get("phase_power", 2)
    i_t, q_t = (m * re).sum(axis=1), (m * im).sum(axis=1)
    out = [(np.arange(F * R), p.reshape(-1)), (np.arange(R), e), (np.arange(R), w),
           (frame0, i_t), (frame0, q_t)]

    def fir(x, taps):
        h = len(taps) // 2
        y = np.zeros(F)
        for k in range(-h, h + 1):
            ok = (t + k >= 0) & (t + k < F)
            y[ok] += taps[k + h] * x[t[ok] + k]
        return y

    filt = {}
    for band in ("resp", "hr"):
        taps = np.asarray(cfg["taps_" + band], dtype=np.float64)
        filt[band] = (fir(i_t, taps), fir(q_t, taps))
        out += [(frame0, filt[band][0]), (frame0, filt[band][1])]
    win = np.asarray(cfg["window"], dtype=np.float64)
    norm = cfg["dft_gain"] / win.sum()
    lanes, xr, xi, fq = [], [], [], []
    dphis = []
    for band, lane0 in (("resp", 0), ("hr", G)):
        fi, fq_ = filt[band]
        fi1, fq1 = np.roll(fi, 1), np.roll(fq_, 1)
        fi1[0] = fq1[0] = 0.0
        y = fq_ * fi1 - fi * fq1
        x = fi * fi1 + fq_ * fq1
        dphi = y * x ** 2 - y ** 3 / 3.0 if cfg["taylor_order"] == 3 else y
        dphis.append((frame0, dphi))
        for j, k in enumerate(cfg["k_" + band]):
            ang = 2.0 * np.pi * k * t / F
            lanes.append(lane0 + j)
            xr.append(norm * np.sum(win * np.cos(ang) * dphi))
            xi.append(-norm * np.sum(win * np.sin(ang) * dphi))
            fq.append(60.0 * k * cfg["fps"] / F)
    out += dphis
    lanes, xr, xi, fq = (np.asarray(v) for v in (lanes, xr, xi, fq))
    pw = xr ** 2 + xi ** 2
    sh = pw ** gamma
    out += [(lanes, xr), (lanes, xi), (lanes, pw), (lanes, sh)]
    n_resp = len(cfg["k_resp"])
    two = np.array([0, G])
    a = np.array([band_gain(cfg, "resp"), band_gain(cfg, "hr")])
    out += [(np.array([0]), np.array([np.sum(np.arange(R) * w) / F ** 2])),
            (np.array([0]), np.array([np.sum(w) / F ** 2])),
            (two, a * np.array([np.sum(fq[:n_resp] * sh[:n_resp]),
                                np.sum(fq[n_resp:] * sh[n_resp:])])),
            (two, a * np.array([np.sum(sh[:n_resp]), np.sum(sh[n_resp:])]))]
    return out
