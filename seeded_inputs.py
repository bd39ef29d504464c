"""Seeded synthetic inputs and parameter sets.

This module is the only code shared by the CPU oracle side (tests, the oracle
baseline timing) and the HIP library side (tests, bench, smoke).  It holds no
CKKS arithmetic: it chooses public parameters (ring degree, prime chains,
digit count, scale) and draws seeded random data (slot vectors, plaintext
matrices, integer residue arrays) that both sides then consume unchanged.

Parameter shapes follow the workloads of the paper (CKKS primer in section 3.2,
parameter table Table 8, ciphertext/key sizes Table 6) with the ring sizes of
the benchmark configurations:

* ``tiny``    N = 2^12, three 30-bit primes, one 60-bit special prime,
               dnum = 3, scale 2^25.  (With a special prime barely above the
               30-bit digits, the uncentred digit's mean term gives key-switching
               noise of ~4e-3 in the slot whose root is nearest 1.)
* ``vital``   N = 2^16, L = 24 (q0 of 60 bits, 23 primes of ~50 bits),
               K = 8 special primes of 60 bits, dnum = 3, scale 2^50.
* ``gesture`` N = 2^16, L = 30, K = 10, dnum = 3, scale 2^50.
* ``mix15``   N = 2^15, L = 12, K = 4, dnum = 3, scale 2^50 (the paper's own
               ring with the gesture pipeline's 12 limbs).
"""
from __future__ import annotations

import numpy as np

__all__ = ["CONFIGS", "params", "is_prime", "uniform_slots", "uniform_matrix",
           "vital_window", "windowed_dft_matrix", "fir_bandpass", "vital_pipeline_config",
           "uniform_residues", "small_ints"]


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 2^64 (bases 2..37)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _primes_near(bits: int, two_n: int, count: int, taken: set[int],
                 alternate: bool) -> list[int]:
    """``count`` primes p = 1 (mod 2N) closest to 2^bits.

    With ``alternate`` the search takes one prime below 2^bits, then one above,
    and so on, so that the product of consecutive primes stays near 2^(2 bits)
    and the scale drifts little after rescaling.  Without it every prime is
    taken below 2^bits (so that it stays under 2^bits).
    """
    out: list[int] = []
    centre = (1 << bits) // two_n * two_n + 1
    down, up = centre, centre + two_n
    side = 0
    while len(out) < count:
        if side == 0 or not alternate:
            while not (is_prime(down) and down not in taken and down < (1 << bits)):
                down -= two_n
            out.append(down)
            taken.add(down)
            down -= two_n
        else:
            while not (is_prime(up) and up not in taken):
                up += two_n
            out.append(up)
            taken.add(up)
            up += two_n
        side ^= 1
    return out


# name -> (log_n, q_layout, p_layout, dnum, scale)
# q_layout/p_layout: list of (bits, count, alternate)
CONFIGS: dict[str, dict] = {
    "tiny": dict(log_n=12, q=[(30, 3, False)], p=[(60, 1, False)], dnum=3,
                 scale=2.0 ** 25),
    "vital": dict(log_n=16, q=[(60, 1, False), (50, 23, True)], p=[(60, 8, False)],
                  dnum=3, scale=2.0 ** 50),
    "gesture": dict(log_n=16, q=[(60, 1, False), (50, 29, True)], p=[(60, 10, False)],
                    dnum=3, scale=2.0 ** 50),
    "mix15": dict(log_n=15, q=[(60, 1, False), (50, 11, True)], p=[(60, 4, False)],
                  dnum=3, scale=2.0 ** 50),
    # a small ring with 8 levels (polynomial evaluation up to degree 64)
    "deep12": dict(log_n=12, q=[(60, 1, False), (50, 7, True)], p=[(60, 3, False)],
                   dnum=3, scale=2.0 ** 50),
    # the gesture circuit's 12 levels on a small ring whose slots hold two
    # 32 x 32 frame blocks (per-frame packing tests; not a secure size)
    "gest12": dict(log_n=12, q=[(60, 1, False), (50, 11, True)], p=[(60, 4, False)],
                   dnum=3, scale=2.0 ** 50),
    # the gesture CNN's 19 levels (+1 of headroom) on a small ring whose slots
    # hold 16 blocks of an 8 x 8 feature map (oracle pins, GPU parity; not a
    # secure size)
    "cnn11": dict(log_n=11, q=[(60, 1, False), (50, 20, True)], p=[(60, 7, False)],
                  dnum=3, scale=2.0 ** 50),
    # smallest and largest supported rings (edge cases of the parity tests)
    "edge11": dict(log_n=11, q=[(60, 1, False), (50, 2, True)], p=[(60, 1, False)],
                   dnum=3, scale=2.0 ** 40),
    "edge17": dict(log_n=17, q=[(60, 1, False), (50, 3, True)], p=[(60, 2, False)],
                   dnum=2, scale=2.0 ** 50),
}

_cache: dict[str, dict] = {}


def params(name: str) -> dict:
    """Public parameter set: {'log_n', 'n', 'q': [...], 'p': [...], 'dnum', 'scale'}.

    Every prime is = 1 (mod 2N) and below 2^61.  The q chain starts with q0.
    """
    if name in _cache:
        return dict(_cache[name])
    cfg = CONFIGS[name]
    two_n = 2 << cfg["log_n"]
    taken: set[int] = set()
    q: list[int] = []
    for bits, count, alt in cfg["q"]:
        q += _primes_near(bits, two_n, count, taken, alt)
    p: list[int] = []
    for bits, count, alt in cfg["p"]:
        p += _primes_near(bits, two_n, count, taken, alt)
    out = dict(name=name, log_n=cfg["log_n"], n=1 << cfg["log_n"], q=q, p=p,
               dnum=cfg["dnum"], scale=cfg["scale"])
    _cache[name] = out
    return dict(out)


def params_with_dnum(name: str, dnum: int) -> dict:
    """The parameter set `name` with another digit count: the same ring and q
    chain, dnum digits and K = ceil(L / dnum) special primes of 60 bits
    (distinct from the chain; the first K of a fixed list of such primes, so
    sets with different dnum share their special primes as far as they go)."""
    base = params(name)
    L = len(base["q"])
    k = -(-L // dnum)
    two_n = 2 * base["n"]
    specials = _primes_near(60, two_n, k, set(base["q"]), False)
    return dict(base, name=f"{name}/dnum{dnum}", dnum=dnum, p=specials)


def params_wide_special(name: str) -> dict:
    """The parameter set `name` with its K special primes moved just below
    2^61 (still = 1 mod 2N and distinct from the chain): moduli at the top of
    the range the library accepts, above the 2^60 bound of its 30-bit
    basis-conversion path."""
    base = params(name)
    two_n = 2 * base["n"]
    specials = _primes_near(61, two_n, len(base["p"]), set(base["q"]), False)
    return dict(base, name=f"{name}/p61", p=specials)


def uniform_slots(n_slots: int, seed: int, lo: float = -1.0, hi: float = 1.0,
                  complex_: bool = False) -> np.ndarray:
    """Slot vector drawn uniformly from [lo, hi) (real, or real+imag parts)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(lo, hi, n_slots)
    if not complex_:
        return re
    return re + 1j * rng.uniform(lo, hi, n_slots)


def uniform_matrix(rows: int, cols: int, seed: int, bound: float) -> np.ndarray:
    """Real matrix with entries uniform in [-bound, bound)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-bound, bound, (rows, cols))


def uniform_residues(moduli, n: int, seed: int, count: int = 1) -> np.ndarray:
    """``count`` stacked arrays of shape [len(moduli)][n], row i uniform in [0, moduli[i])."""
    rng = np.random.default_rng(seed)
    out = np.empty((count, len(moduli), n), dtype=np.uint64)
    for c in range(count):
        for i, m in enumerate(moduli):
            out[c, i] = rng.integers(0, m, n, dtype=np.uint64)
    return out


def small_ints(n: int, seed: int, bound: int) -> np.ndarray:
    """int64 array of n values uniform in [-bound, bound]."""
    rng = np.random.default_rng(seed)
    return rng.integers(-bound, bound + 1, n, dtype=np.int64)


# ---------------------------------------------------------------------------
# Synthetic radar windows (stand-ins for the paper's datasets, Table 2)
# ---------------------------------------------------------------------------

def vital_window(seed: int, frames: int = 200, bins: int = 64, fps: float = 20.0,
                 snr_db: float = 20.0) -> np.ndarray:
    """A vital-sign window: complex range profiles [frames][bins].

    One target range bin (uniform in [8, 56)) carries the chest displacement
    d(t) = A_r sin(2 pi f_r t + p_r) + A_h sin(2 pi f_h t + p_h), with
    respiration f_r ~ U[0.1, 0.5] Hz, A_r ~ U[2, 10] mm and heartbeat
    f_h ~ U[0.8, 2.0] Hz, A_h ~ U[0.1, 0.5] mm, as the phase
    exp(j 4 pi d / lambda) at 60 GHz (lambda ~ 5 mm; the FMCW phase model of
    the paper's Appendix A); every bin gets complex Gaussian noise at the
    given SNR.  The clutter-removed (mean-subtracted, section 3.3.2) and
    normalized (max |z| = 1) window is returned.
    """
    rng = np.random.default_rng(seed)
    lam = 3e8 / 60e9
    t = np.arange(frames) / fps
    fr, ar = rng.uniform(0.1, 0.5), rng.uniform(2e-3, 10e-3)
    fh, ah = rng.uniform(0.8, 2.0), rng.uniform(0.1e-3, 0.5e-3)
    pr, ph = rng.uniform(0, 2 * np.pi, 2)
    d = ar * np.sin(2 * np.pi * fr * t + pr) + ah * np.sin(2 * np.pi * fh * t + ph)
    z = np.zeros((frames, bins), dtype=np.complex128)
    target = rng.integers(8, 56)
    z[:, target] = np.exp(1j * 4 * np.pi * d / lam)
    sigma = 10 ** (-snr_db / 20) / np.sqrt(2)
    z += sigma * (rng.standard_normal(z.shape) + 1j * rng.standard_normal(z.shape))
    z -= z.mean(axis=0, keepdims=True)
    return z / np.abs(z).max()


def windowed_dft_matrix(d: int) -> np.ndarray:
    """W[k, n] = w[n] exp(-j 2 pi sigma(k) n / D) / sum(w) with the Hann
    window w and the fftshift permutation sigma(k) = (k + D/2) mod D (the
    paper's Eq. dft_kernel), normalized so that |W x| <= max|x|."""
    n = np.arange(d)
    w = np.hanning(d)
    sig = (n + d // 2) % d
    return w[None, :] * np.exp(-2j * np.pi * np.outer(sig, n) / d) / w.sum()


# ---- public constants of the vital-sign pipeline (plaintext DSP design) ----

def fir_bandpass(taps: int, lo_hz: float, hi_hz: float, fs: float) -> np.ndarray:
    """Zero-phase band-pass FIR taps h[k], k = -(taps-1)/2 .. (taps-1)/2: the
    difference of two windowed-sinc low-passes (Hamming window), scaled to
    unit gain at the band centre (the paper's K5 filters its soft I/Q into the
    respiration and heart-rate bands)."""
    if taps % 2 == 0:
        raise ValueError("odd tap count")
    k = np.arange(taps) - (taps - 1) // 2

    def lowpass(fc):
        return 2 * fc / fs * np.sinc(2 * fc / fs * k)

    h = (lowpass(hi_hz) - lowpass(lo_hz)) * np.hamming(taps)
    fc = 0.5 * (lo_hz + hi_hz)
    gain = abs(np.sum(h * np.exp(-2j * np.pi * fc / fs * k)))
    return h / gain


def sqrt_poly(degree: int) -> list:
    """Power-basis coefficients c_0 .. c_degree of the least-squares fit of
    sqrt(x) on [0, 1] at 4 (degree + 1) Chebyshev points, through the origin
    (c_0 = 0: a zero sample, e.g. a frame of zero padding, has magnitude 0):
    the polynomial magnitude |z| = sqrt(|z|^2) of a unit-normalized window."""
    k = np.arange(4 * (degree + 1))
    x = 0.5 - 0.5 * np.cos((2 * k + 1) * np.pi / (2 * len(k)))
    basis = np.stack([x ** j for j in range(1, degree + 1)], axis=1)
    c, *_ = np.linalg.lstsq(basis, np.sqrt(x), rcond=None)
    return [0.0] + list(c)


def vital_pipeline_config(frames: int = 200, bins: int = 64, fps: float = 20.0,
                          taps: int = 41, taylor_order: int = 3, fir_gain: float = 5.0,
                          dft_gain: float = 10.0, magnitude_degree: int = 0,
                          gamma: int = 2, fir_backend: str = "toeplitz",
                          phase_power: int = 2) -> dict:
    """The vital-sign pipeline's public parameters (section 3.3.3 example
    pipeline): respiration 0.1-0.6 Hz and heart rate 0.8-2.5 Hz bands, the
    FIR taps of each band (times fir_gain), the Hann window of the phase DFT
    (its weights are w[t] dft_gain / sum w) and the DFT bins k (frequency
    k fps / frames) inside each band.  The two gains are normalization
    constants folded into public weights (as section 3.3.3 folds s^gamma / F
    into W^(1)) so that the cubic Taylor term and the spectra stay near 1 on
    unit-normalized windows.  rate_gain holds one public factor per band,
    folded into the frequency weights and the mask of that band's rate
    average (its numerator and denominator, not their ratio, the rate):
    S = P^gamma is an amplitude^24 quantity whose size spans about 18 decades
    over synthetic windows, and the factors (10^3 respiration, 10^-1 heart
    rate) put the median window's sums near 1, where the decoded sums keep
    1e-3 absolute accuracy and their ratio stays well conditioned against the
    absolute noise of the lane-sum rotations.  With magnitude_degree > 0 the configuration also
    carries the power-basis coefficients of a polynomial magnitude (sqrt_poly),
    which the bin estimate's energy sums instead of the power.  phase_power is
    K4's mask exponent P_phi (2 .. 5)."""
    res = fps / frames
    bands = {"resp": (0.1, 0.6), "hr": (0.8, 2.5)}
    cfg = dict(frames=frames, bins=bins, fps=fps, taylor_order=taylor_order,
               window=np.hanning(frames), dft_gain=dft_gain, gamma=gamma,
               rate_gain={"resp": 1e3, "hr": 1e-1}, fir_backend=fir_backend,
               phase_power=phase_power)
    if magnitude_degree:
        # the bin estimate's energy sums a polynomial magnitude instead of the power
        cfg["mag_coeffs"] = sqrt_poly(magnitude_degree)
    for name, (lo, hi) in bands.items():
        cfg[f"taps_{name}"] = fir_gain * fir_bandpass(taps, lo, hi, fps)
        cfg[f"k_{name}"] = list(range(int(np.ceil(lo / res - 1e-9)),
                                      int(np.floor(hi / res + 1e-9)) + 1))
    return cfg


# ---- synthetic gesture window and the gesture pipeline's public constants ----

def gesture_window(seed: int, frames: int = 30, bins: int = 32, chirps: int = 32,
                   fps: float = 10.0, snr_db: float = 20.0) -> np.ndarray:
    """Range-processed FMCW frames [frames][range bins][chirps] (complex) of
    1-3 point scatterers on random constant-acceleration trajectories (range
    and radial velocity; the range and Doppler spectra of Appendix A), plus
    complex Gaussian noise at snr_db, normalized to max |x| = 1."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 4))
    t = np.arange(frames) / fps
    c = np.arange(chirps)
    x = np.zeros((frames, bins, chirps), dtype=np.complex128)
    for _ in range(k):
        r0 = rng.uniform(4, bins - 4)
        v0 = rng.uniform(-0.4, 0.4)           # Doppler cycles per chirp
        acc = rng.uniform(-0.3, 0.3)
        amp = rng.uniform(0.5, 1.0)
        phi = rng.uniform(0, 2 * np.pi)
        for f in range(frames):
            r = r0 + 3.0 * np.sin(2 * np.pi * 0.3 * t[f] + phi)
            fd = np.clip(v0 + acc * t[f], -0.45, 0.45)
            prof = np.sinc(np.arange(bins) - r)           # range-FFT peak shape
            x[f] += amp * prof[:, None] * np.exp(1j * (2 * np.pi * fd * c + phi))[None, :]
    p_sig = np.mean(np.abs(x) ** 2)
    sigma = np.sqrt(p_sig / 10 ** (snr_db / 10) / 2)
    x += sigma * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    return x / np.abs(x).max()


def gesture_pipeline_config(frames: int = 30, bins: int = 32, chirps: int = 32,
                            hidden=(64, 32), classes: int = 5, seed: int = 77,
                            feature_gain: float = 4.0) -> dict:
    """The gesture pipeline's public parameters (section 3.3.3 example
    pipeline): the Hann window of the Doppler DFT over the chirps (fftshifted,
    normalized by its sum), the notch (the zero-Doppler bin after fftshift,
    reading of Eq. notch_mask for even D), and random public weights of the
    FC network chirps*bins -> hidden[0] -> hidden[1] -> classes (trained
    weights are not available); feature_gain is folded into W1 (the paper
    folds its normalization into W^(1))."""
    rng = np.random.default_rng(seed)
    dims = [bins * chirps, hidden[0], hidden[1], classes]
    ws, bs = [], []
    for i in range(3):
        w = rng.standard_normal((dims[i + 1], dims[i])) / np.sqrt(dims[i])
        if i == 0:
            w = w * feature_gain
        ws.append(w)
        bs.append(rng.uniform(-0.1, 0.1, dims[i + 1]))
    return dict(frames=frames, bins=bins, chirps=chirps, window=np.hanning(chirps),
                notch=[chirps // 2], weights=ws, biases=bs)


def cnn_activation(degree: int = 3, bound: float = 6.0) -> list:
    """Power-basis coefficients of the CNN's degree-3 activation: the
    least-squares fit of the logistic sigmoid on [-bound, bound] (the
    HE-friendly sigmoid of polynomial networks)."""
    x = np.linspace(-bound, bound, 2001)
    y = 1.0 / (1.0 + np.exp(-x))
    c = np.polynomial.polynomial.polyfit(x, y, degree)
    return [float(v) if abs(v) > 1e-12 else 0.0 for v in c]


def gesture_cnn_config(frames: int = 30, bins: int = 32, chirps: int = 32, c1: int = 8,
                       c2: int = 16, hidden: int = 64, classes: int = 10, seed: int = 78,
                       feature_gain: float = 4.0) -> dict:
    """The gesture CNN's public parameters: the front end of the gesture
    pipeline (Doppler DFT window, notch), then two 3 x 3 convolutions with
    stride 2 and zero padding (1 -> c1 -> c2 channels on the bins x chirps
    feature map), 2 x 2 average pooling, dense c2 (bins/8) (chirps/8) ->
    hidden -> classes, with the degree-3 activation after both convolutions
    and the first dense layer.  Weights are random and public (trained ones
    are not available); feature_gain is folded into the first convolution."""
    if bins % 8 or chirps % 8:
        raise ValueError("bins and chirps must be multiples of 8")
    rng = np.random.default_rng(seed)
    conv1 = rng.standard_normal((c1, 3, 3)) / 3.0 * feature_gain
    conv2 = rng.standard_normal((c2, c1, 3, 3)) / np.sqrt(9.0 * c1)
    flat = c2 * (bins // 8) * (chirps // 8)
    dense1 = rng.standard_normal((hidden, flat)) / np.sqrt(flat)
    dense2 = rng.standard_normal((classes, hidden)) / np.sqrt(hidden)
    return dict(frames=frames, bins=bins, chirps=chirps, window=np.hanning(chirps),
                notch=[chirps // 2], conv1=conv1, conv2=conv2, dense1=dense1,
                dense2=dense2, bias1=rng.uniform(-0.1, 0.1, hidden),
                bias2=rng.uniform(-0.1, 0.1, classes), act=cnn_activation())

