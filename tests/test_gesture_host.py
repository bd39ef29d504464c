"""Host-side checks of the gesture pipeline (no GPU): the library's operand
builder against the oracle's, and the oracle pipeline against the same
circuit on plaintext numbers."""
import numpy as np
import pytest

import oracle as O
import seeded_inputs as S
from oracle import gesture as OG
from paper_2603_22437_amd import gesture as HG


@pytest.mark.parametrize("frames,n_slots", [(30, 1 << 15), (14, 1 << 14)])
def test_operand_vectors_match_oracle(frames, n_slots):
    cfg = S.gesture_pipeline_config(frames=frames)
    a = HG.operand_vectors(cfg, n_slots)
    b = OG.operand_vectors(cfg, n_slots)
    assert set(a) == set(b)
    for k in a:
        if isinstance(a[k], dict):
            assert set(a[k]) == set(b[k]), k
            for off in a[k]:
                np.testing.assert_allclose(a[k][off], b[k][off], rtol=0, atol=1e-15)
        else:
            np.testing.assert_allclose(a[k], b[k], rtol=0, atol=1e-15, err_msg=k)
    assert HG.BABY == OG.BABY and HG.DEPTH == OG.DEPTH
    prm = S.params("vital")
    o = O.Oracle(prm)
    assert HG.scales_at_biases(prm["q"], 23, prm["scale"]) == OG.bias_scales(o, 23, prm["scale"])


def test_layout_checks():
    cfg = S.gesture_pipeline_config(frames=30)
    with pytest.raises(ValueError):
        OG.operand_vectors(cfg, 1 << 14)      # 32 x 1024 > 2^14 slots
    with pytest.raises(ValueError):
        HG.operand_vectors(cfg, 1 << 14)


def test_plain_circuit_features():
    """The plaintext mirror's Doppler stage is the windowed, fftshifted DFT
    over chirps (Eq. dft_kernel): a single tone lands on its shifted bin."""
    cfg = S.gesture_pipeline_config(frames=2, bins=2, chirps=32)
    d = cfg["chirps"]
    x = np.zeros((2, 2, d), dtype=np.complex128)
    x[:, :, :] = np.exp(2j * np.pi * 5 * np.arange(d) / d)
    w = np.asarray(cfg["window"])
    sig = (np.arange(d) + d // 2) % d
    spec = (w[None, :] * np.exp(-2j * np.pi * np.outer(sig, np.arange(d)) / d) / w.sum()) @ x[0, 0]
    assert int(np.argmax(np.abs(spec))) == (5 - d // 2) % d


@pytest.mark.slow
def test_oracle_pipeline_decodes_to_plain_circuit():
    prm = S.params("mix15")
    o = O.Oracle(prm)
    s = o.keygen_secret(1)
    cfg = S.gesture_pipeline_config(frames=14)
    x = S.gesture_window(2000, cfg["frames"])
    l0 = o.L - 1
    ops = OG.encode_operands(o, cfg, l0, prm["scale"])
    steps = OG.required_steps(o, cfg, ops)
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5) for k in steps}
    rlk = o.keygen_relin(s, 7)
    re, im = OG.encrypt_window(o, s, x, l0, prm["scale"], 100)
    out = OG.evaluate(o, cfg, ops, re, im, gks, rlk)
    assert out.level == l0 - OG.DEPTH
    classes = cfg["weights"][2].shape[0]
    got = o.decode(o.decrypt(s, out))[:classes].real
    np.testing.assert_allclose(got, OG.plain(cfg, x), rtol=0, atol=1e-6)


def test_library_plain_stages_end_in_the_oracle_logits():
    """The library's plaintext execution (the reference of the per-kernel
    noise table) ends in the oracle's plaintext logits and places every
    stage where the packing puts it."""
    cfg = S.gesture_pipeline_config(frames=30)
    x = S.gesture_window(2005, cfg["frames"])
    st = HG.plain_stages(cfg, x, 1 << 15)
    assert len(st) == 8 + 1
    np.testing.assert_allclose(st[-1][1], OG.plain(cfg, x), rtol=1e-12, atol=1e-12)
    # K3's bins of frame t, range r sit at slot (t R + r) D + k
    t, r, k = 7, 5, 3
    slots, d_re = st[0]
    spec = np.fft.fftshift(np.fft.fft(np.asarray(cfg["window"]) * x[t, r]))
    idx = int(np.flatnonzero(slots == (t * cfg["bins"] + r) * cfg["chirps"] + k)[0])
    assert abs(d_re[idx] - spec[k].real / np.sum(cfg["window"])) < 1e-12


def _gest12_setup(frames_in_plan=2):
    prm = S.params("gest12")
    o = O.Oracle(prm)
    s = o.keygen_secret(1)
    cfg = S.gesture_pipeline_config(frames=frames_in_plan)
    l0 = o.L - 1
    ops = OG.encode_operands(o, cfg, l0, prm["scale"])
    steps = OG.required_steps(o, cfg, ops)
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5) for k in steps}
    rlk = o.keygen_relin(s, 7)
    return prm, o, s, cfg, l0, ops, gks, rlk


def test_oracle_per_frame_packing_decodes_to_plain_circuit():
    """Per-frame packing (one ciphertext pair per frame, section 3.3.2) in the
    oracle: three frames, each through K3 -> K1 -> K6 -> K2 on its own and
    then added and spread over the ring's two blocks of 1024 slots, decode to
    the plaintext circuit's logits over the three frames (N = 2^12)."""
    prm, o, s, cfg, l0, ops, gks, rlk = _gest12_setup()
    x = S.gesture_window(2010, 3)
    # FC1's cyclic diagonals read past the first block only for the features
    # of range bins 0 and 1: the strongest range bin is rolled to bin 0, so a
    # frame sum left unspread (zeros beyond the first block) changes the
    # logits by about 1e-3
    peak = int(np.argmax((np.abs(x) ** 2).sum(axis=(0, 2))))
    x = np.roll(x, -peak, axis=1)
    res, ims = OG.encrypt_frames(o, s, x, l0, prm["scale"], 300)
    out = OG.evaluate_frames(o, cfg, ops, res, ims, gks, rlk)
    assert out.level == l0 - OG.DEPTH
    classes = cfg["weights"][2].shape[0]
    got = o.decode(o.decrypt(s, out))[:classes].real
    np.testing.assert_allclose(got, OG.plain(cfg, x), rtol=0, atol=1e-6)


def test_oracle_per_frame_packing_of_one_frame_is_the_batched_pipeline():
    """With one frame the two packings are the same ciphertext operations:
    bit-identical residues."""
    prm, o, s, cfg, l0, ops, gks, rlk = _gest12_setup()
    x = S.gesture_window(2011, 1)
    re, im = OG.encrypt_window(o, s, x, l0, prm["scale"], 400)
    a = OG.evaluate(o, cfg, ops, re, im, gks, rlk)
    b = OG.evaluate_frames(o, cfg, ops, [re], [im], gks, rlk)
    assert a.level == b.level and a.scale == b.scale
    assert np.array_equal(a.polys, b.polys)
