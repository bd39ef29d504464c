"""The gesture CNN variant on the host: the plaintext network pinned to an
independent formulation (scipy correlation with stride and padding, numpy
pooling), and the oracle's homomorphic composition pinned to the plaintext
network stage by stage (decoded taps at the slots the packing assigns) on a
small ring, N = 2^11 with 21 primes and an 8 x 8 feature map."""
import numpy as np
import pytest
from scipy.signal import correlate2d

import oracle as O
import seeded_inputs as S
from oracle import gesture_cnn as OC


def small_cfg():
    return S.gesture_cnn_config(frames=16, bins=8, chirps=8, c1=4, c2=8, hidden=16,
                                classes=4, seed=5)


def _conv_scipy(img, w):
    """3 x 3 convolution layer, zero padding 1, stride 2, by scipy."""
    out = []
    for o in range(w.shape[0]):
        acc = sum(correlate2d(img[c], w[o, c], mode="same") for c in range(img.shape[0]))
        out.append(acc[::2, ::2])
    return np.array(out)


@pytest.mark.parametrize("cfg", [small_cfg(), S.gesture_cnn_config()], ids=["8x8", "32x32"])
def test_plain_network_matches_scipy_formulation(cfg):
    x = S.gesture_window(2001, cfg["frames"], cfg["bins"], cfg["chirps"])
    st = OC.plain_stages(cfg, x)
    act = lambda v: np.polynomial.polynomial.polyval(v, cfg["act"])
    a1 = act(_conv_scipy(st["feature"][None], cfg["conv1"][:, None]))
    np.testing.assert_allclose(st["a1"], a1, rtol=1e-12, atol=1e-12)
    a2 = act(_conv_scipy(a1, cfg["conv2"]))
    np.testing.assert_allclose(st["a2"], a2, rtol=1e-12, atol=1e-12)
    c2, h, w = a2.shape
    pooled = np.array([[[a2[o, 2 * i:2 * i + 2, 2 * j:2 * j + 2].mean() for j in range(w // 2)]
                        for i in range(h // 2)] for o in range(c2)])
    a3 = act(cfg["dense1"] @ pooled.reshape(-1) + cfg["bias1"])
    np.testing.assert_allclose(st["a3"], a3, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(st["logits"], cfg["dense2"] @ a3 + cfg["bias2"], rtol=1e-12,
                               atol=1e-12)


def test_activation_is_the_sigmoid_fit():
    c = S.cnn_activation()
    assert len(c) == 4 and c[3] != 0
    x = np.linspace(-6, 6, 101)
    assert np.max(np.abs(np.polynomial.polynomial.polyval(x, c) - 1 / (1 + np.exp(-x)))) < 0.1


def test_oracle_cnn_decodes_to_the_plaintext_network_stage_by_stage():
    prm = S.params("cnn11")
    o = O.Oracle(prm)
    cfg = small_cfg()
    s = o.keygen_secret(1)
    l0 = len(prm["q"]) - 1
    ops = OC.encode_operands(o, cfg, l0, prm["scale"])
    gks = {o.galois_element(k): o.keygen_galois(s, o.galois_element(k), 5)
           for k in OC.required_steps(o, cfg, ops)}
    rlk = o.keygen_relin(s, 7)
    # a window with a strong scatterer, so that every stage carries signal
    x = S.gesture_window(2006, cfg["frames"], cfg["bins"], cfg["chirps"])
    v = np.zeros(o.n_slots, dtype=np.complex128)
    v[: x.size] = x.reshape(-1)
    re = o.encrypt_sk(s, o.encode(v.real, prm["scale"], l0), 10)
    im = o.encrypt_sk(s, o.encode(v.imag, prm["scale"], l0), 11)
    taps = []
    logits = OC.evaluate(o, cfg, ops, re, im, gks, rlk, taps)
    assert logits.level == OC.levels(l0, cfg["act"])["out"] == 1
    st = OC.plain_stages(cfg, x)
    for i, (tap, (slots, want)) in enumerate(zip(taps, OC.stage_slots(cfg, o.n_slots, st))):
        got = o.decode(o.decrypt(s, tap)).real[slots]
        assert np.max(np.abs(got - want)) < 1e-6, (i, np.max(np.abs(got - want)))
    got = o.decode(o.decrypt(s, logits)).real[: cfg["dense2"].shape[0]]
    np.testing.assert_allclose(got, st["logits"], rtol=0, atol=1e-6)
    # the taps are informative: the convolutions see the scatterers
    assert np.ptp(st["a1"]) > 0.1 and np.ptp(st["a2"]) > 1e-3
