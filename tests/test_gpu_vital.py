"""The vital-sign pipeline on the GPU (hck_vital_eval).

* N = 2^15, L = 12 (the third-order circuit's 11 levels): residues of all four
  outputs bit-exact (also with the polynomial magnitude option, with
  gamma = 4, with the rotation-based FIR backend and with K4 exponents
  P_phi = 3, 4, 5) against the oracle's pipeline, both sides fed the same
  integer operands (encoded once by the oracle) and the same encrypted
  window; per-frame packing bit-exact against the oracle's per-frame
  composition at N = 2^12.
* N = 2^16, L = 24 (the benchmark ring), with the library's own encoder:
  decoded outputs against the circuit on plaintext numbers.
"""
import numpy as np
import pytest

import oracle as O
import paper_2603_22437_amd as H
import seeded_inputs as S
from oracle import vital as OV
from paper_2603_22437_amd import vital as HV

pytestmark = pytest.mark.gpu


def decoded_tol(v: float) -> float:
    """Decoded-output bound against plaintext: 1e-3 absolute, and 1e-8
    relative for outputs above 10^5.  The rate sums are fourth powers of the
    phase spectrum (S = P^2, P = |X|^2), spanning about 18 decades over
    windows; CKKS noise after a product is relative to its operands' size,
    measured at 2.5e-9 of the value at scale 2^50."""
    return max(1e-3, 1e-8 * abs(v))


def well_conditioned(den: float, ratio: float) -> bool:
    """Whether the client's ratio num / den is asserted to 1e-3: the decoded
    sums carry an absolute noise floor of about 2e-8 (the lane-sum
    rotations), which moves the ratio by about 2e-8 (1 + |ratio|) / den."""
    return den > 1e-4 * (1.0 + abs(ratio))


def _import_plan(ctx, o, cfg, ops):
    """GPU plan holding the oracle's encoded operands."""
    handles = {}
    for name, v in ops.items():
        if isinstance(v, O.LinearTransform):
            res = {g * v.n1 + b: pt.res for g, items in v.groups.items() for b, pt in items}
            handles[name] = ctx.lt_create_from_residues(res, v.n1, v.level, v.scale)
        else:
            handles[name] = ctx.plaintext_import(v.res, v.level, v.scale)
    return H.VitalPlan.build(cfg["frames"], cfg["bins"], cfg["taylor_order"],
                             len(cfg["k_resp"]), len(cfg["k_hr"]), handles,
                             cfg.get("mag_coeffs"), cfg.get("gamma", 2),
                             cfg.get("phase_power", 2))


@pytest.mark.parametrize("order,magnitude,gamma,fir,phase", [
    (3, 0, 2, "toeplitz", 2), (1, 0, 2, "toeplitz", 2), (3, 8, 2, "toeplitz", 2),
    (1, 0, 4, "toeplitz", 2), (3, 0, 2, "rotation", 2), (1, 0, 2, "toeplitz", 3),
    (1, 0, 2, "toeplitz", 4), (1, 0, 2, "toeplitz", 5)])
def test_vital_pipeline_matches_oracle(order, magnitude, gamma, fir, phase):
    prm = S.params("mix15")
    o = O.Oracle(prm)
    ctx = H.Context.from_params(prm)
    s_o = o.keygen_secret(1)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config(taylor_order=order, magnitude_degree=magnitude, gamma=gamma,
                                  fir_backend=fir, phase_power=phase)
    z = S.vital_window(1001, cfg["frames"], cfg["bins"])
    l0 = o.L - 1
    ops = OV.encode_operands(o, cfg, l0)
    plan = _import_plan(ctx, o, cfg, ops)
    steps = OV.required_steps(o, cfg, ops)
    assert ctx.vital_required_steps(plan) == steps
    gko = {o.galois_element(k): o.keygen_galois(s_o, o.galois_element(k), 5) for k in steps}
    rlk_o = o.keygen_relin(s_o, 7)
    gks = ctx.keygen_rotation(sk, steps, 5)
    rlk = ctx.keygen_relin(sk, 7)
    re_o, im_o = OV.encrypt_window(o, s_o, z, l0, prm["scale"], 100)
    re = ctx.ciphertext_import(re_o.polys, l0, re_o.scale)
    im = ctx.ciphertext_import(im_o.polys, l0, im_o.scale)
    got = ctx.vital_eval(plan, re, im, gks, rlk)
    want = OV.evaluate(o, cfg, ops, re_o, im_o, gko, rlk_o)
    for name, g in zip(OV.OUTPUTS, got):
        res, lvl, sc = ctx.ciphertext_export(g)
        assert lvl == want[name].level, name
        assert sc == want[name].scale, name
        assert np.array_equal(res, want[name].polys), name


def test_vital_pipeline_decodes_at_benchmark_ring():
    prm = S.params("vital")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config()
    z = S.vital_window(1002, cfg["frames"], cfg["bins"])
    l0 = len(prm["q"]) - 1
    plan = HV.encode_plan(ctx, cfg, l0)
    gks = ctx.keygen_rotation(sk, ctx.vital_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: z.size] = z.reshape(-1)
    re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], l0), 100)
    im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], l0), 101)
    got = ctx.vital_eval(plan, re, im, gks, rlk)
    want = OV.plain_slots(cfg, z, ctx.n_slots)
    dec = {}
    for name, g in zip(OV.OUTPUTS, got):
        dec[name] = ctx.decode(ctx.decrypt(sk, g)).real
        for slot, v in want[name].items():
            assert abs(dec[name][slot] - v) < decoded_tol(v), (name, slot, dec[name][slot], v)
    # the client's divisions (section 3.3.4)
    checked = 0
    for num, den in (("num_bin", "den_bin"), ("num_rates", "den_rates")):
        for slot in want[num]:
            ratio = want[num][slot] / want[den][slot]
            if well_conditioned(want[den][slot], ratio):
                est = dec[num][slot] / dec[den][slot]
                assert abs(est - ratio) < 1e-3, (num, slot, est, ratio)
                checked += 1
    assert checked == 3    # both rates and the bin on this window


def test_vital_plan_errors():
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    cfg = S.vital_pipeline_config()
    plan = HV.encode_plan(ctx, cfg, len(prm["q"]) - 1)
    bad = H.VitalPlan.build(cfg["frames"], 48, 3, 6, 18, plan._keep)   # bins not 2^k
    with pytest.raises(H.HckError):
        ctx.vital_required_steps(bad)
    sk = ctx.keygen_secret(1)
    rlk = ctx.keygen_relin(sk, 7)
    gks = ctx.keygen_rotation(sk, [1], 5)
    low = ctx.encrypt_sk(sk, ctx.encode(np.zeros(ctx.n_slots), prm["scale"], 5), 3)
    with pytest.raises(H.HckError):   # level 5 < depth 11
        ctx.vital_eval(plan, low, low, gks, rlk)
    top = ctx.encrypt_sk(sk, ctx.encode(np.zeros(ctx.n_slots), prm["scale"],
                                        len(prm["q"]) - 1), 4)
    with pytest.raises(H.HckError):   # keys missing
        ctx.vital_eval(plan, top, top, gks, rlk)
    for e in (1, 6):                  # P_phi outside 2 .. 5
        odd = H.VitalPlan.build(cfg["frames"], cfg["bins"], 3, 6, 18, plan._keep, phase_power=e)
        with pytest.raises(H.HckError):
            ctx.vital_required_steps(odd)


def test_vital_windows_together_match_single_windows():
    """Several windows evaluated together (shared key-switch batches) give
    each window's residues of the single-window evaluation, which the test
    above pins to the oracle."""
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config()
    l0 = len(prm["q"]) - 1
    plan = HV.encode_plan(ctx, cfg, l0)
    gks = ctx.keygen_rotation(sk, ctx.vital_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    res, ims = [], []
    for k in range(3):
        z = S.vital_window(1010 + k, cfg["frames"], cfg["bins"])
        v = np.zeros(ctx.n_slots, dtype=np.complex128)
        v[: z.size] = z.reshape(-1)
        res.append(ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], l0), 400 + k))
        ims.append(ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], l0), 500 + k))
    together = ctx.vital_eval_many(plan, res, ims, gks, rlk)
    for k in range(3):
        alone = ctx.vital_eval(plan, res[k], ims[k], gks, rlk)
        for a, b in zip(alone, together[k]):
            assert np.array_equal(ctx.ciphertext_export(a)[0], ctx.ciphertext_export(b)[0]), k


def test_vital_taps_follow_plaintext_execution():
    """hck_vital_eval_taps: outputs bit-identical to hck_vital_eval's, and
    every kernel's decoded intermediate within the paper's per-kernel
    encryption-noise bound (MSE < 1e-5, section 5.2) of plaintext execution,
    at the depth the circuit assigns it."""
    prm = S.params("vital")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config()
    z = S.vital_window(1004, cfg["frames"], cfg["bins"])
    l0 = len(prm["q"]) - 1
    plan = HV.encode_plan(ctx, cfg, l0)
    gks = ctx.keygen_rotation(sk, ctx.vital_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: z.size] = z.reshape(-1)
    re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], l0), 100)
    im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], l0), 101)
    outs, taps = ctx.vital_eval_taps(plan, re, im, gks, rlk)
    ref = ctx.vital_eval(plan, re, im, gks, rlk)
    for a, b in zip(outs, ref):
        assert np.array_equal(ctx.ciphertext_export(a)[0], ctx.ciphertext_export(b)[0])
    # levels: the bin branch (K1 energy, K2 attention, the bin outputs) runs
    # at levels 3, 2, 1; the rest descends from l0 with the circuit's depth
    levels = [l0 - 1, 3, 2, l0 - 3, l0 - 3, l0 - 4, l0 - 4, l0 - 4, l0 - 4, l0 - 7, l0 - 7,
              l0 - 8, l0 - 8, l0 - 9, l0 - 10, 1, 1, l0 - 11, l0 - 11]
    names = ctx.VITAL_TAPS + plan.OUTPUTS
    for name, c, (slots, want), lv in zip(names, taps + outs,
                                          HV.plain_stages(cfg, z, ctx.n_slots), levels):
        assert c.level == lv, name
        err = ctx.decode(ctx.decrypt(sk, c)).real[slots] - want
        assert np.mean(err ** 2) < 1e-5 and np.max(np.abs(err)) < 1e-3, name


def test_vital_inputs_above_the_plan_level_are_dropped():
    """A plan encoded for inputs at level 12 of 24 (the depth, 11, plus one
    level of headroom for the rate numerators, fourth powers of the spectrum
    times frequencies, whose magnitude depends on the window):
    top-level inputs are dropped to it, giving exactly the residues of inputs
    the caller dropped, and the decoded outputs of the plaintext circuit."""
    prm = S.params("vital")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config()
    top = len(prm["q"]) - 1
    plan = HV.encode_plan(ctx, cfg, 12)
    gks = ctx.keygen_rotation(sk, ctx.vital_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    z = S.vital_window(1005, cfg["frames"], cfg["bins"])
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: z.size] = z.reshape(-1)
    re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], top), 100)
    im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], top), 101)
    got = ctx.vital_eval(plan, re, im, gks, rlk)
    ref = ctx.vital_eval(plan, ctx.drop_level(re, 12), ctx.drop_level(im, 12), gks, rlk)
    for a, b in zip(got, ref):
        assert np.array_equal(ctx.ciphertext_export(a)[0], ctx.ciphertext_export(b)[0])
    assert [c.level for c in got] == [1, 1, 1, 1]
    want = OV.plain_slots(cfg, z, ctx.n_slots)
    dec = {name: ctx.decode(ctx.decrypt(sk, g)).real for name, g in zip(OV.OUTPUTS, got)}
    # every output within the decoded tolerance, and the client's quantity,
    # the rate in beats per minute, within 1e-3 (both bands are well
    # conditioned on this strong window)
    for name in ("num_bin", "den_bin"):
        assert abs(dec[name][0] - want[name][0]) < 1e-3, name
    for name in ("num_rates", "den_rates"):
        for slot, val in want[name].items():
            assert abs(dec[name][slot] - val) < decoded_tol(val), (name, slot, val)
    for slot in want["num_rates"]:
        ratio = want["num_rates"][slot] / want["den_rates"][slot]
        assert well_conditioned(want["den_rates"][slot], ratio), slot
        bpm = dec["num_rates"][slot] / dec["den_rates"][slot]
        assert abs(bpm - ratio) < 1e-3, slot
    low = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], 11), 102)
    with pytest.raises(H.HckError):   # below the plan's level
        ctx.vital_eval(plan, low, low, gks, rlk)


def test_vital_magnitude_option_decodes_at_benchmark_ring():
    """The magnitude option (the bin estimate sums a degree-8 polynomial
    magnitude of the power) at N = 2^16 from plan level 12: outputs decode to
    the same circuit on plaintext numbers, and the bin estimate stays on the
    synthetic target."""
    prm = S.params("vital")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config(magnitude_degree=8)
    plan = HV.encode_plan(ctx, cfg, 12)
    gks = ctx.keygen_rotation(sk, ctx.vital_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    z = S.vital_window(1006, cfg["frames"], cfg["bins"])
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: z.size] = z.reshape(-1)
    top = len(prm["q"]) - 1
    re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], top), 100)
    im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], top), 101)
    got = ctx.vital_eval(plan, re, im, gks, rlk)
    want = OV.plain_slots(cfg, z, ctx.n_slots)
    num, den = (ctx.decode(ctx.decrypt(sk, got[i])).real[0] for i in (0, 1))
    assert abs(num - want["num_bin"][0]) < 1e-3 and abs(den - want["den_bin"][0]) < 1e-3
    target = int(np.argmax(np.abs(z).sum(axis=0)))
    assert abs(num / den - target) < 1.0


def test_vital_per_frame_packing_matches_oracle():
    """Per-frame packing (section 3.3.2) at N = 2^12, L = 12, 32 frames of 32
    bins: the four outputs bit-exact against the oracle's per-frame
    composition, both sides fed the same integer operands and frame pairs."""
    prm = S.params("gest12")
    o = O.Oracle(prm)
    ctx = H.Context.from_params(prm)
    s_o = o.keygen_secret(1)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config(frames=32, bins=32, fps=4.0)
    z = S.vital_window(1003, cfg["frames"], cfg["bins"], fps=cfg["fps"])
    l0 = o.L - 1
    ops = OV.encode_operands(o, cfg, l0)
    plan = _import_plan(ctx, o, cfg, ops)
    steps = OV.frames_required_steps(o, cfg, ops)
    assert ctx.vital_frames_required_steps(plan) == steps
    gko = {o.galois_element(k): o.keygen_galois(s_o, o.galois_element(k), 5) for k in steps}
    rlk_o = o.keygen_relin(s_o, 7)
    gks = ctx.keygen_rotation(sk, steps, 5)
    rlk = ctx.keygen_relin(sk, 7)
    res_o, ims_o = OV.encrypt_frames(o, s_o, z, l0, prm["scale"], 300)
    res = [ctx.ciphertext_import(c.polys, l0, c.scale) for c in res_o]
    ims = [ctx.ciphertext_import(c.polys, l0, c.scale) for c in ims_o]
    got = ctx.vital_eval_frames(plan, res, ims, gks, rlk)
    want = OV.evaluate_frames(o, cfg, ops, res_o, ims_o, gko, rlk_o)
    for name, g in zip(OV.OUTPUTS, got):
        r, lvl, sc = ctx.ciphertext_export(g)
        assert lvl == want[name].level and sc == want[name].scale, name
        assert np.array_equal(r, want[name].polys), name
    with pytest.raises(H.HckError):     # one frame short of the plan's
        ctx.vital_eval_frames(plan, res[:-1], ims[:-1], gks, rlk)


def test_vital_per_frame_packing_decodes_at_benchmark_ring():
    """200 frame pairs of 64 bins at N = 2^16, L = 24 (encrypted at the plan's
    level 12): the outputs decode to the plaintext circuit's numbers."""
    prm = S.params("vital")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config()
    z = S.vital_window(1002, cfg["frames"], cfg["bins"])
    l0 = 12
    plan = HV.encode_plan(ctx, cfg, l0)
    gks = ctx.keygen_rotation(sk, ctx.vital_frames_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    res, ims = [], []
    for t in range(cfg["frames"]):
        v = np.zeros(ctx.n_slots, dtype=np.complex128)
        v[: cfg["bins"]] = z[t]
        res.append(ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], l0), 2 * t))
        ims.append(ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], l0), 2 * t + 1))
    got = ctx.vital_eval_frames(plan, res, ims, gks, rlk)
    want = OV.plain_slots(cfg, z, ctx.n_slots)
    for name, g in zip(OV.OUTPUTS, got):
        dec = ctx.decode(ctx.decrypt(sk, g)).real
        for slot, v in want[name].items():
            assert abs(dec[slot] - v) < decoded_tol(v), (name, slot, dec[slot], v)
