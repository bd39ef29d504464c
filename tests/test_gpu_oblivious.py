"""Data obliviousness of the cloud-side pipelines (Theorem 2; proof in
Appendix D): for two inputs of the same public configuration the execution
trace is the same.

The library's launch trace (hck_trace_*) records, in issue order, every
kernel launch (name, grid, algorithmic bytes, modular multiplications) and
every device allocation and release, as the host issues them.  Each test runs
a pipeline on two different synthetic windows (different scenes, different
encryption randomness) with the same plan and keys, and requires identical
traces, while the encrypted outputs differ.  One untraced window runs first:
the first call on a context allocates its scratch ciphertexts and workspaces,
which later calls reuse (allocation depends on the library's cache state, a
public quantity, not on the data).
"""
import numpy as np
import pytest

import paper_2603_22437_amd as H
import seeded_inputs as S
from paper_2603_22437_amd import gesture as HG
from paper_2603_22437_amd import vital as HV

pytestmark = pytest.mark.gpu


def _encrypt(ctx, sk, x, scale, level, seed):
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: x.size] = x.reshape(-1)
    return (ctx.encrypt_sk(sk, ctx.encode(v.real, scale, level), seed),
            ctx.encrypt_sk(sk, ctx.encode(v.imag, scale, level), seed + 1))


def _traced(ctx, fn):
    ctx.synchronize()
    ctx.trace(True)
    out = fn()
    ctx.trace(False)
    return ctx.trace_read(), out


def _assert_same_trace(t1, t2, kernels):
    assert len(t1) > 0
    if t1 != t2:
        first = next((i for i, (a, b) in enumerate(zip(t1, t2)) if a != b), min(len(t1), len(t2)))
        raise AssertionError(f"traces differ: {len(t1)} vs {len(t2)} records, first at {first}: "
                             f"{t1[first:first + 3]} vs {t2[first:first + 3]}")
    names = {r[0] for r in t1}
    assert kernels <= names, kernels - names


def _outputs(ctx, cts):
    return [ctx.ciphertext_export(c)[0] for c in cts]


def test_vital_pipeline_trace_is_data_independent():
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.vital_pipeline_config()
    l0 = len(prm["q"]) - 1
    plan = HV.encode_plan(ctx, cfg, l0)
    gks = ctx.keygen_rotation(sk, ctx.vital_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    runs = []
    for seed in (3000, 3001, 3002):
        z = S.vital_window(seed, cfg["frames"], cfg["bins"])
        re, im = _encrypt(ctx, sk, z, prm["scale"], l0, seed)
        runs.append(_traced(ctx, lambda: ctx.vital_eval(plan, re, im, gks, rlk)))
    _, (t1, o1), (t2, o2) = runs
    _assert_same_trace(t1, t2, {"ks_modup_strided", "ks_moddown_tail", "lt_inner", "tensor"})
    assert not all(np.array_equal(a, b) for a, b in zip(_outputs(ctx, o1), _outputs(ctx, o2)))


def test_gesture_pipeline_trace_is_data_independent():
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.gesture_pipeline_config(frames=14)
    l0 = len(prm["q"]) - 1
    plan = HG.encode_plan(ctx, cfg, l0, prm["scale"])
    gks = ctx.keygen_rotation(sk, ctx.gesture_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    runs = []
    for seed in (3010, 3011, 3012):
        x = S.gesture_window(seed, cfg["frames"])
        re, im = _encrypt(ctx, sk, x, prm["scale"], l0, seed)
        runs.append(_traced(ctx, lambda: ctx.gesture_eval(plan, re, im, gks, rlk)))
    _, (t1, o1), (t2, o2) = runs
    _assert_same_trace(t1, t2, {"ks_modup_strided", "lt_inner", "tensor"})
    assert not np.array_equal(*_outputs(ctx, [o1, o2]))


def test_gesture_cnn_trace_is_data_independent():
    prm = S.params("cnn11")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    cfg = S.gesture_cnn_config(frames=16, bins=8, chirps=8, c1=4, c2=8, hidden=16,
                              classes=4, seed=5)
    l0 = len(prm["q"]) - 1
    plan = HG.encode_cnn_plan(ctx, cfg, l0, prm["scale"])
    gks = ctx.keygen_rotation(sk, ctx.gesture_cnn_required_steps(plan), 5)
    rlk = ctx.keygen_relin(sk, 7)
    runs = []
    for seed in (3020, 3021, 3022):
        x = S.gesture_window(seed, cfg["frames"], cfg["bins"], cfg["chirps"])
        re, im = _encrypt(ctx, sk, x, prm["scale"], l0, seed)
        runs.append(_traced(ctx, lambda: ctx.gesture_cnn_eval(plan, re, im, gks, rlk)))
    _, (t1, o1), (t2, o2) = runs
    _assert_same_trace(t1, t2, {"ks_modup_strided", "lt_inner", "tensor"})
    assert not np.array_equal(*_outputs(ctx, [o1, o2]))


def test_trace_records_launch_shapes():
    """The records follow the public shape: the same operation at a lower
    level launches fewer rows, and nothing is recorded with the trace off."""
    prm = S.params("tiny")
    ctx = H.Context.from_params(prm)
    sk = ctx.keygen_secret(1)
    top = len(prm["q"]) - 1
    x = S.uniform_residues([int(q) for q in prm["q"]], ctx.n, 5)[0]
    ct = ctx.encrypt_sk(sk, ctx.plaintext_import(x, top, 2.0 ** 25), 9)
    out = ctx.ciphertext()
    ctx.add(ct, ct, out)                     # allocates out
    t_top, _ = _traced(ctx, lambda: ctx.add(ct, ct, out))
    low = ctx.ciphertext()
    ctx.drop_level(ct, 1, low)
    t_low, _ = _traced(ctx, lambda: ctx.add(low, low, out))
    # one launch per polynomial, over the ciphertext's limbs
    assert [r[0] for r in t_top] == [r[0] for r in t_low] == ["addsub", "addsub"]
    assert [r[1] for r in t_top] == [(ctx.n // 256, top + 1, 1)] * 2
    assert [r[1] for r in t_low] == [(ctx.n // 256, 2, 1)] * 2
    assert t_top[0][2] == 24.0 * ctx.n * (top + 1) and t_low[0][2] == 24.0 * ctx.n * 2
    ctx.trace(False)
    ctx.add(ct, ct, out)
    ctx.synchronize()
    assert ctx.trace_read() == t_low
