"""HIP-graph capture of evaluation calls (hck_graph_*).

* One context: the vital pipeline recorded once and replayed on new windows
  written into the same input ciphertexts; every replay's outputs equal, bit
  for bit, the eager call's on the same inputs, with eager work and waits
  between the replays.
* Two contexts on two streams (rings 2^15 and 2^12, one graph handle): a
  vital window on one ring and a gesture window on the other, replayed side
  by side, each equal to its eager result.
* Refusals: a recorded call that would allocate, a replay after a buffer
  was given back, a replay after a context was destroyed.
"""
import numpy as np
import pytest
import torch

import paper_2603_22437_amd as H
import seeded_inputs as S
from paper_2603_22437_amd import gesture as HG
from paper_2603_22437_amd import vital as HV

pytestmark = pytest.mark.gpu


def _slots(ctx, x):
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: x.size] = x.reshape(-1)
    return v


def _encrypt_into(ctx, sk, x, scale, level, seed, re, im):
    v = _slots(ctx, x)
    ctx.encrypt_sk(sk, ctx.encode(v.real, scale, level), seed, out=re)
    ctx.encrypt_sk(sk, ctx.encode(v.imag, scale, level), seed + 1, out=im)


def _export(ctx, cts):
    return [ctx.ciphertext_export(c) for c in cts]


def _same(a, b):
    assert len(a) == len(b)
    for (ra, la, sa), (rb, lb, sb) in zip(a, b):
        assert la == lb and sa == sb
        assert np.array_equal(ra, rb)


class _Vital:
    def __init__(self, prm, seed0):
        self.prm = prm
        self.ctx = H.Context.from_params(prm)
        self.stream = torch.cuda.Stream()
        self.ctx.set_stream(self.stream)
        ctx = self.ctx
        self.sk = ctx.keygen_secret(1)
        self.cfg = S.vital_pipeline_config()
        self.l0 = len(prm["q"]) - 1
        self.plan = HV.encode_plan(ctx, self.cfg, self.l0)
        self.gks = ctx.keygen_rotation(self.sk, ctx.vital_required_steps(self.plan), 5)
        self.rlk = ctx.keygen_relin(self.sk, 7)
        self.re, self.im = ctx.ciphertext(), ctx.ciphertext()
        self.out = [ctx.ciphertext() for _ in range(4)]
        self.load(seed0)

    def load(self, seed):
        z = S.vital_window(seed, self.cfg["frames"], self.cfg["bins"])
        _encrypt_into(self.ctx, self.sk, z, self.prm["scale"], self.l0, seed, self.re, self.im)

    def run(self, out=None):
        return self.ctx.vital_eval(self.plan, self.re, self.im, self.gks, self.rlk,
                                   outputs=self.out if out is None else out)


def test_vital_graph_replays_match_eager():
    v = _Vital(S.params("mix15"), 4000)
    v.run()                                  # allocates every buffer once
    with H.Graph.capture([v.ctx]) as g:
        v.run()
    assert g.info()["contexts"] == 1 and g.info()["nodes"] > 100
    eager_out = [v.ctx.ciphertext() for _ in range(4)]
    for seed in (4001, 4002, 4003):
        v.load(seed)
        g.launch()
        got = _export(v.ctx, v.out)
        v.run(eager_out)                     # eager on the same inputs
        _same(got, _export(v.ctx, eager_out))
        v.ctx.synchronize()
    g.close()


class _Gesture:
    def __init__(self, prm, seed0):
        self.prm = prm
        self.ctx = H.Context.from_params(prm)
        self.stream = torch.cuda.Stream()
        self.ctx.set_stream(self.stream)
        ctx = self.ctx
        self.sk = ctx.keygen_secret(2)
        self.cfg = S.gesture_pipeline_config(frames=4, bins=16, chirps=32)
        self.l0 = len(prm["q"]) - 1
        self.plan = HG.encode_plan(ctx, self.cfg, self.l0, prm["scale"])
        self.gks = ctx.keygen_rotation(self.sk, ctx.gesture_required_steps(self.plan), 5)
        self.rlk = ctx.keygen_relin(self.sk, 7)
        self.re, self.im = ctx.ciphertext(), ctx.ciphertext()
        self.out = ctx.ciphertext()
        self.load(seed0)

    def load(self, seed):
        x = S.gesture_window(seed, self.cfg["frames"], self.cfg["bins"], self.cfg["chirps"])
        _encrypt_into(self.ctx, self.sk, x, self.prm["scale"], self.l0, seed, self.re, self.im)

    def run(self, out=None):
        return self.ctx.gesture_eval(self.plan, self.re, self.im, self.gks, self.rlk,
                                     out=self.out if out is None else out)


def test_two_ring_graph_matches_eager():
    v = _Vital(S.params("mix15"), 4100)
    gw = _Gesture(S.params("gest12"), 4200)
    v.run()
    gw.run()
    with H.Graph.capture([v.ctx, gw.ctx]) as g:
        v.run()
        gw.run()
    assert g.info()["contexts"] == 2
    ev = [v.ctx.ciphertext() for _ in range(4)]
    eg = gw.ctx.ciphertext()
    for k in range(2):
        v.load(4101 + k)
        gw.load(4201 + k)
        g.launch()
        got_v, got_g = _export(v.ctx, v.out), _export(gw.ctx, [gw.out])
        v.run(ev)
        gw.run(eg)
        _same(got_v, _export(v.ctx, ev))
        _same(got_g, _export(gw.ctx, [eg]))
    g.close()


def test_graph_refusals():
    prm = S.params("tiny")
    ctx = H.Context.from_params(prm)
    with pytest.raises(H.HckError):          # the null stream cannot be captured
        with H.Graph.capture([ctx]):
            pass
    stream = torch.cuda.Stream()
    ctx.set_stream(stream)
    sk = ctx.keygen_secret(1)
    top = len(prm["q"]) - 1
    x = S.uniform_residues([int(q) for q in prm["q"]], ctx.n, 5)[0]
    a = ctx.encrypt_sk(sk, ctx.plaintext_import(x, top, 2.0 ** 25), 9)
    out = ctx.ciphertext()
    ctx.add(a, a, out)
    # a recorded call that needs a new buffer is refused
    with pytest.raises(H.HckError):
        with H.Graph.capture([ctx]):
            ctx.add(a, a, ctx.ciphertext())
    # the context still works after a failed capture
    with H.Graph.capture([ctx]) as g:
        ctx.add(a, a, out)
    g.launch()
    want = ctx.ciphertext_export(out)
    g.launch()
    _same([ctx.ciphertext_export(out)], [want])
    # buffers allocated after the capture may come and go
    tmp = ctx.ciphertext()
    ctx.add(a, a, tmp)
    tmp.close()
    g.launch()
    _same([ctx.ciphertext_export(out)], [want])
    # a buffer that existed at the capture, given back, invalidates the graph
    a.close()
    with pytest.raises(H.HckError):
        g.launch()
    g.close()
    a = ctx.encrypt_sk(sk, ctx.plaintext_import(x, top, 2.0 ** 25), 9)
    # destroying the context releases a graph
    with H.Graph.capture([ctx]) as g2:
        ctx.add(a, a, out)
    ctx.synchronize()
    ctx.close()
    with pytest.raises(H.HckError):
        g2.launch()
    g2.close()
