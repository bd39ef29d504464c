"""The serving runtime on the GPU (hck_server_*), at N = 2^15, L = 12.

Tenants register their evaluation keys as exported words; the server loads
them from host memory into HBM when needed.  Every served result is compared
bit for bit with the plain call (hck_vital_eval / hck_gesture_eval) on the
same window with the tenant's original keys: the same result alone and in the
mix, under a budget that forces evictions, and in batches that mix tenants.
A vital and a gesture window served together are also compared bit for bit
with the oracle's pipeline compositions.  Also: imported keys act exactly
like the keys they were exported from.
"""
import numpy as np
import pytest

import paper_2603_22437_amd as H
import seeded_inputs as S
from paper_2603_22437_amd import gesture as HG
from paper_2603_22437_amd import vital as HV

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world():
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    l0 = len(prm["q"]) - 1
    vcfg = S.vital_pipeline_config()
    gcfg = S.gesture_pipeline_config(frames=14)
    vplan = HV.encode_plan(ctx, vcfg, l0)
    gplan = HG.encode_plan(ctx, gcfg, l0, prm["scale"])
    kinds = {0: H.SERVE_VITAL, 1: H.SERVE_VITAL, 2: H.SERVE_GESTURE}
    plans = {H.SERVE_VITAL: vplan, H.SERVE_GESTURE: gplan}
    steps = {H.SERVE_VITAL: ctx.vital_required_steps(vplan),
             H.SERVE_GESTURE: ctx.gesture_required_steps(gplan)}
    tenants = {}
    for t, kind in kinds.items():
        sk = ctx.keygen_secret(10 + t)
        gks = ctx.keygen_rotation(sk, steps[kind], 20 + t)
        rlk = ctx.keygen_relin(sk, 30 + t)
        words = [np.ascontiguousarray(ctx.galois_keys_export(gks, ctx.galois_element(s)))
                 for s in steps[kind]]
        tenants[t] = dict(kind=kind, sk=sk, gks=gks, rlk=rlk, steps=steps[kind],
                          gk_words=words,
                          rlk_words=np.ascontiguousarray(ctx.switch_key_export(rlk)))
    return dict(ctx=ctx, prm=prm, l0=l0, vcfg=vcfg, gcfg=gcfg, plans=plans,
                tenants=tenants)


def _window(w, t, seed):
    """(re, im) ciphertext handles and their exported words for tenant t."""
    ctx, prm, l0 = w["ctx"], w["prm"], w["l0"]
    ten = w["tenants"][t]
    if ten["kind"] == H.SERVE_VITAL:
        z = S.vital_window(seed, w["vcfg"]["frames"], w["vcfg"]["bins"])
    else:
        z = S.gesture_window(seed, w["gcfg"]["frames"])
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: z.size] = z.reshape(-1)
    re = ctx.encrypt_sk(ten["sk"], ctx.encode(v.real, prm["scale"], l0), 2 * seed)
    im = ctx.encrypt_sk(ten["sk"], ctx.encode(v.imag, prm["scale"], l0), 2 * seed + 1)
    return re, im, ctx.ciphertext_export(re)[0], ctx.ciphertext_export(im)[0]


def _direct(w, t, re, im):
    ctx, ten = w["ctx"], w["tenants"][t]
    plan = w["plans"][ten["kind"]]
    if ten["kind"] == H.SERVE_VITAL:
        outs = ctx.vital_eval(plan, re, im, ten["gks"], ten["rlk"])
    else:
        outs = [ctx.gesture_eval(plan, re, im, ten["gks"], ten["rlk"])]
    return [ctx.ciphertext_export(c) for c in outs]


def _serve(w, requests, budget, max_batch=8, max_inflight=16):
    """Serves [(request id, tenant, re words, im words)]; returns the results by id
    and the server's statistics."""
    ctx = w["ctx"]
    srv = H.Server(ctx, budget, max_batch, max_inflight)
    try:
        for t, ten in w["tenants"].items():
            srv.add_tenant(t, ten["kind"], w["plans"][ten["kind"]], ten["steps"],
                           ten["gk_words"], ten["rlk_words"])
        for rid, t, rw, iw in requests:
            srv.submit(rid, t, rw, iw, w["l0"], w["prm"]["scale"])
        done = {}
        while len(done) < len(requests):
            got = srv.poll(timeout_ms=20000)
            assert got, "server made no progress for 20 s"
            for r in got:
                done[r["request"]] = r
        stats = srv.stats()
    finally:
        srv.close()
    return done, stats


def _key_bytes(w, t):
    ten = w["tenants"][t]
    return (len(ten["gk_words"]) + 1) * ten["rlk_words"].nbytes


def test_imported_keys_act_like_the_originals(world):
    w = world
    ctx = w["ctx"]
    ten = w["tenants"][0]
    re, im, _, _ = _window(w, 0, 1200)
    step = ten["steps"][3]
    gks2 = ctx.galois_keys_from_words({ctx.galois_element(s): words
                                       for s, words in zip(ten["steps"], ten["gk_words"])})
    rlk2 = ctx.switch_key_import(ten["rlk_words"])
    assert np.array_equal(ctx.switch_key_export(rlk2), ten["rlk_words"])
    a = ctx.ciphertext_export(ctx.rotate(re, step, ten["gks"]))[0]
    b = ctx.ciphertext_export(ctx.rotate(re, step, gks2))[0]
    assert np.array_equal(a, b)
    m = ctx.mul(re, im)
    assert np.array_equal(ctx.ciphertext_export(ctx.relinearize(m, ten["rlk"]))[0],
                          ctx.ciphertext_export(ctx.relinearize(m, rlk2))[0])
    bad = ten["rlk_words"].copy()
    bad.reshape(-1)[5] = np.uint64(2 ** 63)
    with pytest.raises(H.HckError):
        ctx.switch_key_import(bad)


def test_served_results_equal_plain_calls_alone_and_in_the_mix(world):
    w = world
    wins = {}
    reqs = []
    rid = 0
    for t in (0, 1, 2, 0, 1, 2, 0, 1):
        seed = 1300 + rid
        re, im, rw, iw = _window(w, t, seed)
        wins[rid] = (t, re, im)
        reqs.append((rid, t, rw, iw))
        rid += 1
    # alone: one request, fresh server
    alone, st1 = _serve(w, reqs[:1], budget=1 << 40)
    assert alone[0]["status"] == 0 and alone[0]["batch"] == 1
    # in the mix: all together, generous budget, batches of up to 8
    mixed, st = _serve(w, reqs, budget=1 << 40)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["key_loads"] == 3 and st["evictions"] == 0
    for a, b in zip(alone[0]["outputs"], mixed[0]["outputs"]):
        assert np.array_equal(a, b)
    # windows of both vital tenants shared a batch (their keys differ)
    assert max(r["batch"] for r in mixed.values()) >= 2
    for rid, (t, re, im) in wins.items():
        want = _direct(w, t, re, im)
        got = mixed[rid]
        assert got["status"] == 0, rid
        assert len(got["outputs"]) == len(want)
        for (res, lvl, sc), o, gl, gs in zip(want, got["outputs"], got["levels"], got["scales"]):
            assert gl == lvl and gs == sc
            assert np.array_equal(res, o), (rid, t)


def test_budget_forces_evictions_and_results_stay_exact(world):
    w = world
    window = (2 + 4) * 2 * w["ctx"].L * w["ctx"].n * 8
    # room for one tenant's keys and a few windows at a time
    budget = max(_key_bytes(w, t) for t in w["tenants"]) + 4 * window
    reqs, wins = [], {}
    for rid, t in enumerate((0, 2, 1, 0, 2, 1)):
        re, im, rw, iw = _window(w, t, 1400 + rid)
        wins[rid] = (t, re, im)
        reqs.append((rid, t, rw, iw))
    done, st = _serve(w, reqs, budget=budget, max_batch=4, max_inflight=4)
    assert st["failed"] == 0 and st["completed"] == len(reqs)
    # only one tenant's keys fit at a time: every tenant is loaded, and each
    # switch to another tenant evicts the previous one
    assert st["key_loads"] >= 3 and st["evictions"] >= 2
    assert st["resident_bytes"] <= budget
    for rid, (t, re, im) in wins.items():
        want = _direct(w, t, re, im)
        for (res, _, _), o in zip(want, done[rid]["outputs"]):
            assert np.array_equal(res, o), (rid, t)


def test_server_errors(world):
    w = world
    ctx = w["ctx"]
    ten = w["tenants"][0]
    srv = H.Server(ctx, 1 << 40, 4, 4)
    try:
        with pytest.raises(H.HckError):   # a needed step without a key
            srv.add_tenant(5, H.SERVE_VITAL, w["plans"][H.SERVE_VITAL], ten["steps"][1:],
                           ten["gk_words"][1:], ten["rlk_words"])
        _, _, rw, iw = _window(w, 0, 1500)
        with pytest.raises(H.HckError):   # unknown tenant
            srv.submit(1, 99, rw, iw, w["l0"], w["prm"]["scale"])
        srv.add_tenant(0, H.SERVE_VITAL, w["plans"][H.SERVE_VITAL], ten["steps"],
                       ten["gk_words"], ten["rlk_words"])
        with pytest.raises(H.HckError):   # registered twice
            srv.add_tenant(0, H.SERVE_VITAL, w["plans"][H.SERVE_VITAL], ten["steps"],
                           ten["gk_words"], ten["rlk_words"])
    finally:
        srv.close()
    # a budget below one tenant's keys: the request is rejected, not hung
    srv = H.Server(ctx, _key_bytes(w, 0) // 2, 4, 4)
    try:
        srv.add_tenant(0, H.SERVE_VITAL, w["plans"][H.SERVE_VITAL], ten["steps"],
                       ten["gk_words"], ten["rlk_words"])
        srv.submit(7, 0, rw, iw, w["l0"], w["prm"]["scale"])
        got = srv.poll(timeout_ms=20000)
        assert len(got) == 1 and got[0]["request"] == 7 and got[0]["status"] != 0
    finally:
        srv.close()


def _import_ops(ctx, ops):
    """GPU handles of an oracle-encoded plan's operands (same integers)."""
    import oracle as O
    handles = {}
    for name, v in ops.items():
        if isinstance(v, O.LinearTransform):
            res = {g * v.n1 + b: pt.res for g, items in v.groups.items() for b, pt in items}
            handles[name] = ctx.lt_create_from_residues(res, v.n1, v.level, v.scale)
        else:
            handles[name] = ctx.plaintext_import(v.res, v.level, v.scale)
    return handles


def test_served_windows_match_the_oracle(world):
    """One vital and one gesture window served together (two tenants, one
    server) give the residues of the oracle's pipeline compositions on the
    same encrypted windows: the operands are encoded once by the oracle and
    imported, and the tenants' key words are the oracle's own keys."""
    import oracle as O
    from oracle import gesture as OG
    from oracle import vital as OV
    w = world
    ctx, prm, l0 = w["ctx"], w["prm"], w["l0"]
    o = O.Oracle(prm)
    vcfg, gcfg = w["vcfg"], w["gcfg"]
    vops = OV.encode_operands(o, vcfg, l0)
    gops = OG.encode_operands(o, gcfg, l0, prm["scale"])
    vh, gh = _import_ops(ctx, vops), _import_ops(ctx, gops)
    vplan = H.VitalPlan.build(vcfg["frames"], vcfg["bins"], vcfg["taylor_order"],
                              len(vcfg["k_resp"]), len(vcfg["k_hr"]), vh,
                              vcfg.get("mag_coeffs"), vcfg.get("gamma", 2))
    gplan = H.GesturePlan.build(gcfg["frames"], gcfg["bins"], gcfg["chirps"],
                                gcfg["weights"][0].shape[0], gh)
    cases = {}
    for t, kind, mod, cfg, ops, plan in ((40, H.SERVE_VITAL, OV, vcfg, vops, vplan),
                                         (41, H.SERVE_GESTURE, OG, gcfg, gops, gplan)):
        s_o = o.keygen_secret(60 + t)
        steps = mod.required_steps(o, cfg, ops)
        gko = {o.galois_element(k): o.keygen_galois(s_o, o.galois_element(k), 70 + t)
               for k in steps}
        rlk_o = o.keygen_relin(s_o, 80 + t)
        if kind == H.SERVE_VITAL:
            z = S.vital_window(1600 + t, cfg["frames"], cfg["bins"])
        else:
            z = S.gesture_window(1600 + t, cfg["frames"])
        re_o, im_o = mod.encrypt_window(o, s_o, z, l0, prm["scale"], 90 + 2 * t)
        want = mod.evaluate(o, cfg, ops, re_o, im_o, gko, rlk_o)
        want = [want[n] for n in OV.OUTPUTS] if kind == H.SERVE_VITAL else [want]
        words = [np.ascontiguousarray(gko[o.galois_element(k)], dtype=np.uint64) for k in steps]
        cases[t] = dict(kind=kind, plan=plan, steps=steps, words=words,
                        rlk=np.ascontiguousarray(rlk_o, dtype=np.uint64),
                        re=re_o.polys, im=im_o.polys, want=want)
    srv = H.Server(ctx, 1 << 40, 8, 8)
    try:
        for t, c in cases.items():
            srv.add_tenant(t, c["kind"], c["plan"], c["steps"], c["words"], c["rlk"])
        for t, c in cases.items():
            srv.submit(t, t, c["re"], c["im"], l0, prm["scale"])
        done = {}
        while len(done) < len(cases):
            got = srv.poll(timeout_ms=20000)
            assert got, "server made no progress for 20 s"
            for r in got:
                done[r["request"]] = r
    finally:
        srv.close()
    for t, c in cases.items():
        r = done[t]
        assert r["status"] == 0, t
        assert len(r["outputs"]) == len(c["want"])
        for got, want, lvl, sc in zip(r["outputs"], c["want"], r["levels"], r["scales"]):
            assert lvl == want.level and sc == want.scale, t
            assert np.array_equal(got, want.polys), t
