#!/usr/bin/env python3
"""Benchmark: homomorphic rotations per second at N = 2^16, L = 24 on one MI355X.

One step is one pass of the evaluation hot path over one synthetic vital-sign
window (200 frames x 64 range bins, complex; clutter-removed and normalized;
packed bin-major into a real and an imaginary ciphertext at N = 2^16, L = 24
primes, K = 8 special primes, dnum = 3, scale 2^50):

  * the windowed, fftshifted 200-point DFT of every range bin as the
    block-diagonal plaintext matrices C~ = I_64 (x) Re W and S~ = I_64 (x) Im W
    (the paper's Kernel 3, Eq. dft_re): d_re = C~ v_re - S~ v_im and
    d_im = S~ v_re + C~ v_im by baby-step/giant-step over 2 x 399 cached
    diagonals, with the baby rotations of v_re and v_im shared by both
    outputs and the inner sums of each output combined before its giant
    rotations (automorphisms, batched hybrid key switching, plaintext
    products), then rescale;
  * the power spectrum |d|^2 = d_re^2 + d_im^2 (the paper's energy kernel):
    two tensor products, one relinearization, one rescale.

`value` is rotations per second over the whole timed step (the step's other
work is included in its time).  The dominant kernel's achieved rate is
measured with HIP events on the library's stream; the CPU oracle is timed on a
bounded sample of the same operation on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                       # MI355X HBM3E, GB/s
VALU_LANE_RATE = 256 * 64 * 2.4e9           # full-rate VALU lane operations / s
MAD_PER_MULMOD = 10                         # v_mad_u64_u32 per 61-bit Shoup product
MULMOD_PEAK = VALU_LANE_RATE / MAD_PER_MULMOD

FRAMES, BINS, N1 = 200, 64, 20


def block_diagonals(mat: np.ndarray, blocks: int, n_slots: int) -> dict:
    """Generalized diagonals diag_k[j] = A[j][(j + k) mod n] of
    A = I_blocks (x) mat placed on the first blocks*d slots (zero elsewhere)."""
    d = mat.shape[0]
    out = {}
    k = np.arange(d)
    for off in range(-(d - 1), d):
        col = k + off
        ok = (col >= 0) & (col < d)
        vals = np.where(ok, mat[k, np.clip(col, 0, d - 1)], 0.0)
        v = np.zeros(n_slots)
        v[: blocks * d] = np.tile(vals, blocks)
        if np.any(v):
            out[off] = v
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hoist", action="store_true",
                    help="plain (not hoisted) baby-step rotations")
    ap.add_argument("--no-hoist-giant", action="store_true",
                    help="one ModDown per giant rotation instead of one per output")
    ap.add_argument("--quick", action="store_true",
                    help="timed steps only (for profiler runs): no oracle baseline, "
                         "rotation modes or per-kernel event pass")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the vital-sign pipeline latency measurement")
    ap.add_argument("--pipeline-windows", type=int, default=100,
                    help="timed windows of the vital-sign pipeline")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first copy this many MiB device-to-device (a plain copy of known "
                         "size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the hot path is "
              "single-GPU; see the design notes for how it would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_22437_amd as H
    import seeded_inputs as S

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    prm = S.params("vital")
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    t0 = time.time()
    ctx = H.Context.from_params(prm, 0, stream)
    L, n_slots = len(prm["q"]), prm["n"] // 2
    top = L - 1
    log(f"context N=2^{prm['log_n']} L={L} K={len(prm['p'])} dnum={prm['dnum']} "
        f"({time.time() - t0:.1f}s)")

    # window -> bin-major slots (slot r*200 + t), real and imaginary ciphertexts
    z = S.vital_window(1000, FRAMES, BINS)
    v = np.zeros(n_slots, dtype=np.complex128)
    v[: FRAMES * BINS] = z.T.reshape(-1)
    sk = ctx.keygen_secret(1)
    scale = prm["scale"]
    ct_re = ctx.encrypt_sk(sk, ctx.encode(v.real, scale, top), 100)
    ct_im = ctx.encrypt_sk(sk, ctx.encode(v.imag, scale, top), 101)

    w = S.windowed_dft_matrix(FRAMES)
    lt_c = ctx.lt_create(block_diagonals(w.real, BINS, n_slots), N1, top)
    lt_s = ctx.lt_create(block_diagonals(w.imag, BINS, n_slots), N1, top)
    steps_needed = sorted(set(ctx.lt_required_steps(lt_c)) | set(ctx.lt_required_steps(lt_s)))
    gks = ctx.keygen_rotation(sk, steps_needed, 5)
    rlk = ctx.keygen_relin(sk, 7)
    log(f"setup done: {len(steps_needed)} rotation keys, 2 x {2 * FRAMES - 1} cached diagonals "
        f"({time.time() - t0:.1f}s)")

    # preallocated outputs
    d_re, d_im, t1, t2, p = (ctx.ciphertext() for _ in range(5))
    terms = [(lt_c, 0, 0, 1), (lt_s, 1, 0, -1), (lt_s, 0, 1, 1), (lt_c, 1, 1, 1)]
    babies = sum(1 for b in ctx.lt_required_steps(lt_c) if 0 < b < N1)
    giants = len(ctx.lt_required_steps(lt_c)) - babies
    rot_per_step = 2 * babies + 2 * giants

    def step():
        ctx.lt_eval([ct_re, ct_im], terms, gks, outputs=[d_re, d_im], hoist=not args.no_hoist,
                    hoist_giant=not args.no_hoist_giant)
        ctx.rescale(d_re, d_re)
        ctx.rescale(d_im, d_im)
        ctx.mul(d_re, d_re, t1)
        ctx.mul(d_im, d_im, t2)
        ctx.add(t1, t2, t1)
        ctx.relinearize(t1, rlk, p)
        ctx.rescale(p, p)

    if args.calib_copy_mb:
        src = torch.empty(args.calib_copy_mb << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_mb} MiB done")
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for k in range(args.steps):
        step()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    ms_per_step = float(evs[0].elapsed_time(evs[-1])) / args.steps
    value = rot_per_step * args.steps / wall
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (events), wall {wall:.3f}s")

    # correctness of the measured step: decoded power spectrum vs plaintext math
    got = ctx.decode(ctx.decrypt(sk, p)).real[: FRAMES * BINS].reshape(BINS, FRAMES)
    ref = np.abs(w @ z).T ** 2
    max_err = float(np.max(np.abs(got - ref)))
    log(f"decoded |DFT|^2 max error vs plaintext: {max_err:.3e}")

    if args.quick:
        print(json.dumps({"metric": "rotations/s at N=2^16 L=24", "value": round(value, 2),
                          "unit": "rotations/s", "ms_per_step": round(ms_per_step, 3),
                          "quick": True, "decoded_max_abs_err": max_err}), flush=True)
        return

    # rotation-only throughput: R1 dependent chain, R2 16 ciphertexts with one
    # key (batched key switching), R3 16 ciphertexts with 16 distinct keys
    pool = [ctx.ciphertext() for _ in range(16)]
    for c in pool:
        ctx.add(ct_re, ct_im, c)
    chain_a, chain_b = ctx.ciphertext(), ctx.ciphertext()
    ctx.add(ct_re, ct_im, chain_a)
    distinct = [k for k in steps_needed if k > 0][:16]

    def timed(fn, count):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return count / (time.perf_counter() - t)

    def r1():
        x, y = chain_a, chain_b
        for _ in range(32):
            ctx.rotate(x, 1, gks, y)
            x, y = y, x

    def r2():
        ctx.rotate_many(pool, 1, gks, pool)

    def r3():
        ctx.rotate_steps(pool[:len(distinct)], distinct, gks, pool[:len(distinct)])

    rotation_modes = {"R1_chain_rot_per_s": round(timed(r1, 32), 1),
                      "R2_16ct_one_key_rot_per_s": round(timed(r2, 16), 1),
                      "R3_16ct_16_keys_rot_per_s": round(timed(r3, len(distinct)), 1)}
    log(f"rotation modes: {rotation_modes}")
    ceilings = rotation_ceilings(ctx, prm, rotation_modes, log)

    # per-kernel durations over two more steps (events around every launch)
    ctx.timing(True)
    ctx.timing_reset()
    prof_steps = 2
    for _ in range(prof_steps):
        step()
    ctx.synchronize()
    kernels = {}
    for name in ctx.timing_names():
        kernels[name] = ctx.timing_read(name)
    ctx.timing(False)
    total_ms = sum(k["ms"] for k in kernels.values())
    dom_name, dom = max(kernels.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    gbs = dom["bytes"] / dom["launches"] / (avg_ms * 1e-3) / 1e9
    mms = dom["mulmods"] / dom["launches"] / (avg_ms * 1e-3)
    hbm_frac, alu_frac = gbs / HBM_PEAK_GBS, mms / MULMOD_PEAK
    if alu_frac > hbm_frac:
        roof = {"bound": "alu", "achieved": round(mms / 1e12, 4),
                "peak": round(MULMOD_PEAK / 1e12, 4), "unit": "Tmulmod/s",
                "frac": round(alu_frac, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_frac, 4)}
    roof["traffic"] = measured_traffic(dom_name)
    roof["kernel"] = dom_name
    roof["avg_launch_us"] = round(avg_ms * 1e3, 2)
    roof["share_of_kernel_time"] = round(dom["ms"] / total_ms, 3)
    breakdown = {k: {"ms_per_step": round(v["ms"] / prof_steps, 3), "launches": v["launches"],
                     "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] else None,
                     "Tmulmod/s": round(v["mulmods"] / (v["ms"] * 1e-3) / 1e12, 3)
                     if v["ms"] else None}
                 for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms"])}

    vital = gesture = None
    if not args.no_pipeline:
        vital = vital_pipeline_latency(ctx, prm, sk, rlk, args.pipeline_windows, log)
        gesture = gesture_pipeline_latency(ctx, prm, sk, rlk, args.pipeline_windows, log)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prm, args.cpu_seconds, log)

    line = {
        "metric": "rotations/s at N=2^16 L=24",
        "value": round(value, 2),
        "unit": "rotations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "vital window PSD: 200 frames x 64 bins complex in 2 ciphertexts, "
                        "complex I_64 (x) W_200 windowed DFT by BSGS (2 x 399 cached "
                        f"diagonals, n1={N1}, shared baby steps), rescale, |.|^2 by "
                        "tensor+relin, rescale",
            "ring_log_n": prm["log_n"], "L": L, "K": len(prm["p"]), "dnum": prm["dnum"],
            "rotations_per_step": rot_per_step, "keyswitches_per_step": rot_per_step + 1,
            "hoisted_baby_steps": not args.no_hoist,
            "shared_giant_moddown": not args.no_hoist_giant,
        },
        "decoded_max_abs_err": max_err,
        "window_latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                              "p99": round(float(np.percentile(step_ms, 99)), 3),
                              "windows_per_s": round(args.steps / wall, 2)},
        "rotation_modes": rotation_modes,
        "rotation_ceilings": ceilings,
        "vital_pipeline": vital,
        "gesture_pipeline": gesture,
        "roofline": roof,
        "kernels": breakdown,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_vital_window.md")
KERNEL_SOURCE = {"lt_inner": "lt_kernels.hip", "ks_contig_inner": "ks_fused.hip",
                 "ks_moddown_strided": "ks_fused.hip", "ks_modup_strided": "ks_fused.hip",
                 "ks_moddown_tail": "ks_fused.hip", "ks_inner_gather": "ks_fused.hip",
                 "ks_intt_gather": "ks_fused.hip"}


def source_hash(fname):
    """sha256 prefix over a kernel's source file and the library headers."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2603_22437_amd", "csrc")
    h = hashlib.sha256()
    for f in [fname] + sorted(x for x in os.listdir(csrc) if x.endswith(".h")):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    summary (counts scaled by a plain copy of known size), or None when the
    kernel is not listed or its source changed after the counters were taken."""
    if kernel not in KERNEL_SOURCE or not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 6 and cells[0] == kernel:
            if cells[5] != source_hash(KERNEL_SOURCE[kernel]):
                return None
            return int(cells[4])
    return None


def rotation_ceilings(ctx, prm, modes, log):
    """The two ceilings of one rotation at the top level (N = 2^16, L = 24,
    K = 8, dnum = 3): HBM (ciphertext in + key + ciphertext out at 8 TB/s) and
    the vector-ALU integer rate (modular products per rotation over the
    device's measured Shoup-product rate), with the achieved fraction of each
    for the rotation modes without key reuse (R3) and with it (R2)."""
    n, L, K, dnum = prm["n"], len(prm["q"]), len(prm["p"]), prm["dnum"]
    alpha = -(-L // dnum)
    digits = -(-L // alpha)
    ext = digits * (L + K) - L
    ntts = L + ext + 2 * K + 2 * L                   # INTT d, NTT ext, INTT P, NTT conv
    mulmods = (ntts * (n // 2) * (n.bit_length() - 1)          # butterflies
               + digits * alpha * (L + K - alpha) * n + L * n   # ModUp BConv + digit scale
               + 2 * K * L * n + 2 * K * n                      # ModDown BConv + scale
               + 2 * digits * (L + K) * n                       # key inner product
               + 2 * L * n)                                     # P^-1
    bytes_ = 8 * n * (2 * L + digits * 2 * (L + K) + 2 * L)
    rate = ctx.measure_mulmod_rate() * 1e12
    hbm = HBM_PEAK_GBS * 1e9 / bytes_
    valu = rate / mulmods
    out = {"bytes_per_rotation": bytes_, "mulmods_per_rotation": mulmods,
           "measured_shoup_mulmod_T_per_s": round(rate / 1e12, 3),
           "hbm_ceiling_rot_per_s": round(hbm, 1), "valu_ceiling_rot_per_s": round(valu, 1),
           "R3_frac_of_hbm": round(modes["R3_16ct_16_keys_rot_per_s"] / hbm, 4),
           "R3_frac_of_valu": round(modes["R3_16ct_16_keys_rot_per_s"] / valu, 4),
           "R2_frac_of_valu": round(modes["R2_16ct_one_key_rot_per_s"] / valu, 4)}
    log(f"rotation ceilings: {out}")
    return out


def vital_pipeline_latency(ctx, prm, sk, rlk, windows, log):
    """Latency of the encrypted vital-sign pipeline (K1 -> K2 -> K4 -> K5 ->
    K7 -> K3 -> K1 -> K2 on one 200 x 64 window at N = 2^16, L = 24), per
    window with HIP events, after one warm-up window."""
    import torch
    import seeded_inputs as S
    from paper_2603_22437_amd import vital as HV
    cfg = S.vital_pipeline_config()
    top = len(prm["q"]) - 1
    plan = HV.encode_plan(ctx, cfg, top)
    gks = ctx.keygen_rotation(sk, ctx.vital_required_steps(plan), 5)
    z = S.vital_window(1003, cfg["frames"], cfg["bins"])
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: z.size] = z.reshape(-1)
    re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], top), 200)
    im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], top), 201)
    outs = [ctx.ciphertext() for _ in range(4)]
    stream = torch.cuda.current_stream()
    ctx.vital_eval(plan, re, im, gks, rlk, outs)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(windows + 1)]
    evs[0].record(stream)
    t0 = time.perf_counter()
    for k in range(windows):
        ctx.vital_eval(plan, re, im, gks, rlk, outs)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(windows)])
    # throughput with 8 windows evaluated together (shared key-switch batches)
    batch = 8
    res_b = []
    ims_b = []
    for k in range(batch):
        zk = S.vital_window(1100 + k, cfg["frames"], cfg["bins"])
        vk = np.zeros(ctx.n_slots, dtype=np.complex128)
        vk[: zk.size] = zk.reshape(-1)
        res_b.append(ctx.encrypt_sk(sk, ctx.encode(vk.real, prm["scale"], top), 600 + k))
        ims_b.append(ctx.encrypt_sk(sk, ctx.encode(vk.imag, prm["scale"], top), 700 + k))
    outs_b = ctx.vital_eval_many(plan, res_b, ims_b, gks, rlk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 2
    for _ in range(reps):
        ctx.vital_eval_many(plan, res_b, ims_b, gks, rlk, outs_b)
    torch.cuda.synchronize()
    batched_wps = batch * reps / (time.perf_counter() - t0)
    del outs_b, res_b, ims_b
    noise = kernel_noise(ctx, prm, sk, top, ctx.VITAL_TAPS + plan.OUTPUTS,
                         lambda re_, im_: _flat(ctx.vital_eval_taps(plan, re_, im_, gks, rlk)),
                         lambda zz: HV.plain_stages(cfg, zz, ctx.n_slots),
                         [S.vital_window(1000 + i, cfg["frames"], cfg["bins"]) for i in range(3)])
    got = [ctx.decode(ctx.decrypt(sk, c)).real for c in outs]
    g = HV.lane_group(cfg)
    # the energy-weighted bin estimate must land on the synthetic target bin
    target = int(np.argmax(np.abs(z).sum(axis=0)))
    res = {"windows": windows, "p50_ms": round(float(np.percentile(ms, 50)), 3),
           "p99_ms": round(float(np.percentile(ms, 99)), 3),
           "windows_per_s": round(windows / wall, 2),
           "batched_8_windows_per_s": round(batched_wps, 2),
           "taylor_order": cfg["taylor_order"],
           "rotation_keys": len(gks), "target_bin_true": target,
           "target_bin_est": round(float(got[0][0] / got[1][0]), 4),
           "resp_bpm_est": round(float(got[2][0] / got[3][0]), 3),
           "hr_bpm_est": round(float(got[2][g] / got[3][g]), 3),
           "kernel_noise": noise}
    log(f"vital pipeline: {res}")
    return res


def gesture_pipeline_latency(ctx, prm, sk, rlk, windows, log):
    """Latency of the encrypted gesture pipeline (Doppler DFT, power, notch,
    gamma = 4 attention, frame sum, FC1 -> x^2 -> FC2 -> x^2 -> FC3) on one
    30 frames x 32 range x 32 chirps window at N = 2^16, L = 24, per window
    with HIP events, after one warm-up window."""
    import torch
    import seeded_inputs as S
    from paper_2603_22437_amd import gesture as HG
    cfg = S.gesture_pipeline_config(frames=30)
    top = len(prm["q"]) - 1
    plan = HG.encode_plan(ctx, cfg, top, prm["scale"])
    gks = ctx.keygen_rotation(sk, ctx.gesture_required_steps(plan), 5)
    x = S.gesture_window(2003, cfg["frames"])
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: x.size] = x.reshape(-1)
    re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], top), 300)
    im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], top), 301)
    out = ctx.ciphertext()
    stream = torch.cuda.current_stream()
    ctx.gesture_eval(plan, re, im, gks, rlk, out)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(windows + 1)]
    evs[0].record(stream)
    t0 = time.perf_counter()
    for k in range(windows):
        ctx.gesture_eval(plan, re, im, gks, rlk, out)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(windows)])
    classes = cfg["weights"][2].shape[0]
    logits = ctx.decode(ctx.decrypt(sk, out))[:classes].real
    noise = kernel_noise(ctx, prm, sk, top, ctx.GESTURE_TAPS + ("FC3 logits",),
                         lambda re_, im_: _flat(ctx.gesture_eval_taps(plan, re_, im_, gks, rlk)),
                         lambda xx: HG.plain_stages(cfg, xx, ctx.n_slots),
                         [S.gesture_window(2000 + i, cfg["frames"]) for i in range(3)])
    res = {"windows": windows, "p50_ms": round(float(np.percentile(ms, 50)), 3),
           "p99_ms": round(float(np.percentile(ms, 99)), 3),
           "windows_per_s": round(windows / wall, 2), "rotation_keys": len(gks),
           "frames": cfg["frames"], "classes": classes,
           "predicted_class": int(np.argmax(logits)), "kernel_noise": noise}
    log(f"gesture pipeline: {res}")
    return res


def _flat(result):
    """(outputs, taps) of a *_eval_taps call as one list: taps, then outputs."""
    outs, taps = result
    return list(taps) + (list(outs) if isinstance(outs, (list, tuple)) else [outs])


def kernel_noise(ctx, prm, sk, top, names, run, plain, windows):
    """Per-kernel encryption noise, the method of section 5.2 (Table 3): the
    MSE and max |error| between each decoded intermediate of the encrypted
    pipeline and the same value from plaintext execution, cumulative after
    the preceding kernels, over the given windows; depth = levels consumed."""
    sq = [0.0] * len(names)
    cnt = [0] * len(names)
    mx = [0.0] * len(names)
    depth = [0] * len(names)
    for k, z in enumerate(windows):
        v = np.zeros(ctx.n_slots, dtype=np.complex128)
        v[: z.size] = np.asarray(z).reshape(-1)
        re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], top), 900 + 2 * k)
        im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], top), 901 + 2 * k)
        cts = run(re, im)
        for i, (c, (slots, want)) in enumerate(zip(cts, plain(z))):
            got = ctx.decode(ctx.decrypt(sk, c)).real[slots]
            err = got - want
            sq[i] += float(np.sum(err ** 2))
            cnt[i] += len(slots)
            mx[i] = max(mx[i], float(np.max(np.abs(err))))
            depth[i] = top - c.level
    return [{"stage": n, "mse": float(f"{sq[i] / cnt[i]:.3e}"),
             "max_abs_err": float(f"{mx[i]:.3e}"), "depth": depth[i]}
            for i, n in enumerate(names)]


def cpu_baseline(prm, seconds, log):
    """The oracle's rotation (automorphism + hybrid key switching) of one
    N = 2^16, L = 24 ciphertext at the top level, repeated for ~`seconds`."""
    import oracle as O
    import seeded_inputs as S
    o = O.Oracle(prm)
    s = o.keygen_secret(1)
    g = o.galois_element(1)
    gk = {g: o.keygen_galois(s, g, 5)}
    res = S.uniform_residues(o.qmods(o.L - 1), o.n, 7, count=2)
    ct = O.Ciphertext(res, o.L - 1, 2.0 ** 50)
    n_rot, t0 = 0, time.perf_counter()
    while True:
        ct = o.rotate(ct, 1, gk)
        n_rot += 1
        el = time.perf_counter() - t0
        if el >= seconds or (n_rot >= 1 and el * (n_rot + 1) / n_rot > 2 * seconds):
            break
    log(f"oracle: {n_rot} rotations in {el:.1f}s on {O.num_threads()} threads")
    return {"value": round(n_rot / el, 4), "unit": "rotations/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{n_rot} rotation(s) of one N=2^16, L=24 top-level ciphertext "
                      "(automorphism + hybrid key switching), not the full window step",
            "cpu": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
