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
                    help="timed steps only (for profiler runs): no autotuning, oracle "
                         "baseline, rotation modes or per-kernel event pass")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the vital-sign pipeline latency measurement")
    ap.add_argument("--pipeline-windows", type=int, default=100,
                    help="timed windows of the vital-sign pipeline")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in key-switch batch rule (no autotuning)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the mixed batch (64 windows, rings 2^15 and 2^16)")
    ap.add_argument("--batch-groups", type=int, default=4,
                    help="contexts (streams) per parameter set in the mixed batch")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving measurement (256 tenants, Poisson arrivals)")
    ap.add_argument("--serving-seconds", type=float, default=20.0,
                    help="duration of the synthetic serving traffic")
    ap.add_argument("--microbench", action="store_true",
                    help="only the device's sustained Shoup-product rate and plain "
                         "device-to-device copy rates (the measured ALU and copy ceilings)")
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

    if args.microbench:
        print(json.dumps(microbench(log)), flush=True)
        return

    prm = S.params("vital")
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    t0 = time.time()
    ctx = H.Context.from_params(prm, 0, stream)
    L, n_slots = len(prm["q"]), prm["n"] // 2
    top = L - 1
    log(f"context N=2^{prm['log_n']} L={L} K={len(prm['p'])} dnum={prm['dnum']} "
        f"({time.time() - t0:.1f}s)")
    tuning = None
    if not args.no_autotune and not args.quick:
        t0 = time.time()
        tuned = ctx.autotune_keyswitch()
        tuning = {"keyswitches_per_launch": [tuned[l][0] for l in range(L)],
                  "us_per_keyswitch": [round(tuned[l][1], 1) for l in range(L)],
                  "seconds": round(time.time() - t0, 1)}
        log(f"key-switch schedule tuned in {tuning['seconds']} s: "
            f"{tuning['keyswitches_per_launch']}")

    dnum_tuning = ntt_tuning = None
    if not args.no_autotune and not args.quick:
        dnum_tuning = dnum_autotune(prm, top, log)
        t0 = time.time()
        nt = ctx.autotune_ntt(rows=64)
        ntt_tuning = {"us_per_row_forward_plus_inverse": {f"R1=2^{a}": round(u, 2)
                                                          for a, u in nt["splits"].items()},
                      "chosen_log2_R1": nt["chosen"], "default_log2_R1": (prm["log_n"] + 1) // 2,
                      "seconds": round(time.time() - t0, 1)}
        log(f"NTT split tuning: {ntt_tuning}")

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

    def timed(fn, count, trials=3):
        """rate of the best of `trials` timed calls, after one warm-up call"""
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(trials):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return count / best

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

    # where an R3 rotation's time goes: HIP events around every launch over
    # two more R3 calls, in microseconds per rotation
    ctx.timing(True)
    ctx.timing_reset()
    for _ in range(2):
        r3()
    ctx.synchronize()
    r3_kernels = {}
    for name in ctx.timing_names():
        v = ctx.timing_read(name)
        r3_kernels[name] = {"us_per_rotation": round(v["ms"] * 1e3 / (2 * len(distinct)), 2),
                            "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] else None}
    ctx.timing(False)
    r3_kernels = dict(sorted(r3_kernels.items(), key=lambda kv: -kv[1]["us_per_rotation"]))
    log(f"R3 kernels: {r3_kernels}")
    ceilings = rotation_ceilings(ctx, prm, rotation_modes, log)
    tiny = tiny_end_to_end(log)

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
    # HBM rate from the counters' bytes per launch (the committed FETCH_SIZE /
    # WRITE_SIZE summary) over this run's mean launch time, where the
    # kernel's source is unchanged since: what reaches HBM, without the L2
    # re-reads that algorithmic bytes may count
    for k, v in kernels.items():
        t = measured_traffic(k)
        if t and v["ms"]:
            breakdown[k]["counter_GB/s"] = round(t * v["launches"] / (v["ms"] * 1e-3) / 1e9, 1)

    vital = gesture = gesture_cnn = None
    if not args.no_pipeline:
        vital = vital_pipeline_latency(ctx, prm, sk, rlk, args.pipeline_windows, log)
        # both gesture classifiers run on the gesture parameter set (N = 2^16,
        # L = 30 primes, K = 10, dnum = 3)
        gprm = S.params("gesture")
        gctx = H.Context.from_params(gprm)
        gsk = gctx.keygen_secret(11)
        grlk = gctx.keygen_relin(gsk, 12)
        if not args.no_autotune and not args.quick:
            gctx.autotune_keyswitch()
        gesture = gesture_pipeline_latency(gctx, gprm, gsk, grlk, args.pipeline_windows, log)
        gesture_cnn = gesture_cnn_latency(gctx, gprm, gsk, grlk, args.pipeline_windows, log)
        gctx.close()

    batched = None
    if not args.no_batched and not args.quick:
        batched = batched_mixed_benchmark(args.batch_groups, log)

    serving = None
    if not args.no_serving and not args.quick:
        serving = serving_benchmark(args.serving_seconds, log)

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
            "keyswitch_schedule": "autotuned" if tuning else "built-in rule",
        },
        "autotune": tuning,
        "dnum_tuning": dnum_tuning,
        "ntt_tuning": ntt_tuning,
        "decoded_max_abs_err": max_err,
        "window_latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                              "p99": round(float(np.percentile(step_ms, 99)), 3),
                              "windows_per_s": round(args.steps / wall, 2)},
        "rotation_modes": rotation_modes,
        "R3_kernels_us_per_rotation": r3_kernels,
        "rotation_ceilings": ceilings,
        "tiny_end_to_end": tiny,
        "vital_pipeline": vital,
        "gesture_pipeline": gesture,
        "batched_mixed": batched,
        "serving": serving,
        "roofline": roof,
        # key switching (the hot path's dominant cost) as a whole: full
        # rotations with distinct keys (R3) against both ceilings of one
        # rotation (151 MB at 8 TB/s; 165 M modular products at the measured
        # product rate)
        "roofline_keyswitch": {
            "rotations_per_s": rotation_modes["R3_16ct_16_keys_rot_per_s"],
            "hbm_ceiling_rot_per_s": ceilings["hbm_ceiling_rot_per_s"],
            "frac_of_hbm": ceilings["R3_frac_of_hbm"],
            "valu_ceiling_rot_per_s": ceilings["valu_ceiling_rot_per_s"],
            "frac_of_valu": ceilings["R3_frac_of_valu"]},
        "gesture_cnn_pipeline": gesture_cnn,
        "paper_latencies_context": PAPER_CONTEXT,
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


def tiny_end_to_end(log, reps=50):
    """Latency of the tiny configuration (N = 2^12, L = 3) end to end on the
    GPU: (I_32 (x) M64) x by BSGS (127 diagonals, n1 = 16), rescale, square
    with relinearization, decrypted at scale ~2^50; median over `reps`
    runs."""
    import torch
    import paper_2603_22437_amd as H
    import seeded_inputs as S
    tp = S.params("tiny")
    ctx = H.Context.from_params(tp)
    sk = ctx.keygen_secret(1)
    level = len(tp["q"]) - 1
    n_slots = ctx.n_slots
    mat = S.uniform_matrix(64, 64, 0, 1 / 8)
    j = np.arange(n_slots)
    diags = {}
    for k in range(-63, 64):
        i = j % 64
        ok = (i + k >= 0) & (i + k < 64)
        diags[k % n_slots] = np.where(ok, mat[i, np.clip(i + k, 0, 63)], 0.0)
    lt = ctx.lt_create(diags, 16, level)
    gks = ctx.keygen_rotation(sk, ctx.lt_required_steps(lt), 5)
    rlk = ctx.keygen_relin(sk, 7)
    x = S.uniform_slots(n_slots, 0)
    ct = ctx.encrypt_sk(sk, ctx.encode(x, tp["scale"], level), 3)

    def once():     # decrypted at scale ~2^50 on 2 limbs, with no final rescale
        y = ctx.rescale(ctx.lt_apply(lt, ct, gks))
        return ctx.relinearize(ctx.mul(y, y), rlk)

    out = once()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        t = time.perf_counter()
        out = once()
        ctx.synchronize()
        ms.append((time.perf_counter() - t) * 1e3)
    err = float(np.max(np.abs(ctx.decode(ctx.decrypt(sk, out)).real -
                              (np.kron(np.eye(n_slots // 64), mat) @ x) ** 2)))
    res = {"p50_ms": round(float(np.median(ms)), 3), "reps": reps,
           "decoded_max_abs_err": float(f"{err:.3e}")}
    log(f"tiny end to end: {res}")
    return res


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
    # the circuit needs its depth in levels, plus one of headroom for the rate
    # numerators (fourth powers of the spectrum times frequencies, whose size
    # depends on the window): the plan is encoded for inputs at that level and
    # the top-level inputs are dropped to it
    base = (11 if cfg["taylor_order"] == 3 else 9) + 1
    plan = HV.encode_plan(ctx, cfg, base)
    gks = ctx.keygen_rotation(sk, ctx.vital_required_steps(plan), 5)
    # a window whose two rate averages are well conditioned (their decoded
    # denominators far above the rotations' absolute noise), so that the
    # reported estimates compare with the plaintext circuit's
    z = S.vital_window(1001, cfg["frames"], cfg["bins"])
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
    # the paper's two FIR backends: Toeplitz BSGS (above) against one hoisted
    # rotation per tap
    rcfg = dict(cfg, fir_backend="rotation")
    rplan = HV.encode_plan(ctx, rcfg, base)
    rgks = ctx.keygen_rotation(sk, ctx.vital_required_steps(rplan), 5)
    ctx.vital_eval(rplan, re, im, rgks, rlk, outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fir_windows = 20
    for _ in range(fir_windows):
        ctx.vital_eval(rplan, re, im, rgks, rlk, outs)
    torch.cuda.synchronize()
    rotation_fir_ms = (time.perf_counter() - t0) * 1e3 / fir_windows
    del rgks, rplan
    graph = vital_graph_replay(ctx, plan, re, im, gks, rlk, outs, log)
    per_frame = vital_per_frame(ctx, prm, cfg, plan, sk, rlk, z, base, outs, log)
    ctx.vital_eval(plan, re, im, gks, rlk, outs)
    noise = kernel_noise(ctx, prm, sk, top, base, VITAL_DEPTHS, ctx.VITAL_TAPS + plan.OUTPUTS,
                         lambda re_, im_: _flat(ctx.vital_eval_taps(plan, re_, im_, gks, rlk)),
                         lambda zz: HV.plain_stages(cfg, zz, ctx.n_slots),
                         [S.vital_window(1000 + i, cfg["frames"], cfg["bins"]) for i in range(3)])
    got = [ctx.decode(ctx.decrypt(sk, c)).real for c in outs]
    g = HV.lane_group(cfg)
    plain_out = HV.plain_stages(cfg, z, ctx.n_slots)
    # the energy-weighted bin estimate must land on the synthetic target bin
    target = int(np.argmax(np.abs(z).sum(axis=0)))
    res = {"windows": windows, "p50_ms": round(float(np.percentile(ms, 50)), 3),
           "p99_ms": round(float(np.percentile(ms, 99)), 3),
           "windows_per_s": round(windows / wall, 2),
           "batched_8_windows_per_s": round(batched_wps, 2),
           "rotation_fir_backend_ms_per_window": round(rotation_fir_ms, 3),
           "graph_replay": graph, "per_frame_packing": per_frame,
           "taylor_order": cfg["taylor_order"], "input_level": top, "plan_level": base,
           "rotation_keys": len(gks), "target_bin_true": target,
           "target_bin_est": round(float(got[0][0] / got[1][0]), 4),
           "resp_bpm_est": round(float(got[2][0] / got[3][0]), 3),
           "hr_bpm_est": round(float(got[2][g] / got[3][g]), 3),
           # the same circuit on plaintext numbers; a weak band (tiny
           # numerator and denominator) makes its rate ill-conditioned
           "resp_bpm_plain": round(float(plain_out[-2][1][0] / plain_out[-1][1][0]), 3),
           "hr_bpm_plain": round(float(plain_out[-2][1][1] / plain_out[-1][1][1]), 3),
           "resp_band_den": float(f"{plain_out[-1][1][0]:.3e}"),
           "kernel_noise": noise}
    log(f"vital pipeline: {res}")
    return res


def microbench(log, reps=10):
    """The measured ceilings quoted beside the published peaks: the sustained
    rate of 61-bit Shoup modular products (hck_measure_mulmod_rate: 8
    independent chains per thread, each product fully reduced) and the rate
    of plain device-to-device copies (torch, bytes read + written) of
    several sizes, per HIP-event timing."""
    import torch
    import paper_2603_22437_amd as H
    import seeded_inputs as S
    ctx = H.Context.from_params(S.params("tiny"))
    mulmod = [round(ctx.measure_mulmod_rate(), 4) for _ in range(3)]
    ctx.close()
    copies = {}
    for mib in (256, 1024, 4096):
        src = torch.zeros(mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        copies[f"{mib}_MiB_GBps"] = round(2 * (mib << 20) / sec / 1e9, 1)
        del src, dst
    res = {"metric": "microbench", "shoup_mulmod_T_per_s": mulmod,
           "valu_lane_ops_peak_T_per_s": round(VALU_LANE_RATE / 1e12, 2),
           "copy_read_plus_write": copies, "hbm_peak_GBps": HBM_PEAK_GBS}
    log(f"microbench: {res}")
    return res


def dnum_autotune(prm, level, log, dnums=(2, 3, 4, 6, 8)):
    """The digit-count autotuner (hck_autotune_dnum) over the benchmark ring
    and chain: microseconds per top-level key switch and the switching-key
    size for each dnum (K = ceil(L / dnum) special primes of 60 bits)."""
    import paper_2603_22437_amd as H
    import seeded_inputs as S
    t0 = time.time()
    cands = [S.params_with_dnum(prm["name"], d) for d in dnums]
    r = H.autotune_dnum(cands, level=level, count=8)
    res = {"level": level,
           "candidates": [{"dnum": c["dnum"], "K": len(c["p"]),
                           "us_per_keyswitch": round(u, 1), "key_MiB": round(kb / 2 ** 20, 1)}
                          for c, u, kb in zip(cands, r["us_per_switch"], r["key_bytes"])],
           "fastest_dnum": cands[r["best"]]["dnum"], "benchmark_dnum": prm["dnum"],
           "seconds": round(time.time() - t0, 1)}
    log(f"dnum tuning: {res}")
    return res


def vital_graph_replay(ctx, plan, re, im, gks, rlk, outs, log, windows=20):
    """One vital window issued call by call against the same window recorded
    once into a HIP graph (hck_graph_*) and replayed, both on a stream of the
    context's own: per-window HIP-event latencies (p50)."""
    import torch
    import paper_2603_22437_amd as H
    old = torch.cuda.current_stream()
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    ctx.set_stream(st)
    ctx.vital_eval(plan, re, im, gks, rlk, outs)

    def per_window(fn):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(windows + 1)]
        fn()
        evs[0].record(st)
        for k in range(windows):
            fn()
            evs[k + 1].record(st)
        st.synchronize()
        return float(np.median([evs[k].elapsed_time(evs[k + 1]) for k in range(windows)]))

    eager = per_window(lambda: ctx.vital_eval(plan, re, im, gks, rlk, outs))
    time.sleep(0.05)    # an idle gap that marks the phases apart in a kernel trace
    with H.Graph.capture([ctx]) as g:
        ctx.vital_eval(plan, re, im, gks, rlk, outs)
    replay = per_window(g.launch)
    nodes = g.info()["nodes"]
    g.close()
    st.synchronize()
    ctx.set_stream(old)
    res = {"eager_p50_ms": round(eager, 3), "graph_p50_ms": round(replay, 3),
           "graph_nodes": nodes, "windows": windows}
    log(f"vital graph replay: {res}")
    return res


def vital_per_frame(ctx, prm, cfg, plan, sk, rlk, z, base, outs, log, windows=3):
    """The vital pipeline on per-frame packing (section 3.3.2: one ciphertext
    pair per frame, 200 pairs encrypted at the plan's level) against the
    batched packing's 2 ciphertexts: latency and the largest difference of
    the decoded outputs."""
    import torch
    from paper_2603_22437_amd import vital as HV
    gks = ctx.keygen_rotation(sk, ctx.vital_frames_required_steps(plan), 5)
    res, ims = [], []
    for t in range(cfg["frames"]):
        v = np.zeros(ctx.n_slots, dtype=np.complex128)
        v[: cfg["bins"]] = z[t]
        res.append(ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], base), 3000 + 2 * t))
        ims.append(ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], base), 3001 + 2 * t))
    got = ctx.vital_eval_frames(plan, res, ims, gks, rlk)
    torch.cuda.synchronize()
    ms = []
    for _ in range(windows):
        t0 = time.perf_counter()
        ctx.vital_eval_frames(plan, res, ims, gks, rlk, got)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    a = [ctx.decode(ctx.decrypt(sk, c)).real for c in got]
    b = [ctx.decode(ctx.decrypt(sk, c)).real for c in outs]
    g = HV.lane_group(cfg)
    # relative to each output's size (the rate sums reach 10^6 on strong
    # windows, where CKKS noise is relative to the value)
    diff = max(abs(a[i][s] - b[i][s]) / max(1.0, abs(b[i][s]))
               for i in range(4) for s in ((0,) if i < 2 else (0, g)))
    out = {"windows": windows, "input_ciphertexts": 2 * cfg["frames"],
           "p50_ms": round(float(np.median(ms)), 2), "rotation_keys": len(gks),
           "decoded_max_diff_vs_batched_rel": float(f"{diff:.3e}")}
    log(f"vital per-frame packing: {out}")
    return out


def gesture_pipeline_latency(ctx, prm, sk, rlk, windows, log):
    """Latency of the encrypted gesture pipeline (Doppler DFT, power, notch,
    gamma = 4 attention, frame sum, FC1 -> x^2 -> FC2 -> x^2 -> FC3) on one
    30 frames x 32 range x 32 chirps window at N = 2^16 (the gesture
    parameter set: L = 30, K = 10), per window with HIP events, after one
    warm-up window."""
    import torch
    import seeded_inputs as S
    from paper_2603_22437_amd import gesture as HG
    cfg = S.gesture_pipeline_config(frames=30)
    top = len(prm["q"]) - 1
    base = HG.DEPTH            # plan for inputs at the circuit's depth
    plan = HG.encode_plan(ctx, cfg, base, prm["scale"])
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
    noise = kernel_noise(ctx, prm, sk, top, base, GESTURE_DEPTHS,
                         ctx.GESTURE_TAPS + ("FC3 logits",),
                         lambda re_, im_: _flat(ctx.gesture_eval_taps(plan, re_, im_, gks, rlk)),
                         lambda xx: HG.plain_stages(cfg, xx, ctx.n_slots),
                         [S.gesture_window(2000 + i, cfg["frames"]) for i in range(3)])
    # per-frame packing (section 3.3.2): one ciphertext pair per frame, the
    # same plan; a few windows, each timed with HIP events
    frames = HG.pack_frames(x, ctx.n_slots)
    res_f = [ctx.encrypt_sk(sk, ctx.encode(fv.real, prm["scale"], top), 400 + 2 * f)
             for f, fv in enumerate(frames)]
    ims_f = [ctx.encrypt_sk(sk, ctx.encode(fv.imag, prm["scale"], top), 401 + 2 * f)
             for f, fv in enumerate(frames)]
    out_f = ctx.ciphertext()
    ctx.gesture_eval_frames(plan, res_f, ims_f, gks, rlk, out_f)
    torch.cuda.synchronize()
    pf_windows = 5
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(pf_windows + 1)]
    evs[0].record(stream)
    for k in range(pf_windows):
        ctx.gesture_eval_frames(plan, res_f, ims_f, gks, rlk, out_f)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    ms_f = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(pf_windows)])
    logits_f = ctx.decode(ctx.decrypt(sk, out_f))[:classes].real
    per_frame = {"windows": pf_windows, "input_ciphertexts": 2 * len(frames),
                 "p50_ms": round(float(np.percentile(ms_f, 50)), 3),
                 "vs_batched_latency": round(float(np.percentile(ms_f, 50)
                                                   / np.percentile(ms, 50)), 2),
                 "decoded_max_abs_diff_vs_batched": float(np.abs(logits_f - logits).max())}
    res = {"windows": windows, "p50_ms": round(float(np.percentile(ms, 50)), 3),
           "p99_ms": round(float(np.percentile(ms, 99)), 3),
           "windows_per_s": round(windows / wall, 2), "rotation_keys": len(gks),
           "input_level": top, "plan_level": base,
           "frames": cfg["frames"], "classes": classes,
           "predicted_class": int(np.argmax(logits)), "per_frame_packing": per_frame,
           "kernel_noise": noise}
    log(f"gesture pipeline: {res}")
    return res


def gesture_cnn_latency(ctx, prm, sk, rlk, windows, log):
    """Latency of the gesture classifier's CNN variant (the gesture front end,
    then two 3 x 3 stride-2 convolutions with 8 / 16 channels, pooling, dense
    256 -> 64 -> 10, degree-3 activations; depth 19) on one 30 x 32 x 32
    window at N = 2^16, L = 30, K = 10 from plan level 20, per window with
    HIP events after one warm-up window; decoded logits checked against the
    network on plaintext numbers."""
    import torch
    import seeded_inputs as S
    from paper_2603_22437_amd import gesture as HG
    cfg = S.gesture_cnn_config()
    top = len(prm["q"]) - 1
    base = 20
    plan = HG.encode_cnn_plan(ctx, cfg, base, prm["scale"])
    gks = ctx.keygen_rotation(sk, ctx.gesture_cnn_required_steps(plan), 5)
    x = S.gesture_window(2003, cfg["frames"], cfg["bins"], cfg["chirps"])
    v = np.zeros(ctx.n_slots, dtype=np.complex128)
    v[: x.size] = x.reshape(-1)
    re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], top), 500)
    im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], top), 501)
    out = ctx.ciphertext()
    stream = torch.cuda.current_stream()
    ctx.gesture_cnn_eval(plan, re, im, gks, rlk, out)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(windows + 1)]
    evs[0].record(stream)
    t0 = time.perf_counter()
    for k in range(windows):
        ctx.gesture_cnn_eval(plan, re, im, gks, rlk, out)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(windows)])
    classes = np.shape(cfg["dense2"])[0]
    logits = ctx.decode(ctx.decrypt(sk, out))[:classes].real
    err = float(np.max(np.abs(logits - HG.cnn_plain(cfg, x))))
    res = {"windows": windows, "p50_ms": round(float(np.percentile(ms, 50)), 3),
           "p99_ms": round(float(np.percentile(ms, 99)), 3),
           "windows_per_s": round(windows / wall, 2), "rotation_keys": len(gks),
           "params": "N=2^16, L=30, K=10, dnum=3", "input_level": top, "plan_level": base,
           "depth": 19, "channels": [int(np.shape(cfg["conv1"])[0]),
                                     int(np.shape(cfg["conv2"])[0])],
           "dense": [int(np.shape(cfg["dense1"])[1]), int(np.shape(cfg["dense1"])[0]), classes],
           "decoded_max_abs_err": float(f"{err:.3e}"), "predicted_class": int(np.argmax(logits))}
    log(f"gesture CNN: {res}")
    return res


# The paper's own latencies (RTX 3090 Ti, FIDESlib + OpenFHE, CKKS N = 2^15,
# its datasets; section 5.4 latency table), quoted beside the measured window
# latencies as context: other hardware, other ring, other workload size.
PAPER_CONTEXT = {"hardware": "NVIDIA RTX 3090 Ti (FIDESlib GPU + OpenFHE), CKKS N=2^15",
                 "vital_window_batched_s": 1.21, "vital_window_per_frame_s": 99.48,
                 "gesture_window_batched_s": 5.76, "gesture_window_per_frame_s": 36.56,
                 "gesture_fc_layers_batched_s": 4.5}


# the mixed batch: windows per parameter set (vital windows, gesture windows),
# 40 vital and 24 gesture in all, on rings 2^15 and 2^16 with inputs of 12, 24
# and 30 limbs
MIXED_BATCH = (("mix15", 20, 12), ("vital", 20, 0), ("gesture", 0, 12))


def batched_mixed_benchmark(groups, log, reps=3):
    """64 encrypted windows of mixed shapes (40 vital-sign, 24 gesture; rings
    2^15 and 2^16; inputs of 12, 24 and 30 limbs) evaluated one plain call
    after another on one stream, against the same windows split into
    `groups` groups per parameter set, each group on a context and stream of
    its own (vital windows of a group evaluated together by
    hck_vital_eval_many, so that they share key-switch launches), issued
    eagerly and as one recorded graph set (hck_graph_*).  Every batched
    result equals the sequential one bit for bit."""
    import torch
    import paper_2603_22437_amd as H
    import seeded_inputs as S
    from paper_2603_22437_amd import gesture as HG
    from paper_2603_22437_amd import vital as HV
    t_setup = time.time()
    vcfg = S.vital_pipeline_config()
    vbase = (11 if vcfg["taylor_order"] == 3 else 9) + 1

    class Member:
        """One context evaluating a group of windows of one parameter set."""

        def __init__(self, name, nv, ng, key_words, stream, vseed, gseed):
            prm = S.params(name)
            self.prm = prm
            self.ctx = ctx = H.Context.from_params(prm)
            ctx.set_stream(stream)
            self.stream = stream
            top = len(prm["q"]) - 1
            self.gcfg = S.gesture_pipeline_config(frames=30 if prm["log_n"] == 16 else 14)
            self.vplan = HV.encode_plan(ctx, vcfg, min(vbase, top)) if nv else None
            self.gplan = HG.encode_plan(ctx, self.gcfg, 11, prm["scale"]) if ng else None
            sk = ctx.keygen_secret(1)
            if key_words is None:       # the parameter set's first context makes the keys
                steps = set()
                if nv:
                    steps |= set(ctx.vital_required_steps(self.vplan))
                if ng:
                    steps |= set(ctx.gesture_required_steps(self.gplan))
                gk = ctx.keygen_rotation(sk, sorted(steps), 5)
                rl = ctx.keygen_relin(sk, 7)
                key_words = ({ctx.galois_element(s): ctx.galois_keys_export(gk, ctx.galois_element(s))
                              for s in steps}, ctx.switch_key_export(rl))
            self.key_words = key_words
            self.gks = ctx.galois_keys_from_words(key_words[0])
            self.rlk = ctx.switch_key_import(key_words[1])

            def enc(x, seed):
                v = np.zeros(ctx.n_slots, dtype=np.complex128)
                v[: x.size] = x.reshape(-1)
                return (ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], top), seed),
                        ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], top), seed + 1))
            # window k: scene seed vseed + k (gesture: gseed + k), encryption
            # seeds derived from it, so every context holding that window
            # holds the same ciphertexts
            self.vin = [enc(S.vital_window(vseed + k, vcfg["frames"], vcfg["bins"]),
                            2 * (vseed + k)) for k in range(nv)]
            self.gin = [enc(S.gesture_window(gseed + k, self.gcfg["frames"]),
                            2 * (gseed + k)) for k in range(ng)]
            self.vout = [[ctx.ciphertext() for _ in range(4)] for _ in range(nv)]
            self.gout = [ctx.ciphertext() for _ in range(ng)]

        def plain(self):
            for (re, im), o in zip(self.vin, self.vout):
                self.ctx.vital_eval(self.vplan, re, im, self.gks, self.rlk, o)
            for (re, im), o in zip(self.gin, self.gout):
                self.ctx.gesture_eval(self.gplan, re, im, self.gks, self.rlk, o)

        def batched(self):
            if self.vin:
                self.ctx.vital_eval_many(self.vplan, [a for a, _ in self.vin],
                                         [b for _, b in self.vin], self.gks, self.rlk, self.vout)
            for (re, im), o in zip(self.gin, self.gout):
                self.ctx.gesture_eval(self.gplan, re, im, self.gks, self.rlk, o)

        def results(self):
            return ([[self.ctx.ciphertext_export(c)[0] for c in w] for w in self.vout] +
                    [[self.ctx.ciphertext_export(c)[0]] for c in self.gout])

        def close(self):
            self.ctx.synchronize()
            self.ctx.close()

    def split(total, k):
        return total // groups + (1 if k < total % groups else 0)

    # sequential plain path: one context per parameter set, one stream
    s0 = torch.cuda.Stream()
    seq, words = [], {}
    for name, nv, ng in MIXED_BATCH:
        m = Member(name, nv, ng, None, s0, 10000, 20000)
        words[name] = m.key_words
        seq.append(m)
    # the same windows in groups, each group a context on its own stream
    bat = []
    for name, nv, ng in MIXED_BATCH:
        first_v = first_g = 0
        for k in range(groups):
            gv, gg = split(nv, k), split(ng, k)
            if gv + gg == 0:
                continue
            # this group's windows are the sequential member's windows
            # first_v .. first_v + gv and first_g .. first_g + gg
            m = Member(name, gv, gg, words[name], torch.cuda.Stream(), 10000 + first_v,
                       20000 + first_g)
            bat.append((m, name, first_v, gv, first_g, gg))
            first_v += gv
            first_g += gg
    setup_s = time.time() - t_setup
    windows = sum(nv + ng for _, nv, ng in MIXED_BATCH)
    log(f"mixed batch: {windows} windows, {len(bat)} batched contexts, setup {setup_s:.1f}s")

    def run_seq():
        for m in seq:
            m.plain()

    def run_bat():
        for m, *_ in bat:
            m.batched()

    def timed(fn, streams):
        fn()
        for s in streams:
            s.synchronize()
        best = float("inf")
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            for s in streams:
                s.synchronize()
            best = min(best, time.perf_counter() - t)
        return best

    t_seq = timed(run_seq, [s0])
    streams = [m.stream for m, *_ in bat]
    t_eager = timed(run_bat, streams)
    with H.Graph.capture([m.ctx for m, *_ in bat]) as g:
        run_bat()
    t_graph = timed(g.launch, streams)
    # every batched result equals the sequential one
    exact = True
    for m, name, fv, gv, fg, gg in bat:
        s = next(x for x, (nm, _, _) in zip(seq, MIXED_BATCH) if nm == name)
        got = m.results()
        want_v = [[s.ctx.ciphertext_export(c)[0] for c in w] for w in s.vout[fv: fv + gv]]
        want_g = [[s.ctx.ciphertext_export(c)[0]] for c in s.gout[fg: fg + gg]]
        for a, b in zip(got, want_v + want_g):
            exact = exact and all(np.array_equal(x, y) for x, y in zip(a, b))
    info = g.info()
    g.close()
    for m, *_ in bat:
        m.close()
    for m in seq:
        m.close()
    res = {"windows": windows,
           "mix": [{"params": name, "vital": nv, "gesture": ng} for name, nv, ng in MIXED_BATCH],
           "groups_per_param_set": groups, "batched_contexts": len(streams),
           "sequential_plain_windows_per_s": round(windows / t_seq, 1),
           "batched_eager_windows_per_s": round(windows / t_eager, 1),
           "batched_graph_windows_per_s": round(windows / t_graph, 1),
           "speedup_graph_vs_sequential": round(t_seq / t_graph, 3),
           "speedup_eager_vs_sequential": round(t_seq / t_eager, 3),
           "graph_nodes": info["nodes"], "bit_exact_vs_sequential": bool(exact),
           "setup_s": round(setup_s, 1)}
    log(f"mixed batch: {res}")
    return res


def _pinned_u64(a):
    """A copy of a uint64 array in pinned host memory (asynchronous uploads)."""
    import torch
    t = torch.empty(a.size, dtype=torch.int64, pin_memory=True)
    out = t.numpy().view(np.uint64).reshape(a.shape)
    out[...] = a
    return out, t


def serving_benchmark(seconds, log, tenants=256, key_sets=4, budget_gb=200.0, max_batch=8,
                      max_inflight=32, seed=7):
    """The serving runtime (hck_server) on synthetic traffic, at N = 2^15,
    L = 12, where one tenant's evaluation keys take 0.5-2 GB.

    1. Batched against sequential: 64 mixed windows (40 vital, 24 gesture) of
       64 tenants as plain per-window calls, one after another, and then
       submitted to the server at once (keys resident after a warm-up pass).
    2. Serving: after every tenant's enrollment (its keys uploaded once, by
       one window), Poisson arrivals from `tenants` tenants (70 % vital, 30 %
       gesture) for `seconds`, at 80 % of the batched throughput, under an HBM
       budget of `budget_gb` for resident keys and admitted windows.  Latency is
       submit-to-result per request.  Synthetic tenants draw their keys from
       `key_sets` distinct secret keys (host-memory bound); each tenant still
       holds its own device copy."""
    import torch
    import paper_2603_22437_amd as H
    import seeded_inputs as S
    from paper_2603_22437_amd import gesture as HG
    from paper_2603_22437_amd import vital as HV
    prm = S.params("mix15")
    ctx = H.Context.from_params(prm)
    l0 = len(prm["q"]) - 1
    vcfg = S.vital_pipeline_config()
    gcfg = S.gesture_pipeline_config(frames=14)
    plans = {H.SERVE_VITAL: HV.encode_plan(ctx, vcfg, l0),
             H.SERVE_GESTURE: HG.encode_plan(ctx, gcfg, l0, prm["scale"])}
    steps = {H.SERVE_VITAL: ctx.vital_required_steps(plans[H.SERVE_VITAL]),
             H.SERVE_GESTURE: ctx.gesture_required_steps(plans[H.SERVE_GESTURE])}
    union = sorted(set(steps[H.SERVE_VITAL]) | set(steps[H.SERVE_GESTURE]))
    t0 = time.perf_counter()
    sets, keep = [], []
    for k in range(key_sets):
        sk = ctx.keygen_secret(900 + k)
        gks = ctx.keygen_rotation(sk, union, 910 + k)
        rlk = ctx.keygen_relin(sk, 920 + k)
        words = {}
        for st in union:
            w, t = _pinned_u64(ctx.galois_keys_export(gks, ctx.galois_element(st)))
            words[st] = w
            keep.append(t)
        rw, t = _pinned_u64(ctx.switch_key_export(rlk))
        keep.append(t)
        wins = {}
        for kind in (H.SERVE_VITAL, H.SERVE_GESTURE):
            wins[kind] = []
            for j in range(2):
                sd = 3000 + 10 * k + j
                z = (S.vital_window(sd, vcfg["frames"], vcfg["bins"]) if kind == H.SERVE_VITAL
                     else S.gesture_window(sd, gcfg["frames"]))
                v = np.zeros(ctx.n_slots, dtype=np.complex128)
                v[: z.size] = z.reshape(-1)
                re = ctx.encrypt_sk(sk, ctx.encode(v.real, prm["scale"], l0), 2 * sd)
                im = ctx.encrypt_sk(sk, ctx.encode(v.imag, prm["scale"], l0), 2 * sd + 1)
                wins[kind].append((re, im, ctx.ciphertext_export(re)[0],
                                   ctx.ciphertext_export(im)[0]))
        sets.append(dict(gks=gks, rlk=rlk, words=words, rlk_words=rw, wins=wins))
    kind_of = lambda t: H.SERVE_VITAL if t % 10 < 7 else H.SERVE_GESTURE
    log(f"serving set-up: {key_sets} key sets, {len(union)} rotation keys each, "
        f"{time.perf_counter() - t0:.1f} s")

    # 1. 64 mixed windows: sequential plain calls
    burst = [t for t in range(tenants) if kind_of(t) == H.SERVE_VITAL][:40] + \
            [t for t in range(tenants) if kind_of(t) == H.SERVE_GESTURE][:24]
    def window_of(t, j=0):
        return sets[t % key_sets]["wins"][kind_of(t)][j % 2]
    def sequential(transfers):
        """64 plain calls one after another (keys resident); with transfers,
        each window is also uploaded from and its outputs downloaded to host
        memory, as a caller without the server would."""
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for t in burst:
            ks = sets[t % key_sets]
            re, im, rw, iw = window_of(t)
            if transfers:
                re = ctx.ciphertext_import(rw, l0, prm["scale"])
                im = ctx.ciphertext_import(iw, l0, prm["scale"])
            if kind_of(t) == H.SERVE_VITAL:
                outs = ctx.vital_eval(plans[H.SERVE_VITAL], re, im, ks["gks"], ks["rlk"])
            else:
                outs = [ctx.gesture_eval(plans[H.SERVE_GESTURE], re, im, ks["gks"], ks["rlk"])]
            if transfers:
                for c in outs:
                    ctx.ciphertext_export(c)
        torch.cuda.synchronize()
        return time.perf_counter() - ts

    tuned = ctx.autotune_keyswitch()       # both paths run the tuned schedule
    sequential(False)
    seq_s = sequential(False)
    seq_io_s = sequential(True)
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(budget_gb * 2 ** 30, free - 24 * 2 ** 30))
    srv = H.Server(ctx, budget, max_batch, max_inflight)
    try:
        for t in range(tenants):
            ks = sets[t % key_sets]
            kind = kind_of(t)
            srv.add_tenant(t, kind, plans[kind], steps[kind],
                           [ks["words"][st] for st in steps[kind]], ks["rlk_words"])

        def run_burst(first_id):
            ts = time.perf_counter()
            for i, t in enumerate(burst):
                _, _, rw, iw = window_of(t)
                srv.submit(first_id + i, t, rw, iw, l0, prm["scale"])
            got = []
            while len(got) < len(burst):
                got += srv.poll(timeout_ms=60000)
            return time.perf_counter() - ts, got

        run_burst(0)                       # loads the 64 tenants' keys
        run_burst(500)                     # grows the scratch pool to full batches
        burst_s, got = run_burst(1000)     # keys resident
        assert all(r["status"] == 0 for r in got)
        batched_wps = len(burst) / burst_s
        batches = [r["batch"] for r in got]
        log(f"64 mixed windows: sequential {len(burst) / seq_s:.1f} windows/s, "
            f"served {batched_wps:.1f} windows/s")

        # enrollment: each tenant's evaluation keys are uploaded once, before
        # its traffic (one window per tenant brings them in; all tenants fit
        # the budget, so requests find their keys resident unless evicted)
        t_en = time.perf_counter()
        for t in range(tenants):
            _, _, rw, iw = window_of(t)
            srv.submit(2000 + t, t, rw, iw, l0, prm["scale"])
        done = 0
        while done < tenants:
            got = srv.poll(timeout_ms=60000)
            assert all(r["status"] == 0 for r in got)
            done += len(got)
        enroll_s = time.perf_counter() - t_en
        log(f"enrollment of {tenants} tenants: {enroll_s:.1f} s")

        # 2. Poisson arrivals
        rng = np.random.default_rng(seed)
        rate = 0.8 * batched_wps
        gaps = rng.exponential(1.0 / rate, size=int(rate * seconds * 1.5) + 16)
        arrivals = np.cumsum(gaps)
        arrivals = arrivals[arrivals < seconds]
        who = rng.integers(0, tenants, size=len(arrivals))
        st0 = srv.stats()
        results, lag = [], 0.0
        base = time.perf_counter()
        nxt = 0
        next_log = base + 5.0
        while nxt < len(arrivals) or len(results) < len(arrivals):
            now = time.perf_counter() - base
            while nxt < len(arrivals) and arrivals[nxt] <= now:
                t = int(who[nxt])
                _, _, rw, iw = window_of(t, nxt)
                srv.submit(10000 + nxt, t, rw, iw, l0, prm["scale"])
                lag = max(lag, time.perf_counter() - base - arrivals[nxt])
                nxt += 1
            wait = 0 if nxt >= len(arrivals) else max(0.0, arrivals[nxt] - now)
            got = srv.poll(timeout_ms=int(min(wait, 0.05) * 1000) if nxt < len(arrivals)
                           else 1000)
            for r in got:       # keep the timing records only (a long run would
                r.pop("outputs")  # otherwise hold every window's outputs)
            results += got
            if time.perf_counter() > next_log:
                log(f"serving: {nxt} submitted, {len(results)} done")
                next_log += 5.0
        wall = time.perf_counter() - base
        st1 = srv.stats()
    finally:
        srv.close()
    ok = [r for r in results if r["status"] == 0]
    lat = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in ok])
    vl = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in ok
                   if kind_of(r["tenant"]) == H.SERVE_VITAL])
    gl = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in ok
                   if kind_of(r["tenant"]) == H.SERVE_GESTURE])
    warm = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in ok if not r["key_load"]])
    cold = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in ok if r["key_load"]])
    pct = lambda a, q: round(float(np.percentile(a, q)), 2) if len(a) else None
    out = {
        "ring": "N=2^15, L=12, K=4, dnum=3",
        "tenants": tenants, "mix": "70% vital / 30% gesture",
        "key_gb_per_tenant": {"vital": round((len(steps[H.SERVE_VITAL]) + 1) *
                                             sets[0]["rlk_words"].nbytes / 2 ** 30, 3),
                              "gesture": round((len(steps[H.SERVE_GESTURE]) + 1) *
                                               sets[0]["rlk_words"].nbytes / 2 ** 30, 3)},
        "hbm_budget_gb": round(budget / 2 ** 30, 1),
        "max_batch": max_batch, "max_inflight": max_inflight,
        "keyswitches_per_launch": [tuned[l][0] for l in sorted(tuned)],
        "batched_vs_sequential": {
            "windows": len(burst), "sequential_plain_windows_per_s": round(len(burst) / seq_s, 2),
            "sequential_plain_with_transfers_windows_per_s": round(len(burst) / seq_io_s, 2),
            "served_batched_windows_per_s": round(batched_wps, 2),
            "speedup_vs_plain": round(batched_wps * seq_s / len(burst), 3),
            "speedup_vs_plain_with_transfers": round(batched_wps * seq_io_s / len(burst), 3),
            "mean_batch": round(float(np.mean(batches)), 2)},
        "poisson": {
            "enrollment_s": round(enroll_s, 2),
            "seconds": seconds, "offered_windows_per_s": round(rate, 2),
            "submitted": int(len(arrivals)), "completed": len(ok),
            "failed": len(results) - len(ok),
            "windows_per_s": round(len(ok) / wall, 2),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "vital_p50_ms": pct(vl, 50), "vital_p99_ms": pct(vl, 99),
            "gesture_p50_ms": pct(gl, 50), "gesture_p99_ms": pct(gl, 99),
            "warm_requests": int(len(warm)), "warm_p50_ms": pct(warm, 50),
            "warm_p99_ms": pct(warm, 99),
            "cold_requests": int(len(cold)), "cold_p50_ms": pct(cold, 50),
            "cold_p99_ms": pct(cold, 99),
            "mean_batch": round(float(np.mean([r["batch"] for r in ok])), 2) if ok else None,
            "key_loads": st1["key_loads"] - st0["key_loads"],
            "evictions": st1["evictions"] - st0["evictions"],
            "key_gb_loaded": round((st1["key_bytes_loaded"] - st0["key_bytes_loaded"]) / 2 ** 30,
                                   1),
            "max_submit_lag_ms": round(float(lag) * 1e3, 2)},
    }
    log(f"serving: {out}")
    return out


def _flat(result):
    """(outputs, taps) of a *_eval_taps call as one list: taps, then outputs."""
    outs, taps = result
    return list(taps) + (list(outs) if isinstance(outs, (list, tuple)) else [outs])


# multiplicative depth (products on the path) of each tap and output
VITAL_DEPTHS = [1, 1, 2, 3, 3, 4, 4, 4, 4, 7, 7, 8, 8, 9, 10, 3, 3, 11, 11]
GESTURE_DEPTHS = [1, 1, 2, 3, 5, 6, 7, 9, 11]


def kernel_noise(ctx, prm, sk, top, base, depths, names, run, plain, windows):
    """Per-kernel encryption noise, the method of section 5.2 (Table 3): the
    MSE and max |error| between each decoded intermediate of the encrypted
    pipeline and the same value from plaintext execution, cumulative after
    the preceding kernels, over the given windows (encrypted at level `top`,
    evaluated from the plan's level `base`), with the multiplicative depth
    of the stage and the level its ciphertext ends at."""
    sq = [0.0] * len(names)
    cnt = [0] * len(names)
    mx = [0.0] * len(names)
    level = [0] * len(names)
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
            level[i] = c.level
    return [{"stage": n, "mse": float(f"{sq[i] / cnt[i]:.3e}"),
             "max_abs_err": float(f"{mx[i]:.3e}"), "depth": depths[i], "level": level[i]}
            for i, n in enumerate(names)]


def cpu_baseline(prm, seconds, log):
    """The oracle on the host: the rotation (automorphism + hybrid key
    switching) of one N = 2^16, L = 24 ciphertext at the top level, repeated
    for ~`seconds` on all threads and for 2 rotations on one thread; and the
    tiny configuration end to end (BSGS linear transform, rescale, square
    with relinearization) at N = 2^12."""
    import oracle as O
    import seeded_inputs as S
    o = O.Oracle(prm)
    s = o.keygen_secret(1)
    g = o.galois_element(1)
    gk = {g: o.keygen_galois(s, g, 5)}
    res = S.uniform_residues(o.qmods(o.L - 1), o.n, 7, count=2)
    ct = O.Ciphertext(res, o.L - 1, 2.0 ** 50)

    def rotations(budget, most):
        nonlocal ct
        n_rot, t0 = 0, time.perf_counter()
        while n_rot < most:
            ct = o.rotate(ct, 1, gk)
            n_rot += 1
            el = time.perf_counter() - t0
            if el >= budget or el * (n_rot + 1) / n_rot > 2 * budget:
                break
        return n_rot, el

    threads = O.num_threads()
    n_rot, el = rotations(seconds, 10 ** 6)
    log(f"oracle: {n_rot} rotations in {el:.1f}s on {threads} threads")
    O.set_num_threads(1)
    try:
        n1, el1 = rotations(seconds, 2)
    finally:
        O.set_num_threads(threads)
    log(f"oracle: {n1} rotations in {el1:.1f}s on 1 thread")
    # the tiny configuration end to end
    tp = S.params("tiny")
    ot = O.Oracle(tp)
    st = ot.keygen_secret(1)
    level = ot.L - 1
    x = S.uniform_slots(ot.n_slots, 0)
    mat = S.uniform_matrix(64, 64, 0, 1 / 8)
    diags = {}
    for k in range(-63, 64):
        d = np.zeros(ot.n_slots)
        for j in range(ot.n_slots):
            i = j % 64
            if 0 <= i + k < 64:
                d[j] = mat[i, i + k]
        diags[k % ot.n_slots] = d
    lt = ot.lt_create(diags, 16, level)
    gks = {ot.galois_element(k): ot.keygen_galois(st, ot.galois_element(k), 5)
           for k in ot.lt_required_steps(lt)}
    rlk = ot.keygen_relin(st, 7)
    ctt = ot.encrypt_sk(st, ot.encode(x, tp["scale"], level), 3)
    t0 = time.perf_counter()
    y = ot.rescale(ot.lt_apply(lt, ctt, gks))
    y = ot.relinearize(ot.tensor(y, y), rlk)
    tiny_s = time.perf_counter() - t0
    log(f"oracle: tiny configuration end to end in {tiny_s:.2f}s")
    return {"value": round(n_rot / el, 4), "unit": "rotations/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_rot} rotation(s) of one N=2^16, L=24 top-level ciphertext "
                      "(automorphism + hybrid key switching), not the full window step",
            "single_thread_rotations_per_s": round(n1 / el1, 4),
            "tiny_end_to_end_s": round(tiny_s, 3),
            "tiny_sample": "N=2^12, L=3: (I_32 (x) M64) x by BSGS (127 diagonals, n1=16), "
                           "rescale, square + relinearize",
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
