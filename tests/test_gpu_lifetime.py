"""Handle lifetimes through the C ABI (MI355X).

A context owns the device memory of its objects: destroying it releases the
memory of every handle still alive and detaches those handles, whose own
destroy calls then free only their host records, so destroy calls may come
in any order (a garbage-collected reference cycle, e.g. a traceback that
holds a context and its handles, finalizes them in no fixed order).  Calls
with a detached handle fail with HCK_EINVAL instead of touching freed memory.

Each case runs in a child process and must end normally: exit status 0, or 1
for the deliberately uncaught exception, never a signal.
"""
import os
import subprocess
import sys
import textwrap

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PRELUDE = textwrap.dedent(f"""
    import gc, sys
    sys.path.insert(0, {ROOT!r})
    import numpy as np
    import paper_2603_22437_amd as H
    import seeded_inputs as S
    prm = S.params("tiny")
    z = np.random.default_rng(0).uniform(-1, 1, 1 << (prm["log_n"] - 1))

    def objects(ctx):
        sk = ctx.keygen_secret(1)
        gks = ctx.keygen_rotation(sk, [1, 3], 2)
        rlk = ctx.keygen_relin(sk, 3)
        pt = ctx.encode(z, prm["scale"], len(prm["q"]) - 1)
        ct = ctx.encrypt_sk(sk, pt, 4)
        r = ctx.rotate(ct, 1, gks)
        return [sk, gks, rlk, pt, ct, r]
    print("case start", flush=True)
""")


def run_child(body: str, expect_rc: int = 0, marker: str = "case done"):
    code = PRELUDE + textwrap.dedent(body)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    msg = f"rc={p.returncode}\nstdout:\n{p.stdout[-3000:]}\nstderr:\n{p.stderr[-3000:]}"
    assert p.returncode == expect_rc, msg
    assert marker in p.stdout + p.stderr, msg
    return p


def test_context_closed_before_its_handles():
    run_child("""
        ctx = H.Context.from_params(prm)
        objs = objects(ctx)
        ctx.synchronize()
        ctx.close()
        # detached handles are refused by a live context of the same shape
        ctx2 = H.Context.from_params(prm)
        try:
            ctx2.add(objs[4], objs[4])
            raise SystemExit("a detached handle was accepted")
        except H.HckError as e:
            assert e.code == H.HCK_EINVAL, e
        for o in objs:
            o.close()
        objs = None
        ctx2.close()
        print("case done", flush=True)
    """)


def test_reference_cycle_collected_in_any_order():
    run_child("""
        class Node:
            pass
        for rep in range(4):
            ctx = H.Context.from_params(prm)
            n = Node()
            n.ctx, n.objs, n.me = ctx, objects(ctx), n
            if rep % 2:
                n.objs.reverse()
            ctx = None
            n = None
            gc.collect()
        print("case done", flush=True)
    """)


def test_uncaught_exception_with_live_handles_exits_cleanly():
    # the traceback keeps the frame with the context and its handles alive
    # until interpreter shutdown, which finalizes them
    run_child("""
        def fail():
            ctx = H.Context.from_params(prm)
            objs = objects(ctx)
            server = H.Server(ctx, 1 << 30)
            print("case done", flush=True)
            raise RuntimeError("planned failure with live handles")
        fail()
    """, expect_rc=1)


def test_server_alive_when_its_context_is_closed():
    run_child("""
        ctx = H.Context.from_params(prm)
        objs = objects(ctx)
        server = H.Server(ctx, 1 << 30)
        ctx.close()
        try:
            server.submit(1, 7, np.zeros((2, 3, 4096), np.uint64),
                          np.zeros((2, 3, 4096), np.uint64), 2, 2.0 ** 25)
            raise SystemExit("a server of a destroyed context accepted work")
        except H.HckError:
            pass
        server.close()
        for o in objs:
            o.close()
        print("case done", flush=True)
    """)
