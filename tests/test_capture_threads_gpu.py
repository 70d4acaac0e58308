"""The C ABI under a captured hipGraph and from several host threads at once.

* Graph: the fused, direct, two-pass (caller workspace), width-n and pyramid
  calls are captured once on torch's capture stream and replayed several
  times, with new input copied in eagerly and other eager work between the
  replays; every replay must equal the eager result on the same input.
* Threads: eight host threads call the single-image and batch entry points
  concurrently, each on its own stream and buffers (ctypes releases the GIL,
  so the library's descriptor ring and configuration table see real
  concurrency); every result must equal the one computed alone.
"""
import threading

import numpy as np
import pytest

import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def test_calls_replay_in_a_captured_graph():
    torch = _torch()
    P, R, C = 3, 300, 520
    k = synth.taps_random(3000)
    k7 = synth.taps_random_n(3001, 7)
    a = gu.to_device(synth.image(3002, P, R, C))           # static input of the graph
    tmp = torch.empty(P * R * C, device="cuda")
    outs = {f: torch.empty_like(a) for f in ("fused", "direct", "2pass", "n7")}
    pyr = torch.empty(P, (R + 1) // 2, (C + 1) // 2, device="cuda")

    def calls():
        cs.conv_sep5_1pass(a, outs["fused"], k, cs.CONV_1PASS_FUSED)
        cs.conv_sep5_1pass(a, outs["direct"], k, cs.CONV_1PASS_DIRECT25)
        cs.conv_sep5_2pass(a, outs["2pass"], k, d_tmp=tmp)
        cs.conv_sepn_1pass(a, outs["n7"], k7, cs.CONV_1PASS_FUSED)
        cs.conv_pyr_down(a, pyr, k)

    calls()                        # warm up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            calls()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        a.copy_(gu.to_device(synth.image(3100 + rep, P, R, C)))
        junk = torch.rand(1 << 20, device="cuda").sum()   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = {f: o.clone() for f, o in outs.items()}
        got_pyr = pyr.clone()
        for o in outs.values():
            o.fill_(float("nan"))
        pyr.fill_(float("nan"))
        calls()                    # eager on the same input
        torch.cuda.synchronize()
        for f in outs:
            assert torch.equal(got[f], outs[f]), (rep, f)
        assert torch.equal(got_pyr, pyr), rep
        del junk


def test_concurrent_host_threads():
    torch = _torch()
    T = 8
    rng = np.random.default_rng(3200)
    jobs = []
    for t in range(T):
        R, C = (int(v) for v in rng.integers(64, 400, size=2))
        a = gu.to_device(synth.image(3300 + t, 3, R, C))
        b_imgs = [gu.to_device(synth.image(3400 + 10 * t + i, 3, int(h), int(w)))
                  for i, (h, w) in enumerate(rng.integers(40, 300, size=(20, 2)))]
        k = synth.taps_random(3500 + t)
        jobs.append((a, b_imgs, k))

    def run(job, stream):
        a, b_imgs, k = job
        # allocate on the stream that uses the buffers, so that the caching
        # allocator only reuses them in that stream's order
        with torch.cuda.stream(stream):
            o1 = torch.empty_like(a)
            o2 = torch.empty_like(a)
            ob = [torch.empty_like(x) for x in b_imgs]
            cs.conv_sep5_1pass(a, o1, k, stream=stream)
            cs.conv_sep5_2pass(a, o2, k, stream=stream)
            cs.conv_sep5_batch(b_imgs, ob, [k] * len(b_imgs), stream=stream)
        return o1, o2, ob

    # alone, one after the other
    ref = [run(j, torch.cuda.current_stream()) for j in jobs]
    torch.cuda.synchronize()
    # all at once from T threads, each with its own stream (the inputs were
    # written on the default stream, which is synchronised above)
    results = [None] * T
    errors = []
    streams = [torch.cuda.Stream() for _ in range(T)]
    barrier = threading.Barrier(T)

    def worker(t):
        try:
            torch.cuda.set_device(0)
            barrier.wait()
            for _ in range(3):
                results[t] = run(jobs[t], streams[t])
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(T)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not errors, errors
    torch.cuda.synchronize()
    for t in range(T):
        o1, o2, ob = results[t]
        r1, r2, rb = ref[t]
        assert torch.equal(o1, r1) and torch.equal(o2, r2), t
        assert all(torch.equal(x, y) for x, y in zip(ob, rb)), t
