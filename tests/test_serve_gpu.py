"""Continuous-batching server: every result is the same alone and in the mix,
admission respects the HBM budget, launches overlap, errors are reported."""
import time

import pytest

import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _requests(n, seed, sizes=synth.SERVE_SIZES):
    import numpy as np
    import torch

    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        h, w = sizes[int(rng.integers(0, len(sizes)))]
        a = torch.rand(3, h, w, device="cuda", generator=None)
        reqs.append((a, synth.taps_random(seed * 1000 + i)))
    return reqs


def _wait_all(srv, tickets, timeout_s=60.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t in done:
                continue
            r = srv.poll(t)
            if r is not None:
                done[t] = r
        assert time.time() - t0 < timeout_s, "server did not finish"
    return done


@pytest.mark.parametrize("queue_only", [False, True])
def test_results_alone_equal_results_in_the_mix(queue_only):
    """queue_only = False: submits that find nothing queued and a stream idle
    launch their request themselves; True: every launch by the scheduler."""
    import torch

    torch.manual_seed(0)
    reqs = _requests(40, seed=1)
    alone = []
    for a, k in reqs:
        o = gu.nan_like(a)
        cs.conv_sep5_1pass(a, o, k)
        alone.append(o)
    torch.cuda.synchronize()
    budget = 600 << 20
    srv = cs.conv_serve_create(budget, max_slots=16, n_streams=4, max_batch=8,
                               queue_only=queue_only)
    try:
        outs = [gu.nan_like(a) for a, _ in reqs]
        tickets = []
        for i, (a, k) in enumerate(reqs):
            tickets.append(srv.submit(a, outs[i], k))
            if i % 7 == 3:
                time.sleep(0.0005)  # arrivals while earlier launches run
        times = _wait_all(srv, tickets)
        st = srv.stats()
    finally:
        srv.destroy()
    for o, r in zip(outs, alone):
        assert torch.equal(o, r)
    assert st["completed"] == 40 and st["failed"] == 0
    assert st["max_bytes_in_flight"] <= budget
    assert st["max_slots_in_flight"] <= 16 and st["max_batch"] <= 8
    for t in times.values():
        assert t["submit_ns"] <= t["admit_ns"] <= t["launch_ns"] <= t["done_ns"]
    if queue_only:
        assert st["direct_launches"] == 0
    else:
        assert 1 <= st["direct_launches"] <= st["launches"]
    print("serve stats", st)


def test_drain_sees_direct_launches():
    """A submit that launches its request itself and an immediate drain: the
    drain returns only once that request is done (the scheduler must not
    report idle while a submitter is still launching)."""
    import torch

    srv = cs.conv_serve_create(1 << 30, max_slots=8, n_streams=2, max_batch=4)
    try:
        for i in range(60):
            a = torch.rand(3, 96 + i, 130, device="cuda")
            o = gu.nan_like(a)
            t = srv.submit(a, o, synth.taps_random(7000 + i))
            srv.drain()
            assert srv.poll(t) is not None, i
            assert torch.isfinite(o).all()
        assert srv.stats()["direct_launches"] >= 1
    finally:
        srv.destroy()


def test_budget_limits_admission_and_launches_overlap():
    import torch

    torch.manual_seed(1)
    reqs = _requests(12, seed=2, sizes=((2160, 3840),))
    fp = 2 * 3 * 2160 * 3840 * 4
    srv = cs.conv_serve_create(3 * fp, max_slots=64, n_streams=4, max_batch=1)
    try:
        outs = [gu.nan_like(a) for a, _ in reqs]
        tickets = [srv.submit(a, o, k) for (a, k), o in zip(reqs, outs)]
        _wait_all(srv, tickets)
        st = srv.stats()
    finally:
        srv.destroy()
    assert st["max_bytes_in_flight"] <= 3 * fp
    assert st["max_streams_busy"] >= 2, st   # several launches on the device at once
    for (a, k), o in zip(reqs, outs):
        r = gu.nan_like(a)
        cs.conv_sep5_1pass(a, r, k)
        assert torch.equal(o, r)


def test_errors_and_ticket_lifecycle():
    import torch

    srv = cs.conv_serve_create(1 << 20, max_slots=2, n_streams=1, max_batch=2)
    try:
        big = torch.zeros(3, 512, 512, device="cuda")
        with pytest.raises(cs.ConvError) as e:
            srv.submit(big, torch.zeros_like(big), [1, 4, 6, 4, 1])
        assert e.value.status == cs.CONV_ENOMEM
        with pytest.raises(cs.ConvError) as e:
            srv.submit(big, big, [1, 4, 6, 4, 1])
        assert e.value.status in (cs.CONV_EALIAS, cs.CONV_ENOMEM)
        with pytest.raises(cs.ConvError) as e:
            srv.poll(987654)
        assert e.value.status == cs.CONV_ENOTFOUND
        small = torch.rand(3, 64, 64, device="cuda")
        out = torch.zeros_like(small)
        t = srv.submit(small, out, [1, 4, 6, 4, 1])
        srv.drain()
        assert srv.poll(t) is not None
        with pytest.raises(cs.ConvError):
            srv.poll(t)  # reported once, then forgotten
    finally:
        srv.destroy()


def test_no_producer_wait_mode_after_sync():
    """producer_wait = 0: the caller synchronises its inputs before submitting."""
    import torch

    torch.manual_seed(3)
    reqs = _requests(16, seed=4, sizes=((480, 640), (720, 1280)))
    outs = [gu.nan_like(a) for a, _ in reqs]
    torch.cuda.synchronize()
    srv = cs.conv_serve_create(1 << 30, max_slots=16, n_streams=2, max_batch=8,
                               max_batch_bytes=64 << 20, producer_wait=False)
    try:
        tickets = [srv.submit(a, o, k) for (a, k), o in zip(reqs, outs)]
        _wait_all(srv, tickets)
    finally:
        srv.destroy()
    for (a, k), o in zip(reqs, outs):
        r = gu.nan_like(a)
        cs.conv_sep5_1pass(a, r, k)
        assert torch.equal(o, r)
