"""Batched persistent launch, its captured graph, and the tuner."""
import numpy as np
import pytest

import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def make_batch(n, seed_shapes=3, dtype="f32", scale=1):
    """n uneven images: H, W = 8*U{30..270} // scale (multiple of 8 for scale 1)."""
    shapes = synth.batch_shapes(seed_shapes, n)
    hosts, ins, ks = [], [], []
    for i, (h, w) in enumerate(shapes):
        h, w = max(1, h // scale), max(1, w // scale)
        host = synth.image(100 + i, 3, h, w)
        bits = synth.to_storage(host, dtype)
        hosts.append(bits)
        ins.append(gu.to_device(bits, dtype))
        ks.append(synth.taps_random(200 + i))
    return hosts, ins, ks


def lone(ins, ks, mode=cs.CONV_1PASS_FUSED):
    outs = []
    for a, k in zip(ins, ks):
        o = gu.nan_like(a)
        cs.conv_sep5_1pass(a, o, k, mode)
        outs.append(o)
    return outs


def test_batch_64_uneven_images_matches_lone_and_oracle():
    """The 64-image batch (H, W in 240..2160, multiples of 8, per-image taps)."""
    torch = _torch()
    hosts, ins, ks = make_batch(64)
    outs = [gu.nan_like(a) for a in ins]
    cs.conv_sep5_batch(ins, outs, ks)
    ref_lone = lone(ins, ks)
    for i in range(64):
        assert torch.equal(outs[i], ref_lone[i]), f"image {i}"
    worst = 0.0
    for i in range(0, 64, 3):
        R = hosts[i].shape[1]
        rows = sorted({0, 1, 2, 3, R // 2, R - 3, R - 2, R - 1})
        refs = gu.sample_rows_oracle(hosts[i], ks[i], rows)
        got = outs[i][:, rows, :].cpu().numpy()
        worst = max(worst, gu.check_f32(got, np.stack([refs[y] for y in rows], axis=1)))
    print(f"batch of 64: max rel err on sampled rows {worst:.3e}")


@pytest.mark.parametrize("mode", [cs.CONV_1PASS_FUSED, cs.CONV_1PASS_DIRECT25])
def test_batch_small_full_oracle(mode):
    hosts, ins, ks = make_batch(12, seed_shapes=4, scale=8)
    outs = [gu.nan_like(a) for a in ins]
    cs.conv_sep5_batch(ins, outs, ks, mode=mode)
    for i in range(12):
        gu.check_f32(gu.to_host_bits(outs[i]), gu.oracle_of(hosts[i], ks[i]))
        assert np.array_equal(gu.to_host_bits(outs[i]), gu.to_host_bits(lone([ins[i]], [ks[i]], mode)[0]))


def test_batch_mixed_layouts_and_empty_images():
    torch = _torch()
    shapes = [(3, 50, 301), (1, 4, 64), (3, 0, 10), (2, 77, 256), (3, 130, 517), (1, 1, 1)]
    ins, hosts, ks = [], [], []
    for i, s in enumerate(shapes):
        h = synth.image(300 + i, *s)
        hosts.append(h)
        ins.append(torch.from_numpy(h).cuda())
        ks.append(synth.taps_random(400 + i))
    # one image as an unaligned view (its output is the same view of another buffer)
    big = torch.zeros(3, 130, 520, device="cuda")
    big[:, :, 1:518] = ins[4]
    ins[4] = big[:, :, 1:518]
    outs = [torch.full(a.shape, float("nan"), device="cuda") for a in ins]
    big_out = torch.full((3, 130, 520), 777.0, device="cuda")
    outs[4] = big_out[:, :, 1:518]
    outs[4].fill_(float("nan"))
    cs.conv_sep5_batch(ins, outs, ks)
    assert torch.all(big_out[:, :, 0] == 777.0) and torch.all(big_out[:, :, 518:] == 777.0)
    for i, s in enumerate(shapes):
        if 0 in s:
            continue
        gu.check_f32(outs[i].cpu().numpy(), gu.oracle_of(hosts[i], ks[i]))


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_batch_16bit_matches_lone(dtype):
    torch = _torch()
    hosts, ins, ks = make_batch(10, seed_shapes=5, dtype=dtype, scale=4)
    outs = [gu.nan_like(a) for a in ins]
    cs.conv_sep5_batch(ins, outs, ks)
    for o, r in zip(outs, lone(ins, ks)):
        assert torch.equal(o.view(torch.int16), r.view(torch.int16))


def test_graph_plan_replays_match_eager():
    torch = _torch()
    hosts, ins, ks = make_batch(16, seed_shapes=6, scale=2)
    eager = [gu.nan_like(a) for a in ins]
    cs.conv_sep5_batch(ins, eager, ks)
    outs = [gu.nan_like(a) for a in ins]
    plan = cs.conv_batch_plan_create(ins, outs, ks)
    try:
        for rep in range(4):
            for o in outs:
                o.fill_(float("nan"))
            x = torch.randn(1 << 20, device="cuda")
            (x * 2).sum().item()  # unrelated eager work and a sync between replays
            plan.launch()
            torch.cuda.synchronize()
            for i in range(16):
                assert torch.equal(outs[i], eager[i]), (rep, i)
    finally:
        plan.destroy()


def test_every_batch_tile_config_is_bitwise_identical_and_tuner_runs():
    torch = _torch()
    hosts, ins, ks = make_batch(8, seed_shapes=7, scale=4)
    orig = cs.conv_get_tile_cfg(0, 1)
    orig0 = cs.conv_get_tile_cfg(0, 0)
    base = [gu.nan_like(a) for a in ins]
    cs.conv_sep5_batch(ins, base, ks)
    try:
        for th in (4, 8, 16, 64, 128):
            for w in (1, 2, 4):
                for p in (0, 1, 4, 16):
                    for x in (0, 1, 2, 8):
                        cs.conv_set_tile_cfg(0, 1, th, w, p, x)
                        outs = [gu.nan_like(a) for a in ins]
                        cs.conv_sep5_batch(ins, outs, ks)
                        for o, b in zip(outs, base):
                            assert torch.equal(o, b), (th, w, p, x)
        best, ms = cs.conv_tune(cs.KIND_BATCH, ins, base, ks, reps=2)
        assert best.rows_per_tile >= 1 and ms > 0
        best0, ms0 = cs.conv_tune(cs.KIND_IMAGE, ins[:1], base[:1], ks[:1], reps=2)
        assert best0.rows_per_tile >= 1 and ms0 > 0
        outs = [gu.nan_like(a) for a in ins]
        cs.conv_sep5_batch(ins, outs, ks)
        for o, b in zip(outs, base):
            assert torch.equal(o, b)
    finally:
        cs.conv_set_tile_cfg(0, 1, orig.rows_per_tile, orig.waves_per_wg, orig.persist_wgs_per_cu,
                             orig.xcd_slabs)
        cs.conv_set_tile_cfg(0, 0, orig0.rows_per_tile, orig0.waves_per_wg, 0, orig0.xcd_slabs)
