"""The target workloads at their full sizes, in the launch configurations the
benchmark times: the 64-frame 1024x1024 batch as one launch sequence, an
uneven batch of frames with the mixed workload's sizes (up to 2048x2048), and
three frames in flight on three contexts and streams.  Every frame of a
batch must equal the same frame run alone (bitwise), and sampled frames are
checked in full against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from parity import (check_candidates, check_candidates_exact, check_exempt_bound, check_planes,
                    check_pruned)

pytestmark = pytest.mark.gpu

CAMERA = dict(sigma_min=1.0, sigma_max=30.0, sigma_ratio=1.6, threshold=0.05, overlap=0.5)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def dog():
    import paper_2010_08486_amd as d
    return d


def _oracle_check(c, t, img, prm, natural=True, planes=False):
    """Candidates against the oracle's FP64 cube (near-tie exemptions bounded
    on frames of natural shape) and, with no margin at all, against the
    oracle's local-maximum search on the GPU's own fp32 cube; optionally the
    planes themselves."""
    L_o, D_o, sig = oracle.planes(img, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, 4.0)
    max_abs = float(np.abs(img).max())
    L_g, D_g = c.debug_planes(t, prm)
    D_g = D_g.cpu().numpy()
    if planes:
        check_planes(L_g.cpu().numpy(), D_g, L_o, D_o, sig, max_abs)
    del L_g
    raw = c.debug_candidates(t, prm)
    check_candidates_exact(raw, D_g, prm.threshold)
    exempt = check_candidates(raw, D_o, prm.threshold, sig, max_abs)
    if natural:
        check_exempt_bound(exempt, len(raw))
    return raw, D_o, sig, exempt


def test_batch64_full_size(dog, torch_mod):
    torch = torch_mod
    prm = dog.Params(**CAMERA)
    frames = synth.batch64(n_frames=64)
    dev = [torch.from_numpy(f).cuda() for f in frames]
    print("batch64: 64 frames generated", flush=True)
    with dog.Context(0) as c:
        first, raw_n = c.detect_batch(dev, prm)   # one frame per group, three lanes
        second, _ = c.detect_batch(dev, prm)      # the lanes replay captured graphs
        c.set_batch_grouping(0)
        one, _ = c.detect_batch(dev, prm)         # one launch sequence of 64 frames
        one2, _ = c.detect_batch(dev, prm)        # ... replayed from its graph
        c.set_batch_grouping(3 << 20, 1)          # groups of three, one at a time
        seq, _ = c.detect_batch(dev, prm)
        c.set_batch_grouping(1 << 20, 3)
        for f in range(64):
            alone = c.detect_device(dev[f], prm)
            for other in (second, one, one2, seq):
                assert first[f].tobytes() == alone.tobytes() == other[f].tobytes(), f
        for f in (0, 31, 63):
            raw, D_o, sig, exempt = _oracle_check(c, dev[f], frames[f], prm)
            assert len(raw) == raw_n[f]
            check_pruned(first[f], raw, D_o, prm.threshold, sig, prm.overlap, exempt)
            print("batch64 frame %d: raw %d pruned %d exempt %d" % (f, len(raw), len(first[f]), exempt),
                  flush=True)


def test_uneven_batch_full_sizes(dog, torch_mod):
    torch = torch_mod
    prm = dog.Params(**CAMERA)
    shapes = synth.mixed_shapes()[:32]
    frames = [synth.mixed_frame(f, H, W) for f, (H, W) in enumerate(shapes)]
    dev = [torch.from_numpy(f).cuda() for f in frames]
    print("uneven: %d frames, %.1f Mpx" % (len(frames), sum(h * w for h, w in shapes) / 1e6), flush=True)
    with dog.Context(0) as c:
        res, raw_n = c.detect_batch(dev, prm)
        for f in range(len(frames)):
            assert res[f].tobytes() == c.detect_device(dev[f], prm).tobytes(), (f, shapes[f])
        # the largest square, a 2:1 crop and a mid-size frame against the oracle
        picks = [max(range(len(shapes)), key=lambda i: shapes[i][0] * shapes[i][1] *
                     (shapes[i][0] == shapes[i][1]))]
        picks += [i for i in range(len(shapes)) if shapes[i][0] * 2 == shapes[i][1]][:1]
        picks += [i for i in range(len(shapes)) if shapes[i] == (768, 768)][:1]
        for f in picks:
            raw, D_o, sig, exempt = _oracle_check(c, dev[f], frames[f], prm)
            assert len(raw) == raw_n[f]
            check_pruned(res[f], raw, D_o, prm.threshold, sig, prm.overlap, exempt)
            print("uneven frame %d %s: raw %d pruned %d exempt %d" % (f, shapes[f], len(raw),
                                                                     len(res[f]), exempt), flush=True)


@pytest.mark.parametrize("min_taps", [0, 53, 1])
def test_three_in_flight_full_size(dog, torch_mod, min_taps):
    # the benchmark's timed configuration: three contexts, each on its own
    # stream, steps queued before the previous ones are collected; every
    # plane direct, the five widest planes in the transform domain (the
    # threshold the autotuner picks for this frame), and every plane there
    torch = torch_mod
    prm = dog.Params(**CAMERA)
    imgs = [synth.camera_frame(seed=s) for s in (1, 2, 3, 4, 5)]
    dev = [torch.from_numpy(a).cuda() for a in imgs]
    ctxs = [dog.Context(0) for _ in range(3)]
    for c in ctxs:
        c.set_dct(min_taps)
    streams = [torch.cuda.Stream() for _ in range(3)]
    try:
        ref = [ctxs[0].detect_device(t, prm) for t in dev]
        torch.cuda.synchronize()
        steps, nf = 12, 3
        got = []
        for i in range(nf - 1):
            ctxs[i].detect_device_async(dev[i % 5], prm, stream=streams[i])
        for i in range(nf - 1, steps + nf - 1):
            if i < steps:
                ctxs[i % nf].detect_device_async(dev[i % 5], prm, stream=streams[i % nf])
            got.append(ctxs[(i - nf + 1) % nf].finish())
        for i, b in enumerate(got):
            assert b.tobytes() == ref[i % 5].tobytes(), i
        raw, D_o, sig, exempt = _oracle_check(ctxs[0], dev[1], imgs[1], prm, planes=min_taps > 0)
        check_pruned(ref[1], raw, D_o, prm.threshold, sig, prm.overlap, exempt)
    finally:
        for c in ctxs:
            c.close()


@pytest.mark.parametrize("H,W,n_blobs", [(4096, 4096, 2000), (8, 32768, 60), (32768, 8, 60)])
def test_large_and_extreme_frames(dog, torch_mod, H, W, n_blobs):
    # a frame 16x the benchmark's, and the longest side the library accepts
    # on a frame 8 pixels across (in both orientations), against the oracle
    torch = torch_mod
    prm = dog.Params(**CAMERA)
    print("frame %d x %d" % (H, W), flush=True)
    img = synth.camera_frame(seed=H + W, H=H, W=W, n_blobs=n_blobs)
    t = torch.from_numpy(img).cuda()
    natural = H == W
    with dog.Context(0) as c:
        blobs = c.detect_device(t, prm)
        raw, D_o, sig, exempt = _oracle_check(c, t, img, prm, natural=natural, planes=not natural)
    check_pruned(blobs, raw, D_o, prm.threshold, sig, prm.overlap, exempt)
    print("frame %d x %d: raw %d pruned %d exempt %d" % (H, W, len(raw), len(blobs), exempt), flush=True)
    assert len(blobs) > 0
