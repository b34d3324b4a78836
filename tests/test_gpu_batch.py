"""Uneven batches against the FP64 oracle, frame kinds (pageable host, pinned
host, device) giving identical results, and the server with device frames
and a tight admission budget."""
import numpy as np
import pytest

import oracle
import synth
from parity import check_candidates, check_pruned

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


def _frames():
    shapes = [(96, 160), (128, 128), (64, 256), (200, 100), (256, 64), (33, 47)]
    return [synth.camera_frame(seed=900 + i, H=h, W=w, n_blobs=max(1, h * w // 2000))
            for i, (h, w) in enumerate(shapes)]


def test_uneven_batch_matches_oracle(dog, torch_mod):
    prm = dog.Params(**CAMERA)
    frames = _frames()
    with dog.Context(0) as c:
        blobs, raw = c.detect_batch([torch_mod.from_numpy(f).cuda() for f in frames], prm)
        for f, b, n_raw in zip(frames, blobs, raw):
            L_o, D_o, sig = oracle.planes(f, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, 4.0)
            max_abs = float(np.abs(f).max())
            cand = c.debug_candidates(torch_mod.from_numpy(f).cuda(), prm)
            assert len(cand) == n_raw
            exempt = check_candidates(cand, D_o, prm.threshold, sig, max_abs)
            check_pruned(b, cand, D_o, prm.threshold, sig, prm.overlap, exempt)


def test_frame_kinds_give_identical_results(dog, torch_mod):
    prm = dog.Params(**CAMERA)
    frames = _frames()
    pinned = []
    for f in frames:
        t = torch_mod.empty(f.shape, dtype=torch_mod.float32, pin_memory=True)
        t.copy_(torch_mod.from_numpy(f))
        pinned.append(t)
    dev = [torch_mod.from_numpy(f).cuda() for f in frames]
    mixed = [frames[0], pinned[1], dev[2], pinned[3], frames[4], dev[5]]
    with dog.Context(0) as c:
        a, _ = c.detect_batch(frames, prm)
        b, _ = c.detect_batch(pinned, prm)
        d, _ = c.detect_batch(dev, prm)
        m, _ = c.detect_batch(mixed, prm)
    for i in range(len(frames)):
        assert a[i].tobytes() == b[i].tobytes() == d[i].tobytes() == m[i].tobytes(), i


def test_server_device_frames_and_tight_budget(dog, torch_mod):
    prm = dog.Params(**CAMERA)
    frames = [synth.camera_frame(seed=950 + i, H=1024, W=1024, n_blobs=300) for i in range(3)]
    with dog.Context(0) as c:
        ref = [c.detect_device(torch_mod.from_numpy(f).cuda(), prm) for f in frames]
    dev = [torch_mod.from_numpy(f).cuda() for f in frames]
    # device footprint of a 1024x1024 host frame with 9 Gaussian planes
    # (planes, upload buffer, tables, candidates); the budget admits two at a
    # time, and idle slots give their workspaces back when a third would not fit
    fp_host = dog.footprint(prm, [(1024, 1024)])
    budget = int(2.5 * fp_host)
    sv = dog.Server(prm, slots=2, max_batch_frames=4, hbm_budget_bytes=budget)
    try:
        tickets = [sv.submit(f) for f in dev] + [sv.submit(f) for f in frames]
        for i, tk in enumerate(tickets):
            blobs, info = sv.wait(tk)
            assert info["status"] == 0
            assert blobs.tobytes() == ref[i % len(frames)].tobytes(), i
        st = sv.stats()
        assert st["completed"] == len(tickets)
        assert 0 < st["peak_reserved_bytes"] <= budget
        # what the slots' workspaces really hold stays within the budget too
        assert 0 < st["peak_held_bytes"] <= budget
        assert st["held_bytes"] <= budget
    finally:
        sv.close()


def test_grouped_batch_with_host_and_pinned_frames(dog, torch_mod):
    # frames of 2^20 pixels each form their own groups, run on the lanes; the
    # host and pinned frames are staged on the caller's stream first, and the
    # lanes must see them
    torch = torch_mod
    prm = dog.Params(**CAMERA)
    frames = [synth.camera_frame(seed=1400 + i, H=512, W=2048, n_blobs=200) for i in range(6)]
    pinned = []
    for f in frames:
        t = torch.empty(f.shape, dtype=torch.float32, pin_memory=True)
        t.copy_(torch.from_numpy(f))
        pinned.append(t)
    dev = [torch.from_numpy(f).cuda() for f in frames]
    mixed = [frames[0], pinned[1], dev[2], frames[3], pinned[4], dev[5]]
    with dog.Context(0) as c:
        alone = [c.detect_device(t, prm) for t in dev]
        got, _ = c.detect_batch(mixed, prm)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            got_s, _ = c.detect_batch(mixed, prm)
    for i in range(len(frames)):
        assert got[i].tobytes() == alone[i].tobytes() == got_s[i].tobytes(), i
