"""Serving on the GPU: every request's blob list is the same when served alone,
in a mixed burst of uneven sizes that overlaps on the device, and through
dog_detect_device directly."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CAMERA = dict(sigma_min=1.0, sigma_max=30.0, sigma_ratio=1.6, threshold=0.05, overlap=0.5)


def test_served_alone_equals_mixed_equals_direct():
    import torch

    import paper_2010_08486_amd as dog
    prm = dog.Params(**CAMERA)
    shapes = [(256, 256), (128, 256), (512, 512), (256, 512), (384, 768), (64, 64), (512, 256),
              (1024, 1024)]
    frames = [synth.camera_frame(seed=300 + i, H=h, W=w, n_blobs=max(1, h * w // 2000))
              for i, (h, w) in enumerate(shapes)]
    with dog.Context(0) as ctx:
        direct = [ctx.detect_device(torch.from_numpy(f).cuda(), prm) for f in frames]
    with dog.Server(prm, slots=3, max_batch_frames=3) as sv:
        alone = []
        for f in frames:
            alone.append(sv.wait(sv.submit(f))[0])
        tickets = [sv.submit(f) for f in frames for _ in range(3)]   # each frame 3x, interleaved
        mixed = [sv.wait(t)[0] for t in tickets]
        st = sv.stats()
    assert st["completed"] == len(frames) * 4 and st["failed"] == 0
    for i in range(len(frames)):
        assert alone[i].tobytes() == direct[i].tobytes(), shapes[i]
        for r in range(3):
            assert mixed[i * 3 + r].tobytes() == direct[i].tobytes(), (shapes[i], r)
    assert st["batches"] < len(tickets) + len(frames)      # the burst was batched
