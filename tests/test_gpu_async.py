"""The split entry point (dog_detect_device_async + dog_detect_device_finish):
two contexts used in turn give, frame by frame, exactly the blobs of the
synchronous call and match the FP64 oracle; a context with a launch to finish
refuses other work; finish without a launch is an error; destroying a
context with a launch in flight waits for it."""
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
    shapes = [(256, 256), (200, 300), (1024, 1024), (64, 130), (256, 256), (512, 384), (33, 47)]
    return [synth.camera_frame(seed=1200 + i, H=h, W=w, n_blobs=max(1, h * w // 2000))
            for i, (h, w) in enumerate(shapes)]


def test_pipelined_contexts_match_synchronous(dog, torch_mod):
    prm = dog.Params(**CAMERA)
    frames = [torch_mod.from_numpy(f).cuda() for f in _frames()]
    with dog.Context(0) as c:
        ref = [c.detect_device(t, prm) for t in frames]
    got = [None] * len(frames)
    with dog.Context(0) as a, dog.Context(0) as b:
        ctxs = (a, b)
        ctxs[0].detect_device_async(frames[0], prm)
        for i in range(1, len(frames) + 1):
            if i < len(frames):
                ctxs[i % 2].detect_device_async(frames[i], prm)
            got[i - 1] = ctxs[(i - 1) % 2].finish()
    for i in range(len(frames)):
        assert got[i].tobytes() == ref[i].tobytes(), i


def test_pipelined_result_matches_oracle(dog, torch_mod):
    prm = dog.Params(**CAMERA)
    f = synth.camera_frame(seed=1300, H=192, W=320, n_blobs=40)
    t = torch_mod.from_numpy(f).cuda()
    with dog.Context(0) as c:
        c.detect_device_async(t, prm)
        blobs = c.finish()
        cand = c.debug_candidates(t, prm)
    L_o, D_o, sig = oracle.planes(f, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, 4.0)
    exempt = check_candidates(cand, D_o, prm.threshold, sig, float(np.abs(f).max()))
    check_pruned(blobs, cand, D_o, prm.threshold, sig, prm.overlap, exempt)


def test_side_stream_and_busy_context(dog, torch_mod):
    prm = dog.Params(**CAMERA)
    f = synth.camera_frame(seed=1301, H=256, W=384, n_blobs=50)
    host = torch_mod.from_numpy(f)
    with dog.Context(0) as c:
        ref = c.detect_device(host.cuda(), prm)
        s = torch_mod.cuda.Stream()
        with torch_mod.cuda.stream(s):
            # the input is produced on the side stream; the launch is queued
            # there, after it
            t = torch_mod.empty_like(host, device="cuda")
            t.copy_(host, non_blocking=False)
            t.mul_(1.0)
            c.detect_device_async(t, prm)
        with pytest.raises(dog.DogError) as e:
            c.detect_device(t, prm)
        assert e.value.code == dog.DOG_EBUSY
        with pytest.raises(dog.DogError) as e:
            c.set_variant(9)
        assert e.value.code == dog.DOG_EBUSY
        got = c.finish()
        assert got.tobytes() == ref.tobytes()
        with pytest.raises(dog.DogError) as e:
            c.finish()
        assert e.value.code == dog.DOG_EINVAL
        # the context works normally again
        assert c.detect_device(t, prm).tobytes() == ref.tobytes()


def test_destroy_with_launch_in_flight(dog, torch_mod):
    prm = dog.Params(**CAMERA)
    t = torch_mod.from_numpy(synth.camera_frame(seed=1302, H=1024, W=1024, n_blobs=200)).cuda()
    c = dog.Context(0)
    c.detect_device_async(t, prm)
    c.close()  # waits for the launch before freeing the workspace
    torch_mod.cuda.synchronize()
    with dog.Context(0) as c2:
        assert len(c2.detect_device(t, prm)) > 0
