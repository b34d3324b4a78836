"""dog_preprocess_noalloc, the preprocessing entry point that allocates
nothing (its scratch is a static device array per GPU), against
dog_preprocess on the same inputs: smoothed image, stretched image and
limits bitwise equal, on two calls in a row, the second on a smaller frame
(the array keeps the first call's contents), and on a stream of torch's
besides the current one.  The oracle check of the kernels themselves is
tests/test_gpu_preprocess.py; both entry points run the same kernels."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def dog():
    import paper_2010_08486_amd as d
    return d


def _counts(seed, H, W, n_blobs):
    return (synth.camera_frame(seed=seed, H=H, W=W, n_blobs=n_blobs) * 65535.0).astype(np.float32)


def _pair(dog, torch, img, sigma, saturated, stream=None):
    t = torch.from_numpy(img).cuda()
    H, W = img.shape
    sm_ref = torch.empty((H, W), dtype=torch.float32, device="cuda")
    with dog.Context(0) as c:
        out_ref, (lo, hi) = c.preprocess(t, sigma, saturated, smoothed=sm_ref, limits=True)
    torch.cuda.synchronize()
    out = torch.full((H, W), -1.0, dtype=torch.float32, device="cuda")
    sm = torch.full((H, W), -1.0, dtype=torch.float32, device="cuda")
    lim = torch.full((2,), -1.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    dog.preprocess_noalloc(t, out, smoothed=sm, limits=lim, sigma=sigma, saturated=saturated,
                           stream=stream)
    torch.cuda.synchronize()
    assert sm.cpu().numpy().tobytes() == sm_ref.cpu().numpy().tobytes()
    assert out.cpu().numpy().tobytes() == out_ref.cpu().numpy().tobytes()
    got = lim.cpu().numpy()
    assert got[0] == np.float32(lo) and got[1] == np.float32(hi), (got, lo, hi)
    return got


def test_two_calls_second_smaller(dog, torch_mod):
    big = _counts(70, 1024, 1024, 500)
    small = _counts(71, 200, 333, 40)
    lim1 = _pair(dog, torch_mod, big, 1.0, 0.0035)
    lim2 = _pair(dog, torch_mod, small, 1.0, 0.0035)
    assert lim1[0] != lim2[0] or lim1[1] != lim2[1]
    # no smoothing, then a wider smoothing kernel, on the smaller frame
    _pair(dog, torch_mod, small, 0.0, 0.01)
    _pair(dog, torch_mod, small, 3.0, 0.0035)


def test_in_place_and_on_a_side_stream(dog, torch_mod):
    torch = torch_mod
    img = _counts(72, 384, 640, 100)
    s = torch.cuda.Stream()
    _pair(dog, torch, img, 1.0, 0.0035, stream=s)
    # d_smoothed NULL: the stretch runs in place in d_out
    t = torch.from_numpy(img).cuda()
    with dog.Context(0) as c:
        ref = c.preprocess(t, 1.0, 0.0035)
    out = torch.empty_like(t)
    dog.preprocess_noalloc(t, out, sigma=1.0, saturated=0.0035)
    torch.cuda.synchronize()
    assert out.cpu().numpy().tobytes() == ref.cpu().numpy().tobytes()


def test_rejects_radius_beyond_the_scratch(dog, torch_mod):
    torch = torch_mod
    t = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
    out = torch.empty_like(t)
    with pytest.raises(dog.DogError, match="radius"):
        dog.preprocess_noalloc(t, out, sigma=5.0)
