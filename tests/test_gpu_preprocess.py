"""Preprocessing on the GPU (Sec. 4.1, optional first step) against the FP64
oracle: the smoothed image within the plane tolerance, the stretch limits
exactly the order statistics of the GPU's own fp32 smoothed image (and close
to the oracle's), the stretched image equal to its definition; no smoothing,
no saturation and a constant image as special cases; strided input and
unaligned output buffers; successive calls on two streams; and the detector
run on the preprocessed frame."""
import numpy as np
import pytest

import oracle
import synth
from parity import check_candidates, check_planes

pytestmark = pytest.mark.gpu

TOL = 1e-5


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
    # raw camera counts, before any normalisation
    return (synth.camera_frame(seed=seed, H=H, W=W, n_blobs=n_blobs) * 65535.0).astype(np.float32)


def _check(dog, torch, img, sigma, saturated):
    t = torch.from_numpy(img).cuda()
    H, W = img.shape
    sm = torch.empty((H, W), dtype=torch.float32, device="cuda")
    with dog.Context(0) as c:
        out, (lo, hi) = c.preprocess(t, sigma, saturated, smoothed=sm, limits=True)
        torch.cuda.synchronize()
    S = sm.cpu().numpy()
    O = out.cpu().numpy()
    o_out, o_sm, o_lo, o_hi = oracle.preprocess(img, sigma, saturated)
    scale = float(np.abs(img).max())
    if sigma == 0.0:
        assert np.array_equal(S, img)
    else:
        assert np.all(np.abs(S - o_sm) <= TOL * (np.abs(o_sm) + scale))
    # the limits are exact order statistics of the GPU's own smoothed image
    N = H * W
    m = min(int(np.floor(saturated * N / 2)), (N - 1) // 2)
    srt = np.sort(S.ravel())
    assert lo == srt[m] and hi == srt[N - 1 - m]
    assert abs(lo - o_lo) <= TOL * scale and abs(hi - o_hi) <= TOL * scale
    # the stretch, in fp32 from those limits, and against the oracle's
    if hi > lo:
        exp = np.clip((S - np.float32(lo)) / (np.float32(hi) - np.float32(lo)), 0.0, 1.0)
    else:
        exp = np.zeros_like(S)
    assert np.max(np.abs(O - exp)) <= 2e-7
    assert np.max(np.abs(O - o_out)) <= TOL * max(1.0, scale / max(o_hi - o_lo, 1e-30))
    return O, lo, hi


@pytest.mark.parametrize("shape,sigma,sat", [((1024, 1024), 1.0, 0.0035), ((200, 333), 1.5, 0.0035),
                                             ((64, 97), 0.0, 0.0035), ((256, 256), 2.0, 0.0),
                                             ((1, 130), 1.0, 0.0035), ((77, 1), 3.9, 0.1)])
def test_preprocess_matches_oracle(dog, torch_mod, shape, sigma, sat):
    H, W = shape
    img = _counts(40 + H + W, H, W, max(1, H * W // 2000))
    O, lo, hi = _check(dog, torch_mod, img, sigma, sat)
    assert O.min() >= 0.0 and O.max() <= 1.0


@pytest.mark.parametrize("shape", [(4096, 4096), (3001, 4999)])
def test_preprocess_large_frames(dog, torch_mod, shape):
    # frames large enough that every select-pass thread counts several
    # batches of keys and the stretch sweeps the frame several times (the
    # launch grids are capped at 4096 workgroups); a ragged pixel count
    H, W = shape
    print("preprocess %d x %d" % (H, W), flush=True)
    img = _counts(50 + H, H, W, 400)
    O, lo, hi = _check(dog, torch_mod, img, 1.0, 0.0035)
    assert O.min() >= 0.0 and O.max() <= 1.0 and lo < hi


def test_preprocess_strided_view(dog, torch_mod):
    # a crop of a wider frame: rows of the view are row_stride floats apart
    torch = torch_mod
    img = _counts(80, 120, 200, 20)
    full = torch.from_numpy(img).cuda()
    view = full[:, 13:170]
    with dog.Context(0) as c:
        a, lim_a = c.preprocess(view, 1.0, 0.0035, limits=True)
        b, lim_b = c.preprocess(view.contiguous(), 1.0, 0.0035, limits=True)
        torch.cuda.synchronize()
    assert view.stride(0) == 200 and torch.equal(a, b) and lim_a == lim_b
    o_out, _, o_lo, o_hi = oracle.preprocess(np.ascontiguousarray(img[:, 13:170]), 1.0, 0.0035)
    assert np.max(np.abs(a.cpu().numpy() - o_out)) <= 1e-4


def test_preprocess_unaligned_buffers(dog, torch_mod):
    # output and smoothed buffers 4 bytes off 16-byte alignment (the stretch
    # then moves single values, not 16-byte chunks) and a pixel count that is
    # not a multiple of 4: the same result as aligned buffers
    torch = torch_mod
    img = _counts(90, 123, 77, 15)
    t = torch.from_numpy(img).cuda()
    H, W = img.shape
    buf = torch.empty(H * W + 2, dtype=torch.float32, device="cuda")
    sbuf = torch.empty(H * W + 2, dtype=torch.float32, device="cuda")
    out_u = buf[1:1 + H * W].view(H, W)
    sm_u = sbuf[1:1 + H * W].view(H, W)
    assert out_u.data_ptr() % 16 != 0 and sm_u.data_ptr() % 16 != 0 and (H * W) % 4 != 0
    with dog.Context(0) as c:
        a, lim_a = c.preprocess(t, 1.0, 0.0035, limits=True)
        b, lim_b = c.preprocess(t, 1.0, 0.0035, out=out_u, smoothed=sm_u, limits=True)
        torch.cuda.synchronize()
    assert lim_a == lim_b and torch.equal(a, b)
    o_out, _, _, _ = oracle.preprocess(img, 1.0, 0.0035)
    assert np.max(np.abs(b.cpu().numpy() - o_out)) <= 1e-4


def test_preprocess_constant_image(dog, torch_mod):
    img = np.full((50, 70), 1234.0, np.float32)
    O, lo, hi = _check(dog, torch_mod, img, 1.0, 0.0035)
    assert lo == hi and np.all(O == 0.0)


def test_preprocess_argument_errors(dog, torch_mod):
    t = torch_mod.zeros((16, 16), dtype=torch_mod.float32, device="cuda")
    with dog.Context(0) as c:
        for sigma, sat in ((4.2, 0.0035), (-1.0, 0.0035), (1.0, 1.0), (1.0, -0.1)):
            with pytest.raises(dog.DogError) as e:
                c.preprocess(t, sigma, sat)
            assert e.value.code == dog.DOG_EINVAL


def test_preprocess_two_streams_in_turn(dog, torch_mod):
    # successive calls with different sigmas on two streams share the
    # context's scratch; each must equal the same call made alone
    torch = torch_mod
    imgs = [_counts(60 + i, 300, 400, 60) for i in range(4)]
    ts = [torch.from_numpy(a).cuda() for a in imgs]
    sig = [1.0, 2.0, 0.0, 1.5]
    with dog.Context(0) as c:
        ref = [c.preprocess(t, s, 0.0035).clone() for t, s in zip(ts, sig)]
        torch.cuda.synchronize()
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        outs = []
        for i, (t, s) in enumerate(zip(ts, sig)):
            outs.append(c.preprocess(t, s, 0.0035, stream=streams[i % 2]))
        torch.cuda.synchronize()
    for r, o in zip(ref, outs):
        assert torch.equal(r, o)


def test_detector_on_preprocessed_frame(dog, torch_mod):
    # the paper's pipeline: preprocess, then detect (same stream); the
    # detector part against the oracle on the preprocessed frame
    torch = torch_mod
    img = _counts(70, 256, 320, 40)
    prm = dog.Params(1.0, 30.0, 1.6, 0.1, 0.5)
    with dog.Context(0) as c:
        pre = c.preprocess(torch.from_numpy(img).cuda(), 1.0, 0.0035)
        blobs = c.detect_device(pre, prm)
        raw = c.debug_candidates(pre, prm)
        L_g, D_g = c.debug_planes(pre, prm)
        torch.cuda.synchronize()
    P = pre.cpu().numpy()
    L_o, D_o, sig = oracle.planes(P, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, 4.0)
    check_planes(L_g.cpu().numpy(), D_g.cpu().numpy(), L_o, D_o, sig, 1.0)
    check_candidates(raw, D_o, prm.threshold, sig, 1.0)
    assert len(blobs) > 0
