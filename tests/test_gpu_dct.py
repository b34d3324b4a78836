"""The transform-domain blur of the widest planes (Sec. 4.1: the convolution
taken through a fast Fourier transform, whose cost does not grow with
sigma), against the FP64 oracle: planes within the plane tolerance, the
local-maximum decision exact on the GPU's own cube, near-tie exemptions
bounded, pruned lists as the oracle prunes.  Frames whose sides are powers of
two take the path; others stay direct and must be unaffected."""
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


def _parity(dog, torch, img, prm, min_taps, natural=True):
    t = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    L_o, D_o, sig = oracle.planes(img, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, 4.0)
    max_abs = float(np.abs(img).max())
    with dog.Context(0) as c:
        L_d, _ = c.debug_planes(t, prm)             # every plane direct
        raw_d = c.debug_candidates(t, prm)
        c.set_dct(min_taps)
        L_g, D_g = c.debug_planes(t, prm)
        torch.cuda.synchronize()
        L_g, D_g, L_d = L_g.cpu().numpy(), D_g.cpu().numpy(), L_d.cpu().numpy()
        eL, eD = check_planes(L_g, D_g, L_o, D_o, sig, max_abs)
        raw = c.debug_candidates(t, prm)
        check_candidates_exact(raw, D_g, prm.threshold)
        exempt = check_candidates(raw, D_o, prm.threshold, sig, max_abs)
        if natural:
            # near ties are a property of the frame: at most 1 % of the
            # candidates, or as many as the direct blur has on the same frame
            exempt_d = check_candidates(raw_d, D_o, prm.threshold, sig, max_abs)
            check_exempt_bound(exempt, len(raw), exempt_d)
        blobs = c.detect_device(t, prm)
        check_pruned(blobs, raw, D_o, prm.threshold, sig, prm.overlap, exempt)
        ms, n = c.kernel_times_all()
    radii = dog.plan_info(prm)["radii"]
    taken = [p for p in range(len(radii)) if 2 * radii[p] + 1 >= min_taps]
    for p in range(len(radii)):
        if p not in taken:   # planes left to the direct blur are unchanged
            assert L_g[p].tobytes() == L_d[p].tobytes(), p
    return raw, blobs, exempt, eL, eD, taken


@pytest.mark.parametrize("H,W", [(1024, 1024), (512, 1024), (2048, 1024), (1024, 2048), (256, 256)])
def test_transform_planes_camera_frames(dog, torch_mod, H, W):
    prm = dog.Params(**CAMERA)
    img = synth.camera_frame(seed=H * 7 + W, H=H, W=W, n_blobs=max(20, H * W // 2000))
    raw, blobs, exempt, eL, eD, taken = _parity(dog, torch_mod, img, prm, 200)
    print("dct %dx%d planes %s: raw %d pruned %d exempt %d, err L %.2e D %.2e"
          % (H, W, taken, len(raw), len(blobs), exempt, eL, eD), flush=True)
    assert taken == [7, 8]


def test_every_plane_in_the_transform_domain(dog, torch_mod):
    prm = dog.Params(**CAMERA)
    img = synth.camera_frame(seed=41, H=512, W=512, n_blobs=150)
    raw, blobs, exempt, eL, eD, taken = _parity(dog, torch_mod, img, prm, 1)
    assert taken == list(range(9))
    print("dct all planes: raw %d exempt %d err L %.2e D %.2e" % (len(raw), exempt, eL, eD))


def test_radius_beyond_the_frame(dog, torch_mod):
    # 64 x 128 frame with radii up to 172: the kernel wraps the period 2N
    # several times, which the transfer function includes
    prm = dog.Params(**CAMERA)
    img = synth.camera_frame(seed=42, H=64, W=128, n_blobs=6)
    _parity(dog, torch_mod, img, prm, 100, natural=False)


def test_small_ladder_and_paper_ladder(dog, torch_mod):
    prm = dog.Params(1.0, 8.0, 1.6, 0.1, 0.5)
    img = synth.small_frame(seed=5)          # 256 x 256, radii up to 42
    _parity(dog, torch_mod, img, prm, 50)
    # Eq. 1 ladder, truncate 5: the oracle on the same sigmas
    prm = dog.Params.paper(1.0, 30.0, 10, threshold=0.05)
    img = synth.camera_frame(seed=43, H=512, W=512, n_blobs=150)
    t = torch_mod.from_numpy(img).cuda()
    sig = oracle.sigmas_arithmetic(1.0, 30.0, 10)
    L_o, D_o = oracle.planes_sigmas(img, sig, 5.0)
    with dog.Context(0) as c:
        c.set_dct(150)
        L_g, D_g = c.debug_planes(t, prm)
        check_planes(L_g.cpu().numpy(), D_g.cpu().numpy(), L_o, D_o, sig, float(img.max()))
        raw = c.debug_candidates(t, prm)
        check_candidates_exact(raw, D_g.cpu().numpy(), prm.threshold)


def test_batches_graphs_and_other_shapes(dog, torch_mod):
    # a batch of power-of-two and other frames: each frame equals the frame
    # alone, graph replays equal eager launches, other shapes stay direct
    torch = torch_mod
    prm = dog.Params(**CAMERA)
    shapes = [(1024, 1024), (768, 768), (512, 1024), (384, 768), (256, 256)]
    frames = [synth.mixed_frame(i, H, W) for i, (H, W) in enumerate(shapes)]
    dev = [torch.from_numpy(f).cuda() for f in frames]
    with dog.Context(0) as plain, dog.Context(0) as c:
        c.set_dct(200)
        alone = [c.detect_device(t, prm) for t in dev]
        for g in (1 << 20, 0):
            c.set_batch_grouping(g)
            for _ in range(3):            # the second and third replay a graph
                got, _ = c.detect_batch(dev, prm)
                for i in range(len(frames)):
                    assert got[i].tobytes() == alone[i].tobytes(), (g, shapes[i])
        for i, (H, W) in enumerate(shapes):
            if (H & (H - 1)) or (W & (W - 1)):
                assert alone[i].tobytes() == plain.detect_device(dev[i], prm).tobytes()


@pytest.mark.parametrize("min_taps", [200, 1])
def test_transform_kernel_times(dog, torch_mod, min_taps):
    # min_taps 1: every plane in the transform domain, so the blur passes
    # have no direct tiles and time only the transform jobs they run
    prm = dog.Params(**CAMERA)
    img = synth.camera_frame(seed=1)
    t = torch_mod.from_numpy(img).cuda()
    with dog.Context(0) as c:
        c.set_dct(min_taps)
        c.set_profiling(True)
        for _ in range(5):
            c.detect_device(t, prm)
        ms, n = c.kernel_times_all()
    assert n == 5
    us = {k: round(m / n * 1e3, 2) for k, m in zip(dog.Context.KERNEL_NAMES, ms)}
    print("kernel us with the transform path (min_taps %d):" % min_taps, us, flush=True)
    # the transform jobs run in the blur passes' launches when the variant's
    # kernels take their line length, else in launches of their own
    assert us["pass1"] + us["fft1"] > 0 and us["pass2"] + us["fft2"] > 0 and us["nms"] > 0
    assert all(m >= 0 for m in ms)


@pytest.mark.parametrize("H,W", [(512, 1024), (1024, 512), (1024, 1024)])
def test_merged_and_separate_launches_agree(dog, torch_mod, H, W):
    # the transform jobs inside the blur launches (variant 8) and in launches
    # of their own (variant 13: two waves per workgroup, too few for the jobs'
    # groups; variant 14: cost-balanced direct tiles) give bitwise the same
    # planes, every plane in the transform domain and with the direct planes
    # beside; a workgroup that loads its four column jobs' lines together
    # must not let a wave overwrite the staging buffer before every wave has
    # read it
    prm = dog.Params(**CAMERA)
    img = synth.mixed_frame(2, H, W)
    t = torch_mod.from_numpy(img).cuda()
    for min_taps in (1, 200):
        out = []
        for v in (8, 13, 14):
            with dog.Context(0) as c:
                c.set_variant(v)
                c.set_dct(min_taps)
                L, _ = c.debug_planes(t, prm)
                out.append(L.cpu().numpy())
        for i in (1, 2):
            assert out[0].tobytes() == out[i].tobytes(), (H, W, min_taps, i)
