"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Planes within 1e-5 relative (scaled, see parity.py); blob lists identical
except voxels within the fp32/FP64 decision margin of a tie or of the
threshold; pruned lists equal.  Also edge shapes (1x1, thin, ragged tiles,
radius larger than the image, row stride > width), candidate overflow,
determinism, kernel-variant invariance and batch == single frame.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import (check_candidates, check_candidates_exact, check_exempt_bound, check_planes,
                    check_pruned)

pytestmark = pytest.mark.gpu

SMALL = dict(sigma_min=1.0, sigma_max=8.0, sigma_ratio=1.6, threshold=0.1, overlap=0.5)
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


@pytest.fixture(scope="module")
def ctx(dog, torch_mod):
    c = dog.Context(0)
    yield c
    c.close()


def _dev(torch, img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _full_parity(dog, ctx, torch, img, prm_kw, check_plane=True, natural=False):
    prm = dog.Params(**prm_kw)
    t = _dev(torch, img)
    L_o, D_o, sig = oracle.planes(img, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, 4.0)
    max_abs = float(np.abs(img).max())
    L_g, D_g = ctx.debug_planes(t, prm)
    torch.cuda.synchronize()
    D_g = D_g.cpu().numpy()
    if check_plane:
        check_planes(L_g.cpu().numpy(), D_g, L_o, D_o, sig, max_abs)
    raw = ctx.debug_candidates(t, prm)
    check_candidates_exact(raw, D_g, prm.threshold)
    exempt = check_candidates(raw, D_o, prm.threshold, sig, max_abs)
    if natural:
        check_exempt_bound(exempt, len(raw))
    pruned = ctx.detect_device(t, prm)
    check_pruned(pruned, raw, D_o, prm.threshold, sig, prm.overlap, exempt)
    return raw, pruned, exempt


def test_small_frame_parity(dog, ctx, torch_mod):
    img = synth.small_frame(seed=0)
    raw, pruned, exempt = _full_parity(dog, ctx, torch_mod, img, SMALL, natural=True)
    print("small: raw %d pruned %d exempt %d" % (len(raw), len(pruned), exempt))
    assert len(pruned) >= 10


def test_camera_frame_parity_full_size(dog, ctx, torch_mod):
    img = synth.camera_frame(seed=1)
    raw, pruned, exempt = _full_parity(dog, ctx, torch_mod, img, CAMERA, natural=True)
    print("camera 1024^2: raw %d pruned %d exempt %d" % (len(raw), len(pruned), exempt))
    assert len(pruned) >= 100


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (3, 1), (7, 5), (2, 130), (97, 131), (64, 64),
                                   (65, 63), (130, 257), (33, 300)])
def test_edge_shapes_parity(dog, ctx, torch_mod, shape):
    H, W = shape
    img = synth.small_frame(seed=H * 1000 + W, H=H, W=W, n_blobs=max(1, H * W // 800))
    _full_parity(dog, ctx, torch_mod, img, SMALL)


def test_radius_larger_than_image(dog, ctx, torch_mod):
    # sigma up to ~43 (radius 172) on a 20 x 300 crop: rows reflect many times
    img = synth.camera_frame(seed=5, H=20, W=300, n_blobs=3)
    _full_parity(dog, ctx, torch_mod, img, CAMERA)


def test_row_stride_greater_than_width(dog, ctx, torch_mod):
    torch = torch_mod
    img = synth.small_frame(seed=12, H=90, W=70, n_blobs=6)
    wide = np.zeros((90, 101), np.float32)
    wide[:, :70] = img
    wide[:, 70:] = 7.0          # must never be read
    t = _dev(torch, wide)[:, :70]
    assert t.stride(0) == 101
    prm = dog.Params(**SMALL)
    got = ctx.detect_device(t, prm)
    ref = ctx.detect_device(_dev(torch, img), prm)
    assert got.tobytes() == ref.tobytes()
    L_o, D_o, sig = oracle.planes(img, 1, 8, 1.6)
    L_g, D_g = ctx.debug_planes(t, prm)
    check_planes(L_g.cpu().numpy(), D_g.cpu().numpy(), L_o, D_o, sig, float(img.max()))


def test_candidate_overflow_all_ties(dog, ctx, torch_mod):
    # a zero image has D == 0 everywhere: with a negative threshold every
    # voxel ties with its neighbourhood, far beyond the initial capacity
    torch = torch_mod
    img = np.zeros((256, 256), np.float32)
    prm = dog.Params(1, 8, 1.6, -1.0, 1.0)
    raw = ctx.debug_candidates(_dev(torch, img), prm)
    assert len(raw) == 256 * 256 * 5
    exp = np.array([(y, x, i) for y in range(256) for x in range(256) for i in range(5)])
    got = np.stack([raw["y"], raw["x"], raw["scale"]], 1)
    assert np.array_equal(got, exp)
    assert np.all(raw["response"] == 0)
    # and a normal frame right after still matches
    test_small_frame_parity(dog, ctx, torch)


def test_overflow_of_one_tile_below_capacity(dog, torch_mod):
    # a 64x64 zero frame with a negative threshold: 20,480 tied candidates,
    # below the initial capacity of a new context but far above what one
    # workgroup's LDS buffer holds, so most records take the direct path to
    # the global list; every one must reach the host list
    torch = torch_mod
    img = np.zeros((64, 64), np.float32)
    prm = dog.Params(1, 8, 1.6, -1.0, 1.0)
    with dog.Context(0) as c:
        for _ in range(2):   # the second call reads back a larger first slice
            raw = c.debug_candidates(_dev(torch, img), prm)
            assert len(raw) == 64 * 64 * 5
            exp, _ = oracle.nms(np.zeros((5, 64, 64)), -1.0)
            got = np.stack([raw["y"], raw["x"], raw["scale"]], 1)
            assert np.array_equal(got, exp)
            assert np.all(raw["response"] == 0)
            blobs = c.detect_device(_dev(torch, img), prm)   # overlap 1: no pruning
            assert blobs.tobytes() == raw.tobytes()


def test_overflowing_and_normal_tiles_in_one_frame(dog, torch_mod):
    # a camera frame with a 200 x 200 constant block: more than the widest
    # radius (42) inside the block every plane is constant, so each DoG plane
    # is constant there and ties across the whole interior; with a negative
    # threshold every voxel of each plane that is a maximum across scales is
    # a local maximum, so the tiles over the interior hold more records than
    # their LDS buffers and are walked again straight to the global list,
    # while the other tiles flush as usual.  The records are exactly the
    # local maxima of the GPU's own DoG cube.
    torch = torch_mod
    img = synth.camera_frame(seed=21, H=384, W=384, n_blobs=70)
    img[100:300, 20:220] = 0.25
    prm = dog.Params(1, 8, 1.6, -1.0, 1.0)
    with dog.Context(0) as c:
        t = _dev(torch, img)
        raw = c.debug_candidates(t, prm)
        _, D_g = c.debug_planes(t, prm)
        check_candidates_exact(raw, D_g.cpu().numpy(), prm.threshold)
        inside = (raw["y"] >= 190) & (raw["y"] < 210) & (raw["x"] >= 110) & (raw["x"] < 130)
        n_in = int(inside.sum())   # whole planes of the 20 x 20 centre
        assert n_in >= 400 and n_in % 400 == 0
        assert c.detect_device(t, prm).tobytes() == raw.tobytes()   # overlap 1: no pruning
        assert c.debug_candidates(t, prm).tobytes() == raw.tobytes()


def test_repeat_runs_bitwise_identical(dog, ctx, torch_mod):
    img = synth.camera_frame(seed=3, H=512, W=384, n_blobs=120)
    t = _dev(torch_mod, img)
    prm = dog.Params(**CAMERA)
    a = ctx.debug_candidates(t, prm)
    b = ctx.debug_candidates(t, prm)
    assert a.tobytes() == b.tobytes()
    La, Da = ctx.debug_planes(t, prm)
    Lb, Db = ctx.debug_planes(t, prm)
    assert torch_mod.equal(La, Lb) and torch_mod.equal(Da, Db)


@pytest.mark.parametrize("shape", [(200, 300), (192, 320)])
def test_all_variants_bitwise_identical(dog, ctx, torch_mod, shape):
    # (200, 300): 4-byte loads in pass 1 (width not a multiple of 64);
    # (192, 320): 16-byte loads in pass 1 for the LDS-staged variants
    img = synth.camera_frame(seed=4, H=shape[0], W=shape[1], n_blobs=40)
    t = _dev(torch_mod, img)
    prm = dog.Params(**CAMERA)
    ctx.set_variant(0)
    L0, D0 = ctx.debug_planes(t, prm)
    c0 = ctx.debug_candidates(t, prm)
    try:
        for v in range(1, dog.num_variants()):
            ctx.set_variant(v)
            L, D = ctx.debug_planes(t, prm)
            c = ctx.debug_candidates(t, prm)
            assert torch_mod.equal(L, L0) and torch_mod.equal(D, D0), dog.variant_info(v)
            assert c.tobytes() == c0.tobytes(), dog.variant_info(v)
    finally:
        ctx.set_variant(-1)


def test_batch_equals_single_frames(dog, ctx, torch_mod):
    shapes = [(256, 256), (128, 512), (300, 200), (64, 64), (512, 256)]
    frames = [synth.camera_frame(seed=50 + i, H=h, W=w, n_blobs=h * w // 2000 + 1)
              for i, (h, w) in enumerate(shapes)]
    prm = dog.Params(**CAMERA)
    singles = [ctx.detect_device(_dev(torch_mod, f), prm) for f in frames]
    host_batch, raw_counts = ctx.detect_batch(frames, prm)
    dev_batch, _ = ctx.detect_batch([_dev(torch_mod, f) for f in frames], prm)
    for s, hb, db in zip(singles, host_batch, dev_batch):
        assert s.tobytes() == hb.tobytes() == db.tobytes()
    assert all(r >= len(s) for r, s in zip(raw_counts, singles))


def test_host_entry_point_matches_device(dog, ctx, torch_mod):
    img = synth.small_frame(seed=21)
    got = dog.detect(img, 1.0, 8.0, 1.6, 0.1, 0.5)
    ref = ctx.detect_device(_dev(torch_mod, img), dog.Params(**SMALL))
    assert got.tobytes() == ref.tobytes()


def test_invalid_device_arguments(dog, ctx, torch_mod):
    t = _dev(torch_mod, np.zeros((8, 8), np.float32))
    with pytest.raises(dog.DogError) as e:
        ctx.detect_device(t, dog.Params(sigma_min=0.0))
    assert e.value.code == dog.DOG_EINVAL
    with pytest.raises(dog.DogError):
        dog.detect(np.zeros((0, 5), np.float32), 1, 8)


def test_graph_replays_match_eager_launches(dog, torch_mod):
    # the captured sequence is replayed with new frame pointers; every replay,
    # with eager work and synchronisations in between, must equal the eager path
    torch = torch_mod
    frames = [synth.camera_frame(seed=70 + i, H=300, W=260, n_blobs=40) for i in range(3)]
    prm = dog.Params(**CAMERA)
    with dog.Context(0) as eager:
        eager.set_graph_mode(False)
        ref = [eager.detect_device(_dev(torch, f), prm) for f in frames]
        ref_batch, _ = eager.detect_batch(frames, prm)
    dev = [_dev(torch, f) for f in frames]
    with dog.Context(0) as g:
        for rep in range(4):
            for i, t in enumerate(dev):
                got = g.detect_device(t, prm)
                assert got.tobytes() == ref[i].tobytes(), (rep, i)
                float((t * 2.0).sum().item())      # eager torch work on the same stream
                torch.cuda.synchronize()
            got_b, _ = g.detect_batch(dev, prm)
            for i in range(3):
                assert got_b[i].tobytes() == ref_batch[i].tobytes() == ref[i].tobytes()


def test_kernel_timing_in_both_launch_modes(dog, torch_mod):
    img = synth.camera_frame(seed=9, H=512, W=512, n_blobs=100)
    t = _dev(torch_mod, img)
    prm = dog.Params(**CAMERA)
    with dog.Context(0) as c:
        for graphs in (True, False):
            c.set_graph_mode(graphs)
            c.set_profiling(True)
            for _ in range(3):
                c.detect_device(t, prm)
            ms, n = c.kernel_times()
            c.set_profiling(False)
            assert n == 3
            assert all(m > 0 for m in ms), ms


def test_input_written_on_default_stream_is_seen(dog, ctx, torch_mod):
    # the frame is written by torch on the default stream behind a long
    # matrix product; the detector must be ordered after that write
    torch = torch_mod
    img = synth.camera_frame(seed=77, H=512, W=512, n_blobs=80)
    prm = dog.Params(**CAMERA)
    ref = ctx.detect_device(_dev(torch, img), prm)
    src = _dev(torch, img)
    dst = torch.zeros_like(src)
    torch.cuda.synchronize()
    a = torch.randn(4096, 4096, device="cuda")
    for _ in range(4):
        a = a @ a
        a = a / a.abs().max()
    dst.copy_(src)
    got = ctx.detect_device(dst, prm)
    assert got.tobytes() == ref.tobytes()
    float(a.sum().item())
