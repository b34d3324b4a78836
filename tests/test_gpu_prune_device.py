"""Device-side overlap pruning and radius histogram (Sec. 4.1: pruning or
coalescing overlapping blobs and histogramming their radii, steps the paper
notes could move to the GPU), through dog_prune_device, against the FP64
oracle's pruning and histogram of the same candidate lists.  The lists are
the GPU detector's own raw candidates, given to the device in shuffled order
(the kernel sorts them)."""
import numpy as np
import pytest

import oracle
import synth

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


@pytest.fixture(scope="module")
def ctx(dog, torch_mod):
    c = dog.Context(0)
    yield c
    c.close()


def _ladder(dog, prm):
    info = dog.plan_info(prm)
    return np.asarray(info["sigmas"], np.float64), info["k"]


def _expected(dog, prm, raw):
    """The oracle's pruning (or coalescing) of the sorted raw list and the
    oracle's histogram of the survivors' output sigmas."""
    sig, k = _ladder(dog, prm)
    s64 = sig[raw["scale"]]
    if prm.coalesce:
        keep, s_out = oracle.prune(raw["y"], raw["x"], s64, prm.overlap, coalesce=True)
        out_sigma = s_out[keep].astype(np.float32)
    else:
        keep = oracle.prune(raw["y"], raw["x"], s64, prm.overlap)
        out_sigma = s64[keep].astype(np.float32)
    exp = raw[keep].copy()
    exp["sigma"] = out_sigma
    hist = oracle.radius_histogram(sig[:k], out_sigma.astype(np.float64))
    return exp, hist


def _check(dog, ctx, prm, raw, seed=0):
    """raw: blobs sorted by (y, x, scale) with their ladder sigmas."""
    rng = np.random.default_rng(seed)
    shuffled = raw[rng.permutation(len(raw))]
    got, hist = ctx.prune_device(shuffled, prm)
    exp, exp_hist = _expected(dog, prm, raw)
    assert got.tobytes() == exp.tobytes()
    assert np.array_equal(hist, exp_hist)
    # and the library's host step gives the same list
    assert dog.prune(prm, shuffled).tobytes() == got.tobytes()
    return got


@pytest.mark.parametrize("H,W,n_blobs", [(1024, 1024, 500), (2048, 2048, 2000), (4096, 4096, 2000),
                                         (768, 1536, 600)])
def test_device_prune_of_detector_candidates(dog, ctx, torch_mod, H, W, n_blobs):
    prm = dog.Params(**CAMERA)
    img = synth.camera_frame(seed=H + 3 * W, H=H, W=W, n_blobs=n_blobs)
    t = torch_mod.from_numpy(img).cuda()
    raw = ctx.debug_candidates(t, prm)
    got = _check(dog, ctx, prm, raw)
    print("device prune %dx%d: raw %d kept %d" % (H, W, len(raw), len(got)), flush=True)
    assert 0 < len(got) < len(raw)
    # the detector's own pruned list is the same
    assert ctx.detect_device(t, prm).tobytes() == got.tobytes()


@pytest.mark.parametrize("overlap", [0.0, 0.2, 0.9, 1.0])
def test_device_prune_overlap_limits(dog, ctx, torch_mod, overlap):
    prm = dog.Params(**dict(CAMERA, overlap=overlap))
    img = synth.camera_frame(seed=77, H=512, W=512, n_blobs=300)
    raw = ctx.debug_candidates(torch_mod.from_numpy(img).cuda(), prm)
    got = _check(dog, ctx, prm, raw, seed=3)
    if overlap == 1.0:
        assert got.tobytes() == raw.tobytes()


def test_device_coalescing_paper_configuration(dog, ctx, torch_mod):
    # Eq. 1 ladder with n_bin = 10, truncate 5, coalescing by averaging the
    # radius: sigmas change as blobs merge, and later pairs see the new ones
    prm = dog.Params.paper(1.0, 30.0, 10, threshold=0.05)
    for seed, (H, W) in ((1, (1024, 1024)), (2, (2048, 2048))):
        img = synth.camera_frame(seed=seed, H=H, W=W, n_blobs=500 * (H * W) // (1 << 20))
        t = torch_mod.from_numpy(img).cuda()
        raw = ctx.debug_candidates(t, prm)
        got = _check(dog, ctx, prm, raw, seed=seed)
        assert np.any(got["sigma"] != np.asarray(_ladder(dog, prm)[0], np.float32)[got["scale"]])
        assert ctx.detect_device(t, prm).tobytes() == got.tobytes()
        print("device coalescing %dx%d: raw %d kept %d" % (H, W, len(raw), len(got)), flush=True)


def test_device_prune_hand_cases(dog, ctx):
    prm = dog.Params(**CAMERA)
    B = dog.BLOB_DTYPE
    # empty list, one blob
    got, hist = ctx.prune_device(np.empty(0, B), prm)
    assert len(got) == 0 and not hist.any()
    one = np.array([(5, 7, 3, 0.0, 0.25)], B)
    got, hist = ctx.prune_device(one, prm)
    assert len(got) == 1 and hist[3] == 1 and hist.sum() == 1
    # concentric blobs of scales 2 and 5: the smaller goes; equal scales at
    # the same centre cannot occur, equal scales one pixel apart: the later goes
    pair = np.array([(100, 100, 2, 0.0, 2.0), (100, 100, 5, 0.0, 1.0), (100, 101, 2, 0.0, 3.0)], B)
    pair["sigma"] = np.asarray(_ladder(dog, prm)[0], np.float32)[pair["scale"]]
    got = _check(dog, ctx, prm, pair)
    assert [tuple(r) for r in got[["y", "x", "scale"]]] == [(100, 100, 5)]
    # blobs at the corners of the largest frame
    far = np.array([(0, 0, 0, 0.0, 1.0), (0, 32767, 4, 0.0, 1.0), (32767, 32767, 7, 0.0, 1.0)], B)
    far["sigma"] = np.asarray(_ladder(dog, prm)[0], np.float32)[far["scale"]]
    _check(dog, ctx, prm, far)


def test_device_prune_errors_and_large_lists(dog, ctx):
    prm = dog.Params(**CAMERA)
    B = dog.BLOB_DTYPE
    bad = np.array([(1, 1, 8, 0.0, 1.0)], B)           # scale k = 8 is outside 0..7
    with pytest.raises(dog.DogError) as e:
        ctx.prune_device(bad, prm)
    assert e.value.code == dog.DOG_EINVAL
    bad = np.array([(-1, 1, 0, 0.0, 1.0)], B)
    with pytest.raises(dog.DogError):
        ctx.prune_device(bad, prm)
    # a list larger than one workgroup holds takes the host steps, same result
    rng = np.random.default_rng(5)
    n = 9000
    many = np.zeros(n, B)
    many["y"] = rng.integers(0, 3000, n)
    many["x"] = rng.integers(0, 3000, n)
    many["scale"] = rng.integers(0, 8, n)
    many["response"] = rng.random(n, dtype=np.float32)
    _, idx = np.unique(many["y"].astype(np.int64) * 100000 + many["x"] * 10 + many["scale"],
                       return_index=True)
    many = many[np.sort(idx)]
    order = np.lexsort((many["scale"], many["x"], many["y"]))
    raw = many[order]
    raw["sigma"] = np.asarray(_ladder(dog, prm)[0], np.float32)[raw["scale"]]
    _check(dog, ctx, prm, raw)


@pytest.mark.parametrize("coalesce", [False, True])
def test_device_prune_blob_with_more_than_64_pairs(dog, ctx, coalesce):
    # Blob A (sigma 16.8) is visited first; 70 small blobs (sigma 1, 3 px
    # apart, so they do not touch each other) inside its disk come next in
    # visiting order, then blob B (sigma 26.8) overlapping A, then more small
    # blobs.  A removes the 70 small ones (its pairs span two groups of 64)
    # and is removed at its pair with B; B then removes the later small blobs
    # inside its disk, and the last row, outside both disks, stays.  The
    # result is the oracle's in both modes.
    prm = dog.Params(**dict(CAMERA, coalesce=coalesce))
    sig = _ladder(dog, prm)[0]
    rows = [(100, 500, 6)]
    rows += [(y, x, 0) for y in (101, 104, 107, 110, 113) for x in range(480, 522, 3)]
    rows += [(115, 500, 7)]
    rows += [(y, x, 0) for y in (116, 119, 160) for x in range(480, 522, 3)]
    B = dog.BLOB_DTYPE
    raw = np.zeros(len(rows), B)
    raw["y"] = [r[0] for r in rows]
    raw["x"] = [r[1] for r in rows]
    raw["scale"] = [r[2] for r in rows]
    raw["response"] = np.linspace(0.1, 1.0, len(rows), dtype=np.float32)
    raw = raw[np.lexsort((raw["scale"], raw["x"], raw["y"]))]
    raw["sigma"] = np.asarray(sig, np.float32)[raw["scale"]]
    got = _check(dog, ctx, prm, raw, seed=11)
    kept = {(int(r["y"]), int(r["x"]), int(r["scale"])) for r in got}
    assert (100, 500, 6) not in kept and (115, 500, 7) in kept
    assert all((160, x, 0) in kept for x in range(480, 522, 3))
    if not coalesce:   # (coalescing shrinks A as it goes, so it stops removing)
        assert not any((y, x, 0) in kept
                       for y in (101, 104, 107, 110, 113) for x in range(480, 522, 3))
