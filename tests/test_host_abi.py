"""CPU tests of the library boundary: it loads, exports every symbol the
header declares, validates arguments, and its host steps (ladder plan,
pruning) agree with the oracle.  No kernel is launched."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2010_08486_amd as dog


def test_library_exports_every_header_symbol():
    L = dog.lib()
    names = dog.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
        assert ctypes.cast(getattr(L, n), ctypes.c_void_p).value


@pytest.mark.parametrize("p", [(1, 8, 1.6), (1, 30, 1.6), (2.0, 2.0, 1.6), (0.7, 13.0, 1.25),
                               (1.0, 1.6 ** 4 * 0.999, 1.6)])
def test_plan_matches_oracle_ladder(p):
    info = dog.plan_info(dog.Params(p[0], p[1], p[2], 0.1, 0.5, 4.0))
    s = oracle.sigmas_geometric(*p)
    assert info["k"] == oracle.num_dog_planes(*p) == len(s) - 1
    assert np.array_equal(info["sigmas"], s)
    assert info["radii"].tolist() == [oracle.radius(x, 4.0) for x in s]


@pytest.mark.parametrize("bad", [dict(sigma_min=0.0), dict(sigma_min=-1.0), dict(sigma_max=0.5),
                                 dict(sigma_ratio=1.0), dict(sigma_ratio=0.9),
                                 dict(threshold=float("nan")), dict(overlap=1.5),
                                 dict(overlap=-0.1), dict(truncate=-1.0),
                                 dict(sigma_min=1.0, sigma_max=1e9, sigma_ratio=1.01)])
def test_invalid_params_rejected(bad):
    kw = dict(sigma_min=1.0, sigma_max=8.0, sigma_ratio=1.6, threshold=0.1, overlap=0.5, truncate=4.0)
    kw.update(bad)
    with pytest.raises(dog.DogError) as e:
        dog.plan_info(dog.Params(**kw))
    assert e.value.code == dog.DOG_EINVAL


@pytest.mark.parametrize("seed,overlap", [(0, 0.5), (1, 0.5), (2, 0.0), (3, 0.9), (4, 1.0)])
def test_prune_matches_oracle(seed, overlap):
    rng = np.random.default_rng(seed)
    n = 400
    prm = dog.Params(1, 30, 1.6, 0.05, overlap)
    sig = dog.plan_info(prm)["sigmas"]
    b = np.zeros(n, dog.BLOB_DTYPE)
    b["y"] = rng.integers(0, 120, n)
    b["x"] = rng.integers(0, 120, n)
    b["scale"] = rng.integers(0, 8, n)
    # unique voxels, as the detector produces
    _, u = np.unique(b[["y", "x", "scale"]], return_index=True)
    b = b[np.sort(u)]
    rng.shuffle(b)
    got = dog.prune(prm, b)
    order = np.lexsort((b["scale"], b["x"], b["y"]))
    s = b[order]
    keep = oracle.prune(s["y"], s["x"], sig[s["scale"]], overlap)
    exp = s[keep]
    assert got[["y", "x", "scale"]].tolist() == exp[["y", "x", "scale"]].tolist()
    assert np.all(got["sigma"] == sig[got["scale"]].astype(np.float32))


def test_footprint_grows_with_frames():
    prm = dog.Params(1, 30, 1.6, 0.05, 0.5)
    one = dog.footprint(prm, [(1024, 1024)])
    two = dog.footprint(prm, [(1024, 1024), (512, 2048)])
    assert one >= 2 * 9 * 1024 * 1024 * 4
    assert two > one


def test_no_gpu_context_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except ImportError:
        pass
    with pytest.raises(dog.DogError) as e:
        dog.Context()
    assert e.value.code in (dog.DOG_EDEVICE, dog.DOG_EINVAL)
    assert dog.lib().dog_last_error()


@pytest.mark.parametrize("p", [(1.0, 30.0, 10), (1.0, 8.0, 7), (2.0, 2.0, 3), (0.5, 12.0, 40)])
def test_arithmetic_plan_matches_oracle_ladder(p):
    # Sec. 4 Eq. 1 with the paper's truncate 5
    prm = dog.Params(p[0], p[1], 1.6, 0.1, 0.5, 5.0, "arithmetic", p[2], True)
    info = dog.plan_info(prm)
    s = oracle.sigmas_arithmetic(*p)
    assert info["k"] == p[2] == len(s) - 1
    assert np.array_equal(info["sigmas"], s)
    assert info["radii"].tolist() == [oracle.radius(x, 5.0) for x in s]
    assert dog.plan_info(dog.Params.paper())["k"] == 10


@pytest.mark.parametrize("bad", [dict(ladder="arithmetic", n_bin=0), dict(ladder="arithmetic", n_bin=64),
                                 dict(ladder="arithmetic", n_bin=-3)])
def test_invalid_arithmetic_params_rejected(bad):
    kw = dict(sigma_min=1.0, sigma_max=8.0, sigma_ratio=1.6, threshold=0.1, overlap=0.5, truncate=5.0)
    kw.update(bad)
    with pytest.raises(dog.DogError) as e:
        dog.plan_info(dog.Params(**kw))
    assert e.value.code == dog.DOG_EINVAL
    # sigma_ratio is not used by the arithmetic ladder
    dog.plan_info(dog.Params(1.0, 8.0, 0.5, 0.1, 0.5, 5.0, "arithmetic", 4))
    c = dog.Params(1.0, 8.0).c()
    for field, v in (("ladder", 2), ("coalesce", 2), ("reserved", 1)):
        raw = dog.dog_params(c.sigma_min, c.sigma_max, c.sigma_ratio, c.threshold, c.overlap,
                             c.truncate, 0, 0, 0, 0)
        setattr(raw, field, v)
        k = ctypes.c_int32(0)
        assert dog.lib().dog_plan_info(ctypes.byref(raw), ctypes.byref(k), None, None, 0) == dog.DOG_EINVAL


@pytest.mark.parametrize("seed,overlap,ladder", [(0, 0.5, "geometric"), (1, 0.5, "arithmetic"),
                                                 (2, 0.0, "arithmetic"), (3, 0.9, "geometric")])
def test_coalescing_prune_matches_oracle(seed, overlap, ladder):
    rng = np.random.default_rng(seed)
    n = 400
    prm = (dog.Params(1, 30, 1.6, 0.05, overlap, 4.0, "geometric", 0, True) if ladder == "geometric"
           else dog.Params(1, 30, 1.6, 0.05, overlap, 5.0, "arithmetic", 10, True))
    sig = dog.plan_info(prm)["sigmas"]
    k = len(sig) - 1
    b = np.zeros(n, dog.BLOB_DTYPE)
    b["y"] = rng.integers(0, 120, n)
    b["x"] = rng.integers(0, 120, n)
    b["scale"] = rng.integers(0, k, n)
    _, u = np.unique(b[["y", "x", "scale"]], return_index=True)
    b = b[np.sort(u)]
    rng.shuffle(b)
    got = dog.prune(prm, b)
    order = np.lexsort((b["scale"], b["x"], b["y"]))
    s = b[order]
    keep, s_out = oracle.prune(s["y"], s["x"], sig[s["scale"]], overlap, coalesce=True)
    exp = s[keep]
    assert got[["y", "x", "scale"]].tolist() == exp[["y", "x", "scale"]].tolist()
    assert np.array_equal(got["sigma"], s_out[keep].astype(np.float32))
    if overlap < 1.0 and len(exp) < len(s):
        # some survivors really were coalesced (their sigma left the ladder)
        assert np.any(got["sigma"] != sig[got["scale"]].astype(np.float32))


@pytest.mark.parametrize("seed,ladder", [(0, "geometric"), (1, "arithmetic")])
def test_radius_histogram_matches_oracle(seed, ladder):
    rng = np.random.default_rng(seed)
    prm = (dog.Params(1, 30, 1.6, 0.05, 0.5) if ladder == "geometric"
           else dog.Params.paper(1.0, 30.0, 10))
    sig = dog.plan_info(prm)["sigmas"]
    k = len(sig) - 1
    b = np.zeros(500, dog.BLOB_DTYPE)
    # ladder sigmas and coalesced means between them (as float32, like the output)
    b["sigma"] = np.where(rng.random(500) < 0.5, sig[rng.integers(0, k, 500)],
                          rng.uniform(0.5, sig[k - 1] * 1.2, 500)).astype(np.float32)
    got = dog.radius_histogram(prm, b)
    exp = oracle.radius_histogram(sig[:k], b["sigma"].astype(np.float64))
    assert got.tolist() == exp.tolist() and got.sum() == 500
    assert dog.radius_histogram(prm, b[:0]).tolist() == [0] * k


@pytest.mark.parametrize("coalesce", [False, True])
@pytest.mark.parametrize("spread", [(64, 4000), (700, 700), (3000, 40)])
def test_prune_wide_frames_match_oracle(coalesce, spread):
    # frames much wider than the largest touching distance: the host scan
    # skips distant columns, which must not change which blobs survive
    H, W = spread
    rng = np.random.default_rng(H + W + coalesce)
    n = 2500
    prm = dog.Params(1, 30, 1.6, 0.05, 0.5, 4.0, "geometric", 0, coalesce)
    sig = dog.plan_info(prm)["sigmas"]
    b = np.zeros(n, dog.BLOB_DTYPE)
    b["y"] = rng.integers(0, H, n)
    b["x"] = rng.integers(0, W, n) - W // 3     # columns on both sides of 0
    b["scale"] = rng.integers(0, 8, n)
    _, u = np.unique(b[["y", "x", "scale"]], return_index=True)
    b = b[np.sort(u)]
    rng.shuffle(b)
    got = dog.prune(prm, b)
    s = b[np.lexsort((b["scale"], b["x"], b["y"]))]
    keep, s_out = oracle.prune(s["y"], s["x"], sig[s["scale"]], 0.5, coalesce=True) if coalesce else \
        (oracle.prune(s["y"], s["x"], sig[s["scale"]], 0.5), sig[s["scale"]])
    exp = s[keep]
    assert 0 < len(exp) < len(s)
    assert got[["y", "x", "scale"]].tolist() == exp[["y", "x", "scale"]].tolist()
    assert np.array_equal(got["sigma"], s_out[keep].astype(np.float32))


@pytest.mark.parametrize("coalesce", [False, True])
def test_prune_extreme_coordinates(coalesce):
    # clusters spread over the whole int32 range: the packed sort key does
    # not fit in 64 bits (the three-field sort runs), coordinate differences
    # exceed int32, and blobs in a cluster still overlap
    rng = np.random.default_rng(11 + coalesce)
    n = 400
    prm = dog.Params(1, 30, 1.6, 0.05, 0.5, 4.0, "geometric", 0, coalesce)
    sig = dog.plan_info(prm)["sigmas"]
    centres = rng.integers(-2**31 + 100, 2**31 - 100, (25, 2))
    # two clusters at the two ends of the row range: their int32 row
    # difference would wrap to a few pixels
    centres[0] = (-2**31 + 8, 0)
    centres[1] = (2**31 - 9, 0)
    pick = rng.integers(0, 25, n)
    b = np.zeros(n, dog.BLOB_DTYPE)
    b["y"] = centres[pick, 0] + rng.integers(-8, 9, n)
    b["x"] = centres[pick, 1] + rng.integers(-8, 9, n)
    b["scale"] = rng.integers(0, 8, n)
    _, u = np.unique(b[["y", "x", "scale"]], return_index=True)
    b = b[np.sort(u)]
    rng.shuffle(b)
    got = dog.prune(prm, b)
    s = b[np.lexsort((b["scale"], b["x"], b["y"]))]
    keep, s_out = oracle.prune(s["y"], s["x"], sig[s["scale"]], 0.5, coalesce=True) if coalesce else \
        (oracle.prune(s["y"], s["x"], sig[s["scale"]], 0.5), sig[s["scale"]])
    exp = s[keep]
    assert 0 < len(exp) < len(s)
    assert got[["y", "x", "scale"]].tolist() == exp[["y", "x", "scale"]].tolist()
    assert np.array_equal(got["sigma"], s_out[keep].astype(np.float32))
