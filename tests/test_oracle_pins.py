"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics,
not by the oracle itself (CPU only).

Each test names what it pins:
  P1 kernel weights: normalisation, symmetry, Gaussian ratios, radius rule
  P2 a delta image reproduces the kernel (interior and reflected at a border)
  P3 separable blur == brute-force 2-D convolution on tiny images
  P4 blur == scipy.ndimage.gaussian_filter; max filter == scipy maximum_filter
  P5 a planted Gaussian blob is found once, at its centre, at the scale the
     continuum closed form predicts, with the closed-form response
  P6 invariances (translation, intensity scaling, transpose, constant image)
  P7 local-maximum search == brute force with a library max filter; plateaus
  P8 lens area vs quadrature and closed forms; pruning invariants
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ---------------------------------------------------------------- P1 weights
@pytest.mark.parametrize("sigma", [0.5, 1.0, 1.6, 2.56, 4.096, 10.48576, 42.94967296])
def test_p1_weights_normalised_symmetric_gaussian(sigma):
    r = oracle.radius(sigma, 4.0)
    w = oracle.weights(sigma, r)
    assert len(w) == 2 * r + 1
    assert abs(w.sum() - 1.0) <= (2 * r + 1) * 2.0 ** -52
    assert np.array_equal(w, w[::-1])
    j = np.arange(-r, r + 1)
    ratio = w / w[r]
    np.testing.assert_allclose(ratio, np.exp(-j * j / (2 * sigma * sigma)), rtol=1e-14, atol=0)


def test_p1_radius_rule_and_ladders():
    # radius = truncate*sigma rounded to nearest (Sec. 4.1 samples out to truncate*sigma)
    assert oracle.radius(1.0, 4.0) == 4
    assert oracle.radius(1.125, 4.0) == 5          # 4.5 rounds up
    assert oracle.radius(1.1, 4.0) == 4            # 4.4 rounds down
    assert oracle.radius(1.0, 5.0) == 5
    # geometric ladders of the two workloads (1..8 and 1..30, ratio 1.6)
    assert oracle.num_dog_planes(1, 8, 1.6) == 5
    assert oracle.num_dog_planes(1, 30, 1.6) == 8
    s = oracle.sigmas_geometric(1, 30, 1.6)
    np.testing.assert_allclose(s, 1.6 ** np.arange(9), rtol=1e-15)
    assert [oracle.radius(x) for x in s] == [4, 6, 10, 16, 26, 42, 67, 107, 172]
    assert [oracle.radius(x) for x in oracle.sigmas_geometric(1, 8, 1.6)] == [4, 6, 10, 16, 26, 42]
    # degenerate ladder sigma_min == sigma_max: one DoG plane
    assert oracle.num_dog_planes(2.0, 2.0, 1.6) == 1
    # Sec. 4 Eq. 1 (arithmetic): sigma_1 = min, step (max-min)/n_bin
    np.testing.assert_allclose(oracle.sigmas_arithmetic(1, 8, 7), np.arange(1, 9), rtol=0, atol=1e-15)


def test_p1_weights_match_library_kernel():
    # scipy's 1-D Gaussian filter of a centred delta returns its truncated kernel
    for sigma in (1.0, 2.56, 10.48576):
        r = oracle.radius(sigma)
        n = 4 * r + 3
        d = np.zeros(n)
        d[n // 2] = 1.0
        k = ndi.gaussian_filter1d(d, sigma, truncate=4.0, mode="reflect")
        np.testing.assert_allclose(k[n // 2 - r:n // 2 + r + 1], oracle.weights(sigma, r),
                                   rtol=1e-13, atol=1e-17)
        assert np.all(k[:n // 2 - r] == 0) and np.all(k[n // 2 + r + 1:] == 0)


# ---------------------------------------------------------------- P2 delta
def test_p2_interior_delta_gives_outer_product():
    sigma = 2.56
    r = oracle.radius(sigma)
    H, W = 41, 37
    img = np.zeros((H, W))
    cy, cx = 20, 18
    img[cy, cx] = 1.0
    L = oracle.blur(img, sigma)
    w = oracle.weights(sigma, r)
    expect = np.zeros((H, W))
    expect[cy - r:cy + r + 1, cx - r:cx + r + 1] = np.outer(w, w)
    np.testing.assert_allclose(L, expect, rtol=0, atol=1e-15)


def test_p2_border_delta_is_reflected():
    # half-sample symmetric reflection: a delta at index 0 is also seen at -1,
    # so the response along an axis is w[t] + w[t+1] (w symmetric).
    sigma = 1.6
    r = oracle.radius(sigma)
    H, W = 30, 30
    img = np.zeros((H, W))
    img[0, 0] = 1.0
    L = oracle.blur(img, sigma)
    w = oracle.weights(sigma, r)
    prof = np.zeros(W)
    for t in range(r + 1):
        prof[t] = w[r + t] + (w[r + t + 1] if t + 1 <= r else 0.0)
    np.testing.assert_allclose(L, np.outer(prof, prof), rtol=0, atol=1e-15)


def test_reflect_map_examples():
    # x[-1] = x[0], x[-2] = x[1], x[n] = x[n-1], period 2n, n = 1 maps to 0
    n = 4
    got = [oracle.reflect(t, n) for t in range(-9, 13)]
    ext = np.pad(np.arange(n), 9, mode="symmetric")
    assert got == list(ext[:22])
    assert all(oracle.reflect(t, 1) == 0 for t in range(-5, 6))


# ---------------------------------------------------------------- P3 brute force
def _brute_2d(img, sigma, truncate=4.0):
    r = int(math.floor(truncate * sigma + 0.5))
    j = np.arange(-r, r + 1)
    g = np.exp(-j * j / (2 * sigma * sigma))
    k2 = np.outer(g, g) / np.outer(g, g).sum()
    P = np.pad(img, r, mode="symmetric")
    H, W = img.shape
    out = np.zeros((H, W))
    for a in range(2 * r + 1):
        for b in range(2 * r + 1):
            out += k2[a, b] * P[a:a + H, b:b + W]
    return out


@pytest.mark.parametrize("shape,sigma", [((7, 5), 1.0), ((1, 9), 1.6), ((3, 1), 1.0),
                                         ((3, 1), 3.0), ((2, 6), 2.56), ((5, 4), 4.096),
                                         ((1, 1), 1.6), ((11, 13), 1.6)])
def test_p3_separable_equals_bruteforce_2d(shape, sigma):
    rng = np.random.default_rng(7)
    img = rng.uniform(-1, 1, shape)
    np.testing.assert_allclose(oracle.blur(img, sigma), _brute_2d(img, sigma), rtol=0, atol=1e-13)


# ---------------------------------------------------------------- P4 library
@pytest.mark.parametrize("sigma", [1.0, 1.6, 4.096, 10.48576])
def test_p4_blur_matches_scipy(sigma):
    rng = np.random.default_rng(11)
    img = rng.uniform(0, 1, (48, 40))
    ref = ndi.gaussian_filter(img, sigma, mode="reflect", truncate=4.0)
    np.testing.assert_allclose(oracle.blur(img, sigma), ref, rtol=0, atol=1e-13)


def test_p4_planes_and_dog_match_scipy():
    img = synth.small_frame(seed=3, H=64, W=48, n_blobs=5)
    L, D, s = oracle.planes(img, 1.0, 8.0, 1.6)
    assert L.shape == (6, 64, 48) and D.shape == (5, 64, 48)
    for i, sg in enumerate(s):
        ref = ndi.gaussian_filter(img.astype(np.float64), sg, mode="reflect", truncate=4.0)
        np.testing.assert_allclose(L[i], ref, rtol=0, atol=1e-13)
    for i in range(5):
        np.testing.assert_allclose(D[i], s[i] * (L[i] - L[i + 1]), rtol=0, atol=0)


# ---------------------------------------------------------------- P5 planted blob
def _closed_form_dog(s, sig):
    """Continuum response at the centre of a unit Gaussian blob of std s:
    a blob blurred by sigma has centre height s^2/(s^2+sigma^2)."""
    return np.array([sig[i] * s * s * (1.0 / (s * s + sig[i] ** 2) - 1.0 / (s * s + sig[i + 1] ** 2))
                     for i in range(len(sig) - 1)])


@pytest.mark.parametrize("ladder,s,N", [((1, 8), 1.0, 96), ((1, 8), 2.0, 96), ((1, 8), 3.0, 128),
                                        ((1, 8), 5.0, 160), ((1, 30), 1.5, 160),
                                        ((1, 30), 6.0, 256), ((1, 30), 14.0, 448)])
def test_p5_planted_blob_scale_and_response(ladder, s, N):
    smin, smax = ladder
    c = N // 2
    amp = 1.0
    img = synth.planted_blob(N, N, c, c, s, amp)
    blobs, raw, D, sig = oracle.detect(img, smin, smax, 1.6, threshold=0.02, overlap=0.5,
                                       return_raw=True)
    cf = _closed_form_dog(s, sig)
    i_star = int(np.argmax(cf))
    assert len(raw) == 1, raw
    assert (raw["y"][0], raw["x"][0], raw["scale"][0]) == (c, c, i_star)
    # the image is stored in fp32 and the kernels are truncated: 1e-3 relative
    np.testing.assert_allclose(D[:, c, c], cf * amp, rtol=2e-3, atol=2e-4)
    # blob radius sqrt(2)*sigma (Sec. 3) with sigma the detected ladder value
    assert raw["sigma"][0] == sig[i_star]


# ---------------------------------------------------------------- P6 invariances
def _blobs_on_zero(H, W, pts):
    return synth.render_blobs(H, W, [p[0] for p in pts], [p[1] for p in pts],
                              [p[2] for p in pts], [1.0] * len(pts)).astype(np.float32)


def test_p6_translation():
    pts = [(40, 40, 2.0), (52, 70, 3.0), (80, 45, 1.5)]
    a = _blobs_on_zero(160, 160, pts)
    b = _blobs_on_zero(160, 160, [(y + 7, x + 11, s) for y, x, s in pts])
    ra = oracle.detect(a, 1, 4, 1.6, threshold=0.02)
    rb = oracle.detect(b, 1, 4, 1.6, threshold=0.02)
    assert len(ra) >= 3
    assert np.array_equal(ra["y"] + 7, rb["y"]) and np.array_equal(ra["x"] + 11, rb["x"])
    assert np.array_equal(ra["scale"], rb["scale"])


def test_p6_intensity_scaling():
    img = synth.small_frame(seed=5, H=96, W=96, n_blobs=8)
    ra = oracle.detect(img, 1, 8, 1.6, threshold=0.1)
    rb = oracle.detect((img * np.float32(2.0)).astype(np.float32), 1, 8, 1.6, threshold=0.2)
    assert len(ra) > 0
    for f in ("y", "x", "scale"):
        assert np.array_equal(ra[f], rb[f])
    np.testing.assert_array_equal(ra["response"] * 2.0, rb["response"])


def test_p6_transpose():
    img = synth.small_frame(seed=9, H=80, W=64, n_blobs=8)
    ra = oracle.detect(img, 1, 8, 1.6, threshold=0.1, overlap=1.0)
    rb = oracle.detect(np.ascontiguousarray(img.T), 1, 8, 1.6, threshold=0.1, overlap=1.0)
    A = sorted(zip(ra["y"], ra["x"], ra["scale"]))
    B = sorted(zip(rb["x"], rb["y"], rb["scale"]))
    assert len(A) > 0 and A == B


def test_p6_constant_image_has_no_blobs():
    img = np.full((50, 40), 0.7, np.float32)
    assert len(oracle.detect(img, 1, 8, 1.6, threshold=0.1)) == 0
    L, D, _ = oracle.planes(img, 1, 8, 1.6)
    np.testing.assert_allclose(L, float(np.float32(0.7)), rtol=1e-14)
    assert np.abs(D).max() < 1e-13


# ---------------------------------------------------------------- P7 NMS
@pytest.mark.parametrize("seed", range(5))
def test_p7_nms_matches_library_max_filter(seed):
    rng = np.random.default_rng(seed)
    k, H, W = 4, 9, 7
    D = rng.uniform(-1, 1, (k, H, W))
    D = np.round(D * 4) / 4          # many exact ties
    thr = -0.3
    M = ndi.maximum_filter(D, size=3, mode="constant", cval=-np.inf)
    expect = sorted((int(y), int(x), int(i)) for i, y, x in zip(*np.nonzero((D == M) & (D > thr))))
    yxi, resp = oracle.nms(D, thr)
    assert [tuple(r) for r in yxi.tolist()] == expect
    for (y, x, i), v in zip(yxi, resp):
        assert v == D[i, y, x]
        assert oracle.neigh_max(D, i, y, x) == M[i, y, x]


def test_p7_plateau_reports_all_tied_voxels_and_strict_threshold():
    D = np.zeros((3, 6, 6))
    D[1, 2:4, 2:4] = 0.5              # a 2x2 plateau: four tied maxima
    D[0, 0, 5] = 0.1                  # equals the threshold: not kept (strict)
    yxi, _ = oracle.nms(D, 0.1)
    assert [tuple(r) for r in yxi.tolist()] == [(2, 2, 1), (2, 3, 1), (3, 2, 1), (3, 3, 1)]
    # edge planes and borders are eligible
    E = np.zeros((2, 3, 3))
    E[0, 0, 0] = 1.0
    E[1, 2, 2] = 2.0
    yxi, _ = oracle.nms(E, 0.0)
    assert [tuple(r) for r in yxi.tolist()] == [(0, 0, 0), (2, 2, 1)]


# ---------------------------------------------------------------- P8 overlap
def _lens_quadrature(d, r1, r2, n=4001):
    # integrate the chord length of disk 2 inside disk 1 along x
    x = np.linspace(-r1, r1, n)
    h1 = np.sqrt(np.maximum(r1 * r1 - x * x, 0))
    h2 = np.sqrt(np.maximum(r2 * r2 - (x - d) ** 2, 0))
    return np.trapezoid(2 * np.minimum(h1, h2) * ((np.abs(x - d) <= r2)), x)


@pytest.mark.parametrize("d,r1,r2", [(1.0, 2.0, 2.0), (2.5, 2.0, 1.5), (3.0, 3.0, 1.0),
                                     (0.7, 1.0, 3.0), (4.0, 2.5, 2.0)])
def test_p8_lens_area_vs_quadrature(d, r1, r2):
    assert abs(oracle.lens_area(d, r1, r2) - _lens_quadrature(d, r1, r2)) < 2e-4 * math.pi * min(r1, r2) ** 2


def test_p8_lens_closed_forms():
    r = 2.0
    for d in (0.3, 1.0, 2.5, 3.9):
        eq = 2 * r * r * math.acos(d / (2 * r)) - 0.5 * d * math.sqrt(4 * r * r - d * d)
        assert abs(oracle.lens_area(d, r, r) - eq) < 1e-12
    assert oracle.lens_area(5.0, 2.0, 3.0) == 0.0
    assert oracle.lens_area(6.0, 2.0, 3.0) == 0.0
    assert oracle.lens_area(0.5, 1.0, 3.0) == pytest.approx(math.pi)
    assert oracle.overlap_fraction(10, 10, 2.0, 10, 10, 5.0) == pytest.approx(1.0)
    assert oracle.overlap_fraction(0, 0, 1.0, 0, 100, 1.0) == 0.0


def test_p8_prune_rules():
    # two concentric blobs: the smaller sigma is removed
    keep = oracle.prune([5, 5], [5, 5], [1.0, 2.0], 0.5)
    assert keep.tolist() == [False, True]
    keep = oracle.prune([5, 5], [5, 5], [2.0, 1.0], 0.5)
    assert keep.tolist() == [True, False]
    # equal sigma: the later one goes
    keep = oracle.prune([5, 5], [5, 6], [3.0, 3.0], 0.5)
    assert keep.tolist() == [True, False]
    # overlap >= 1 disables pruning; far apart blobs are kept
    assert oracle.prune([5, 5], [5, 5], [1.0, 2.0], 1.0).tolist() == [True, True]
    assert oracle.prune([0, 50], [0, 50], [1.0, 1.0], 0.0).tolist() == [True, True]
    # chain A(sigma 2)-B(sigma 3)-C(sigma 2): B removes A, then B removes C
    keep = oracle.prune([10, 10, 10], [10, 12, 14], [2.0, 3.0, 2.0], 0.5)
    assert keep.tolist() == [False, True, False]


def test_p8_prune_invariants_random():
    rng = np.random.default_rng(4)
    n = 300
    pts = sorted(zip(rng.integers(0, 60, n).tolist(), rng.integers(0, 60, n).tolist(),
                     rng.integers(0, 5, n).tolist()))
    y = np.array([p[0] for p in pts])
    x = np.array([p[1] for p in pts])
    s = 1.6 ** np.array([p[2] for p in pts])
    keep = oracle.prune(y, x, s, 0.5)
    idx = np.nonzero(keep)[0]
    # no surviving pair overlaps more than the limit
    for a in range(len(idx)):
        for b in range(a + 1, len(idx)):
            i, j = idx[a], idx[b]
            assert oracle.overlap_fraction(y[i], x[i], s[i], y[j], x[j], s[j]) <= 0.5
    # every removed blob overlaps (> limit) some blob of larger-or-equal sigma
    for i in np.nonzero(~keep)[0]:
        assert any(oracle.overlap_fraction(y[i], x[i], s[i], y[j], x[j], s[j]) > 0.5 and s[j] >= s[i]
                   for j in range(n) if j != i)


def test_p8_coalesce_rules():
    # Sec. 4.1: overlapping blobs are coalesced by averaging the radius
    # (reading R7b: the blob with the smaller sigma goes, the other takes the
    # mean sigma, and later pairs see the new sigma)
    keep, s = oracle.prune([5, 5], [5, 5], [1.0, 3.0], 0.5, coalesce=True)
    assert keep.tolist() == [False, True] and s[1] == 2.0
    keep, s = oracle.prune([5, 5], [5, 5], [3.0, 1.0], 0.5, coalesce=True)
    assert keep.tolist() == [True, False] and s[0] == 2.0
    # chain A(2)-B(3)-C(2) on a row, 2 px apart: B absorbs A (sigma 2.5),
    # then C (sigma 2.25)
    keep, s = oracle.prune([10, 10, 10], [10, 12, 14], [2.0, 3.0, 2.0], 0.5, coalesce=True)
    assert keep.tolist() == [False, True, False] and s[1] == 2.25
    # the shrunken blob no longer reaches a third one: A(1) and B(4)
    # concentric, C(1.5) 4 px away overlaps B(4) by 0.93 but B(2.5) by 0.31
    y, x, sg = [10, 10, 10], [10, 10, 14], [1.0, 4.0, 1.5]
    assert oracle.overlap_fraction(10, 10, 4.0, 10, 14, 1.5) > 0.5
    assert oracle.overlap_fraction(10, 10, 2.5, 10, 14, 1.5) < 0.5
    assert oracle.prune(y, x, sg, 0.5).tolist() == [False, True, False]
    keep, s = oracle.prune(y, x, sg, 0.5, coalesce=True)
    assert keep.tolist() == [False, True, True] and s[1] == 2.5 and s[2] == 1.5
    # overlap >= 1: nothing changes
    keep, s = oracle.prune([5, 5], [5, 5], [1.0, 3.0], 1.0, coalesce=True)
    assert keep.tolist() == [True, True] and s.tolist() == [1.0, 3.0]


def test_p8_coalesce_reduces_to_prune_for_equal_sigmas():
    # with one sigma for every blob the mean is that sigma, so coalescing
    # keeps exactly the blobs pruning keeps
    rng = np.random.default_rng(5)
    pts = sorted(set(zip(rng.integers(0, 40, 200).tolist(), rng.integers(0, 40, 200).tolist())))
    y = np.array([p[0] for p in pts])
    x = np.array([p[1] for p in pts])
    s = np.full(len(pts), 2.56)
    keep_c, s_c = oracle.prune(y, x, s, 0.5, coalesce=True)
    assert keep_c.tolist() == oracle.prune(y, x, s, 0.5).tolist()
    assert np.all(s_c == 2.56)


def test_p1_arithmetic_ladder_of_the_paper():
    # Sec. 4 Eq. 1 with n_bin = 10 over 1..30: step 2.9, last sigma = max
    s = oracle.sigmas_arithmetic(1.0, 30.0, 10)
    assert len(s) == 11 and s[0] == 1.0 and s[-1] == 30.0
    np.testing.assert_allclose(np.diff(s), 2.9, rtol=1e-14)
    # n_bin = 1: just the two ends
    assert oracle.sigmas_arithmetic(2.0, 5.0, 1).tolist() == [2.0, 5.0]


def test_r11_stretch_on_a_permutation():
    # no smoothing, distinct values 0..N-1: with N = 10000 and 0.35 %
    # saturation, m = floor(17.5) = 17 pixels below lo at each end
    rng = np.random.default_rng(7)
    img = rng.permutation(10000).astype(np.float32).reshape(100, 100)
    out, sm, lo, hi = oracle.preprocess(img, sigma=0.0, saturated=0.0035)
    assert (lo, hi) == (17.0, 9982.0)
    np.testing.assert_array_equal(sm, img.astype(np.float64))
    np.testing.assert_allclose(out, np.clip((img.astype(np.float64) - 17.0) / 9965.0, 0.0, 1.0),
                               rtol=0, atol=1e-15)
    assert int((out == 0.0).sum()) == 18 and int((out == 1.0).sum()) == 18
    # no saturation: the stretch spans the full range
    _, _, lo0, hi0 = oracle.preprocess(img, sigma=0.0, saturated=0.0)
    assert (lo0, hi0) == (0.0, 9999.0)


def test_r11_smoothing_matches_scipy_and_limits_match_numpy():
    from scipy import ndimage
    img = synth.camera_frame(seed=8, H=96, W=80, n_blobs=10) * 65535.0
    out, sm, lo, hi = oracle.preprocess(img.astype(np.float32), sigma=1.5, saturated=0.0035)
    ref = ndimage.gaussian_filter(img.astype(np.float32).astype(np.float64), 1.5,
                                  mode="reflect", truncate=4.0)
    np.testing.assert_allclose(sm, ref, rtol=1e-12, atol=1e-9)
    m = int(np.floor(0.0035 * sm.size / 2))
    srt = np.sort(sm.ravel())
    assert lo == srt[m] and hi == srt[-1 - m]
    assert out.min() == 0.0 and out.max() == 1.0


def test_r11_constant_image_and_affine_invariance():
    out, _, lo, hi = oracle.preprocess(np.full((20, 30), 7.0, np.float32), sigma=1.0)
    assert lo == hi == pytest.approx(7.0) and np.all(out == 0.0)
    img = synth.small_frame(seed=9, H=64, W=64).astype(np.float32)
    a, _, _, _ = oracle.preprocess(img, sigma=1.0)
    b, _, _, _ = oracle.preprocess((img * 4.0 + 3.0).astype(np.float32), sigma=1.0)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-6)


def test_r12_radius_histogram():
    # Sec. 4.1: bin centres at the ladder radii sqrt(2)*sigma_i
    lad = [1.0, 2.0, 4.0]
    # blobs exactly at the ladder sigmas land in their own bins
    assert oracle.radius_histogram(lad, [1.0, 4.0, 4.0, 2.0, 1.0]).tolist() == [2, 1, 2]
    # coalesced sigmas go to the nearest centre: 1.4 -> 1, 1.6 -> 2, 3.1 -> 4;
    # a tie (1.5, midway between 1 and 2) goes to the lower bin
    assert oracle.radius_histogram(lad, [1.4, 1.6, 3.1, 1.5]).tolist() == [2, 1, 1]
    # beyond the ends: the end bins
    assert oracle.radius_histogram(lad, [0.1, 50.0]).tolist() == [1, 0, 1]
    assert oracle.radius_histogram(lad, []).tolist() == [0, 0, 0]


# ------------------------------------------------- the one-call C detector
# orc_detect composes ladder, planes, local maxima, threshold and pruning a
# second time inside the C oracle (it is what the CPU baseline times).  It
# must return exactly what the composition of the pinned pieces above
# returns: same (y, x, scale) triples, same sigma and response bits.
def _one_call_equals_composition(img, smin, smax, thr, overlap):
    comp = oracle.detect(img, smin, smax, 1.6, threshold=thr, overlap=overlap)
    one = oracle.detect_c(img, smin, smax, 1.6, threshold=thr, overlap=overlap)
    assert len(one) == len(comp)
    for f in ("y", "x", "scale"):
        assert np.array_equal(one[f], comp[f]), f
    assert one["sigma"].tobytes() == comp["sigma"].tobytes()
    assert one["response"].tobytes() == comp["response"].tobytes()
    return len(one)


@pytest.mark.parametrize("case", ["small", "ragged"])
def test_one_call_detector_equals_composition_small(case):
    if case == "small":
        img = synth.small_frame(seed=0)                      # 256x256, ladder 1..8
        n = _one_call_equals_composition(img, 1.0, 8.0, 0.1, 0.5)
    else:
        img = synth.small_frame(seed=7, H=97, W=131, n_blobs=9)
        n = _one_call_equals_composition(img, 1.0, 8.0, 0.1, 0.5)
    assert n > 0


@pytest.mark.parametrize("overlap", [0.5, 1.0])
def test_one_call_detector_equals_composition_camera_frame(overlap):
    img = synth.camera_frame(seed=1)                         # 1024x1024, ladder 1..30
    n = _one_call_equals_composition(img, 1.0, 30.0, 0.05, overlap)
    assert n > 100
