"""GPU parity for the paper's own configuration: the arithmetic ladder of
Sec. 4 Eq. 1 (n_bin + 1 sigmas), truncate 5, and coalescing of overlapping
blobs by averaging the radius (Sec. 4.1), against the FP64 oracle on the same
ladder.  Includes a ladder of more than 10 Gaussian planes (the local-maximum
kernel's rolling form) and a ragged frame."""
import numpy as np
import pytest

import oracle
import synth
from parity import check_candidates, check_candidates_exact, check_exempt_bound, check_planes

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


def _parity(dog, torch, img, prm, natural=False):
    t = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    sig = oracle.sigmas_arithmetic(prm.sigma_min, prm.sigma_max, prm.n_bin)
    L_o, D_o = oracle.planes_sigmas(img, sig, prm.truncate)
    max_abs = float(np.abs(img).max())
    with dog.Context(0) as c:
        L_g, D_g = c.debug_planes(t, prm)
        torch.cuda.synchronize()
        D_g = D_g.cpu().numpy()
        check_planes(L_g.cpu().numpy(), D_g, L_o, D_o, sig, max_abs)
        raw = c.debug_candidates(t, prm)
        check_candidates_exact(raw, D_g, prm.threshold)
        exempt = check_candidates(raw, D_o, prm.threshold, sig, max_abs)
        if natural:
            check_exempt_bound(exempt, len(raw))
        blobs = c.detect_device(t, prm)
    # coalescing of the oracle's own list (or, with voxels in the decision
    # margin, of the GPU's raw list) must give the same blobs and sigmas
    if exempt == 0:
        yxi, _ = oracle.nms(D_o, prm.threshold)
        ry, rx, ri = yxi[:, 0], yxi[:, 1], yxi[:, 2]
    else:
        ry, rx, ri = raw["y"], raw["x"], raw["scale"]
    keep, s_out = oracle.prune(ry, rx, sig[ri], prm.overlap, coalesce=True)
    exp = list(zip(ry[keep].tolist(), rx[keep].tolist(), ri[keep].tolist()))
    got = list(zip(blobs["y"].tolist(), blobs["x"].tolist(), blobs["scale"].tolist()))
    assert got == exp
    assert np.array_equal(blobs["sigma"], s_out[keep].astype(np.float32))
    return raw, blobs, exempt


def test_paper_ladder_small_frame(dog, torch_mod):
    prm = dog.Params.paper(sigma_min=1.0, sigma_max=8.0, n_bin=7, threshold=0.1)
    raw, blobs, exempt = _parity(dog, torch_mod, synth.small_frame(seed=21), prm)
    print("paper ladder 1..8/7: raw %d coalesced %d exempt %d" % (len(raw), len(blobs), exempt))
    assert len(blobs) >= 10 and len(blobs) < len(raw)


def test_paper_ladder_many_planes_ragged(dog, torch_mod):
    # 13 Gaussian planes, sigma up to 30 (radius 150) on a 200 x 333 frame
    prm = dog.Params.paper(sigma_min=1.0, sigma_max=30.0, n_bin=12, threshold=0.05)
    img = synth.camera_frame(seed=22, H=200, W=333, n_blobs=40)
    raw, blobs, exempt = _parity(dog, torch_mod, img, prm)
    print("paper ladder 1..30/12: raw %d coalesced %d exempt %d" % (len(raw), len(blobs), exempt))
    assert len(blobs) >= 5


def test_paper_ladder_pruning_mode_and_variants(dog, torch_mod):
    # the same ladder with plain pruning, and every kernel variant bitwise equal
    prm = dog.Params(1.0, 30.0, 1.6, 0.05, 0.5, 5.0, "arithmetic", 10, False)
    img = synth.camera_frame(seed=23, H=256, W=256, n_blobs=40)
    t = torch_mod.from_numpy(img).cuda()
    with dog.Context(0) as c:
        ref = c.detect_device(t, prm)
        L0, _ = c.debug_planes(t, prm)
        L0 = L0.cpu().numpy()
        for v in range(dog.num_variants()):
            c.set_variant(v)
            assert c.detect_device(t, prm).tobytes() == ref.tobytes(), v
            L, _ = c.debug_planes(t, prm)
            assert L.cpu().numpy().tobytes() == L0.tobytes(), v
    sig = oracle.sigmas_arithmetic(1.0, 30.0, 10)
    assert np.all(ref["sigma"] == sig[ref["scale"]].astype(np.float32))


def test_paper_configuration_at_the_benchmark_size(dog, torch_mod):
    # the configuration the benchmark times: 1024x1024 camera frame, Eq. 1
    # ladder with n_bin = 10 over 1..30 (11 planes, radius up to 150),
    # truncate 5, coalescing, threshold 0.05
    prm = dog.Params.paper(1.0, 30.0, 10, threshold=0.05)
    img = synth.camera_frame(seed=1)
    raw, blobs, exempt = _parity(dog, torch_mod, img, prm, natural=True)
    print("paper configuration 1024^2: raw %d coalesced %d exempt %d" % (len(raw), len(blobs), exempt))
    assert len(blobs) >= 100
