"""Parity helpers: compare the HIP path's planes and blob lists with the FP64
oracle under the stated tolerances.

Planes (relative 1e-5, scaled so the bound holds where the value is near 0):
    |L_gpu - L_orc| <= 1e-5 * (|L_orc| + max|I|)
    |D_gpu - D_orc| <= 1e-5 * (|D_orc| + sigma_i * max|I|)
Blob lists: identical, except a voxel may appear on one side only when the
oracle's FP64 cube puts it within delta_i = 2e-5 * sigma_i * max|I| of a tie
with its largest neighbour or of the threshold (a decision fp32 cannot take
the same way as FP64 there).  On frames of natural shape such voxels must
stay rare (MAX_EXEMPT_FRACTION of the candidates).

Margin-free check: on the GPU's own fp32 DoG cube the local-maximum decision
has a single right answer.  Widening fp32 to FP64 keeps equality and order,
and the kernel compares with the largest float <= threshold, so the oracle's
local-maximum search run on that cube must return exactly the GPU's
candidates, with their responses bit for bit.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

PLANE_RTOL = 1e-5
MARGIN = 2e-5
MAX_EXEMPT_FRACTION = 0.01


def check_candidates_exact(gpu_raw, D_gpu, thr):
    """gpu_raw: the GPU's candidates (sorted by y, x, scale); D_gpu: the same
    kernels' fp32 DoG cube (k, H, W).  No exemptions."""
    D = np.asarray(D_gpu, np.float32).astype(np.float64)
    yxi, resp = oracle.nms(D, thr)
    got = np.stack([np.asarray(gpu_raw["y"]), np.asarray(gpu_raw["x"]),
                    np.asarray(gpu_raw["scale"])], 1).astype(np.int64)
    assert got.shape == yxi.shape, "GPU %d candidates, oracle on the GPU cube %d" % (
        len(got), len(yxi))
    assert np.array_equal(got, yxi.astype(np.int64)), "candidate sets differ"
    assert np.array_equal(np.asarray(gpu_raw["response"], np.float64), resp), "responses differ"
    return len(yxi)


def check_exempt_bound(exempt, n_raw, reference=0):
    """Near-tie exemptions on a frame of natural shape: at most 1 % of the
    candidates, rounded up to a whole voxel, or `reference` (the count of
    another path on the same frame, whose own near ties bound the frame's)."""
    allowed = max(math.ceil(MAX_EXEMPT_FRACTION * max(n_raw, 1)), reference)
    assert exempt <= allowed, "%d of %d candidates exempt (at most %d)" % (exempt, n_raw, allowed)


def check_planes(L_gpu, D_gpu, L_orc, D_orc, sigmas, max_abs):
    L_gpu = np.asarray(L_gpu, np.float64)
    D_gpu = np.asarray(D_gpu, np.float64)
    errL = np.abs(L_gpu - L_orc) / (np.abs(L_orc) + max_abs)
    assert errL.max() <= PLANE_RTOL, "L plane error %.3g" % errL.max()
    k = D_orc.shape[0]
    worst = 0.0
    for i in range(k):
        e = np.abs(D_gpu[i] - D_orc[i]) / (np.abs(D_orc[i]) + sigmas[i] * max_abs)
        worst = max(worst, float(e.max()))
    assert worst <= PLANE_RTOL, "D plane error %.3g" % worst
    return float(errL.max()), worst


def neighbour_max_excluding(D, i, y, x):
    k, H, W = D.shape
    m = -np.inf
    for ii in range(max(0, i - 1), min(k, i + 2)):
        for yy in range(max(0, y - 1), min(H, y + 2)):
            for xx in range(max(0, x - 1), min(W, x + 2)):
                if (ii, yy, xx) != (i, y, x):
                    m = max(m, D[ii, yy, xx])
    return m


def check_candidates(gpu_raw, D_orc, thr, sigmas, max_abs):
    """gpu_raw: blob array (y, x, scale, sigma, response) before pruning.
    Returns the number of exempt voxels."""
    yxi, resp = oracle.nms(D_orc, thr)
    o = {(int(a), int(b), int(c)): r for (a, b, c), r in zip(yxi, resp)}
    g = {(int(b["y"]), int(b["x"]), int(b["scale"])): float(b["response"]) for b in gpu_raw}
    assert len(g) == len(gpu_raw), "duplicate GPU candidates"
    exempt = 0
    for v in set(g) ^ set(o):
        y, x, i = v
        d = D_orc[i, y, x]
        delta = MARGIN * sigmas[i] * max_abs
        near_tie = abs(d - neighbour_max_excluding(D_orc, i, y, x)) < delta
        near_thr = abs(d - thr) < delta
        assert near_tie or near_thr, "voxel %s only on %s side (D=%.9g)" % (
            v, "GPU" if v in g else "oracle", d)
        exempt += 1
    for v in set(g) & set(o):
        y, x, i = v
        assert abs(g[v] - o[v]) <= PLANE_RTOL * (abs(o[v]) + sigmas[i] * max_abs), v
    if len(gpu_raw):
        assert np.all(gpu_raw["sigma"] == np.asarray(sigmas, np.float32)[gpu_raw["scale"]])
    return exempt


def check_pruned(gpu_pruned, gpu_raw, D_orc, thr, sigmas, overlap, exempt):
    """With no exempt voxels the pruned list must equal the oracle's; with
    some, the oracle's pruning of the GPU's own raw list must equal it."""
    if exempt == 0:
        yxi, _ = oracle.nms(D_orc, thr)
        raw_y, raw_x, raw_i = yxi[:, 0], yxi[:, 1], yxi[:, 2]
    else:
        raw_y, raw_x, raw_i = gpu_raw["y"], gpu_raw["x"], gpu_raw["scale"]
    keep = oracle.prune(raw_y, raw_x, np.asarray(sigmas)[raw_i], overlap)
    exp = list(zip(raw_y[keep].tolist(), raw_x[keep].tolist(), raw_i[keep].tolist()))
    got = list(zip(gpu_pruned["y"].tolist(), gpu_pruned["x"].tolist(), gpu_pruned["scale"].tolist()))
    assert got == exp
