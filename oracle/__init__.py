"""FP64 CPU oracle of the Difference-of-Gaussians blob detector.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the GPU library never does, and the
two share no code.  The arithmetic lives in ``dog_oracle.c`` (plain C, FP64);
this module is argument marshalling through ctypes.

Every function follows arXiv:2010.08486: the scale space of Sec. 3, the sigma
ladder of Sec. 4 Eq. 1 (geometric form, reading R1 in ``dog_oracle.c``), the
truncated Gaussian kernels of Sec. 4.1, the scaled adjacent differences of
Sec. 4 Eq. 2-3, the 3x3x3 local-maximum search of Sec. 4 with the Thresh mask
of Sec. 4.1, and the overlap pruning of Sec. 4.1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dog_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile dog_oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
             "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    vp = ctypes.c_void_p
    sig = {
        "orc_set_threads": (None, [ctypes.c_int]),
        "orc_get_threads": (ctypes.c_int, []),
        "orc_num_dog_planes": (ctypes.c_int, [dbl, dbl, dbl]),
        "orc_sigmas_geometric": (None, [dbl, dbl, ctypes.c_int, vp]),
        "orc_sigmas_arithmetic": (None, [dbl, dbl, ctypes.c_int, vp]),
        "orc_radius": (ctypes.c_int, [dbl, dbl]),
        "orc_weights": (None, [dbl, ctypes.c_int, vp]),
        "orc_reflect": (i64, [i64, i64]),
        "orc_blur": (None, [vp, i64, i64, dbl, dbl, vp, vp]),
        "orc_planes_sigmas": (ctypes.c_int, [vp, i64, i64, i64, ctypes.c_int, vp, dbl, vp, vp]),
        "orc_planes": (ctypes.c_int, [vp, i64, i64, i64, dbl, dbl, dbl, dbl, vp, vp]),
        "orc_neigh_max": (dbl, [vp, ctypes.c_int, i64, i64, ctypes.c_int, i64, i64]),
        "orc_nms": (i64, [vp, ctypes.c_int, i64, i64, dbl, vp, vp, i64]),
        "orc_lens_area": (dbl, [dbl, dbl, dbl]),
        "orc_overlap_fraction": (dbl, [dbl, dbl, dbl, dbl, dbl, dbl]),
        "orc_prune": (i64, [i64, vp, vp, vp, dbl, vp]),
        "orc_prune_coalesce": (i64, [i64, vp, vp, vp, dbl, vp, vp]),
        "orc_preprocess": (ctypes.c_int, [vp, i64, i64, i64, dbl, dbl, vp, vp, vp]),
        "orc_radius_histogram": (None, [ctypes.c_int, vp, i64, vp, vp]),
        "orc_detect": (i64, [vp, i64, i64, i64, dbl, dbl, dbl, dbl, dbl, dbl,
                             vp, vp, vp, i64, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def num_dog_planes(smin: float, smax: float, ratio: float) -> int:
    """k, the number of DoG planes of the geometric ladder."""
    return int(_load().orc_num_dog_planes(smin, smax, ratio))


def sigmas_geometric(smin: float, smax: float, ratio: float) -> np.ndarray:
    """The k+1 Gaussian standard deviations smin*ratio^i."""
    k = num_dog_planes(smin, smax, ratio)
    out = np.empty(k + 1, np.float64)
    _load().orc_sigmas_geometric(smin, ratio, k, _p(out))
    return out


def sigmas_arithmetic(smin: float, smax: float, n_bin: int) -> np.ndarray:
    """Sec. 4, Eq. 1: n_bin+1 equally spaced standard deviations."""
    out = np.empty(n_bin + 1, np.float64)
    _load().orc_sigmas_arithmetic(smin, smax, int(n_bin), _p(out))
    return out


def radius(sigma: float, truncate: float = 4.0) -> int:
    return int(_load().orc_radius(sigma, truncate))


def weights(sigma: float, r: int) -> np.ndarray:
    """Truncated normalised Gaussian, index j+r for j=-r..r."""
    w = np.empty(2 * r + 1, np.float64)
    _load().orc_weights(sigma, int(r), _p(w))
    return w


def reflect(t: int, n: int) -> int:
    return int(_load().orc_reflect(int(t), int(n)))


def blur(img: np.ndarray, sigma: float, truncate: float = 4.0) -> np.ndarray:
    """Separable truncated Gaussian blur of a float64 image (reflect borders)."""
    a = np.ascontiguousarray(img, dtype=np.float64)
    H, W = a.shape
    tmp = np.empty_like(a)
    out = np.empty_like(a)
    _load().orc_blur(_p(a), H, W, sigma, truncate, _p(tmp), _p(out))
    return out


def _as_f32(image) -> np.ndarray:
    a = np.asarray(image)
    if a.dtype != np.float32:
        raise TypeError("oracle takes fp32 images, got %s" % a.dtype)
    if a.ndim != 2:
        raise ValueError("image must be 2-D")
    return np.ascontiguousarray(a)


def planes_sigmas(image: np.ndarray, sigmas, truncate: float = 4.0):
    """L (n_g planes) and D (n_g-1 planes) for an explicit sigma list."""
    a = _as_f32(image)
    s = np.ascontiguousarray(sigmas, dtype=np.float64)
    H, W = a.shape
    n_g = len(s)
    L = np.empty((n_g, H, W), np.float64)
    D = np.empty((n_g - 1, H, W), np.float64)
    rc = _load().orc_planes_sigmas(_p(a), H, W, W, n_g, _p(s), truncate, _p(L), _p(D))
    if rc != 0:
        raise ValueError("bad oracle input")
    return L, D


def planes(image: np.ndarray, smin: float, smax: float, ratio: float, truncate: float = 4.0):
    """Return (L, D, sigmas) for the geometric ladder."""
    s = sigmas_geometric(smin, smax, ratio)
    L, D = planes_sigmas(image, s, truncate)
    return L, D, s


def neigh_max(D: np.ndarray, i: int, y: int, x: int) -> float:
    d = np.ascontiguousarray(D, dtype=np.float64)
    k, H, W = d.shape
    return float(_load().orc_neigh_max(_p(d), k, H, W, int(i), int(y), int(x)))


def nms(D: np.ndarray, threshold: float):
    """Local maxima above threshold: (yxi int32 [n,3], response float64 [n])."""
    d = np.ascontiguousarray(D, dtype=np.float64)
    k, H, W = d.shape
    lib = _load()
    n = int(lib.orc_nms(_p(d), k, H, W, threshold, None, None, 0))
    yxi = np.empty((max(n, 1), 3), np.int32)
    resp = np.empty(max(n, 1), np.float64)
    lib.orc_nms(_p(d), k, H, W, threshold, _p(yxi), _p(resp), n)
    return yxi[:n], resp[:n]


def lens_area(d: float, r1: float, r2: float) -> float:
    return float(_load().orc_lens_area(d, r1, r2))


def overlap_fraction(y1, x1, s1, y2, x2, s2) -> float:
    return float(_load().orc_overlap_fraction(y1, x1, s1, y2, x2, s2))


def prune(y, x, sigma, overlap: float, coalesce: bool = False):
    """Keep mask (bool) after overlap pruning of blobs given in (y, x, scale)
    order.  With coalesce (Sec. 4.1, averaging the radius), returns
    (keep mask, final sigma of every blob)."""
    yy = np.ascontiguousarray(y, dtype=np.int32)
    xx = np.ascontiguousarray(x, dtype=np.int32)
    ss = np.ascontiguousarray(sigma, dtype=np.float64)
    n = len(yy)
    keep = np.empty(max(n, 1), np.uint8)
    if coalesce:
        out = np.empty(max(n, 1), np.float64)
        _load().orc_prune_coalesce(n, _p(yy), _p(xx), _p(ss), overlap, _p(keep), _p(out))
        return keep[:n].astype(bool), out[:n]
    _load().orc_prune(n, _p(yy), _p(xx), _p(ss), overlap, _p(keep))
    return keep[:n].astype(bool)


def preprocess(image: np.ndarray, sigma: float = 1.0, saturated: float = 0.0035):
    """Preprocessing of Sec. 4.1 (reading R11): (stretched output, smoothed
    image, lo, hi), all FP64."""
    a = _as_f32(image)
    H, W = a.shape
    out = np.empty((H, W), np.float64)
    sm = np.empty((H, W), np.float64)
    lh = np.empty(2, np.float64)
    if _load().orc_preprocess(_p(a), H, W, W, sigma, saturated, _p(sm), _p(out), _p(lh)) != 0:
        raise ValueError("bad oracle input")
    return out, sm, float(lh[0]), float(lh[1])


def radius_histogram(ladder, blob_sigma) -> np.ndarray:
    """Counts of blob radii per ladder radius sqrt(2)*sigma_i (nearest
    centre; reading R12).  ladder: the k DoG-scale sigmas."""
    lad = np.ascontiguousarray(ladder, dtype=np.float64)
    bs = np.ascontiguousarray(blob_sigma, dtype=np.float64)
    out = np.empty(len(lad), np.int64)
    _load().orc_radius_histogram(len(lad), _p(lad), len(bs), _p(bs) if len(bs) else None, _p(out))
    return out


BLOB_DTYPE = np.dtype([("y", np.int32), ("x", np.int32), ("scale", np.int32),
                       ("sigma", np.float64), ("response", np.float64)])


def detect(image: np.ndarray, sigma_min: float, sigma_max: float, sigma_ratio: float = 1.6,
           threshold: float = 0.1, overlap: float = 0.5, truncate: float = 4.0,
           return_raw: bool = False):
    """Whole detector: blobs after pruning as a structured array sorted by
    (y, x, scale).  With return_raw, also the blobs before pruning and the
    DoG cube."""
    a = _as_f32(image)
    L, D, s = planes(a, sigma_min, sigma_max, sigma_ratio, truncate)
    yxi, resp = nms(D, threshold)
    raw = np.empty(len(resp), BLOB_DTYPE)
    raw["y"], raw["x"], raw["scale"] = yxi[:, 0], yxi[:, 1], yxi[:, 2]
    raw["sigma"] = s[yxi[:, 2]] if len(resp) else np.empty(0)
    raw["response"] = resp
    keep = prune(raw["y"], raw["x"], raw["sigma"], overlap)
    out = raw[keep]
    if return_raw:
        return out, raw, D, s
    return out


def detect_c(image: np.ndarray, sigma_min: float, sigma_max: float, sigma_ratio: float = 1.6,
             threshold: float = 0.1, overlap: float = 0.5, truncate: float = 4.0,
             cap: int = 1 << 16):
    """The same detector run entirely inside the C oracle (one call); used for
    the CPU-baseline timing.  Returns the pruned blob array."""
    a = _as_f32(image)
    H, W = a.shape
    lib = _load()
    while True:
        yxi = np.empty((cap, 3), np.int32)
        sig = np.empty(cap, np.float64)
        resp = np.empty(cap, np.float64)
        nraw = ctypes.c_int64(0)
        m = int(lib.orc_detect(_p(a), H, W, W, sigma_min, sigma_max, sigma_ratio,
                               threshold, overlap, truncate, _p(yxi), _p(sig), _p(resp),
                               cap, ctypes.byref(nraw)))
        if m < 0:
            raise ValueError("bad oracle input")
        if m <= cap:
            break
        cap = m
    out = np.empty(m, BLOB_DTYPE)
    out["y"], out["x"], out["scale"] = yxi[:m, 0], yxi[:m, 1], yxi[:m, 2]
    out["sigma"], out["response"] = sig[:m], resp[:m]
    return out
