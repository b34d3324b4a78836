"""Python binding of libdog.so, the MI355X Difference-of-Gaussians blob detector.

Argument marshalling only: every step of the detector runs in the library's
HIP kernels and host runtime (see include/dog.h).  The names mirror the C ABI.
PyTorch is used for device memory and streams when device tensors are passed.

    import paper_2010_08486_amd as dog
    blobs = dog.detect(img, 1.0, 30.0, 1.6, threshold=0.05, overlap=0.5)
    ctx = dog.Context()
    blobs = ctx.detect_device(cuda_tensor, dog.Params(1, 30, 1.6, 0.05, 0.5))
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdog.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dog.h")

DOG_OK, DOG_EINVAL, DOG_ENOMEM, DOG_EDEVICE, DOG_EBUSY, DOG_EAGAIN, DOG_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6

BLOB_DTYPE = np.dtype([("y", np.int32), ("x", np.int32), ("scale", np.int32),
                       ("sigma", np.float32), ("response", np.float32)])


class DogError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class dog_params(ctypes.Structure):
    _fields_ = [("sigma_min", ctypes.c_double), ("sigma_max", ctypes.c_double),
                ("sigma_ratio", ctypes.c_double), ("threshold", ctypes.c_double),
                ("overlap", ctypes.c_double), ("truncate", ctypes.c_double),
                ("ladder", ctypes.c_int32), ("n_bin", ctypes.c_int32),
                ("coalesce", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class dog_blob(ctypes.Structure):
    _fields_ = [("y", ctypes.c_int32), ("x", ctypes.c_int32), ("scale", ctypes.c_int32),
                ("sigma", ctypes.c_float), ("response", ctypes.c_float)]


class dog_frame(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("height", ctypes.c_int64), ("width", ctypes.c_int64),
                ("row_stride", ctypes.c_int64), ("on_device", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class dog_result(ctypes.Structure):
    _fields_ = [("blobs", ctypes.POINTER(dog_blob)), ("count", ctypes.c_int64),
                ("raw_count", ctypes.c_int64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t_arrive_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class dog_server_opts(ctypes.Structure):
    _fields_ = [("max_batch_frames", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("dry_run", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("max_wait_ms", ctypes.c_double),
                ("dry_run_us_per_mpx", ctypes.c_double), ("tune_cache", ctypes.c_char_p),
                ("max_batch_pixels", ctypes.c_int64)]


class dog_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "rejected",
                                               "queued", "running", "batches")] + \
               [(n, ctypes.c_double) for n in ("mean_batch_frames", "p50_ms", "p99_ms", "mean_ms",
                                                "max_ms", "frames_per_s")] + \
               [("reserved_bytes", ctypes.c_uint64), ("peak_reserved_bytes", ctypes.c_uint64),
                ("held_bytes", ctypes.c_uint64), ("peak_held_bytes", ctypes.c_uint64),
                ("admission_waits", ctypes.c_int64)]


@dataclass
class Params:
    """Detector hyper-parameters; defaults follow Sec. 4.1 (threshold 0.1,
    overlap 0.5) and the geometric ladder ratio 1.6 with truncate 4.
    ladder = "arithmetic" takes the paper's Eq. 1 ladder of n_bin + 1 sigmas
    (sigma_ratio unused); coalesce = True merges overlapping blobs by
    averaging the radius instead of removing the smaller one."""
    sigma_min: float = 1.0
    sigma_max: float = 30.0
    sigma_ratio: float = 1.6
    threshold: float = 0.1
    overlap: float = 0.5
    truncate: float = 4.0
    ladder: str = "geometric"
    n_bin: int = 0
    coalesce: bool = False

    @classmethod
    def paper(cls, sigma_min: float = 1.0, sigma_max: float = 30.0, n_bin: int = 10,
              threshold: float = 0.1, overlap: float = 0.5) -> "Params":
        """The paper's own configuration: arithmetic ladder (Eq. 1),
        truncate 5, coalescing by averaging the radius (Sec. 4.1)."""
        return cls(sigma_min, sigma_max, 1.6, threshold, overlap, 5.0, "arithmetic", n_bin, True)

    def c(self) -> dog_params:
        """The C struct (cached while the values stay the same)."""
        if self.ladder not in ("geometric", "arithmetic"):
            raise ValueError("ladder must be 'geometric' or 'arithmetic'")
        key = (self.sigma_min, self.sigma_max, self.sigma_ratio, self.threshold, self.overlap,
               self.truncate, 1 if self.ladder == "arithmetic" else 0, int(self.n_bin),
               1 if self.coalesce else 0, 0)
        cached = self.__dict__.get("_c")
        if cached is None or cached[0] != key:
            cached = (key, dog_params(*key))
            self.__dict__["_c"] = cached
        return cached[1]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libdog.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdog.so is not built: run `python -m paper_2010_08486_amd.build` "
                           "(the detector has no non-HIP fallback)")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, u64, vp, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double
    pblob = ctypes.POINTER(ctypes.POINTER(dog_blob))
    pi64 = ctypes.POINTER(i64)
    sig = {
        "dog_detect": (i32, [vp, i64, i64, i64, dbl, dbl, dbl, dbl, dbl, pblob, pi64]),
        "dog_blobs_free": (None, [vp]),
        "dog_last_error": (ctypes.c_char_p, []),
        "dog_version": (ctypes.c_char_p, []),
        "dog_context_create": (i32, [ctypes.c_int, u64, ctypes.POINTER(vp)]),
        "dog_context_destroy": (None, [vp]),
        "dog_footprint": (i32, [ctypes.POINTER(dog_params), i32, pi64, pi64, ctypes.POINTER(u64)]),
        "dog_detect_device": (i32, [vp, vp, i64, i64, i64, ctypes.POINTER(dog_params), vp, pblob, pi64]),
        "dog_detect_device_async": (i32, [vp, vp, i64, i64, i64, ctypes.POINTER(dog_params), vp]),
        "dog_detect_device_finish": (i32, [vp, pblob, pi64]),
        "dog_preprocess": (i32, [vp, vp, i64, i64, i64, dbl, dbl, vp, vp, vp, vp]),
        "dog_preprocess_noalloc": (i32, [vp, i64, i64, i64, dbl, dbl, vp, vp, vp, vp]),
        "dog_detect_batch": (i32, [vp, i32, ctypes.POINTER(dog_frame), ctypes.POINTER(dog_params), vp,
                                   ctypes.POINTER(dog_result)]),
        "dog_results_free": (None, [ctypes.POINTER(dog_result), i32]),
        "dog_debug_planes": (i32, [vp, vp, i64, i64, i64, ctypes.POINTER(dog_params), vp, vp,
                                   ctypes.POINTER(i32)]),
        "dog_debug_candidates": (i32, [vp, vp, i64, i64, i64, ctypes.POINTER(dog_params), pblob, pi64]),
        "dog_plan_info": (i32, [ctypes.POINTER(dog_params), ctypes.POINTER(i32),
                                ctypes.POINTER(dbl), ctypes.POINTER(i32), i32]),
        "dog_prune": (i32, [ctypes.POINTER(dog_params), vp, i64, pi64]),
        "dog_radius_histogram": (i32, [ctypes.POINTER(dog_params), vp, i64, pi64]),
        "dog_prune_device": (i32, [vp, ctypes.POINTER(dog_params), vp, i64, vp, pblob, pi64, pi64]),
        "dog_server_create": (i32, [ctypes.c_int, ctypes.POINTER(dog_params),
                                    ctypes.POINTER(dog_server_opts), ctypes.POINTER(vp)]),
        "dog_server_submit": (i32, [vp, ctypes.POINTER(dog_frame), ctypes.POINTER(u64)]),
        "dog_server_poll": (i32, [vp, u64, ctypes.POINTER(dog_result)]),
        "dog_server_wait": (i32, [vp, u64, ctypes.POINTER(dog_result)]),
        "dog_server_drain": (i32, [vp]),
        "dog_server_stats": (i32, [vp, ctypes.POINTER(dog_stats)]),
        "dog_server_destroy": (None, [vp]),
        "dog_num_variants": (ctypes.c_int, []),
        "dog_variant_info": (ctypes.c_int, [ctypes.c_int] + [ctypes.POINTER(i32)] * 4),
        "dog_set_variant": (ctypes.c_int, [vp, ctypes.c_int]),
        "dog_set_profiling": (ctypes.c_int, [vp, i32]),
        "dog_set_graph_mode": (ctypes.c_int, [vp, i32]),
        "dog_set_batch_grouping": (ctypes.c_int, [vp, i64, i32]),
        "dog_kernel_times": (ctypes.c_int, [vp, ctypes.POINTER(dbl), pi64]),
        "dog_kernel_times_all": (ctypes.c_int, [vp, ctypes.POINTER(dbl), i32, pi64]),
        "dog_set_dct": (ctypes.c_int, [vp, i32]),
        "dog_autotune": (i32, [vp, ctypes.POINTER(dog_params), vp, i64, i64, i64, i32,
                               ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
        "dog_autotune_save": (i32, [vp, ctypes.c_char_p]),
        "dog_autotune_load": (i32, [vp, ctypes.c_char_p]),
        "dog_autotune_choice": (i32, [vp, ctypes.POINTER(dog_params), i64, i64, ctypes.POINTER(i32)]),
        "dog_autotune_transform": (i32, [vp, ctypes.POINTER(dog_params), i64, i64, ctypes.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions declared in include/dog.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dog_[a-z0-9_]+)\s*\(", txt)))


def _check(rc: int) -> None:
    if rc != DOG_OK:
        raise DogError(rc, lib().dog_last_error().decode())


def _blobs(ptr, n: int) -> np.ndarray:
    out = np.empty(n, BLOB_DTYPE)
    if n:
        ctypes.memmove(out.ctypes.data, ptr, n * BLOB_DTYPE.itemsize)
    lib().dog_blobs_free(ctypes.cast(ptr, ctypes.c_void_p))
    return out


def version() -> str:
    return lib().dog_version().decode()


def detect(image: np.ndarray, sigma_min: float, sigma_max: float, sigma_ratio: float = 1.6,
           threshold: float = 0.1, overlap: float = 0.5) -> np.ndarray:
    """dog_detect on a host fp32 image (2-D, row stride taken from the array)."""
    a = np.asarray(image)
    if a.dtype != np.float32 or a.ndim != 2:
        raise TypeError("image must be a 2-D float32 array")
    if a.strides[1] != 4 or a.strides[0] % 4:
        a = np.ascontiguousarray(a)
    H, W = a.shape
    p = ctypes.POINTER(dog_blob)()
    n = ctypes.c_int64(0)
    _check(lib().dog_detect(a.ctypes.data, H, W, a.strides[0] // 4, sigma_min, sigma_max, sigma_ratio,
                            threshold, overlap, ctypes.byref(p), ctypes.byref(n)))
    return _blobs(p, n.value)


def num_variants() -> int:
    return int(lib().dog_num_variants())


def variant_info(v: int) -> dict:
    vals = [ctypes.c_int32() for _ in range(4)]
    _check(lib().dog_variant_info(v, *[ctypes.byref(x) for x in vals]))
    return dict(zip(("S", "waves", "strips", "nms_rows"), (x.value for x in vals)))


def _tensor_image(t):
    """(pointer, H, W, row_stride) of a 2-D float32 CUDA tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or t.stride(1) != 1:
        raise TypeError("expected a 2-D float32 tensor with unit column stride")
    return t.data_ptr(), t.shape[0], t.shape[1], t.stride(0)


def _stream_ptr(stream=None, device=None):
    """The HIP stream the library runs on: the given torch stream, else the
    current one of `device` (0 = the null stream), so the detector is ordered
    after the work that produced the input."""
    import torch
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return ctypes.c_void_p(raw(torch.cuda.current_device() if device is None else device))
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """dog_context: device workspace, pinned staging and a stream."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self._h = ctypes.c_void_p()
        self._inflight = None
        _check(lib().dog_context_create(device, budget_bytes, ctypes.byref(self._h)))
        self.device = device

    def close(self) -> None:
        if self._h:
            lib().dog_context_destroy(self._h)  # waits for a launch not yet finished
            self._h = ctypes.c_void_p()
        self._inflight = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def set_variant(self, v: int) -> None:
        _check(lib().dog_set_variant(self._h, v))

    def autotune(self, image, params: Params, reps: int = 5):
        """dog_autotune on a 2-D float32 CUDA tensor.  Returns (winning
        variant, list of mean microseconds per variant)."""
        import torch
        ptr, H, W, st = _tensor_image(image)
        torch.cuda.synchronize(image.device)
        nv = num_variants()
        us = (ctypes.c_double * nv)()
        v = ctypes.c_int32(-1)
        prm = params.c()
        _check(lib().dog_autotune(self._h, ctypes.byref(prm), ptr, H, W, st, reps, ctypes.byref(v), us))
        return v.value, list(us)

    def autotune_save(self, path: str) -> None:
        _check(lib().dog_autotune_save(self._h, os.fsencode(path)))

    def autotune_load(self, path: str) -> None:
        _check(lib().dog_autotune_load(self._h, os.fsencode(path)))

    def autotune_transform(self, params: Params, height: int, width: int) -> int:
        """The transform threshold (kernel taps) used for frames of this shape."""
        v = ctypes.c_int32(0)
        prm = params.c()
        _check(lib().dog_autotune_transform(self._h, ctypes.byref(prm), height, width, ctypes.byref(v)))
        return v.value

    def autotune_choice(self, params: Params, height: int, width: int) -> int:
        v = ctypes.c_int32(-1)
        prm = params.c()
        _check(lib().dog_autotune_choice(self._h, ctypes.byref(prm), height, width, ctypes.byref(v)))
        return v.value

    def set_batch_grouping(self, max_group_pixels: int, lanes: int = 3) -> None:
        """Frames per launch sequence in detect_batch (by pixels; 0 = one
        sequence) and how many sequences run at once."""
        _check(lib().dog_set_batch_grouping(self._h, int(max_group_pixels), int(lanes)))

    def set_graph_mode(self, on: bool) -> None:
        _check(lib().dog_set_graph_mode(self._h, 1 if on else 0))

    def set_profiling(self, on: bool) -> None:
        _check(lib().dog_set_profiling(self._h, 1 if on else 0))

    def kernel_times(self):
        """(ms per kernel summed [pass1, pass2, nms], number of launch sequences)."""
        ms = (ctypes.c_double * 3)()
        n = ctypes.c_int64(0)
        _check(lib().dog_kernel_times(self._h, ms, ctypes.byref(n)))
        return list(ms), n.value

    KERNEL_NAMES = ("pass1", "pass2", "nms", "fft1", "fft2")

    def kernel_times_all(self):
        """(ms per kernel summed, in KERNEL_NAMES order, number of launch sequences)."""
        ms = (ctypes.c_double * len(self.KERNEL_NAMES))()
        n = ctypes.c_int64(0)
        _check(lib().dog_kernel_times_all(self._h, ms, len(ms), ctypes.byref(n)))
        return list(ms), n.value

    def set_dct(self, min_taps: int) -> None:
        """dog_set_dct: planes whose kernels have at least min_taps taps are
        blurred in the cosine-transform domain (power-of-two frames); 0 = never,
        -1 = the autotuner's choice per frame shape (the default)."""
        _check(lib().dog_set_dct(self._h, int(min_taps)))

    def detect_device(self, image, params: Params, stream=None) -> np.ndarray:
        ptr, H, W, st = _tensor_image(image)
        p = ctypes.POINTER(dog_blob)()
        n = ctypes.c_int64(0)
        prm = params.c()
        _check(lib().dog_detect_device(self._h, ptr, H, W, st, ctypes.byref(prm),
                                       _stream_ptr(stream, image.device.index),
                                       ctypes.byref(p), ctypes.byref(n)))
        return _blobs(p, n.value)

    def detect_device_async(self, image, params: Params, stream=None) -> None:
        """Queue the detector on `image` and return; `finish()` collects the
        blobs.  The tensor is held until then."""
        ptr, H, W, st = _tensor_image(image)
        prm = params.c()
        _check(lib().dog_detect_device_async(self._h, ptr, H, W, st, ctypes.byref(prm),
                                             _stream_ptr(stream, image.device.index)))
        self._inflight = image

    def finish(self) -> np.ndarray:
        """Blobs of the launch queued by `detect_device_async`."""
        p = ctypes.POINTER(dog_blob)()
        n = ctypes.c_int64(0)
        try:
            _check(lib().dog_detect_device_finish(self._h, ctypes.byref(p), ctypes.byref(n)))
        finally:
            self._inflight = None
        return _blobs(p, n.value)

    def preprocess(self, image, sigma: float = 1.0, saturated: float = 0.0035, out=None,
                   smoothed=None, stream=None, limits: bool = False):
        """Smoothing and contrast stretch of a device image (Sec. 4.1): returns
        the stretched CUDA tensor, and (lo, hi) when `limits` is set."""
        import torch
        ptr, H, W, st = _tensor_image(image)
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=image.device)
        lim = (ctypes.c_float * 2)() if limits else None
        _check(lib().dog_preprocess(self._h, ptr, H, W, st, float(sigma), float(saturated),
                                    out.data_ptr(),
                                    smoothed.data_ptr() if smoothed is not None else None,
                                    lim, _stream_ptr(stream, image.device.index)))
        if limits:
            return out, (lim[0], lim[1])
        return out

    def debug_candidates(self, image, params: Params) -> np.ndarray:
        import torch
        ptr, H, W, st = _tensor_image(image)
        torch.cuda.synchronize(image.device)
        p = ctypes.POINTER(dog_blob)()
        n = ctypes.c_int64(0)
        prm = params.c()
        _check(lib().dog_debug_candidates(self._h, ptr, H, W, st, ctypes.byref(prm),
                                          ctypes.byref(p), ctypes.byref(n)))
        return _blobs(p, n.value)

    def prune_device(self, blobs, params: Params, stream=None):
        """dog_prune_device: sort, overlap-prune and histogram a blob list on
        the GPU.  blobs: a BLOB_DTYPE array (copied to the device first) or a
        CUDA uint8 tensor holding such records.  Returns (survivors,
        histogram of k int64)."""
        import torch
        if isinstance(blobs, torch.Tensor):
            d = blobs
            n = d.numel() // BLOB_DTYPE.itemsize
        else:
            b = np.ascontiguousarray(np.array(blobs, dtype=BLOB_DTYPE))
            n = len(b)
            d = torch.from_numpy(b.view(np.uint8).reshape(-1)).cuda()
        k = plan_info(params)["k"]
        hist = np.zeros(k, np.int64)
        p = ctypes.POINTER(dog_blob)()
        cnt = ctypes.c_int64(0)
        prm = params.c()
        st = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _check(lib().dog_prune_device(self._h, ctypes.byref(prm), d.data_ptr() if n else None, n,
                                      st, ctypes.byref(p), ctypes.byref(cnt),
                                      hist.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return _blobs(p, cnt.value), hist

    def debug_planes(self, image, params: Params):
        """(L, D) as CUDA tensors: (k+1, H, W) and (k, H, W) fp32."""
        import torch
        ptr, H, W, st = _tensor_image(image)
        k = plan_info(params)["k"]
        L = torch.empty((k + 1, H, W), dtype=torch.float32, device=image.device)
        D = torch.empty((k, H, W), dtype=torch.float32, device=image.device)
        kk = ctypes.c_int32(0)
        prm = params.c()
        torch.cuda.synchronize(image.device)
        _check(lib().dog_debug_planes(self._h, ptr, H, W, st, ctypes.byref(prm), L.data_ptr(),
                                      D.data_ptr(), ctypes.byref(kk)))
        assert kk.value == k
        return L, D

    def detect_batch(self, frames, params: Params, stream=None):
        """dog_detect_batch over a list of 2-D float32 frames: numpy arrays
        (host), pinned CPU tensors (page-locked host, uploaded by DMA) or CUDA
        tensors (device).  Returns (list of blob arrays, list of raw counts)."""
        n = len(frames)
        arr = (dog_frame * max(n, 1))()
        keep = []
        for i, fr in enumerate(frames):
            if isinstance(fr, np.ndarray):
                a = fr
                if a.dtype != np.float32 or a.ndim != 2:
                    raise TypeError("frames must be 2-D float32")
                if a.strides[1] != 4 or a.strides[0] % 4:
                    a = np.ascontiguousarray(a)
                keep.append(a)
                arr[i] = dog_frame(a.ctypes.data, a.shape[0], a.shape[1], a.strides[0] // 4, 0, 0)
            elif not fr.is_cuda:
                import torch
                if (not fr.is_pinned() or fr.dtype != torch.float32 or fr.dim() != 2
                        or fr.stride(1) != 1):
                    raise TypeError("CPU tensor frames must be pinned 2-D float32 with unit column stride")
                arr[i] = dog_frame(fr.data_ptr(), fr.shape[0], fr.shape[1], fr.stride(0), 2, 0)
            else:
                ptr, H, W, st = _tensor_image(fr)
                arr[i] = dog_frame(ptr, H, W, st, 1, 0)
        res = (dog_result * max(n, 1))()
        prm = params.c()
        s = _stream_ptr(stream) if any(not isinstance(f, np.ndarray) for f in frames) else None
        rc = lib().dog_detect_batch(self._h, n, arr, ctypes.byref(prm), s, res)
        out, raw = [], []
        for i in range(n):
            if res[i].status != DOG_OK:
                lib().dog_results_free(res, n)
                _check(rc if rc != DOG_OK else res[i].status)
            b = np.empty(res[i].count, BLOB_DTYPE)
            if res[i].count:
                ctypes.memmove(b.ctypes.data, res[i].blobs, res[i].count * BLOB_DTYPE.itemsize)
            out.append(b)
            raw.append(int(res[i].raw_count))
        lib().dog_results_free(res, n)
        _check(rc)
        return out, raw


def preprocess_noalloc(image, out, smoothed=None, limits=None, sigma: float = 1.0,
                       saturated: float = 0.0035, stream=None) -> None:
    """dog_preprocess_noalloc: the preprocessing of Context.preprocess into
    caller-allocated CUDA tensors, with no allocation by the library (its
    scratch is a static device array of the current GPU).  out (and
    smoothed, if given): float32 tensors of the image's shape with dense
    rows; limits: a float32 CUDA tensor of 2 elements receiving (lo, hi).
    Queued on `stream` (default: the current stream); nothing is waited for."""
    import torch
    ptr, H, W, st = _tensor_image(image)
    for t in (out, smoothed):
        if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda or
                              t.dtype != torch.float32 or tuple(t.shape) != (H, W) or
                              not t.is_contiguous()):
            raise TypeError("out and smoothed must be dense float32 CUDA tensors of the image's shape")
    if limits is not None and (not isinstance(limits, torch.Tensor) or not limits.is_cuda or
                               limits.dtype != torch.float32 or limits.numel() < 2 or
                               not limits.is_contiguous()):
        raise TypeError("limits must be a float32 CUDA tensor of 2 elements")
    _check(lib().dog_preprocess_noalloc(ptr, H, W, st, float(sigma), float(saturated),
                                        out.data_ptr(),
                                        smoothed.data_ptr() if smoothed is not None else None,
                                        limits.data_ptr() if limits is not None else None,
                                        _stream_ptr(stream, image.device.index)))


def prune(params: Params, blobs: np.ndarray) -> np.ndarray:
    """dog_prune: sort and overlap-prune a blob array (host step)."""
    b = np.ascontiguousarray(np.array(blobs, dtype=BLOB_DTYPE))
    n = ctypes.c_int64(0)
    prm = params.c()
    _check(lib().dog_prune(ctypes.byref(prm), b.ctypes.data, len(b), ctypes.byref(n)))
    return b[:n.value].copy()


def radius_histogram(params: Params, blobs: np.ndarray) -> np.ndarray:
    """Blob counts per ladder radius sqrt(2)*sigma_i (nearest centre), k bins."""
    b = np.ascontiguousarray(blobs, dtype=BLOB_DTYPE)
    k = plan_info(params)["k"]
    out = np.zeros(k, np.int64)
    prm = params.c()
    _check(lib().dog_radius_histogram(ctypes.byref(prm), b.ctypes.data if len(b) else None,
                                      len(b), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out


def plan_info(params: Params) -> dict:
    """The library's ladder for these parameters: k, sigmas (k+1), radii (k+1)."""
    cap = 64
    k = ctypes.c_int32(0)
    sig = (ctypes.c_double * cap)()
    rad = (ctypes.c_int32 * cap)()
    prm = params.c()
    _check(lib().dog_plan_info(ctypes.byref(prm), ctypes.byref(k), sig, rad, cap))
    n = k.value + 1
    return {"k": k.value, "sigmas": np.array(sig[:n]), "radii": np.array(rad[:n])}


def footprint(params: Params, shapes) -> int:
    hs = (ctypes.c_int64 * max(len(shapes), 1))(*[s[0] for s in shapes])
    ws = (ctypes.c_int64 * max(len(shapes), 1))(*[s[1] for s in shapes])
    out = ctypes.c_uint64(0)
    prm = params.c()
    _check(lib().dog_footprint(ctypes.byref(prm), len(shapes), hs, ws, ctypes.byref(out)))
    return int(out.value)


class Server:
    """dog_server: continuous batching of host frames (see include/dog.h)."""

    def __init__(self, params: Params, device: int = 0, max_batch_frames: int = 16,
                 slots: int = 3, queue_capacity: int = 4096, hbm_budget_bytes: int = 0,
                 max_wait_ms: float = 0.0, dry_run: bool = False,
                 dry_run_us_per_mpx: float = 0.0, tune_cache: str | None = None,
                 max_batch_pixels: int = 0):
        self._h = ctypes.c_void_p()
        self._held = {}
        opts = dog_server_opts(max_batch_frames, slots, queue_capacity, 1 if dry_run else 0,
                               hbm_budget_bytes, max_wait_ms, dry_run_us_per_mpx,
                               os.fsencode(tune_cache) if tune_cache else None,
                               max_batch_pixels)
        prm = params.c()
        _check(lib().dog_server_create(device, ctypes.byref(prm), ctypes.byref(opts),
                                       ctypes.byref(self._h)))

    def close(self) -> None:
        if self._h:
            lib().dog_server_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, frame) -> int:
        """Queue a 2-D float32 frame: a numpy array (copied at once) or a CUDA
        tensor (borrowed: held here until its result is taken)."""
        if isinstance(frame, np.ndarray):
            a = frame
            if a.dtype != np.float32 or a.ndim != 2:
                raise TypeError("frames must be 2-D float32 arrays")
            if a.strides[1] != 4 or a.strides[0] % 4:
                a = np.ascontiguousarray(a)
            fr = dog_frame(a.ctypes.data, a.shape[0], a.shape[1], a.strides[0] // 4, 0, 0)
            hold = None
        else:
            ptr, H, W, st = _tensor_image(frame)
            fr = dog_frame(ptr, H, W, st, 1, 0)
            hold = frame
            import torch
            torch.cuda.current_stream(frame.device).synchronize()  # pixels written before the server reads
        t = ctypes.c_uint64(0)
        _check(lib().dog_server_submit(self._h, ctypes.byref(fr), ctypes.byref(t)))
        if hold is not None:
            self._held[int(t.value)] = hold
        return int(t.value)

    @staticmethod
    def _unpack(r: dog_result):
        b = np.empty(r.count, BLOB_DTYPE)
        if r.count:
            ctypes.memmove(b.ctypes.data, r.blobs, r.count * BLOB_DTYPE.itemsize)
        lib().dog_blobs_free(ctypes.cast(r.blobs, ctypes.c_void_p))
        info = {"status": int(r.status), "raw_count": int(r.raw_count),
                "t_arrive_ns": int(r.t_arrive_ns), "t_done_ns": int(r.t_done_ns)}
        return b, info

    def poll(self, ticket: int):
        """(blobs, info) if done, None if still pending; raises on unknown tickets."""
        r = dog_result()
        rc = lib().dog_server_poll(self._h, ticket, ctypes.byref(r))
        if rc == DOG_EAGAIN:
            return None
        self._held.pop(ticket, None)
        _check(rc)
        return self._unpack(r)

    def wait(self, ticket: int):
        r = dog_result()
        rc = lib().dog_server_wait(self._h, ticket, ctypes.byref(r))
        self._held.pop(ticket, None)
        _check(rc)
        return self._unpack(r)

    def drain(self) -> None:
        _check(lib().dog_server_drain(self._h))

    def stats(self) -> dict:
        st = dog_stats()
        _check(lib().dog_server_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in dog_stats._fields_}
