"""Thin ctypes binding of libfse.so (the C ABI in include/fse.h).

Functions keep the ABI's names and only marshal arguments; all work happens
in the library's HIP kernels.  PyTorch supplies device memory and streams.
Loading fails loudly when the built library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfse.so")

FSE_OK = 0
FSE_ERR_INVALID_ARG = -1
FSE_ERR_UNSUPPORTED = -2
FSE_ERR_BUDGET = -3
FSE_ERR_OUT_OF_MEMORY = -4
FSE_ERR_DEVICE = -5
FSE_ERR_TIMEOUT = -6
FSE_ERR_NOT_FOUND = -7
FSE_ERR_BUSY = -8
FSE_ERR_CANCELLED = -9

FSE_PREC_F64, FSE_PREC_F32, FSE_PREC_BF16X3 = 0, 1, 2
FSE_SCHED_PERSISTENT, FSE_SCHED_WAVEFRONT, FSE_SCHED_PER_BLOCK = 0, 1, 2
FSE_WHOLE, FSE_TILED, FSE_TILED_VERTICAL = 0, 1, 2
FSE_ORDER_RASTER, FSE_ORDER_OPTIMIZED = 0, 1
FSE_MAX_CLASSES = 3

EXPORTED = [
    "fse_status_string", "fse_params_default", "fse_plan_tiles", "fse_extrapolate", "fse_extrapolate_batch",
    "fse_last_stats", "fse_release", "fse_serve_create", "fse_serve_submit", "fse_serve_poll", "fse_serve_wait",
    "fse_serve_destroy", "fse_plan_create", "fse_plan_execute", "fse_plan_destroy", "fse_plan_stats",
    "fse_autotune", "fse_plan_tiles_vertical", "fse_serve_cancel", "fse_extrapolate_noalloc",
    "fse_autotune_overlapped",
]

FSE_NOALLOC_SCRATCH_BYTES = 32 << 20


class fse_image_t(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch", ctypes.c_int64)]


class fse_mask_t(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch", ctypes.c_int64)]


class fse_tile_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("x", "y", "w", "h", "ox", "oy", "ow", "oh")]


class fse_class_t(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("border", ctypes.c_int32), ("iters", ctypes.c_int32)]


class fse_params_t(ctypes.Structure):
    _fields_ = [
        ("n_classes", ctypes.c_int32),
        ("classes", fse_class_t * FSE_MAX_CLASSES),
        ("rho", ctypes.c_double), ("gamma", ctypes.c_double), ("recon_weight", ctypes.c_double),
        ("precision", ctypes.c_int32), ("schedule", ctypes.c_int32), ("tiling", ctypes.c_int32),
        ("n_tiles", ctypes.c_int32), ("overlap", ctypes.c_int32), ("align", ctypes.c_int32),
        ("workgroups", ctypes.c_int32), ("block_waves", ctypes.c_int32),
        ("trace_sel", ctypes.c_void_p), ("trace_stride", ctypes.c_int32), ("trace_capacity", ctypes.c_int64),
        ("order", ctypes.c_int32),
    ]


class fse_run_stats_t(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("n_lost_pixels", ctypes.c_int64), ("n_degenerate", ctypes.c_int64),
                ("n_jobs", ctypes.c_int64), ("wavefront_keys", ctypes.c_int32), ("host_plan_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("device_error", ctypes.c_int32)]


class fse_serve_config_t(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32), ("device", ctypes.c_int32),
                ("workgroups", ctypes.c_int32)]


class fse_request_stats_t(ctypes.Structure):
    _fields_ = [("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
                ("n_blocks", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded libfse.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfse.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2207_00238_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        st = ctypes.c_int32
        L.fse_status_string.restype = ctypes.c_char_p
        L.fse_status_string.argtypes = [st]
        L.fse_params_default.restype = st
        L.fse_params_default.argtypes = [P(fse_params_t)]
        L.fse_plan_tiles.restype = st
        L.fse_plan_tiles.argtypes = [ctypes.c_int32] * 5 + [P(fse_tile_t)]
        L.fse_plan_tiles_vertical.restype = st
        L.fse_plan_tiles_vertical.argtypes = [ctypes.c_int32] * 5 + [P(fse_tile_t)]
        L.fse_extrapolate.restype = st
        L.fse_extrapolate.argtypes = [P(fse_image_t), P(fse_mask_t), P(fse_params_t), P(fse_image_t), ctypes.c_void_p]
        L.fse_extrapolate_noalloc.restype = st
        L.fse_extrapolate_noalloc.argtypes = [P(fse_image_t), P(fse_mask_t), P(fse_params_t), P(fse_image_t),
                                              ctypes.c_void_p]
        L.fse_extrapolate_batch.restype = st
        L.fse_extrapolate_batch.argtypes = [ctypes.c_int32, P(fse_image_t), P(fse_mask_t), P(fse_params_t),
                                            P(fse_image_t), ctypes.c_void_p]
        L.fse_last_stats.restype = st
        L.fse_last_stats.argtypes = [P(fse_run_stats_t)]
        L.fse_release.restype = st
        L.fse_release.argtypes = []
        L.fse_serve_create.restype = st
        L.fse_serve_create.argtypes = [P(fse_serve_config_t), P(ctypes.c_void_p)]
        L.fse_serve_submit.restype = st
        L.fse_serve_submit.argtypes = [ctypes.c_void_p, P(fse_image_t), P(fse_mask_t), P(fse_params_t),
                                       P(fse_image_t), P(ctypes.c_uint64)]
        L.fse_serve_poll.restype = st
        L.fse_serve_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, P(ctypes.c_int32), P(fse_request_stats_t)]
        L.fse_serve_wait.restype = st
        L.fse_serve_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, P(fse_request_stats_t)]
        L.fse_serve_cancel.restype = st
        L.fse_serve_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.fse_serve_destroy.restype = st
        L.fse_serve_destroy.argtypes = [ctypes.c_void_p]
        L.fse_autotune.restype = st
        L.fse_autotune.argtypes = [ctypes.c_int32, P(fse_image_t), P(fse_mask_t), P(fse_params_t), P(fse_image_t),
                                   ctypes.c_void_p, P(fse_params_t)]
        L.fse_autotune_overlapped.restype = st
        L.fse_autotune_overlapped.argtypes = [ctypes.c_int32, P(fse_image_t), P(fse_mask_t), P(fse_params_t),
                                              P(fse_image_t), ctypes.c_int32, P(fse_params_t)]
        L.fse_plan_create.restype = st
        L.fse_plan_create.argtypes = [ctypes.c_int32, P(fse_mask_t), P(fse_params_t), P(ctypes.c_void_p)]
        L.fse_plan_execute.restype = st
        L.fse_plan_execute.argtypes = [ctypes.c_void_p, P(fse_image_t), P(fse_image_t), ctypes.c_void_p]
        L.fse_plan_destroy.restype = st
        L.fse_plan_destroy.argtypes = [ctypes.c_void_p]
        L.fse_plan_stats.restype = st
        L.fse_plan_stats.argtypes = [ctypes.c_void_p, P(fse_run_stats_t)]
        _lib = L
    return _lib


class FseError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = lib().fse_status_string(status).decode()
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")
        self.status = status


def check(status: int, what: str = "") -> None:
    if status != FSE_OK:
        raise FseError(status, what)


# ---------------------------------------------------------------------------
# ABI entry points (same names, argument marshalling only)
# ---------------------------------------------------------------------------

def fse_params_default(**overrides) -> fse_params_t:
    p = fse_params_t()
    check(lib().fse_params_default(ctypes.byref(p)), "fse_params_default")
    classes = overrides.pop("classes", None)
    if classes is not None:
        p.n_classes = len(classes)
        for i, (B, b, K) in enumerate(classes):
            p.classes[i].block, p.classes[i].border, p.classes[i].iters = B, b, K
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def fse_plan_tiles(W: int, H: int, N: int, d: int, align: int = 1):
    tiles = (fse_tile_t * N)()
    check(lib().fse_plan_tiles(W, H, N, d, align, tiles), "fse_plan_tiles")
    return [((t.x, t.y, t.w, t.h), (t.ox, t.oy, t.ow, t.oh)) for t in tiles]


def fse_plan_tiles_vertical(W: int, H: int, N: int, d: int, align: int = 1):
    tiles = (fse_tile_t * N)()
    check(lib().fse_plan_tiles_vertical(W, H, N, d, align, tiles), "fse_plan_tiles_vertical")
    return [((t.x, t.y, t.w, t.h), (t.ox, t.oy, t.ow, t.oh)) for t in tiles]


def _image(t) -> fse_image_t:
    assert t.dim() == 2 and t.is_cuda and t.stride(1) == 1
    import torch
    assert t.dtype == torch.float32
    return fse_image_t(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0))


def _mask(t) -> fse_mask_t:
    assert t.dim() == 2 and t.is_cuda and t.stride(1) == 1
    import torch
    assert t.dtype == torch.uint8
    return fse_mask_t(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def fse_extrapolate(image, mask, params: fse_params_t, out, stream=None) -> None:
    """image, out: (H, W) float32 CUDA tensors; mask: (H, W) uint8 (1 = lost)."""
    im, mk, ot = _image(image), _mask(mask), _image(out)
    check(lib().fse_extrapolate(ctypes.byref(im), ctypes.byref(mk), ctypes.byref(params), ctypes.byref(ot),
                                _stream(stream)), "fse_extrapolate")


def fse_extrapolate_noalloc(image, mask, params: fse_params_t, out, stream=None) -> None:
    """fse_extrapolate with the library's fixed device scratch (no allocation)."""
    im, mk, ot = _image(image), _mask(mask), _image(out)
    check(lib().fse_extrapolate_noalloc(ctypes.byref(im), ctypes.byref(mk), ctypes.byref(params), ctypes.byref(ot),
                                        _stream(stream)), "fse_extrapolate_noalloc")


def fse_extrapolate_batch(images, masks, params: fse_params_t, outs, stream=None) -> None:
    n = len(images)
    ims = (fse_image_t * n)(*[_image(t) for t in images])
    mks = (fse_mask_t * n)(*[_mask(t) for t in masks])
    ots = (fse_image_t * n)(*[_image(t) for t in outs])
    check(lib().fse_extrapolate_batch(n, ims, mks, ctypes.byref(params), ots, _stream(stream)),
          "fse_extrapolate_batch")


def fse_last_stats() -> dict:
    s = fse_run_stats_t()
    check(lib().fse_last_stats(ctypes.byref(s)), "fse_last_stats")
    return {k: getattr(s, k) for k, _ in fse_run_stats_t._fields_}


def fse_release() -> None:
    check(lib().fse_release(), "fse_release")


def extrapolate(image, mask, params: fse_params_t | None = None, stream=None):
    """Convenience: allocate the output and run fse_extrapolate."""
    import torch
    out = torch.empty_like(image)
    fse_extrapolate(image, mask, params if params is not None else fse_params_default(), out, stream)
    return out


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

def fse_serve_create(hbm_budget_bytes: int, max_slots: int = 4, device: int = 0, workgroups: int = 0):
    cfg = fse_serve_config_t(hbm_budget_bytes, max_slots, device, workgroups)
    h = ctypes.c_void_p()
    check(lib().fse_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "fse_serve_create")
    return h


def fse_serve_submit(server, image, mask, params: fse_params_t, out) -> int:
    """Queue one request.  The tensors must stay alive until it is done, and
    image and mask must already hold their final contents: the server's
    streams are not ordered after the caller's (synchronise first)."""
    im, mk, ot = _image(image), _mask(mask), _image(out)
    t = ctypes.c_uint64()
    check(lib().fse_serve_submit(server, ctypes.byref(im), ctypes.byref(mk), ctypes.byref(params), ctypes.byref(ot),
                                 ctypes.byref(t)), "fse_serve_submit")
    return t.value


def _req_stats(st) -> dict:
    return {k: getattr(st, k) for k, _ in fse_request_stats_t._fields_}


def fse_serve_poll(server, ticket: int):
    done = ctypes.c_int32()
    st = fse_request_stats_t()
    check(lib().fse_serve_poll(server, ticket, ctypes.byref(done), ctypes.byref(st)), "fse_serve_poll")
    return bool(done.value), _req_stats(st)


def fse_serve_wait(server, ticket: int, timeout_us: int = -1) -> dict:
    st = fse_request_stats_t()
    check(lib().fse_serve_wait(server, ticket, timeout_us, ctypes.byref(st)), "fse_serve_wait")
    return _req_stats(st)


def fse_serve_cancel(server, ticket: int) -> bool:
    """Withdraw a queued request: True when withdrawn (its wait then raises
    with FSE_ERR_CANCELLED), False when it was already admitted into a launch
    (it completes normally)."""
    s = lib().fse_serve_cancel(server, ticket)
    if s == FSE_ERR_BUSY:
        return False
    check(s, "fse_serve_cancel")
    return True


def fse_serve_destroy(server) -> None:
    check(lib().fse_serve_destroy(server), "fse_serve_destroy")


# ---------------------------------------------------------------------------
# prepared plans (HIP graph replay)
# ---------------------------------------------------------------------------

def fse_plan_create(masks, params: fse_params_t):
    n = len(masks)
    mks = (fse_mask_t * n)(*[_mask(t) for t in masks])
    h = ctypes.c_void_p()
    check(lib().fse_plan_create(n, mks, ctypes.byref(params), ctypes.byref(h)), "fse_plan_create")
    return h


def fse_plan_execute(plan, images, outs, stream=None) -> None:
    n = len(images)
    ims = (fse_image_t * n)(*[_image(t) for t in images])
    ots = (fse_image_t * n)(*[_image(t) for t in outs])
    check(lib().fse_plan_execute(plan, ims, ots, _stream(stream)), "fse_plan_execute")


def fse_plan_stats(plan) -> dict:
    """Plan statistics and the device error word of its last execution
    (waits for that execution)."""
    s = fse_run_stats_t()
    check(lib().fse_plan_stats(plan, ctypes.byref(s)), "fse_plan_stats")
    return {k: getattr(s, k) for k, _ in fse_run_stats_t._fields_}


def fse_plan_destroy(plan) -> None:
    check(lib().fse_plan_destroy(plan), "fse_plan_destroy")


def fse_autotune(images, masks, params: fse_params_t, outs, stream=None) -> fse_params_t:
    """Fastest schedule (n_tiles when 0 in a tiled mode, block_waves,
    workgroups) for this batch; outs receive results."""
    n = len(images)
    ims = (fse_image_t * n)(*[_image(t) for t in images])
    mks = (fse_mask_t * n)(*[_mask(t) for t in masks])
    ots = (fse_image_t * n)(*[_image(t) for t in outs])
    best = fse_params_t()
    check(lib().fse_autotune(n, ims, mks, ctypes.byref(params), ots, _stream(stream), ctypes.byref(best)),
          "fse_autotune")
    return best


def fse_autotune_overlapped(images, masks, params: fse_params_t, outs, streams: int) -> fse_params_t:
    """Fastest schedule for `streams` consecutive calls in flight; outs receive results."""
    n = len(images)
    ims = (fse_image_t * n)(*[_image(t) for t in images])
    mks = (fse_mask_t * n)(*[_mask(t) for t in masks])
    ots = (fse_image_t * n)(*[_image(t) for t in outs])
    best = fse_params_t()
    check(lib().fse_autotune_overlapped(n, ims, mks, ctypes.byref(params), ots, streams, ctypes.byref(best)),
          "fse_autotune_overlapped")
    return best
