"""MI355X-native image-based invasion percolation (IBIP).

Thin Python binding over the C ABI of ``libibip_hip.so`` (``include/ibip.h``).
PyTorch supplies device memory and the stream; every step of the computation
runs in the library's HIP kernels. There is no CPU fallback: if the library is
missing or no GPU is present, the calls raise.

    import paper_2101_03240_amd as ibip
    dt2 = ibip.edt(image)                         # exact squared EDT
    r = ibip.invade(image, inlets)                # step / radius / saturation / Pc
    t = ibip.trap(r["seq"], outlets)              # trapped defender, re-ranked steps
    m = ibip.opening_drainage(image, inlets, T)   # pressure-based MIO drainage

Image tensors are ``torch.uint8`` on a ROCm device with shape (X, Y, Z) or
(Y, Z) (a 2D image, X = 1); nonzero = pore. uint32 outputs are returned in
``torch.int32`` tensors holding the same bits (every value fits below 2^31 for
the supported sizes).
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = ["edt", "edt_noalloc", "invade", "invade_resume", "invade_batch", "set_tuning", "get_tuning", "cached_tuning", "Server", "trap", "saturation", "remap_steps", "compare_opening", "opening_drainage",
           "IbipError", "library_path", "load_library", "enable_timing", "get_timing", "reset_timing",
           "probe_claim_latency"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libibip_hip.so")
_lib = None
_lock = threading.Lock()
_ctx = {}

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOSOLID", -4: "EDEVICE", -5: "ECAPACITY",
           -6: "ECANCELLED"}


class IbipError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _Dims(ctypes.Structure):
    _fields_ = [("X", ctypes.c_int32), ("Y", ctypes.c_int32), ("Z", ctypes.c_int32)]


class _Timing(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("edt_ms", "setup_ms", "loop_ms", "loop_kernel_ms", "wide_kernel_ms",
                                                "paint_ms", "steps_ms", "trap_ms", "mio_ms")] + \
               [(n, ctypes.c_int64) for n in ("loop_launches", "wide_launches", "steps", "popped", "relax_sweeps",
                                                "wide_centres")]


class _Job(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("inlets", ctypes.c_void_p), ("dims", _Dims),
                ("max_steps", ctypes.c_int64), ("seq", ctypes.c_void_p), ("rad2", ctypes.c_void_p),
                ("centre_step", ctypes.c_void_p), ("M", ctypes.c_void_p), ("sat", ctypes.c_void_p),
                ("n_steps", ctypes.c_int64), ("status", ctypes.c_int32)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32), ("lookahead", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "cancelled", "pending", "running",
                                                "bytes_in_use", "peak_bytes", "peak_running")]


class _Tuning(ctypes.Structure):
    _fields_ = [("edt_tile_y", ctypes.c_int32), ("edt_tile_x", ctypes.c_int32), ("batch_wide", ctypes.c_int64)]


def _tuning_struct(t: dict | None) -> "_Tuning":
    t = t or {}
    unknown = set(t) - {"edt_tile_y", "edt_tile_x", "batch_wide"}
    if unknown:
        raise ValueError(f"unknown tuning keys {sorted(unknown)}")
    return _Tuning(int(t.get("edt_tile_y", 0)), int(t.get("edt_tile_x", 0)), int(t.get("batch_wide", 0)))


class _InvadeOpts(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int64), ("sigma", ctypes.c_double),
                ("theta_rad", ctypes.c_double), ("voxel_size", ctypes.c_double)]


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load ``libibip_hip.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise IbipError(-4, f"{_LIB_PATH} is missing; build it with paper_2101_03240_amd.build.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.ibip_ctx_create.argtypes = [ctypes.POINTER(P), i32, P]
        lib.ibip_ctx_destroy.argtypes = [P]
        lib.ibip_ctx_set_stream.argtypes = [P, P]
        lib.ibip_last_error.argtypes = [P]
        lib.ibip_last_error.restype = ctypes.c_char_p
        lib.ibip_ctx_scratch_bytes.argtypes = [P]
        lib.ibip_ctx_scratch_bytes.restype = i64
        lib.ibip_edt.argtypes = [P, P, _Dims, P]
        lib.ibip_edt_noalloc.argtypes = [P, P, _Dims, P, P]
        lib.ibip_edt_noalloc.restype = i32
        lib.ibip_invade.argtypes = [P, P, P, _Dims, ctypes.POINTER(_InvadeOpts), P, P, P, ctypes.POINTER(i64)]
        lib.ibip_invade_resume.argtypes = [P, P, P, _Dims, ctypes.POINTER(_InvadeOpts), P, i64, P, P, P,
                                           ctypes.POINTER(i64)]
        lib.ibip_invade_resume.restype = i32
        lib.ibip_get_steps.argtypes = [P, P, P, P, P, i64]
        lib.ibip_trap.argtypes = [P, P, P, _Dims, P, P, ctypes.POINTER(i64)]
        lib.ibip_opening_drainage.argtypes = [P, P, P, _Dims, P, i32, P, P]
        lib.ibip_invade_batch.argtypes = [P, ctypes.POINTER(_Job), i32]
        lib.ibip_invade_batch.restype = i32
        lib.ibip_server_create.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(_ServerOpts)]
        lib.ibip_server_submit.argtypes = [P, ctypes.POINTER(_Job), ctypes.POINTER(i64)]
        lib.ibip_server_poll.argtypes = [P, i64, ctypes.POINTER(i32)]
        lib.ibip_server_wait.argtypes = [P, i64, ctypes.POINTER(_Job), ctypes.POINTER(ctypes.c_double)]
        lib.ibip_server_cancel.argtypes = [P, i64]
        lib.ibip_server_stats_get.argtypes = [P, ctypes.POINTER(_ServerStats)]
        lib.ibip_server_last_error.argtypes = [P]
        lib.ibip_server_last_error.restype = ctypes.c_char_p
        lib.ibip_server_destroy.argtypes = [P]
        for fn in (lib.ibip_server_create, lib.ibip_server_submit, lib.ibip_server_poll, lib.ibip_server_wait,
                   lib.ibip_server_cancel, lib.ibip_server_stats_get, lib.ibip_server_destroy):
            fn.restype = i32
        lib.ibip_saturation.argtypes = [P, P, _Dims, P, i64, ctypes.POINTER(_InvadeOpts), P, P, P, P]
        lib.ibip_saturation.restype = i32
        lib.ibip_remap_steps.argtypes = [P, P, P, _Dims, P, i64, i64, P]
        lib.ibip_remap_steps.restype = i32
        lib.ibip_ctx_set_readings.argtypes = [P, ctypes.c_uint32]
        lib.ibip_compare_opening.argtypes = [P, P, P, P, _Dims, P, P, i32, P, P]
        lib.ibip_compare_opening.restype = i32
        lib.ibip_ctx_set_readings.restype = i32
        lib.ibip_ctx_set_tuning.argtypes = [P, ctypes.POINTER(_Tuning)]
        lib.ibip_ctx_set_tuning.restype = i32
        lib.ibip_ctx_get_tuning.argtypes = [P, ctypes.POINTER(_Tuning)]
        lib.ibip_ctx_get_tuning.restype = i32
        lib.ibip_server_set_tuning.argtypes = [P, ctypes.POINTER(_Tuning)]
        lib.ibip_server_set_tuning.restype = i32
        lib.ibip_ctx_enable_timing.argtypes = [P, i32]
        lib.ibip_ctx_get_timing.argtypes = [P, ctypes.POINTER(_Timing)]
        lib.ibip_ctx_reset_timing.argtypes = [P]
        lib.ibip_probe_claim_latency.argtypes = [P, i64, i32, ctypes.POINTER(ctypes.c_double)]
        for fn in (lib.ibip_ctx_enable_timing, lib.ibip_ctx_get_timing, lib.ibip_ctx_reset_timing,
                   lib.ibip_probe_claim_latency):
            fn.restype = i32
        for fn in (lib.ibip_ctx_create, lib.ibip_ctx_destroy, lib.ibip_ctx_set_stream, lib.ibip_edt,
                   lib.ibip_invade, lib.ibip_get_steps, lib.ibip_trap, lib.ibip_opening_drainage):
            fn.restype = i32
        _lib = lib
    return _lib


def _torch():
    import torch
    return torch


# Launch parameters from the autotuner's cache (autotune.py), applied per call
# by the image's size class unless the thread set its own with set_tuning.
_tuned = {"loaded": False, "doc": None}
_manual = set()  # context keys whose tuning the caller set


def _tuning_doc():
    if not _tuned["loaded"]:
        _tuned["loaded"] = True
        try:
            from . import autotune
            torch = _torch()
            _tuned["doc"] = autotune.load(torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName)
        except Exception:
            _tuned["doc"] = None
    return _tuned["doc"]


def _auto_tuning(shape, batch: bool = False) -> dict | None:
    doc = _tuning_doc()
    if doc is None:
        return None
    from .autotune import size_class
    t = dict(doc.get("edt", {}).get(size_class(shape), {}))
    t = {k: t[k] for k in ("edt_tile_y", "edt_tile_x") if k in t}
    if batch and "batch" in doc:
        t["batch_wide"] = int(doc["batch"]["batch_wide"])
    return t or None


def cached_tuning(shape, batch: bool = False) -> dict:
    """The launch parameters the autotuner's cache holds for an image of
    `shape` on the current GPU (with `batch`, also the batch's wide-step
    threshold); empty when there is no cache for this GPU."""
    return _auto_tuning(tuple(shape), batch=batch) or {}


def _apply_auto(ctx, shape):
    """Set the cached tuning of this shape's size class on the context, unless
    the calling thread chose its own."""
    if ctx.value in _manual:
        return
    t = _auto_tuning(shape)
    if t is not None:
        load_library().ibip_ctx_set_tuning(ctx, ctypes.byref(_tuning_struct(t)))


def _context(device) -> ctypes.c_void_p:
    """The calling thread's context on `device` (a context holds scratch
    buffers and is used by one thread at a time, so each host thread gets its
    own; calls from two threads on two streams then run concurrently)."""
    torch = _torch()
    lib = load_library()
    idx = device.index if device.index is not None else torch.cuda.current_device()
    key = (idx, threading.get_ident())
    ctx = _ctx.get(key)
    if ctx is None:
        ctx = ctypes.c_void_p()
        st = lib.ibip_ctx_create(ctypes.byref(ctx), idx, None)
        if st != 0:
            raise IbipError(st, f"cannot create a context on device {idx}")
        _ctx[key] = ctx
    stream = torch.cuda.current_stream(idx).cuda_stream
    lib.ibip_ctx_set_stream(ctx, ctypes.c_void_p(stream))
    return ctx


READ_INTEGER_BALL, READ_MASK_INLETS, READ_TRAP26 = 1, 2, 4


def _readings(ctx, integer_ball: bool = False, mask_inlets: bool = False, connectivity: int = 6):
    """Set the context's readings of the ambiguous passages for the next call."""
    if connectivity not in (6, 26):
        raise ValueError("connectivity must be 6 or 26")
    flags = ((READ_INTEGER_BALL if integer_ball else 0) | (READ_MASK_INLETS if mask_inlets else 0) |
             (READ_TRAP26 if connectivity == 26 else 0))
    _check(load_library().ibip_ctx_set_readings(ctx, flags), ctx)


def _check(st: int, ctx):
    if st != 0:
        msg = load_library().ibip_last_error(ctx)
        raise IbipError(st, msg.decode() if msg else "")


def _dims_of(t) -> tuple[_Dims, tuple]:
    if t.dim() == 2:
        shape = (1,) + tuple(t.shape)
    elif t.dim() == 3:
        shape = tuple(t.shape)
    else:
        raise ValueError("expected a 2D or 3D tensor")
    return _Dims(*shape), shape


def _dev_u8(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a torch tensor on a GPU device")
    if t.dtype != torch.uint8:
        t = (t != 0).to(torch.uint8)
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def edt(image):
    """Exact squared distance from every voxel to the nearest solid voxel
    (Section 2.1, Figure 2(b)); 0 on solid. Returns int32 bits of uint32."""
    torch = _torch()
    image = _dev_u8(image, "image")
    dims, shape = _dims_of(image)
    ctx = _context(image.device)
    _apply_auto(ctx, shape)
    out = torch.empty(image.shape, dtype=torch.int32, device=image.device)
    _check(load_library().ibip_edt(ctx, _ptr(image), dims, _ptr(out)), ctx)
    return out


def edt_noalloc(image, out=None, solid_flag=None):
    """``edt`` through ibip_edt_noalloc, which allocates no device memory
    (its intermediate distances live in the library's fixed scratch; images
    of at most 2^24 voxels). ``out`` (int32, the image's shape) and
    ``solid_flag`` (int32, one entry) may be given to avoid allocations here
    too. Returns (dt2, solid_flag); solid_flag[0] == 0 means the image holds
    no solid voxel. Does not synchronise."""
    torch = _torch()
    image = _dev_u8(image, "image")
    dims, shape = _dims_of(image)
    ctx = _context(image.device)
    _apply_auto(ctx, shape)
    if out is None:
        out = torch.empty(image.shape, dtype=torch.int32, device=image.device)
    if solid_flag is None:
        solid_flag = torch.empty(1, dtype=torch.int32, device=image.device)
    _check(load_library().ibip_edt_noalloc(ctx, _ptr(image), dims, _ptr(out), _ptr(solid_flag)), ctx)
    return out, solid_flag


def invade_resume(image, inlets, checkpoint, k_done: int, **kw):
    """Continue an invasion from a checkpoint (ibip_invade_resume):
    ``checkpoint`` is the ``centre_step`` of an ``invade(..., max_steps=k_done)``
    on the same inputs that returned K = k_done. Takes the keyword arguments
    of ``invade`` (``max_steps`` counts from step 1) and returns the same
    dict, over the whole invasion."""
    ck = _dev_i32(checkpoint, "checkpoint")
    if ck.numel() != image.numel():
        raise ValueError("the checkpoint must have the image's shape")
    return invade(image, inlets, _resume=(ck, int(k_done)), **kw)


def invade(image, inlets, max_steps: int = 0, sigma: float = 1.0, theta_rad: float = 0.0,
           voxel_size: float = 1.0, rad2: bool = True, centre_step: bool = True, steps: bool = True,
           integer_ball: bool = False, mask_inlets: bool = False, _resume=None):
    """The invasion loop of Section 2.1 with the per-step arrays of Sections
    2.2.1-2.2.2. Returns a dict with ``seq`` (int32: -1 solid, 0 uninvaded,
    k = step), ``rad2``, ``centre_step``, ``K`` and, when ``steps``, the
    per-step ``M``, ``n_new``, ``sat`` and ``pc`` (device tensors).
    ``integer_ball`` paints footnote 1's integer sphere; ``mask_inlets`` lets
    only pore inlet voxels seed (variant readings)."""
    torch = _torch()
    image = _dev_u8(image, "image")
    inlets = _dev_u8(inlets, "inlets")
    if inlets.shape != image.shape:
        raise ValueError("inlets must have the image's shape")
    dims, shape = _dims_of(image)
    dev = image.device
    ctx = _context(dev)
    _readings(ctx, integer_ball=integer_ball, mask_inlets=mask_inlets)
    _apply_auto(ctx, shape)
    lib = load_library()
    seq = torch.empty(image.shape, dtype=torch.int32, device=dev)
    r2 = torch.empty(image.shape, dtype=torch.int32, device=dev) if rad2 else None
    cs = torch.empty(image.shape, dtype=torch.int32, device=dev) if centre_step else None
    opts = _InvadeOpts(int(max_steps), float(sigma), float(theta_rad), float(voxel_size))
    K = ctypes.c_int64(0)
    if _resume is None:
        _check(lib.ibip_invade(ctx, _ptr(image), _ptr(inlets), dims, ctypes.byref(opts), _ptr(seq),
                               _ptr(r2) if r2 is not None else None, _ptr(cs) if cs is not None else None,
                               ctypes.byref(K)), ctx)
    else:
        cs_in, k_done = _resume
        _check(lib.ibip_invade_resume(ctx, _ptr(image), _ptr(inlets), dims, ctypes.byref(opts), _ptr(cs_in),
                                      int(k_done), _ptr(seq), _ptr(r2) if r2 is not None else None,
                                      _ptr(cs) if cs is not None else None, ctypes.byref(K)), ctx)
    out = {"seq": seq, "rad2": r2, "centre_step": cs, "K": int(K.value)}
    if steps:
        k = max(int(K.value), 1)
        M = torch.empty(k, dtype=torch.int32, device=dev)
        n_new = torch.empty(k, dtype=torch.int64, device=dev)
        sat = torch.empty(k, dtype=torch.float64, device=dev)
        pc = torch.empty(k, dtype=torch.float64, device=dev)
        _check(lib.ibip_get_steps(ctx, _ptr(M), _ptr(n_new), _ptr(sat), _ptr(pc), k), ctx)
        kk = int(K.value)
        out.update(M=M[:kk], n_new=n_new[:kk], sat=sat[:kk], pc=pc[:kk])
    return out


def set_tuning(tuning: dict | None = None, device=None):
    """Launch parameters for the calling thread's context (ibip_ctx_set_tuning):
    ``edt_tile_y`` (32 or 64), ``edt_tile_x`` (16 or 32), ``batch_wide`` (a
    batch job's steps above it run over the whole GPU; negative: never).
    Missing keys or None: defaults. Results never depend on them."""
    torch = _torch()
    ctx = _context(torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device()))
    t = _tuning_struct(tuning)
    _check(load_library().ibip_ctx_set_tuning(ctx, ctypes.byref(t)), ctx)
    # None hands the choice back to the autotuner's cache
    if tuning is None:
        _manual.discard(ctx.value)
    else:
        _manual.add(ctx.value)


def get_tuning(device=None) -> dict:
    torch = _torch()
    ctx = _context(torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device()))
    t = _Tuning()
    _check(load_library().ibip_ctx_get_tuning(ctx, ctypes.byref(t)), ctx)
    return {n: getattr(t, n) for n, _ in _Tuning._fields_}


def invade_batch(images, inlets, max_steps=0, rad2: bool = True, centre_step: bool = True, M: bool = True,
                 sat: bool = False, raise_on_error: bool = True, tuning: dict | None = None):
    """ibip_invade over a list of images of uneven size in one call (the step
    loops of all jobs run in one launch; a job's step above the wide
    threshold continues over the whole GPU). ``inlets`` is a list of masks of
    matching shapes; ``max_steps`` an int or a list. ``tuning`` (keys of
    ``set_tuning``) applies to this call only. Returns a list of dicts like
    ``invade`` (``seq``, ``rad2``, ``centre_step``, ``K``, ``M``, ``sat``)
    plus each job's ``status``."""
    torch = _torch()
    n = len(images)
    if len(inlets) != n:
        raise ValueError("one inlets mask per image")
    ms = list(max_steps) if isinstance(max_steps, (list, tuple)) else [int(max_steps)] * n
    imgs = [_dev_u8(t, "image") for t in images]
    inls = [_dev_u8(t, "inlets") for t in inlets]
    if n == 0:
        return []
    dev = imgs[0].device
    ctx = _context(dev)
    jobs = (_Job * n)()
    outs = []
    for i, (im, il) in enumerate(zip(imgs, inls)):
        if il.shape != im.shape:
            raise ValueError("inlets must have the image's shape")
        dims, _ = _dims_of(im)
        o = {"seq": torch.empty(im.shape, dtype=torch.int32, device=dev),
             "rad2": torch.empty(im.shape, dtype=torch.int32, device=dev) if rad2 else None,
             "centre_step": torch.empty(im.shape, dtype=torch.int32, device=dev) if centre_step else None,
             "M": torch.empty(max(im.numel(), 1), dtype=torch.int32, device=dev) if M else None,
             "sat": torch.empty(max(im.numel(), 1), dtype=torch.float64, device=dev) if sat else None}
        outs.append(o)
        jobs[i].image = im.data_ptr()
        jobs[i].inlets = il.data_ptr()
        jobs[i].dims = dims
        jobs[i].max_steps = int(ms[i])
        for f in ("seq", "rad2", "centre_step", "M", "sat"):
            setattr(jobs[i], f, o[f].data_ptr() if o[f] is not None else None)
    lib = load_library()
    saved = None
    if tuning is None and ctx.value not in _manual:
        tuning = _auto_tuning(max((tuple(t.shape) for t in imgs), key=lambda sh: max(sh)), batch=True)
    if tuning is not None:
        saved = _Tuning()
        _check(lib.ibip_ctx_get_tuning(ctx, ctypes.byref(saved)), ctx)
        t = _tuning_struct(tuning)
        _check(lib.ibip_ctx_set_tuning(ctx, ctypes.byref(t)), ctx)
    try:
        st = lib.ibip_invade_batch(ctx, jobs, n)
    finally:
        if saved is not None:
            lib.ibip_ctx_set_tuning(ctx, ctypes.byref(saved))
    if st != 0 and raise_on_error:
        _check(st, ctx)
    for i, o in enumerate(outs):
        k = int(jobs[i].n_steps)
        o["K"] = k
        o["status"] = int(jobs[i].status)
        if o["M"] is not None:
            o["M"] = o["M"][:k]
        if o["sat"] is not None:
            o["sat"] = o["sat"][:k]
    return outs


class Server:
    """Continuous-batching invasion server (``ibip_server_*``). ``submit``
    queues one image and returns a ticket at once; ``wait`` returns the
    ``invade``-style result dict with ``status``, ``K`` and ``latency_ms``."""

    def __init__(self, device=0, hbm_budget_bytes: int = 8 << 30, max_inflight: int = 16, lookahead: int = 8):
        torch = _torch()
        self._lib = load_library()
        self._dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = self._dev.index if self._dev.index is not None else torch.cuda.current_device()
        self._h = ctypes.c_void_p()
        opts = _ServerOpts(int(hbm_budget_bytes), int(max_inflight), int(lookahead))
        st = self._lib.ibip_server_create(ctypes.byref(self._h), idx, ctypes.byref(opts))
        if st != 0:
            raise IbipError(st, "cannot create the server")
        self._live = {}
        self.tuning = {}  # the launch parameters last set (empty: the library's defaults)
        doc = _tuning_doc()
        if doc is not None and "serve" in doc:
            t = dict(doc.get("edt", {}).get("large", {}))
            t = {k: t[k] for k in ("edt_tile_y", "edt_tile_x") if k in t}
            t["batch_wide"] = int(doc["serve"]["serve_wide"])
            self.set_tuning(t)

    def submit(self, image, inlets, max_steps: int = 0, rad2: bool = True, centre_step: bool = True,
               M: bool = True) -> int:
        torch = _torch()
        image = _dev_u8(image, "image")
        inlets = _dev_u8(inlets, "inlets")
        if inlets.shape != image.shape:
            raise ValueError("inlets must have the image's shape")
        dims, _ = _dims_of(image)
        dev = image.device
        o = {"image": image, "inlets": inlets,
             "seq": torch.empty(image.shape, dtype=torch.int32, device=dev),
             "rad2": torch.empty(image.shape, dtype=torch.int32, device=dev) if rad2 else None,
             "centre_step": torch.empty(image.shape, dtype=torch.int32, device=dev) if centre_step else None,
             "M": torch.empty(max(image.numel(), 1), dtype=torch.int32, device=dev) if M else None}
        # inputs must be in place before the server's streams read them
        torch.cuda.current_stream(dev).synchronize()
        job = _Job()
        job.image = image.data_ptr()
        job.inlets = inlets.data_ptr()
        job.dims = dims
        job.max_steps = int(max_steps)
        for f in ("seq", "rad2", "centre_step", "M"):
            setattr(job, f, o[f].data_ptr() if o[f] is not None else None)
        job.sat = None
        t = ctypes.c_int64(0)
        st = self._lib.ibip_server_submit(self._h, ctypes.byref(job), ctypes.byref(t))
        if st != 0:
            raise IbipError(st, (self._lib.ibip_server_last_error(self._h) or b"").decode())
        self._live[int(t.value)] = o
        return int(t.value)

    def set_tuning(self, tuning: dict | None = None):
        """Launch parameters of the jobs admitted from now on (keys of
        ``set_tuning``; ``batch_wide`` applies to the served jobs)."""
        t = _tuning_struct(tuning)
        st = self._lib.ibip_server_set_tuning(self._h, ctypes.byref(t))
        if st != 0:
            raise IbipError(st, "bad tuning")
        self.tuning = dict(tuning or {})

    def done(self, ticket: int) -> bool:
        d = ctypes.c_int32(0)
        st = self._lib.ibip_server_poll(self._h, int(ticket), ctypes.byref(d))
        if st != 0:
            raise IbipError(st, "unknown ticket")
        return bool(d.value)

    def wait(self, ticket: int) -> dict:
        job = _Job()
        lat = ctypes.c_double(0.0)
        self._lib.ibip_server_wait(self._h, int(ticket), ctypes.byref(job), ctypes.byref(lat))
        o = self._live.pop(int(ticket))
        k = int(job.n_steps)
        res = {"seq": o["seq"], "rad2": o["rad2"], "centre_step": o["centre_step"],
               "M": o["M"][:k] if o["M"] is not None else None, "K": k, "status": int(job.status),
               "latency_ms": float(lat.value)}
        return res

    def cancel(self, ticket: int) -> bool:
        return self._lib.ibip_server_cancel(self._h, int(ticket)) == 0

    def stats(self) -> dict:
        s = _ServerStats()
        self._lib.ibip_server_stats_get(self._h, ctypes.byref(s))
        return {n: getattr(s, n) for n, _ in _ServerStats._fields_}

    def close(self):
        if self._h:
            self._lib.ibip_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def trap(seq, outlets, seq_trapped: bool = True, connectivity: int = 6):
    """Defender trapping and re-ranking (Section 2.2.3). Returns a dict with
    ``trapped`` (uint8), ``seq_trapped`` (int32) and ``K_after``.
    ``connectivity`` 26 connects voxels across edges and corners (variant)."""
    torch = _torch()
    if not isinstance(seq, torch.Tensor) or not seq.is_cuda or seq.dtype != torch.int32:
        raise ValueError("seq must be an int32 torch tensor on a GPU device")
    seq = seq.contiguous()
    outlets = _dev_u8(outlets, "outlets")
    if outlets.shape != seq.shape:
        raise ValueError("outlets must have the shape of seq")
    dims, shape = _dims_of(seq)
    dev = seq.device
    ctx = _context(dev)
    _readings(ctx, connectivity=connectivity)
    tr = torch.empty(seq.shape, dtype=torch.uint8, device=dev)
    st = torch.empty(seq.shape, dtype=torch.int32, device=dev) if seq_trapped else None
    K = ctypes.c_int64(0)
    _check(load_library().ibip_trap(ctx, _ptr(seq), _ptr(outlets), dims, _ptr(tr),
                                    _ptr(st) if st is not None else None, ctypes.byref(K)), ctx)
    return {"trapped": tr, "seq_trapped": st, "K_after": int(K.value)}


def _dev_i32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32:
        raise ValueError(f"{name} must be an int32 torch tensor on a GPU device")
    return t.contiguous()


def saturation(seq, M, sigma: float = 1.0, theta_rad: float = 0.0, voxel_size: float = 1.0,
               satmap: bool = True) -> dict:
    """Per-step arrays and the saturation map of a step labelling (Sections
    2.2.1-2.2.2, Figure 5 left): the sequence of ``invade``, or the re-ranked
    one of ``trap`` with the radii of ``remap_steps`` for the trapping-aware
    curve. Returns ``n_new``, ``sat``, ``pc`` (K entries) and ``satmap``
    (float64, -1 solid, 0 uninvaded, else the saturation after the voxel's
    step)."""
    torch = _torch()
    seq = _dev_i32(seq, "seq")
    dev = seq.device
    M = M.to(device=dev, dtype=torch.int32).contiguous()
    K = int(M.numel())
    dims, _ = _dims_of(seq)
    ctx = _context(dev)
    n_new = torch.empty(max(K, 1), dtype=torch.int64, device=dev)
    sat = torch.empty(max(K, 1), dtype=torch.float64, device=dev)
    pc = torch.empty(max(K, 1), dtype=torch.float64, device=dev)
    sm = torch.empty(seq.shape, dtype=torch.float64, device=dev) if satmap else None
    opts = _InvadeOpts(0, float(sigma), float(theta_rad), float(voxel_size))
    _check(load_library().ibip_saturation(ctx, _ptr(seq), dims, _ptr(M), K, ctypes.byref(opts), _ptr(n_new),
                                          _ptr(sat), _ptr(pc), _ptr(sm) if sm is not None else None), ctx)
    return {"n_new": n_new[:K], "sat": sat[:K], "pc": pc[:K], "satmap": sm}


def remap_steps(seq, seq_trapped, M, K_after: int):
    """Squared radius of each step that survives trapping, in re-ranked order
    (Section 2.2.3); int32 tensor of K_after entries (uint32 values)."""
    torch = _torch()
    seq = _dev_i32(seq, "seq")
    st = _dev_i32(seq_trapped, "seq_trapped")
    if st.shape != seq.shape:
        raise ValueError("seq_trapped must have the shape of seq")
    dev = seq.device
    M = M.to(device=dev, dtype=torch.int32).contiguous()
    dims, _ = _dims_of(seq)
    ctx = _context(dev)
    out = torch.empty(max(int(K_after), 1), dtype=torch.int32, device=dev)
    _check(load_library().ibip_remap_steps(ctx, _ptr(seq), _ptr(st), dims, _ptr(M), int(M.numel()), int(K_after),
                                           _ptr(out)), ctx)
    return out[:int(K_after)]


def opening_drainage(image, inlets, thresholds, mask_inlets: bool = False):
    """Pressure-based drainage by morphological image opening (Section 2.4.1)
    at the squared radii ``thresholds`` (strictly decreasing, >= 1). Returns a
    dict with ``mio_r2`` (int32 bits of uint32) and ``mio_sat`` (list).
    ``mask_inlets``: only pore inlet voxels seed (variant reading)."""
    torch = _torch()
    image = _dev_u8(image, "image")
    inlets = _dev_u8(inlets, "inlets")
    if inlets.shape != image.shape:
        raise ValueError("inlets must have the image's shape")
    dims, shape = _dims_of(image)
    dev = image.device
    ctx = _context(dev)
    _readings(ctx, mask_inlets=mask_inlets)
    _apply_auto(ctx, shape)
    T = [int(t) for t in thresholds]
    arr = (ctypes.c_uint32 * max(len(T), 1))(*T)
    sat = (ctypes.c_double * max(len(T), 1))()
    out = torch.empty(image.shape, dtype=torch.int32, device=dev)
    _check(load_library().ibip_opening_drainage(ctx, _ptr(image), _ptr(inlets), dims, ctypes.cast(arr, ctypes.c_void_p),
                                                len(T), _ptr(out), ctypes.cast(sat, ctypes.c_void_p)), ctx)
    return {"mio_r2": out, "mio_sat": [sat[i] for i in range(len(T))]}


def compare_opening(satmap, mio_r2, thresholds, mio_sat, trapped=None) -> dict:
    """Equal-saturation comparison of IBIP with the opening (Section 3.1.1,
    Figures 8 and 9): at each opening level i, ``disagree[i]`` voxels lie in
    exactly one of {0 < satmap <= mio_sat[i]} and {mio_r2 >= thresholds[i]},
    and ``mio_trapped[i]`` of the opening's voxels are ``trapped`` (zeros
    without it). Returns int64 tensors of one entry per level."""
    torch = _torch()
    if not isinstance(satmap, torch.Tensor) or not satmap.is_cuda or satmap.dtype != torch.float64:
        raise ValueError("satmap must be a float64 torch tensor on a GPU device")
    satmap = satmap.contiguous()
    r2 = _dev_i32(mio_r2, "mio_r2")
    if r2.shape != satmap.shape:
        raise ValueError("mio_r2 must have the shape of satmap")
    if trapped is not None:
        trapped = _dev_u8(trapped, "trapped")
        if trapped.shape != satmap.shape:
            raise ValueError("trapped must have the shape of satmap")
    dims, _ = _dims_of(satmap)
    dev = satmap.device
    ctx = _context(dev)
    T = [int(t) for t in thresholds]
    S = [float(x) for x in mio_sat]
    if len(T) != len(S) or not T:
        raise ValueError("thresholds and mio_sat need one entry per level")
    tarr = (ctypes.c_uint32 * len(T))(*T)
    sarr = (ctypes.c_double * len(S))(*S)
    dis = torch.empty(len(T), dtype=torch.int64, device=dev)
    mt = torch.zeros(len(T), dtype=torch.int64, device=dev)
    _check(load_library().ibip_compare_opening(
        ctx, _ptr(satmap), _ptr(r2), _ptr(trapped) if trapped is not None else None, dims,
        ctypes.cast(tarr, ctypes.c_void_p), ctypes.cast(sarr, ctypes.c_void_p), len(T), _ptr(dis),
        _ptr(mt) if trapped is not None else None), ctx)
    return {"disagree": dis, "mio_trapped": mt}


def enable_timing(enable: bool = True, device=None):
    """Turn the library's per-phase HIP-event timing on or off (see
    ibip_timing) for the calling thread's context."""
    torch = _torch()
    ctx = _context(torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device()))
    _check(load_library().ibip_ctx_enable_timing(ctx, 1 if enable else 0), ctx)


def reset_timing(device=None):
    torch = _torch()
    ctx = _context(torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device()))
    _check(load_library().ibip_ctx_reset_timing(ctx), ctx)


def probe_claim_latency(span_bytes: int, n_chain: int = 20000, device=None) -> float:
    """Average time (ns) of one claim in a chain of dependent atomics through
    a buffer of ``span_bytes`` (ibip_probe_claim_latency)."""
    torch = _torch()
    ctx = _context(torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device()))
    ns = ctypes.c_double(0.0)
    _check(load_library().ibip_probe_claim_latency(ctx, int(span_bytes), int(n_chain), ctypes.byref(ns)), ctx)
    return ns.value


def get_timing(device=None) -> dict:
    """Accumulated phase times (ms) and counters of the calling thread's
    context since its last reset."""
    torch = _torch()
    ctx = _context(torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device()))
    t = _Timing()
    _check(load_library().ibip_ctx_get_timing(ctx, ctypes.byref(t)), ctx)
    return {name: getattr(t, name) for name, _ in _Timing._fields_}
