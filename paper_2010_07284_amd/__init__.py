"""Python binding of libvlg, the MI355X spatial model checker (C ABI in
include/vlg.h).  Argument marshalling only: parsing, planning and every
operator run inside the library and its HIP kernels.  PyTorch provides device
memory and the stream.

    ctx = create()                       # device 0, torch's current stream
    img = load_image(ctx, tensor)        # (C,H,W) or (H,W), float32 / uint8
    f = compile_formula(ctx, src)
    masks = check_all(ctx, f, img)       # list of packed int64 [H, ceil(W/64)] tensors
    m = check(ctx, f, img, 0, fmt="u8")  # uint8 [H, W] tensor of 0/1
"""
import ctypes

from . import _lib
from ._lib import LIB_PATH, VlgError  # noqa: F401

MODES = {"perop": 0, "fused": 1, "graph": 2}
FMTS = {"packed": 0, "u8": 1}


def _torch():
    import torch
    return torch


class Context:
    def __init__(self, handle, device, stream):
        self.handle = handle
        self.device = device
        self.stream = stream

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None and _lib.loaded():
            _lib.lib().vlg_destroy(h)


class Image:
    def __init__(self, handle, shape, dtype):
        self.handle = handle
        self.shape = shape  # (C, H, W)
        self.dtype = dtype

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None and _lib.loaded():
            _lib.lib().vlg_image_free(h)


class Formula:
    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None and _lib.loaded():
            _lib.lib().vlg_formula_free(h)


def create(device=0, stream=None):
    """vlg_create on `device`, enqueueing on `stream` (a torch.cuda.Stream;
    default: a new stream, since graph capture needs a non-default stream).
    Results are ready after sync(ctx) or after waiting on ctx.stream."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.Stream(device)
    h = ctypes.c_void_p()
    _lib.call("vlg_create", ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
    return Context(h, device, stream)


def sync(ctx):
    """vlg_sync: raises VlgError (code -6, VLG_ENOCONV) when a labelling loop
    of the work since the last synchronisation stopped at its iteration cap."""
    _lib.call("vlg_sync", ctx.handle)


def set_loop_cap(ctx, cap):
    """vlg_set_loop_cap: iteration cap of the labelling loops (0 = default)."""
    _lib.call("vlg_set_loop_cap", ctx.handle, int(cap))


class _Ordered:
    """Stream ordering around a call that reads or writes caller tensors: the
    context's stream first waits for torch's current stream (pending writes
    to the outputs, e.g. a fill), and torch's current stream then waits for
    the context's stream, so torch work issued later sees the results.  Both
    are asynchronous."""

    def __init__(self, ctx):
        self.ctx = ctx

    def __enter__(self):
        torch = _torch()
        self.cur = torch.cuda.current_stream(self.ctx.device)
        if self.cur.cuda_stream != self.ctx.stream.cuda_stream:
            self.ctx.stream.wait_stream(self.cur)
        return self

    def __exit__(self, *exc):
        if exc[0] is None and self.cur.cuda_stream != self.ctx.stream.cuda_stream:
            self.cur.wait_stream(self.ctx.stream)
        return False


def set_mode(ctx, mode):
    _lib.call("vlg_set_mode", ctx.handle, MODES[mode] if isinstance(mode, str) else int(mode))


def load_image(ctx, t):
    """vlg_load_image from a torch tensor or numpy array, (C,H,W) or (H,W),
    float32, uint8 or uint16, host or device."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.from_numpy(t)
    if t.dim() == 2:
        t = t.unsqueeze(0)
    codes = {torch.float32: 0, torch.uint8: 1, torch.uint16: 2}
    if t.dim() != 3 or t.dtype not in codes:
        raise ValueError("image must be (C,H,W) float32, uint8 or uint16")
    t = t.contiguous()
    C, H, W = t.shape
    dtype = codes[t.dtype]
    where = 1 if t.is_cuda else 0
    if where == 1:
        # the library copies on its own stream: torch's pending writes first
        torch.cuda.current_stream(t.device).synchronize()
    h = ctypes.c_void_p()
    _lib.call("vlg_load_image", ctx.handle, ctypes.c_void_p(t.data_ptr()), dtype, C, H, W, W, where,
              ctypes.byref(h))
    if where == 1:
        sync(ctx)  # the source tensor may be released by the caller
    return Image(h, (C, H, W), t.dtype)


def load_volume(ctx, t):
    """vlg_load_volume from a torch tensor or numpy array, (C,D,H,W) or
    (D,H,W), float32, uint8 or uint16, host or device.  The returned image's
    shape is (C, D*H, W) for mask allocation; image.depth holds D."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.from_numpy(t)
    if t.dim() == 3:
        t = t.unsqueeze(0)
    codes = {torch.float32: 0, torch.uint8: 1, torch.uint16: 2}
    if t.dim() != 4 or t.dtype not in codes:
        raise ValueError("volume must be (C,D,H,W) float32, uint8 or uint16")
    t = t.contiguous()
    C, D, H, W = t.shape
    where = 1 if t.is_cuda else 0
    if where == 1:
        torch.cuda.current_stream(t.device).synchronize()
    h = ctypes.c_void_p()
    _lib.call("vlg_load_volume", ctx.handle, ctypes.c_void_p(t.data_ptr()), codes[t.dtype], C, D, H, W, where,
              ctypes.byref(h))
    if where == 1:
        sync(ctx)
    im = Image(h, (C, D * H, W), t.dtype)
    im.depth = D
    return im


def ccl_labels3(ctx, mask, depth, height, width, out=None):
    """vlg_ccl_labels3 of a packed device volume mask -> int32 [D, H, W] labels
    (smallest linear index of each 26-component, -1 for background)."""
    torch = _torch()
    if out is None:
        out = torch.empty((depth, height, width), dtype=torch.int32, device=mask.device)
    with _Ordered(ctx):
        _lib.call("vlg_ccl_labels3", ctx.handle, ctypes.c_void_p(mask.data_ptr()), depth, height, width,
                  ctypes.c_void_p(out.data_ptr()))
    return out


def compile_formula(ctx, src):
    h = ctypes.c_void_p()
    _lib.call("vlg_compile_formula", ctx.handle if ctx else None, src.encode(), ctypes.byref(h))
    return Formula(h)


def formula_info(f):
    st = _lib.FormulaStats()
    _lib.call("vlg_formula_info", f.handle, ctypes.byref(st))
    return {name: getattr(st, name) for name, _ in _lib.FormulaStats._fields_}


def formula_plan(f, mode="fused", fuse_halo=8):
    """vlg_formula_plan: the kernel schedule of every output as a dict."""
    import json
    need = ctypes.c_int64()
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _lib.call("vlg_formula_plan", f.handle, m, fuse_halo, None, 0, ctypes.byref(need))
    buf = ctypes.create_string_buffer(need.value)
    _lib.call("vlg_formula_plan", f.handle, m, fuse_halo, buf, need.value, ctypes.byref(need))
    return json.loads(buf.value.decode())


def output_names(f):
    n = formula_info(f)["outputs"]
    L = _lib.lib()
    return [L.vlg_formula_output_name(f.handle, i).decode() for i in range(n)]


def _alloc_out(img, fmt, device):
    torch = _torch()
    C, H, W = img.shape
    if fmt == "packed":
        return torch.empty((H, (W + 63) // 64), dtype=torch.int64, device=device)
    return torch.empty((H, W), dtype=torch.uint8, device=device)


def check(ctx, f, img, output_index=0, out=None, fmt="packed"):
    """vlg_check: one output into a device tensor (allocated if `out` is None)."""
    if out is None:
        out = _alloc_out(img, fmt, f"cuda:{ctx.device}")
    where = 1 if out.is_cuda else 0
    with _Ordered(ctx):
        _lib.call("vlg_check", ctx.handle, f.handle, img.handle, output_index, ctypes.c_void_p(out.data_ptr()),
                  FMTS[fmt], where)
    return out


def check_all(ctx, f, img, outs=None, fmt="packed"):
    """vlg_check_all: every output in one evaluation."""
    n = formula_info(f)["outputs"]
    if outs is None:
        outs = [_alloc_out(img, fmt, f"cuda:{ctx.device}") for _ in range(n)]
    where = 1 if outs[0].is_cuda else 0
    arr = (ctypes.c_void_p * n)(*[o.data_ptr() if o is not None else None for o in outs])
    with _Ordered(ctx):
        _lib.call("vlg_check_all", ctx.handle, f.handle, img.handle, arr, FMTS[fmt], where)
    return outs


def check_batch(ctx, f, imgs, outs=None, fmt="packed"):
    """vlg_check_batch: every output of f on each image; returns a list (per
    image) of lists (per output)."""
    n = formula_info(f)["outputs"]
    if outs is None:
        outs = [[_alloc_out(im, fmt, f"cuda:{ctx.device}") for _ in range(n)] for im in imgs]
    present = [o for row in outs for o in row if o is not None]
    where = 1 if not present or present[0].is_cuda else 0
    flat = [o.data_ptr() if o is not None else None for row in outs for o in row]
    arr = (ctypes.c_void_p * len(flat))(*flat)
    harr = (ctypes.c_void_p * len(imgs))(*[im.handle.value for im in imgs])
    with _Ordered(ctx):
        _lib.call("vlg_check_batch", ctx.handle, f.handle, harr, len(imgs), arr, FMTS[fmt], where)
    return outs


def ccl_labels(ctx, mask, height, width, out=None):
    """vlg_ccl_labels of a packed device mask -> int32 [H, W] labels (smallest
    row-major index of each component, -1 for background)."""
    torch = _torch()
    if out is None:
        out = torch.empty((height, width), dtype=torch.int32, device=mask.device)
    with _Ordered(ctx):
        _lib.call("vlg_ccl_labels", ctx.handle, ctypes.c_void_p(mask.data_ptr()), height, width,
                  ctypes.c_void_p(out.data_ptr()))
    return out


def ccl_labels_noalloc(ctx, mask, height, width, out):
    """vlg_ccl_labels_noalloc: the labelling of ccl_labels into the caller's
    int32 [H, W] device tensor `out`, with the library allocating nothing
    (its arrays live in a fixed per-GPU device array; VLG_ESHAPE beyond it)."""
    with _Ordered(ctx):
        _lib.call("vlg_ccl_labels_noalloc", ctx.handle, ctypes.c_void_p(mask.data_ptr()), height, width,
                  ctypes.c_void_p(out.data_ptr()))
    return out


NOALLOC_SCRATCH_BYTES = 40 << 20


def ccl_labels_pj(ctx, mask, height, width, reconnect_every=0, out=None):
    """vlg_ccl_labels_pj: the paper's pointer-jumping labelling of a packed
    device mask -> (int32 [H, W] labels = largest row-major index of each
    component, -1 background; {"main_iterations", "rounds", "launches"})."""
    torch = _torch()
    if out is None:
        out = torch.empty((height, width), dtype=torch.int32, device=mask.device)
    st = _lib.PjStats()
    with _Ordered(ctx):
        _lib.call("vlg_ccl_labels_pj", ctx.handle, ctypes.c_void_p(mask.data_ptr()), height, width,
                  int(reconnect_every), ctypes.c_void_p(out.data_ptr()), ctypes.byref(st))
    return out, {name: getattr(st, name) for name, _ in _lib.PjStats._fields_}


def profile_step(ctx, f, img, kind, reps=20):
    """vlg_profile_step: (mean ms of one launch of the first `kind` step,
    repeated back to back without per-launch events; its algorithmic bytes)."""
    ms, b = ctypes.c_double(), ctypes.c_double()
    _lib.call("vlg_profile_step", ctx.handle, f.handle, img.handle, kind.encode(), int(reps), ctypes.byref(ms),
              ctypes.byref(b))
    return ms.value, b.value


def stream_copy(ctx, dst, src, width=16, reps=5):
    """vlg_stream_copy: mean ms of one copy of src into dst (device tensors of
    equal byte size) with the library's non-temporal copy kernel."""
    ms = ctypes.c_double()
    nbytes = src.numel() * src.element_size()
    _lib.call("vlg_stream_copy", ctx.handle, ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
              nbytes, int(width), int(reps), ctypes.byref(ms))
    return ms.value


def ccl_counters(ctx):
    c = _lib.CclCounters()
    _lib.call("vlg_ccl_read_counters", ctx.handle, ctypes.byref(c))
    return {name: getattr(c, name) for name, _ in _lib.CclCounters._fields_}


def profile(ctx, f, img, iters=5):
    """vlg_profile: per kernel kind {name: (launches, ms_total, algorithmic_bytes)}
    from HIP events around each step of the fused schedule."""
    arr = (_lib.KernelTime * 16)()
    n = ctypes.c_int()
    _lib.call("vlg_profile", ctx.handle, f.handle, img.handle, iters, arr, 16, ctypes.byref(n))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].ms, arr[i].bytes) for i in range(n.value)}


def profile_batch(ctx, f, imgs, iters=3):
    """vlg_profile_batch: per kernel kind {name: (launches, ms_total,
    algorithmic_bytes)} of the batched schedule over the images."""
    arr = (_lib.KernelTime * 16)()
    n = ctypes.c_int()
    harr = (ctypes.c_void_p * len(imgs))(*[im.handle.value for im in imgs])
    _lib.call("vlg_profile_batch", ctx.handle, f.handle, harr, len(imgs), iters, arr, 16, ctypes.byref(n))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].ms, arr[i].bytes) for i in range(n.value)}


TUNABLES = {"ccl_tile_rows": 0, "near_band_rows": 1, "batch_grid": 2, "ccl_lanes": 3, "fuse_halo": 4,
            "ccl_algo": 5, "pj_reconnect": 6, "arith_kernel": 7}
CCL_UNION_FIND, CCL_POINTER_JUMPING = 1, 2
ARITH_INTERPRETER, ARITH_COMPILED = 1, 2


def set_tunable(ctx, name, value):
    """vlg_set_tunable: force a tunable (0 = back to the tuning table)."""
    _lib.call("vlg_set_tunable", ctx.handle, TUNABLES[name], int(value))


def get_tunable(ctx, name, height, width):
    v = ctypes.c_int()
    _lib.call("vlg_get_tunable", ctx.handle, TUNABLES[name], height, width, ctypes.byref(v))
    return v.value


def autotune(ctx, f, img, iters=5):
    """vlg_autotune: {tunable: (best, {candidate: ms})} for img's shape class."""
    arr = (_lib.TuneReport * 8)()
    n = ctypes.c_int()
    _lib.call("vlg_autotune", ctx.handle, f.handle, img.handle, iters, arr, 8, ctypes.byref(n))
    names = {v: k for k, v in TUNABLES.items()}
    return {names[arr[i].which]: (arr[i].best, {arr[i].candidates[j]: arr[i].ms[j] for j in range(arr[i].n)})
            for i in range(n.value)}


def autotune_batch(ctx, f, imgs, iters=3):
    """vlg_autotune_batch: {tunable: (best, {candidate: ms})} for the batch class
    of `imgs` (ms per batched evaluation of every output on all images)."""
    arr = (_lib.TuneReport * 4)()
    n = ctypes.c_int()
    harr = (ctypes.c_void_p * len(imgs))(*[im.handle.value for im in imgs])
    _lib.call("vlg_autotune_batch", ctx.handle, f.handle, harr, len(imgs), iters, arr, 4, ctypes.byref(n))
    names = {v: k for k, v in TUNABLES.items()}
    return {names[arr[i].which]: (arr[i].best, {arr[i].candidates[j]: arr[i].ms[j] for j in range(arr[i].n)})
            for i in range(n.value)}


def tune_save(ctx, path):
    _lib.call("vlg_tune_save", ctx.handle, path.encode())


def tune_load(ctx, path):
    _lib.call("vlg_tune_load", ctx.handle, path.encode())


def evaluation_bytes(f, img):
    """vlg_evaluation_bytes: device workspace of one evaluation of f on img."""
    b = ctypes.c_int64()
    _lib.call("vlg_evaluation_bytes", f.handle, img.handle, ctypes.byref(b))
    return b.value


class Server:
    """Serving loop (vlg_server_*): continuous batching with HBM-footprint
    admission.  submit() returns at once; wait() blocks for one request and
    returns (queue_ms, run_ms)."""

    def __init__(self, device=0, slots=4, budget_bytes=8 << 30):
        h = ctypes.c_void_p()
        _lib.call("vlg_server_create", ctypes.byref(h), device, slots, int(budget_bytes))
        self.handle = h
        self.device = device
        self._keep = {}

    def submit(self, f, img, outs):
        # slot streams live inside the library: pending torch writes to the
        # output buffers (e.g. a fill) must be complete before they are handed over
        if any(o is not None and o.is_cuda for o in outs):
            _torch().cuda.current_stream(self.device).synchronize()
        arr = (ctypes.c_void_p * len(outs))(*[o.data_ptr() if o is not None else None for o in outs])
        rid = ctypes.c_int64()
        _lib.call("vlg_server_submit", self.handle, f.handle, img.handle, arr, ctypes.byref(rid))
        self._keep[rid.value] = (f, img, outs)  # keep buffers alive until waited
        return rid.value

    def wait(self, rid):
        q, r = ctypes.c_double(), ctypes.c_double()
        try:
            _lib.call("vlg_server_wait", self.handle, rid, ctypes.byref(q), ctypes.byref(r))
        finally:
            self._keep.pop(rid, None)
        return q.value, r.value

    def stats(self):
        st = _lib.ServerStats()
        _lib.call("vlg_server_read_stats", self.handle, ctypes.byref(st))
        return {n: getattr(st, n) for n, _ in _lib.ServerStats._fields_}

    def close(self):
        h, self.handle = self.handle, None
        if h:
            _lib.call("vlg_server_destroy", h)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None and _lib.loaded():
            self.close()


def unpack(words, height, width):
    """Packed int64 words (torch or numpy, [H, ceil(W/64)]) -> numpy uint8 [H, W]."""
    import numpy as np
    a = words.cpu().numpy() if hasattr(words, "cpu") else np.asarray(words)
    if height == 0 or width == 0:
        return np.zeros((height, width), np.uint8)
    bits = np.unpackbits(a.astype("<i8").view(np.uint8).reshape(height, -1), axis=1, bitorder="little")
    return bits[:, :width].copy()


def pack(mask):
    """numpy uint8 [H, W] of 0/1 -> numpy int64 [H, ceil(W/64)] packed words."""
    import numpy as np
    H, W = mask.shape
    wpr = (W + 63) // 64
    padded = np.zeros((H, wpr * 64), np.uint8)
    padded[:, :W] = mask
    return np.packbits(padded, axis=1, bitorder="little").view("<i8").reshape(H, wpr).copy()


__all__ = ["create", "sync", "set_loop_cap", "set_mode", "load_image", "compile_formula", "formula_info", "formula_plan", "output_names",
           "check", "check_all", "check_batch", "ccl_labels", "ccl_labels_noalloc", "ccl_labels_pj", "ccl_labels3", "load_volume", "ccl_counters", "profile", "profile_batch", "profile_step", "stream_copy", "set_tunable", "get_tunable", "autotune", "tune_save",
           "tune_load", "autotune_batch", "Server", "evaluation_bytes", "unpack", "pack", "VlgError",
           "LIB_PATH"]
