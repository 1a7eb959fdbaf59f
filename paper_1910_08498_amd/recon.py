"""Python binding of librecon.so: argument marshalling only.

Functions carry the names of the C ABI in include/recon.h.  Every step of the
insertion path runs in the library's HIP kernels; PyTorch only supplies device
memory (tensors) and the current HIP stream.  If the library is not built,
importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so the library shares torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librecon.so")

RECON_OK, RECON_EINVAL, RECON_ENOMEM, RECON_EDEVICE, RECON_ECONFIG = 0, -1, -2, -3, -4
RECON_SLICE_C64, RECON_SLICE_F16, RECON_SLICE_BF16 = 0, 1, 2
RECON_VARIANT_AUTO, RECON_VARIANT_NAIVE, RECON_VARIANT_BINNED, RECON_VARIANT_SLAB = 0, 1, 2, 3
RECON_WEIGHTS_DEFAULT, RECON_WEIGHTS_TABLE, RECON_WEIGHTS_OTF = 0, 1, 2
RECON_TRAVERSAL_COLUMNS_SECOND, RECON_TRAVERSAL_SPATIAL_QUEUE = 1, 2


class recon_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("blob_radius", ctypes.c_float), ("blob_alpha", ctypes.c_float),
                ("blob_order", ctypes.c_int32), ("table_size", ctypes.c_int32),
                ("table_lerp", ctypes.c_int32), ("r_max", ctypes.c_float),
                ("slice_dtype", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class recon_config(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("waves_per_block", ctypes.c_int32), ("group", ctypes.c_int32),
                ("inner_chunk", ctypes.c_int32), ("split", ctypes.c_int32),
                ("slab_flags", ctypes.c_int32), ("cu_count", ctypes.c_int32), ("weights", ctypes.c_int32),
                ("traversal", ctypes.c_int32), ("reserved", ctypes.c_int32 * 7)]


class recon_tune_opts(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("target_ns_per_slice", ctypes.c_double), ("order_count", ctypes.c_int32),
                ("reserved1", ctypes.c_int32), ("order", ctypes.POINTER(ctypes.c_int32)),
                ("reserved", ctypes.c_int32 * 4)]


class recon_tune_info(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int32), ("steps_done", ctypes.c_int32), ("space_size", ctypes.c_int32),
                ("best_index", ctypes.c_int32), ("best_ns_per_slice", ctypes.c_double),
                ("mean_ns_per_slice", ctypes.c_double), ("best", recon_config)]


class ReconError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"recon error {status}: {msg}")
        self.status = status


_lib = None


def load_library():
    """Loads librecon.so once; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    P, vp, sz = ctypes.POINTER, ctypes.c_void_p, ctypes.c_size_t
    i32 = ctypes.c_int32
    sig = {
        "recon_default_params": ([i32, P(recon_params)], i32),
        "recon_query_sizes": ([P(recon_params), P(sz), P(sz), P(sz)], i32),
        "recon_init": ([P(recon_params), vp, vp, vp, sz, vp, P(vp)], i32),
        "recon_init_static": ([P(recon_params), vp, vp, vp, P(vp)], i32),
        "recon_reset": ([vp], i32),
        "recon_insert_batch": ([vp, vp, vp, vp, i32], i32),
        "recon_finalize": ([vp, vp, ctypes.c_float], i32),
        "recon_set_config": ([vp, P(recon_config)], i32),
        "recon_get_config": ([vp, P(recon_config)], i32),
        "recon_set_stream": ([vp, vp], i32),
        "recon_set_timing_events": ([vp, vp, vp], i32),
        "recon_tune_space_size": ([vp, P(i32)], i32),
        "recon_tune_space_config": ([vp, i32, P(recon_config)], i32),
        "recon_tune_begin": ([vp, P(recon_tune_opts)], i32),
        "recon_tune_get_info": ([vp, P(recon_tune_info)], i32),
        "recon_tune_end": ([vp], i32),
        "recon_tune_invocations": ([ctypes.c_double] * 4 + [P(ctypes.c_double)], i32),
        "recon_tune_steps": ([ctypes.c_double] * 2 + [P(ctypes.c_double)], i32),
        "recon_batch_query_size": ([P(vp), i32, P(sz)], i32),
        "recon_batch_create": ([P(vp), i32, vp, sz, P(vp)], i32),
        "recon_batch_insert": ([vp, P(vp), P(vp), P(vp), P(i32)], i32),
        "recon_batch_destroy": ([vp], None),
        "recon_mlp_sizes": ([i32, i32, i32, i32, P(sz), P(sz)], i32),
        "recon_mlp_forward": ([vp, i32, i32, i32, vp, i32, vp, vp, vp], i32),
        "recon_mlp_train_step": ([vp, i32, i32, i32, vp, vp, i32, ctypes.c_float, vp, vp, vp, vp], i32),
        "recon_stats": ([vp, P(ctypes.c_uint64), P(ctypes.c_uint64)], i32),
        "recon_destroy": ([vp], None),
        "recon_last_error": ([], ctypes.c_char_p),
        "recon_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != RECON_OK:
        raise ReconError(status, load_library().recon_last_error().decode())


def _ptr(t):
    """Device pointer of a tensor (None -> NULL)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# same-named wrappers of the C ABI
# ---------------------------------------------------------------------------
def recon_default_params(n: int) -> recon_params:
    p = recon_params()
    _check(load_library().recon_default_params(int(n), ctypes.byref(p)))
    return p


def recon_query_sizes(p: recon_params):
    g, w, ws = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().recon_query_sizes(ctypes.byref(p), ctypes.byref(g), ctypes.byref(w), ctypes.byref(ws)))
    return g.value, w.value, ws.value


def recon_init(p: recon_params, G, W, ws, stream=None):
    ctx = ctypes.c_void_p()
    _check(load_library().recon_init(ctypes.byref(p), _ptr(G), _ptr(W), _ptr(ws), ws.numel() * ws.element_size(),
                                     _stream(stream), ctypes.byref(ctx)))
    return ctx


def recon_init_static(p: recon_params, G, W, stream=None):
    ctx = ctypes.c_void_p()
    _check(load_library().recon_init_static(ctypes.byref(p), _ptr(G), _ptr(W), _stream(stream), ctypes.byref(ctx)))
    return ctx


def recon_reset(ctx):
    _check(load_library().recon_reset(ctx))


def recon_insert_batch(ctx, slices, scales, quats, count: int):
    _check(load_library().recon_insert_batch(ctx, _ptr(slices), _ptr(scales), _ptr(quats), int(count)))


def recon_finalize(ctx, V, w_threshold: float = 0.0):
    _check(load_library().recon_finalize(ctx, _ptr(V), float(w_threshold)))


def recon_set_config(ctx, cfg: recon_config | None):
    _check(load_library().recon_set_config(ctx, None if cfg is None else ctypes.byref(cfg)))


def recon_get_config(ctx) -> recon_config:
    c = recon_config()
    _check(load_library().recon_get_config(ctx, ctypes.byref(c)))
    return c


def recon_set_stream(ctx, stream=None):
    _check(load_library().recon_set_stream(ctx, _stream(stream)))


def recon_set_timing_events(ctx, start=None, stop=None):
    """start/stop: torch.cuda.Event objects (or None to disable)."""
    sp = None if start is None else ctypes.c_void_p(start.cuda_event)
    tp = None if stop is None else ctypes.c_void_p(stop.cuda_event)
    _check(load_library().recon_set_timing_events(ctx, sp, tp))


def recon_tune_space_size(ctx) -> int:
    n = ctypes.c_int32()
    _check(load_library().recon_tune_space_size(ctx, ctypes.byref(n)))
    return n.value


def recon_tune_space_config(ctx, index: int) -> recon_config:
    c = recon_config()
    _check(load_library().recon_tune_space_config(ctx, int(index), ctypes.byref(c)))
    return c


def recon_tune_begin(ctx, max_steps: int = 0, seed: int = 0, target_ns_per_slice: float = 0.0, order=None):
    """order: optional sequence of tuning-space indices to try in that order."""
    o = recon_tune_opts()
    o.max_steps, o.seed, o.target_ns_per_slice = int(max_steps), int(seed), float(target_ns_per_slice)
    keep = None
    if order is not None:
        keep = (ctypes.c_int32 * len(order))(*[int(k) for k in order])
        o.order_count = len(order)
        o.order = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int32))
    _check(load_library().recon_tune_begin(ctx, ctypes.byref(o)))


def recon_tune_get_info(ctx) -> recon_tune_info:
    i = recon_tune_info()
    _check(load_library().recon_tune_get_info(ctx, ctypes.byref(i)))
    return i


def recon_tune_end(ctx):
    _check(load_library().recon_tune_end(ctx))


def recon_tune_invocations(rp: float, s: float, t_avg: float, t_well: float) -> float:
    out = ctypes.c_double()
    _check(load_library().recon_tune_invocations(rp, s, t_avg, t_well, ctypes.byref(out)))
    return out.value


def recon_tune_steps(r: float, p: float) -> float:
    out = ctypes.c_double()
    _check(load_library().recon_tune_steps(r, p, ctypes.byref(out)))
    return out.value


def _ctx_array(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))()
    for i, c in enumerate(ctxs):
        arr[i] = c.value if isinstance(c, ctypes.c_void_p) else c
    return arr


def recon_batch_query_size(ctxs) -> int:
    n = ctypes.c_size_t()
    _check(load_library().recon_batch_query_size(_ctx_array(ctxs), len(ctxs), ctypes.byref(n)))
    return n.value


def recon_batch_create(ctxs, ws):
    b = ctypes.c_void_p()
    _check(load_library().recon_batch_create(_ctx_array(ctxs), len(ctxs), _ptr(ws), ws.numel() * ws.element_size(),
                                             ctypes.byref(b)))
    return b


def recon_batch_insert(batch, slices, scales, quats, counts):
    """slices, quats: lists of device tensors (or None); scales: list or None."""
    k = len(counts)
    sl = (ctypes.c_void_p * k)(*[None if t is None else t.data_ptr() for t in slices])
    qt = (ctypes.c_void_p * k)(*[None if t is None else t.data_ptr() for t in quats])
    sc = None if scales is None else (ctypes.c_void_p * k)(*[None if t is None else t.data_ptr() for t in scales])
    cn = (ctypes.c_int32 * k)(*[int(c) for c in counts])
    _check(load_library().recon_batch_insert(batch, sl, sc, qt, cn))


def recon_batch_destroy(batch):
    load_library().recon_batch_destroy(batch)


def recon_mlp_sizes(n_in: int, n_hidden: int, n_out: int, batch: int):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().recon_mlp_sizes(n_in, n_hidden, n_out, batch, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def recon_mlp_forward(params, n_in, n_hidden, n_out, x, batch, ws, probs, stream=None):
    _check(load_library().recon_mlp_forward(_ptr(params), n_in, n_hidden, n_out, _ptr(x), batch, _ptr(ws),
                                            _ptr(probs), _stream(stream)))


def recon_mlp_train_step(params, n_in, n_hidden, n_out, x, y, batch, lr, ws, loss=None, grads=None, stream=None):
    _check(load_library().recon_mlp_train_step(_ptr(params), n_in, n_hidden, n_out, _ptr(x), _ptr(y), batch,
                                               float(lr), _ptr(ws), _ptr(loss), _ptr(grads), _stream(stream)))


def recon_stats(ctx):
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load_library().recon_stats(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def recon_destroy(ctx):
    load_library().recon_destroy(ctx)


def recon_version() -> str:
    return load_library().recon_version().decode()


# ---------------------------------------------------------------------------
# convenience owner of the device buffers
# ---------------------------------------------------------------------------
class Reconstruction:
    """Owns G, W and the workspace as torch tensors on `device` and a context.

    insert() hands slices and quaternions (device tensors) to the library in
    chunks of at most max_batch; finalize() returns V as a complex64 tensor.
    static_workspace=True takes the library's static workspace
    (recon_init_static) instead of allocating one."""

    def __init__(self, n: int, device="cuda", stream=None, static_workspace=False, **overrides):
        load_library()
        self.params = recon_default_params(n)
        for k, v in overrides.items():
            setattr(self.params, k, v)
        gb, wb, wsb = recon_query_sizes(self.params)
        dim = n + 1
        self.device = torch.device(device)
        self.G = torch.empty((dim, dim, dim), dtype=torch.complex64, device=self.device)
        self.W = torch.empty((dim, dim, dim), dtype=torch.float32, device=self.device)
        assert self.G.numel() * 8 == gb and self.W.numel() * 4 == wb
        self.stream = stream
        if static_workspace:
            self.ws = None
            self.ctx = recon_init_static(self.params, self.G, self.W, stream)
        else:
            self.ws = torch.empty(wsb, dtype=torch.uint8, device=self.device)
            self.ctx = recon_init(self.params, self.G, self.W, self.ws, stream)
        self._keep = []

    @property
    def n(self) -> int:
        return int(self.params.n)

    def set_config(self, **kw):
        cfg = recon_get_config(self.ctx)
        for k, v in kw.items():
            setattr(cfg, k, v)
        recon_set_config(self.ctx, cfg)

    def config(self) -> dict:
        c = recon_get_config(self.ctx)
        return {k: getattr(c, k) for k, _ in recon_config._fields_ if k != "reserved"}

    def insert(self, slices, quats, scales=None):
        S = int(quats.shape[0])
        if S == 0:
            return
        n, w = self.n, self.n // 2 + 1
        if slices.device != self.device or quats.device != self.device:
            raise ValueError("slices and quaternions must be on the reconstruction's device")
        if tuple(quats.shape) != (S, 4) or quats.dtype != torch.float32 or not quats.is_contiguous():
            raise ValueError("quats must be a contiguous float32 [S, 4] tensor")
        dt = int(self.params.slice_dtype)
        want = {RECON_SLICE_C64: (torch.complex64, (S, n, w)), RECON_SLICE_F16: (torch.float16, (S, n, w, 2)),
                RECON_SLICE_BF16: (torch.bfloat16, (S, n, w, 2))}[dt]
        if slices.dtype != want[0] or tuple(slices.shape) != want[1] or not slices.is_contiguous():
            raise ValueError(f"slices must be a contiguous {want[0]} tensor of shape {want[1]}")
        if dt == RECON_SLICE_F16 and (scales is None or scales.dtype != torch.float32 or scales.shape != (S,)):
            raise ValueError("half-precision slices need float32 scales of shape [S]")
        mb = int(self.params.max_batch)
        for s0 in range(0, S, mb):
            s1 = min(S, s0 + mb)
            recon_insert_batch(self.ctx, slices[s0:s1], None if scales is None else scales[s0:s1],
                               quats[s0:s1], s1 - s0)

    def finalize(self, w_threshold: float = 0.0, out=None):
        V = out if out is not None else torch.empty_like(self.G)
        recon_finalize(self.ctx, V, w_threshold)
        return V

    def reset(self):
        recon_reset(self.ctx)

    def stats(self):
        return recon_stats(self.ctx)

    def close(self):
        if self.ctx is not None:
            recon_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
