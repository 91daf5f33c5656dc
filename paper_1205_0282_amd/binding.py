"""Python binding of the brickcast C ABI (``include/brickcast.h``).

Argument marshalling only: every step of the ray caster runs in the HIP
library.  PyTorch provides the device memory the library asks for and the
stream frames are enqueued on.  There is no fallback: if the library has not
been built, :func:`load_library` raises :class:`LibraryMissing`.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbrickcast.so")

BC_OK, BC_E_ARG, BC_E_STATE, BC_E_NOMEM, BC_E_HIP, BC_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FORMATS = {"f32": 0, "f16": 1, "fp8": 2}
SRC_DTYPES = {"f32": 0, "f16": 1}

EXPORTS = [
    "bc_create", "bc_destroy", "bc_last_error", "bc_plan", "bc_bind_memory", "bc_load_bricks",
    "bc_set_transfer_function", "bc_set_view", "bc_render_frame", "bc_get_frame_stats",
    "bc_get_bricks", "bc_get_visibility_order", "bc_get_rects", "bc_read_brick",
    "bc_enable_timing", "bc_get_timing", "bc_set_option",
    "bc_cnn_plan", "bc_cnn_bind", "bc_cnn_set_weights", "bc_cnn_get_weights", "bc_cnn_forward",
    "bc_cnn_gradients", "bc_cnn_train_step", "bc_set_learned", "bc_autotune", "bc_get_frame_times",
    "bc_set_operator", "bc_render_frame_static",
]
BC_STATIC_MAX_TILES = 65536
CNN_N_PARAMS = 15056
BC_OPT_EMPTY_SKIP, BC_OPT_RENDER_WORKGROUPS, BC_OPT_SAMPLE_CHUNK, BC_OPT_GRAPH, BC_OPT_XCD_QUEUES = 0, 1, 2, 3, 4
BC_OPT_TILE_WIDTH = 5
BC_OP_COMPOSITE, BC_OP_MIP = 0, 1
BC_STEP_FIXED, BC_STEP_PER_VOXEL = 0, 1


class LibraryMissing(RuntimeError):
    pass


class BrickcastError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"brickcast error {code}: {msg}")
        self.code = code


class VolumeDesc(C.Structure):
    _fields_ = [("global_dims", C.c_int64 * 3), ("share_lo", C.c_int64 * 3), ("share_hi", C.c_int64 * 3),
                ("brick_dims", C.c_int32 * 3), ("ghost", C.c_int32), ("storage", C.c_int32),
                ("src_dtype", C.c_int32)]


class View(C.Structure):
    _fields_ = [("modelview", C.c_double * 16), ("projection", C.c_double * 16), ("width", C.c_int32),
                ("height", C.c_int32), ("step", C.c_double), ("ert_threshold", C.c_double)]


class FrameStats(C.Structure):
    _fields_ = [("nominal_samples", C.c_uint64), ("evaluated_samples", C.c_uint64),
                ("n_tiles", C.c_uint32), ("fell_back", C.c_int32), ("psnr_db", C.c_float),
                ("reserved", C.c_uint32)]


_LIB = None


def load_library(path: str = LIB_PATH):
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} is not built; run `python -m paper_1205_0282_amd.build`")
    # PyTorch first: its HIP runtime is then the one the library binds to (a
    # second runtime loaded ahead of PyTorch's leaves PyTorch without devices)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, I, I64, D, F = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_float
    sig = {
        "bc_create": (I, [I, C.POINTER(P)]),
        "bc_destroy": (None, [P]),
        "bc_last_error": (C.c_char_p, [P]),
        "bc_plan": (I, [P, C.POINTER(VolumeDesc), I, I, I, I64, C.POINTER(C.c_size_t)]),
        "bc_bind_memory": (I, [P, C.POINTER(P), C.POINTER(C.c_size_t)]),
        "bc_load_bricks": (I, [P, P, C.POINTER(C.c_int64), I]),
        "bc_set_transfer_function": (I, [P, C.POINTER(F), I, D, D, D]),
        "bc_set_view": (I, [P, C.POINTER(View), I]),
        "bc_render_frame": (I, [P, P, P]),
        "bc_render_frame_static": (I, [P, P, P]),
        "bc_get_frame_stats": (I, [P, C.POINTER(FrameStats)]),
        "bc_get_bricks": (I, [P, C.POINTER(C.c_int32), C.POINTER(F), C.POINTER(F), I, C.POINTER(I)]),
        "bc_get_visibility_order": (I, [P, I, C.POINTER(C.c_int32), I]),
        "bc_get_rects": (I, [P, I, C.POINTER(C.c_int32), I]),
        "bc_read_brick": (I, [P, I, P, C.c_size_t, C.POINTER(C.c_int32)]),
        "bc_enable_timing": (I, [P, I]),
        "bc_set_option": (I, [P, I, I64]),
        "bc_cnn_plan": (I, [P, I, I, I, C.POINTER(C.c_size_t)]),
        "bc_set_learned": (I, [P, I, D, D, I]),
        "bc_set_operator": (I, [P, I, I]),
        "bc_autotune": (I, [P, P, P, I, C.POINTER(C.c_int64)]),
        "bc_get_frame_times": (I, [P, C.POINTER(C.c_double), I, C.POINTER(I)]),
        "bc_cnn_bind": (I, [P, P, C.c_size_t]),
        "bc_cnn_set_weights": (I, [P, C.POINTER(F), C.POINTER(F), C.POINTER(F), C.c_size_t, I64]),
        "bc_cnn_get_weights": (I, [P, C.POINTER(F), C.POINTER(F), C.POINTER(F), C.c_size_t, C.POINTER(I64)]),
        "bc_cnn_forward": (I, [P, P, P, I, I, I, P]),
        "bc_cnn_gradients": (I, [P, P, P, I, I, I, C.POINTER(F), C.POINTER(F)]),
        "bc_cnn_train_step": (I, [P, P, P, I, I, I, F, C.POINTER(F), P]),
        "bc_get_timing": (I, [P, C.POINTER(C.c_double), C.POINTER(I)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _view_struct(v) -> View:
    s = View()
    s.modelview[:] = [float(x) for x in np.asarray(v.modelview, dtype=np.float64).reshape(16)]
    s.projection[:] = [float(x) for x in np.asarray(v.projection, dtype=np.float64).reshape(16)]
    s.width, s.height = int(v.width), int(v.height)
    s.step, s.ert_threshold = float(v.step), float(v.ert)
    return s


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class BrickCaster:
    """One context on one GPU: plan, bind (torch-allocated), load, set the
    transfer function and views, render."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.bc_create(device, C.byref(h))
        if rc != BC_OK:
            raise BrickcastError(rc, self.lib.bc_last_error(None).decode())
        self.h = h
        self.regions = None
        self.n_views = 0
        self.width = self.height = 0

    # ------------------------------------------------------------ plumbing
    def _check(self, rc):
        if rc != BC_OK:
            raise BrickcastError(rc, self.lib.bc_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.bc_destroy(self.h)
            self.h = None
        self.regions = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- plan
    def plan(self, global_dims, brick_dims, storage="f32", src_dtype="f32", share=None,
             max_views=1, max_w=1920, max_h=1080, max_tiles=0):
        d = VolumeDesc()
        d.global_dims[:] = [int(x) for x in global_dims]
        lo, hi = share if share is not None else ((0, 0, 0), tuple(global_dims))
        d.share_lo[:] = [int(x) for x in lo]
        d.share_hi[:] = [int(x) for x in hi]
        d.brick_dims[:] = [int(x) for x in brick_dims]
        d.ghost = 1
        d.storage = FORMATS[storage] if isinstance(storage, str) else int(storage)
        d.src_dtype = SRC_DTYPES[src_dtype] if isinstance(src_dtype, str) else int(src_dtype)
        sizes = (C.c_size_t * 4)()
        self._check(self.lib.bc_plan(self.h, C.byref(d), max_views, max_w, max_h, int(max_tiles), sizes))
        self.desc = d
        self.storage = storage
        self.src_dtype = src_dtype
        self.planned_sizes = [int(s) for s in sizes]
        return self.planned_sizes

    def bind(self):
        import torch
        dev = torch.device("cuda", self.device)
        self.regions = [torch.empty(max(s, 256), dtype=torch.uint8, device=dev) for s in self.planned_sizes]
        ptrs = (C.c_void_p * 4)(*[r.data_ptr() for r in self.regions])
        sizes = (C.c_size_t * 4)(*[r.numel() for r in self.regions])
        self._check(self.lib.bc_bind_memory(self.h, ptrs, sizes))

    # ---------------------------------------------------------------- load
    def load(self, volume):
        """volume: numpy array (host) or torch tensor (device), [z][y][x],
        covering the share plus its ghost halo clamped to the cube."""
        import torch
        if isinstance(volume, torch.Tensor):
            assert volume.is_cuda and volume.dtype == (torch.float32 if self.src_dtype == "f32" else torch.float16)
            strides = (C.c_int64 * 3)(volume.stride(2), volume.stride(1), volume.stride(0))
            self._check(self.lib.bc_load_bricks(self.h, C.c_void_p(volume.data_ptr()), strides, 1))
        else:
            v = np.asarray(volume)
            assert v.dtype == (np.float32 if self.src_dtype == "f32" else np.float16)
            es = v.itemsize
            strides = (C.c_int64 * 3)(v.strides[2] // es, v.strides[1] // es, v.strides[0] // es)
            self._check(self.lib.bc_load_bricks(self.h, C.c_void_p(v.ctypes.data), strides, 0))

    # ------------------------------------------------------------ requests
    def set_transfer_function(self, rgba, vmin, vmax, dt_ref=1.0):
        t = np.ascontiguousarray(rgba, dtype=np.float32)
        self._check(self.lib.bc_set_transfer_function(self.h, _ptr(t, C.c_float), t.shape[0],
                                                      float(vmin), float(vmax), float(dt_ref)))

    def set_views(self, views):
        arr = (View * len(views))(*[_view_struct(v) for v in views])
        self._check(self.lib.bc_set_view(self.h, arr, len(views)))
        self.n_views = len(views)
        self.width, self.height = int(views[0].width), int(views[0].height)

    def render(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.n_views, self.height, self.width, 4), dtype=torch.float32,
                              device=torch.device("cuda", self.device))
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.bc_render_frame(self.h, C.c_void_p(out.data_ptr()), C.c_void_p(st)))
        return out

    def render_static(self, out=None, stream=None):
        """bc_render_frame_static: the same frame with the sub-image tiles in
        the library's fixed device array (no allocation by the library)."""
        import torch
        if out is None:
            out = torch.empty((self.n_views, self.height, self.width, 4), dtype=torch.float32,
                              device=torch.device("cuda", self.device))
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.bc_render_frame_static(self.h, C.c_void_p(out.data_ptr()), C.c_void_p(st)))
        return out

    # ------------------------------------------------------------- queries
    def stats(self):
        s = FrameStats()
        self._check(self.lib.bc_get_frame_stats(self.h, C.byref(s)))
        return {"nominal_samples": int(s.nominal_samples), "evaluated_samples": int(s.evaluated_samples),
                "n_tiles": int(s.n_tiles), "fell_back": int(s.fell_back), "psnr_db": float(s.psnr_db)}

    def set_option(self, option, value):
        self._check(self.lib.bc_set_option(self.h, int(option), int(value)))

    def enable_timing(self, on=True, stages=True):
        """Opens a timing window: events around every stage (stages=True) or
        only around the ray-casting kernel (stages=False, fewer events
        between the frame's kernels); on=False closes it."""
        self._check(self.lib.bc_enable_timing(self.h, 0 if not on else (1 if stages else 2)))

    def timing(self):
        """(summed ms of set-up, ray casting, compositing; frames) since
        enable_timing."""
        ms = (C.c_double * 3)()
        n = C.c_int()
        self._check(self.lib.bc_get_timing(self.h, ms, C.byref(n)))
        return [float(x) for x in ms], int(n.value)

    def autotune(self, out=None, frames=3, stream=None):
        """Times every candidate launch shape on the current views and keeps
        the fastest; returns (chunk, workgroups, tile width)."""
        import torch
        if out is None:
            out = torch.empty((self.n_views, self.height, self.width, 4), dtype=torch.float32,
                              device=torch.device("cuda", self.device))
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        ch = (C.c_int64 * 3)()
        self._check(self.lib.bc_autotune(self.h, C.c_void_p(out.data_ptr()), C.c_void_p(st), int(frames), ch))
        return int(ch[0]), int(ch[1]), int(ch[2])

    def set_operator(self, op="composite", step="fixed"):
        """op: "composite" or "mip"; step: "fixed" (the views' step) or "voxel"
        (one sample per voxel slice along each ray's dominant axis)."""
        ops = {"composite": BC_OP_COMPOSITE, "mip": BC_OP_MIP}
        steps = {"fixed": BC_STEP_FIXED, "voxel": BC_STEP_PER_VOXEL}
        if isinstance(op, str) and op not in ops or isinstance(step, str) and step not in steps:
            raise ValueError(f"unknown operator {op!r} or step policy {step!r}")
        o = ops[op] if isinstance(op, str) else int(op)
        st = steps[step] if isinstance(step, str) else int(step)
        self._check(self.lib.bc_set_operator(self.h, o, st))

    def set_learned(self, enable=True, coarse_step=2.0, psnr_threshold_db=40.0, validate_stride=8):
        self._check(self.lib.bc_set_learned(self.h, 1 if enable else 0, float(coarse_step),
                                            float(psnr_threshold_db), int(validate_stride)))

    # -------------------------------------------------------- upsampler
    def cnn_setup(self, max_n, max_h, max_w):
        import torch
        nb = C.c_size_t()
        self._check(self.lib.bc_cnn_plan(self.h, max_n, max_h, max_w, C.byref(nb)))
        self.cnn_ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=torch.device("cuda", self.device))
        self._check(self.lib.bc_cnn_bind(self.h, C.c_void_p(self.cnn_ws.data_ptr()), self.cnn_ws.numel()))

    def cnn_set_weights(self, w, adam_m=None, adam_v=None, step=0):
        w = np.ascontiguousarray(w, dtype=np.float32)
        m = None if adam_m is None else np.ascontiguousarray(adam_m, dtype=np.float32)
        v = None if adam_v is None else np.ascontiguousarray(adam_v, dtype=np.float32)
        self._check(self.lib.bc_cnn_set_weights(self.h, _ptr(w, C.c_float), None if m is None else _ptr(m, C.c_float),
                                                None if v is None else _ptr(v, C.c_float), w.size, int(step)))

    def cnn_get_weights(self):
        w = np.zeros(CNN_N_PARAMS, np.float32)
        m = np.zeros(CNN_N_PARAMS, np.float32)
        v = np.zeros(CNN_N_PARAMS, np.float32)
        step = C.c_int64()
        self._check(self.lib.bc_cnn_get_weights(self.h, _ptr(w, C.c_float), _ptr(m, C.c_float), _ptr(v, C.c_float),
                                                CNN_N_PARAMS, C.byref(step)))
        return w, m, v, int(step.value)

    def cnn_forward(self, coarse, out=None, stream=None):
        """coarse: (n, h, w, 4) float32 CUDA tensor -> (n, 2h, 2w, 4)."""
        import torch
        n, h, w, _ = coarse.shape
        if out is None:
            out = torch.empty((n, 2 * h, 2 * w, 4), dtype=torch.float32, device=coarse.device)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.bc_cnn_forward(self.h, C.c_void_p(coarse.data_ptr()), C.c_void_p(out.data_ptr()),
                                            n, h, w, C.c_void_p(st)))
        return out

    def cnn_gradients(self, coarse, target):
        import torch
        torch.cuda.synchronize()
        n, h, w, _ = coarse.shape
        g = np.zeros(CNN_N_PARAMS, np.float32)
        loss = C.c_float()
        self._check(self.lib.bc_cnn_gradients(self.h, C.c_void_p(coarse.data_ptr()), C.c_void_p(target.data_ptr()),
                                              n, h, w, _ptr(g, C.c_float), C.byref(loss)))
        return g, float(loss.value)

    def cnn_train_step(self, coarse, target, lr=1e-3, want_loss=True, stream=None):
        import torch
        n, h, w, _ = coarse.shape
        loss = C.c_float()
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.bc_cnn_train_step(self.h, C.c_void_p(coarse.data_ptr()), C.c_void_p(target.data_ptr()),
                                               n, h, w, float(lr), C.byref(loss) if want_loss else None,
                                               C.c_void_p(st)))
        return float(loss.value) if want_loss else None

    def frame_times(self, cap=4096):
        """Whole-frame ms of every frame timed since enable_timing."""
        ms = (C.c_double * cap)()
        n = C.c_int()
        self._check(self.lib.bc_get_frame_times(self.h, ms, cap, C.byref(n)))
        return [float(ms[i]) for i in range(min(cap, n.value))]

    def bricks(self):
        n = C.c_int()
        self._check(self.lib.bc_get_bricks(self.h, None, None, None, 0, C.byref(n)))
        lohi = np.zeros((n.value, 6), np.int32)
        so = np.zeros((n.value, 2), np.float32)
        mm = np.zeros((n.value, 2), np.float32)
        self._check(self.lib.bc_get_bricks(self.h, _ptr(lohi, C.c_int32), _ptr(so, C.c_float),
                                           _ptr(mm, C.c_float), n.value, C.byref(n)))
        return lohi, so, mm

    def visibility_order(self, view=0):
        n = self.bricks()[0].shape[0]
        o = np.zeros(n, np.int32)
        self._check(self.lib.bc_get_visibility_order(self.h, view, _ptr(o, C.c_int32), n))
        return o

    def rects(self, view=0):
        n = self.bricks()[0].shape[0]
        r = np.zeros((n, 4), np.int32)
        self._check(self.lib.bc_get_rects(self.h, view, _ptr(r, C.c_int32), n))
        return r

    def read_brick(self, b):
        dims = (C.c_int32 * 3)()
        self._check(self.lib.bc_read_brick(self.h, b, None, 0, dims))
        gx, gy, gz = dims[0], dims[1], dims[2]
        dt = {"f32": np.float32, "f16": np.uint16, "fp8": np.uint8}[self.storage]
        buf = np.zeros((gx // 4) * (gy // 4) * (gz // 4) * 80, dtype=dt)
        self._check(self.lib.bc_read_brick(self.h, b, C.c_void_p(buf.ctypes.data), buf.nbytes, dims))
        return buf, (gx, gy, gz)


def unswizzle(buf, padded_dims):
    """Stored brick elements -> array [z][y][x] of the padded ghosted brick.
    Layout: 4x4x4 micro-blocks in row-major order, each 16 rows (y, then z) of
    5 elements, x fastest, the fifth repeating the first voxel of the next
    micro-block along x.  For layout tests."""
    gx, gy, gz = padded_dims
    mbx, mby, mbz = gx // 4, gy // 4, gz // 4
    e = np.arange(mbx * mby * mbz * 80)
    mbi, inn = e // 80, e % 80
    row, wx = inn // 5, inn % 5
    keep = wx < 4
    x = (mbi % mbx) * 4 + wx
    y = ((mbi // mbx) % mby) * 4 + (row & 3)
    z = (mbi // (mbx * mby)) * 4 + (row >> 2)
    out = np.zeros((gz, gy, gx), dtype=buf.dtype)
    out[z[keep], y[keep], x[keep]] = buf[keep]
    return out


def row_tails(buf, padded_dims):
    """The fifth element of every stored row, with the voxel it repeats (the
    first voxel of the next micro-block along x, or the row's last voxel at
    the end of the padded brick), both as flat arrays.  For layout tests."""
    gx, gy, gz = padded_dims
    full = unswizzle(buf, padded_dims)
    mbx, mby, mbz = gx // 4, gy // 4, gz // 4
    e = np.arange(mbx * mby * mbz * 80)
    mbi, inn = e // 80, e % 80
    row, wx = inn // 5, inn % 5
    t = wx == 4
    x = np.minimum((mbi % mbx) * 4 + 4, gx - 1)
    y = ((mbi // mbx) % mby) * 4 + (row & 3)
    z = (mbi // (mbx * mby)) * 4 + (row >> 2)
    return buf[t], full[z[t], y[t], x[t]]
