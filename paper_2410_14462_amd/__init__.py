"""Python binding of liblv.so, the gfx950 library for learning-free feature
uplifting onto Gaussian Splatting scenes and graph diffusion (LUDVIG,
arXiv 2410.14462).  Argument marshalling only: every step of the computation
runs in the library's HIP kernels.  PyTorch supplies device memory and the
current stream.  The names follow include/lv.h.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblv.so")

LV_F32, LV_BF16, LV_FP8_E4M3 = 0, 1, 2
# the same element types in the pixel-block layout of lv_encode_map
LV_F32_PX8, LV_BF16_PX8, LV_FP8_E4M3_PX8 = 3, 4, 5
LV_ERR_CANCELLED = 5
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
LV_ACCUM_COUNTS = 1
LV_ACCUM_DETERMINISTIC = 2
LV_GRAPH_SPATIAL_COSINE, LV_GRAPH_FEATURE_RBF = 0, 1
_DTYPES = {"f32": LV_F32, "bf16": LV_BF16, "fp8": LV_FP8_E4M3,
           "f32_px8": LV_F32_PX8, "bf16_px8": LV_BF16_PX8, "fp8_px8": LV_FP8_E4M3_PX8}


class LvError(RuntimeError):
    pass


class lv_camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("znear", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class lv_view_debug(ctypes.Structure):
    _fields_ = [("visible", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("rect", ctypes.c_void_p),
                ("rec", ctypes.c_void_p), ("tile_start", ctypes.c_void_p), ("ids", ctypes.c_void_p),
                ("ids_capacity", ctypes.c_int64)]


class lv_feature_set(ctypes.Structure):
    _fields_ = [("acc", ctypes.c_void_p), ("maps", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("stride", ctypes.c_int32)]


class lv_graph_opts(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("bandwidth", ctypes.c_float), ("unary", ctypes.c_void_p),
                ("binarize", ctypes.c_float)]


class lv_scene_opts(ctypes.Structure):
    _fields_ = [("alpha_max", ctypes.c_float), ("alpha_min", ctypes.c_float), ("t_eps", ctypes.c_float),
                ("dilation", ctypes.c_float), ("tile", ctypes.c_int32), ("flags", ctypes.c_uint32)]


LV_SCENE_CALLER_ORDER = 1


class lv_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("workers", ctypes.c_int32),
                ("max_sets", ctypes.c_int32), ("max_channels", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("scratch_bytes", ctypes.c_int64)]


class lv_request(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("cams", ctypes.c_void_p), ("m", ctypes.c_int32),
                ("maps", ctypes.c_void_p), ("stride", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("scales", ctypes.c_void_p), ("D", ctypes.c_int32), ("out_feat", ctypes.c_void_p),
                ("out_wsum", ctypes.c_void_p), ("tag", ctypes.c_uint64), ("stream", ctypes.c_void_p)]


class lv_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("t_submit", ctypes.c_int64), ("t_start", ctypes.c_int64), ("t_end", ctypes.c_int64),
                ("t_admit", ctypes.c_int64), ("bytes", ctypes.c_int64), ("D", ctypes.c_int32),
                ("views", ctypes.c_int32)]


class lv_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("passes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64), ("budget", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("peak_device_bytes", ctypes.c_int64)]


class lv_uplift_set(ctypes.Structure):
    _fields_ = [("maps", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("D", ctypes.c_int32),
                ("out_feat", ctypes.c_void_p), ("out_wsum", ctypes.c_void_p)]


class lv_uplift_stats(ctypes.Structure):
    _fields_ = [("views", ctypes.c_int64), ("pairs", ctypes.c_int64), ("visible", ctypes.c_int64),
                ("covered_pixels", ctypes.c_int64), ("contributions", ctypes.c_int64),
                ("partial_sums", ctypes.c_int64)]


assert ctypes.sizeof(lv_camera) == 80

_lib = None


def lib():
    """Load liblv.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LvError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_14462_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        sig = {
            "lv_last_error": ([], ctypes.c_char_p),
            "lv_version": ([], ctypes.c_char_p),
            "lv_scene_create": ([P, P, P, P, i64, ctypes.POINTER(lv_scene_opts), P, ctypes.POINTER(P)], i32),
            "lv_accum_export": ([P, P, P, P, P], i32),
            "lv_accum_import": ([P, P, P, P, P], i32),
            "lv_scene_destroy": ([P], i32),
            "lv_scene_size": ([P], i64),
            "lv_uplift": ([P, P, i32, P, i32, P, i32, P, P, P], i32),
            "lv_accum_create": ([P, i32, u32, P, ctypes.POINTER(P)], i32),
            "lv_accum_reset": ([P, P], i32),
            "lv_uplift_accumulate": ([P, P, i32, P, i32, P, P], i32),
            "lv_accum_finalize": ([P, P, P, P, P], i32),
            "lv_accum_counts": ([P, P, P], i32),
            "lv_accum_finalize_count": ([P, P, P], i32),
            "lv_prune_by_weight": ([P, i64, i64, P, P], i32),
            "lv_graph_build_knn": ([P, P, i32, i32, ctypes.POINTER(lv_graph_opts), P, ctypes.POINTER(P)], i32),
            "lv_anchor_init": ([P, i64, ctypes.c_float, P, P], i32),
            "lv_reach_unary": ([P, P, i64, i32, P, P], i32),
            "lv_graph_csr": ([P, ctypes.POINTER(i64), ctypes.POINTER(i64), P, P, P, P], i32),
            "lv_accum_destroy": ([P], i32),
            "lv_encode": ([P, i64, i32, i32, P, P, P], i32),
            "lv_encode_noalloc": ([P, i64, i32, i32, P, P, P], i32),
            "lv_encode_map": ([P, i32, i32, i32, i32, P, P, P], i32),
            "lv_graph_create_csr": ([i64, i64, P, P, P, i32, P, ctypes.POINTER(P)], i32),
            "lv_graph_destroy": ([P], i32),
            "lv_diffuse": ([P, P, P, i32, i32, i32, P, P], i32),
            "lv_debug_view": ([P, P, ctypes.POINTER(lv_view_debug), ctypes.POINTER(i64)], i32),
            "lv_accum_stats": ([P, ctypes.POINTER(lv_uplift_stats)], i32),
            "lv_uplift_sets": ([P, P, i32, P, i32, i32, P], i32),
            "lv_uplift_accumulate_sets": ([P, i32, P, i32, i32, P], i32),
            "lv_profile_start": ([], i32),
            "lv_profile_stop": ([ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double), P, i64], i32),
            "lv_render": ([P, P, i32, P, i32, P, P, P], i32),
            "lv_server_create": ([ctypes.POINTER(lv_server_opts), ctypes.POINTER(P)], i32),
            "lv_server_submit": ([P, ctypes.POINTER(lv_request)], i32),
            "lv_server_poll": ([P, P, i32, ctypes.POINTER(i32)], i32),
            "lv_server_drain": ([P], i32),
            "lv_server_stats_get": ([P, ctypes.POINTER(lv_server_stats)], i32),
            "lv_server_destroy": ([P], i32),
            "lv_server_cancel": ([P, ctypes.c_uint64], i32),
            "lv_set_allocator": ([ALLOC_FN, FREE_FN, P], i32),
            "lv_release_scratch": ([P, i32], i32),
            "lv_memory_stats": ([ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return ["lv_last_error", "lv_version", "lv_scene_create", "lv_scene_destroy", "lv_scene_size",
            "lv_uplift", "lv_accum_create", "lv_accum_reset", "lv_uplift_accumulate",
            "lv_accum_finalize", "lv_accum_counts", "lv_accum_destroy", "lv_encode", "lv_encode_noalloc",
            "lv_encode_map",
            "lv_graph_create_csr", "lv_graph_destroy", "lv_diffuse", "lv_debug_view",
            "lv_accum_stats", "lv_profile_start", "lv_profile_stop", "lv_uplift_sets",
            "lv_uplift_accumulate_sets", "lv_render", "lv_server_create", "lv_server_submit", "lv_server_poll",
            "lv_server_drain", "lv_server_stats_get", "lv_server_destroy", "lv_accum_finalize_count",
            "lv_prune_by_weight", "lv_graph_build_knn", "lv_graph_csr", "lv_anchor_init", "lv_reach_unary",
            "lv_server_cancel", "lv_set_allocator", "lv_release_scratch", "lv_memory_stats",
            "lv_accum_export", "lv_accum_import"]


def _check(status):
    if status != 0:
        msg = lib().lv_last_error().decode(errors="replace")
        raise LvError(f"lv status {status}: {msg}")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f32(t, shape=None):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise LvError("expected a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise LvError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


def camera_struct(cam):
    c = lv_camera()
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.znear = float(cam.znear)
    c.width, c.height, c.reserved = int(cam.width), int(cam.height), 0
    return c


_CAM_DTYPE = np.dtype([("R", np.float32, 9), ("t", np.float32, 3), ("f", np.float32, 5),
                       ("wh", np.int32, 3)])
assert _CAM_DTYPE.itemsize == ctypes.sizeof(lv_camera)


def camera_array(cams):
    """lv_camera[m] (same layout as the C struct), filled column-wise."""
    m = len(cams)
    a = np.zeros(max(1, m), _CAM_DTYPE)
    if m:
        a["R"][:m] = np.asarray([c.R for c in cams], np.float32).reshape(m, 9)
        a["t"][:m] = np.asarray([c.t for c in cams], np.float32).reshape(m, 3)
        a["f"][:m] = np.asarray([(c.fx, c.fy, c.cx, c.cy, c.znear) for c in cams], np.float32)
        a["wh"][:m, :2] = np.asarray([(c.width, c.height) for c in cams], np.int64)
    return (lv_camera * max(1, m)).from_buffer(a)


class Cameras:
    """A camera rig marshalled once into lv_camera[m]; accepted wherever a
    list of cameras is (saves the per-call marshalling of the rig)."""

    def __init__(self, cams):
        self.cams = list(cams)
        self.array = camera_array(self.cams)

    def __len__(self):
        return len(self.cams)

    def __getitem__(self, i):
        return self.cams[i]

    def __iter__(self):
        return iter(self.cams)


class Maps:
    """Contiguous maps [H, W, D] of one dtype, validated and marshalled once
    into a device-pointer table (the tensors are kept alive; they must keep
    their storage, not be resized or re-allocated in place, while the table
    is in use); accepted wherever a list of maps is."""

    def __init__(self, maps, dtype="f32"):
        self.maps = list(maps)
        self.dtype = _DTYPES[dtype]
        self.table = _map_table(self.maps, self.dtype)

    def __len__(self):
        return len(self.maps)

    def __getitem__(self, i):
        return self.maps[i]


def _cams(cams):
    return cams.array if isinstance(cams, Cameras) else camera_array(cams)


def _maps(maps, dtype):
    if isinstance(maps, Maps):
        if maps.dtype != dtype:
            raise LvError("map table built for another dtype")
        return maps.table
    return _map_table(maps, dtype)


def _elem_torch(dtype):
    """torch dtypes accepted for maps of an lv dtype (either layout)."""
    import torch
    return {LV_F32: (torch.float32,), LV_BF16: (torch.bfloat16,),
            LV_FP8_E4M3: (torch.uint8, getattr(torch, "float8_e4m3fn", torch.uint8))}[dtype % 3]


def _map_channels(mp, dtype):
    """D of a map: [H, W, D] (HWC) or [H, ceil(W/8), D, 8] (pixel blocks)."""
    return int(mp.shape[2]) if dtype >= LV_F32_PX8 else int(mp.shape[-1])


def _map_table(maps, dtype):
    want = _elem_torch(dtype)
    tab = (ctypes.c_void_p * max(1, len(maps)))()
    for i, mp in enumerate(maps):
        if not (mp.is_cuda and mp.is_contiguous() and mp.dtype in want):
            raise LvError(f"map {i}: expected a contiguous CUDA tensor of {want}")
        tab[i] = mp.data_ptr()
    return tab


# lv_scene_opts defaults: the FP32 literals 0.99f, 1/255.f, 1e-4f, 0.3f and 16
SCENE_DEFAULTS = (float(np.float32(0.99)), float(np.float32(1.0) / np.float32(255.0)),
                  float(np.float32(1e-4)), float(np.float32(0.3)), 16)


class Scene:
    """lv_scene: Gaussians resident on the GPU (means, scales, quats, opacity)."""

    def __init__(self, means, scales, quats, opacity, opts=None, order="morton"):
        """opts: None or a dict of lv_scene_opts fields (alpha_max, alpha_min,
        t_eps, dilation, tile).  order: "morton" (the library's default
        storage order) or "caller" (LV_SCENE_CALLER_ORDER)."""
        n = means.shape[0]
        _dev_f32(means, (n, 3)); _dev_f32(scales, (n, 3)); _dev_f32(quats, (n, 4)); _dev_f32(opacity, (n,))
        if order not in ("morton", "caller"):
            raise ValueError(f"order must be 'morton' or 'caller', not {order!r}")
        h = ctypes.c_void_p()
        o = None
        if opts is not None or order == "caller":
            opts = opts or {}
            o = lv_scene_opts(*[opts.get(k, d) for k, d in (("alpha_max", SCENE_DEFAULTS[0]),
                                                               ("alpha_min", SCENE_DEFAULTS[1]),
                                                               ("t_eps", SCENE_DEFAULTS[2]),
                                                               ("dilation", SCENE_DEFAULTS[3]),
                                                               ("tile", SCENE_DEFAULTS[4]))],
                              LV_SCENE_CALLER_ORDER if order == "caller" else 0)
        _check(lib().lv_scene_create(_ptr(means), _ptr(scales), _ptr(quats), _ptr(opacity), n,
                                     ctypes.byref(o) if o is not None else None, _stream(),
                                     ctypes.byref(h)))
        self.handle, self.n = h, n

    @classmethod
    def from_arrays(cls, scene, device="cuda", order="morton"):
        import torch
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)
        return cls(f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacity), order=order)

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lv_scene_destroy(self.handle)
            self.handle = None

    __del__ = close

    def uplift(self, cams, maps, dtype="f32", scales=None, out=None, wsum=None):
        """Eq. (3): returns (f [n,D] f32, beta [n] f32)."""
        import torch
        dt = _DTYPES[dtype]
        D = _map_channels(maps[0], dt) if maps else (out.shape[1] if out is not None else 1)
        if out is None:
            out = torch.empty((self.n, D), device="cuda", dtype=torch.float32)
        if wsum is None:
            wsum = torch.empty((self.n,), device="cuda", dtype=torch.float32)
        ca = _cams(cams)
        tab = _maps(maps, dt)
        _check(lib().lv_uplift(self.handle, ca, len(cams), tab, dt, _ptr(scales), D, _ptr(out),
                               _ptr(wsum), _stream()))
        return out, wsum

    def render(self, cams, g, alpha=True, outs=None):
        """Eq. (4): g [n, D] f32 -> ([H, W, D] per camera, [H, W] opacity per camera).
        outs: optional (maps, opacities) to write into (opacities [] when alpha
        is False), each shaped as above."""
        import torch
        if g.dim() == 1:
            g = g[:, None]
        _dev_f32(g, (self.n, g.shape[1]))
        D = g.shape[1]
        if outs is not None:
            outs, alps = outs
            if len(outs) != len(cams) or (alpha and len(alps) != len(cams)):
                raise LvError("render: one output (and opacity) per camera")
            for c, o in zip(cams, outs):
                _dev_f32(o, (c.height, c.width, D))
            if alpha:
                for c, a in zip(cams, alps):
                    _dev_f32(a, (c.height, c.width))
        else:
            outs = [torch.empty((c.height, c.width, D), device="cuda") for c in cams]
            alps = [torch.empty((c.height, c.width), device="cuda") for c in cams] if alpha else []
        to = (ctypes.c_void_p * max(1, len(cams)))(*[o.data_ptr() for o in outs])
        ta = (ctypes.c_void_p * max(1, len(cams)))(*[a.data_ptr() for a in alps]) if alpha else None
        _check(lib().lv_render(self.handle, _cams(cams), len(cams), _ptr(g), D, to, ta, _stream()))
        return outs, alps

    def uplift_sets(self, cams, sets, dtype="f32", outs=None):
        """Several feature sets over the same views in one pass.  sets: list of
        map lists (or (maps, scales) pairs).  Returns [(f, beta)] per set."""
        import torch
        dt = _DTYPES[dtype]
        arr = (lv_uplift_set * len(sets))()
        keep, res = [], []
        for k, st in enumerate(sets):
            maps, scales = st if isinstance(st, tuple) else (st, None)
            D = _map_channels(maps[0], dt)
            f, b = outs[k] if outs is not None else (
                torch.empty((self.n, D), device="cuda", dtype=torch.float32),
                torch.empty((self.n,), device="cuda", dtype=torch.float32))
            tab = _maps(maps, dt)
            keep.append(tab)
            arr[k] = lv_uplift_set(ctypes.cast(tab, ctypes.c_void_p),
                                   None if scales is None else scales.data_ptr(), D,
                                   f.data_ptr(), b.data_ptr())
            res.append((f, b))
        _check(lib().lv_uplift_sets(self.handle, _cams(cams), len(cams), arr, len(sets), dt,
                                    _stream()))
        return res

    def debug_view(self, cam):
        """Structure of one view (synchronous, host arrays)."""
        n = self.n
        TX, TY = -(-cam.width // 16), -(-cam.height // 16)
        vis = np.zeros(n, np.uint8)
        depth = np.zeros(n, np.uint32)
        rect = np.zeros((n, 4), np.int32)
        rec = np.zeros((n, 8), np.float32)
        ts = np.zeros(TX * TY + 1, np.int64)
        dbg = lv_view_debug(vis.ctypes.data, depth.ctypes.data, rect.ctypes.data, rec.ctypes.data,
                            ts.ctypes.data, None, 0)
        P = ctypes.c_int64()
        c = camera_struct(cam)
        _check(lib().lv_debug_view(self.handle, ctypes.byref(c), ctypes.byref(dbg), ctypes.byref(P)))
        ids = np.zeros(max(1, P.value), np.int32)
        dbg.ids, dbg.ids_capacity = ids.ctypes.data, P.value
        _check(lib().lv_debug_view(self.handle, ctypes.byref(c), ctypes.byref(dbg), ctypes.byref(P)))
        return dict(visible=vis.astype(bool), depth=depth, rect=rect, rec=rec, tile_start=ts,
                    ids=ids[:P.value])


class Accum:
    """lv_accum: streaming accumulator U = W^T F, beta (and counts)."""

    def __init__(self, scene, D, counts=False, deterministic=False):
        """deterministic: U in 64-bit fixed point (LV_ACCUM_DETERMINISTIC),
        the same bit for bit whatever the order of the updates."""
        h = ctypes.c_void_p()
        flags = (LV_ACCUM_COUNTS if counts else 0) | (LV_ACCUM_DETERMINISTIC if deterministic else 0)
        _check(lib().lv_accum_create(scene.handle, D, flags, _stream(), ctypes.byref(h)))
        self.handle, self.scene, self.D, self.flags = h, scene, D, flags

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lv_accum_destroy(self.handle)
            self.handle = None

    __del__ = close

    def reset(self):
        _check(lib().lv_accum_reset(self.handle, _stream()))

    def add(self, cams, maps, dtype="f32", scales=None):
        dt = _DTYPES[dtype]
        _check(lib().lv_uplift_accumulate(self.handle, _cams(cams), len(cams),
                                          _maps(maps, dt), dt, _ptr(scales), _stream()))

    def finalize(self, want_sum=False):
        import torch
        n = self.scene.n
        f = torch.empty((n, self.D), device="cuda", dtype=torch.float32)
        b = torch.empty((n,), device="cuda", dtype=torch.float32)
        u = torch.empty((n, self.D), device="cuda", dtype=torch.float32) if want_sum else None
        _check(lib().lv_accum_finalize(self.handle, _ptr(f), _ptr(b), _ptr(u), _stream()))
        return (f, b, u) if want_sum else (f, b)

    def stats(self):
        st = lv_uplift_stats()
        _check(lib().lv_accum_stats(self.handle, ctypes.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in lv_uplift_stats._fields_}

    def counts(self):
        import torch
        c = torch.empty((self.scene.n,), device="cuda", dtype=torch.int32)
        _check(lib().lv_accum_counts(self.handle, _ptr(c), _stream()))
        return c

    def export(self):
        """Checkpoint: (U [n, D] float32, or int64 fixed point for a
        deterministic accumulator; beta [n] int64 holding the uint64 fixed
        point; counts [n] int32 or None), in the caller's Gaussian order."""
        import torch
        n = self.scene.n
        det = bool(self.flags & LV_ACCUM_DETERMINISTIC)
        U = torch.empty((n, self.D), device="cuda", dtype=torch.int64 if det else torch.float32)
        beta = torch.empty((n,), device="cuda", dtype=torch.int64)
        counts = torch.empty((n,), device="cuda", dtype=torch.int32) if self.flags & LV_ACCUM_COUNTS else None
        _check(lib().lv_accum_export(self.handle, _ptr(U), _ptr(beta), _ptr(counts), _stream()))
        return U, beta, counts

    def load(self, U, beta, counts=None):
        """Resume from export()'s tensors (same scene, D and flags)."""
        _check(lib().lv_accum_import(self.handle, _ptr(U), _ptr(beta), _ptr(counts), _stream()))

    def finalize_count(self):
        """lv_accum_finalize_count: f = U / count (needs counts=True)."""
        import torch
        f = torch.empty((self.scene.n, self.D), device="cuda", dtype=torch.float32)
        _check(lib().lv_accum_finalize_count(self.handle, _ptr(f), _stream()))
        return f


def anchor_init(g, fraction=0.1):
    """lv_anchor_init: g0 keeps the ceil(fraction npos) largest positive
    entries of g (float32 [n] on the device), 0 elsewhere."""
    import torch
    _dev_f32(g)
    g0 = torch.empty_like(g)
    _check(lib().lv_anchor_init(_ptr(g), g.numel(), float(fraction), _ptr(g0), _stream()))
    return g0


def reach_unary(gT, unary):
    """lv_reach_unary: h = unary where gT > 0, else 0 (gT [n] or [n, D])."""
    import torch
    _dev_f32(gT)
    _dev_f32(unary)
    n = unary.numel()
    D = 1 if gT.dim() == 1 else gT.shape[1]
    h = torch.empty_like(gT)
    _check(lib().lv_reach_unary(_ptr(gT), _ptr(unary), n, D, _ptr(h), _stream()))
    return h


def prune_by_weight(wsum, k):
    """lv_prune_by_weight: uint8 mask [n] of the k Gaussians with the largest
    wsum (device FP32 [n]), ties to the lower index."""
    import torch
    _dev_f32(wsum)
    n = wsum.numel()
    keep = torch.empty((n,), device="cuda", dtype=torch.uint8)
    _check(lib().lv_prune_by_weight(_ptr(wsum), n, int(k), _ptr(keep), _stream()))
    return keep


def _slice_table(maps, dtype, D):
    """Maps of one set for lv_feature_set: each [H, W, D] (None: the set does
    not take that view), channels contiguous, pixels `stride` elements apart
    (a channel slice [..., :D] of a wider map is accepted).  Returns (table,
    stride)."""
    want = _elem_torch(dtype)
    px8 = dtype >= LV_F32_PX8
    tab = (ctypes.c_void_p * max(1, len(maps)))()
    stride = None
    for i, mp in enumerate(maps):
        if mp is None:
            tab[i] = None
            continue
        if px8:  # [H, ceil(W/8), D, 8], or a channel slice [..., :D, :] of a wider map
            ok = mp.is_cuda and mp.dtype in want and mp.dim() == 4 and mp.shape[2] == D and mp.shape[3] == 8
            st = mp.stride() if ok else (0, 0, 0, 0)
            px = st[1] // 8 if ok else 0
            ok = ok and st[3] == 1 and (st[2] == 8 or D == 1) and st[1] == 8 * px and px >= D \
                and st[0] == st[1] * mp.shape[1]
        elif mp.is_cuda and mp.dtype in want and mp.dim() == 3 and mp.shape[2] == D and mp.is_contiguous():
            ok, px = True, D
        else:  # a channel slice: channels adjacent, rows of W pixels
            ok = mp.is_cuda and mp.dtype in want and mp.dim() == 3 and mp.shape[2] == D
            st = mp.stride() if ok else (0, 0, 0)
            px = st[1]
            ok = ok and (st[2] == 1 or D == 1) and px >= D and st[0] == px * mp.shape[1]
        if not ok or (stride is not None and px != stride):
            raise LvError(f"map {i}: expected a CUDA [H, W, {D}] tensor of {want} with "
                          f"contiguous channels and one pixel stride per set")
        stride = px
        tab[i] = mp.data_ptr()
    return tab, (stride or D)


def accumulate_sets(cams, sets, dtype="f32"):
    """sets: list of (Accum, maps[, scales]) sharing one scene; one pass.
    maps[v] may be None (the set does not take view v) or a channel slice of a
    wider map."""
    dt = _DTYPES[dtype]
    arr = (lv_feature_set * len(sets))()
    keep = []
    for k, st in enumerate(sets):
        acc, maps = st[0], st[1]
        scales = st[2] if len(st) > 2 else None
        tab, stride = _slice_table(maps, dt, acc.D)
        keep.append(tab)
        arr[k] = lv_feature_set(acc.handle.value, ctypes.cast(tab, ctypes.c_void_p),
                                None if scales is None else scales.data_ptr(), stride)
    _check(lib().lv_uplift_accumulate_sets(_cams(cams), len(cams), arr, len(sets), dt,
                                           _stream()))


def profile_start():
    _check(lib().lv_profile_start())


def profile_stop(capacity=4096):
    """-> list of blend-launch durations (ms), in launch order, since profile_start()."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    per = np.zeros(capacity, np.float64)
    _check(lib().lv_profile_stop(ctypes.byref(n), ctypes.byref(ms), per.ctypes.data, capacity))
    return [float(x) for x in per[:min(n.value, capacity)]]


def encode(src, dtype):
    """Encode an FP32 map [..., D] to 'bf16' or 'fp8' (+ per-channel scales);
    the '_px8' types take one map [H, W, D] and return it in the pixel-block
    layout, shape [H, ceil(W/8), D, 8]."""
    import torch
    _dev_f32(src)
    D = src.shape[-1]
    pixels = src.numel() // D
    dt = _DTYPES[dtype]
    if dt >= LV_F32_PX8:
        if src.dim() != 3:
            raise LvError("pixel-block encoding takes one map [H, W, D]")
        H, W = src.shape[0], src.shape[1]
        el = _elem_torch(dt)
        dst = torch.empty((H, (W + 7) // 8, D, 8), device="cuda",
                          dtype=torch.uint8 if el[0] == torch.uint8 else el[0])
        scales = torch.empty((D,), device="cuda", dtype=torch.float32) if dt == LV_FP8_E4M3_PX8 else None
        _check(lib().lv_encode_map(_ptr(src), H, W, D, dt, _ptr(dst), _ptr(scales), _stream()))
        return dst, scales
    if dt == LV_BF16:
        dst = torch.empty(src.shape, device="cuda", dtype=torch.bfloat16)
        scales = None
    elif dt == LV_FP8_E4M3:
        dst = torch.empty(src.shape, device="cuda", dtype=torch.uint8)
        scales = torch.empty((D,), device="cuda", dtype=torch.float32)
    else:
        dst = torch.empty_like(src)
        scales = None
    _check(lib().lv_encode(_ptr(src), pixels, D, dt, _ptr(dst), _ptr(scales), _stream()))
    return dst, scales


class Graph:
    """lv_graph: CSR matrix over the Gaussians (int32 row_ptr/col, f32 or bf16 values)."""

    def __init__(self, row_ptr, col, val):
        import torch
        n = row_ptr.shape[0] - 1
        nnz = col.shape[0]
        dt = LV_BF16 if val.dtype == torch.bfloat16 else LV_F32
        if val.dtype not in (torch.float32, torch.bfloat16):
            raise LvError("graph values must be float32 or bfloat16")
        h = ctypes.c_void_p()
        _check(lib().lv_graph_create_csr(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(val), dt, _stream(),
                                         ctypes.byref(h)))
        self.handle, self.n, self.dtype = h, n, dt

    @classmethod
    def knn(cls, scene, feats, k=16, kind="spatial_cosine", bandwidth=1.0, unary=None, binarize=0.0):
        """lv_graph_build_knn: the kNN diffusion graph over the scene's centres
        with feature weights (feats [n, D] float32 on the device); kind
        "feature_rbf" gives the paper's Eq. 7 / Eq. 9 weights (bandwidth,
        unary P [n] float32 on the device or None, binarize threshold)."""
        _dev_f32(feats)
        if unary is not None:
            _dev_f32(unary)
        D = 1 if feats.dim() == 1 else feats.shape[1]
        kinds = {"spatial_cosine": LV_GRAPH_SPATIAL_COSINE, "feature_rbf": LV_GRAPH_FEATURE_RBF}
        o = lv_graph_opts(kinds[kind], float(bandwidth), None if unary is None else unary.data_ptr(),
                          float(binarize))
        h = ctypes.c_void_p()
        _check(lib().lv_graph_build_knn(scene.handle, _ptr(feats), D, int(k), ctypes.byref(o), _stream(),
                                        ctypes.byref(h)))
        g = cls.__new__(cls)
        g.handle, g.n, g.dtype = h, scene.n, LV_F32
        return g

    def csr(self):
        """(row_ptr int32 [n+1], col int32 [nnz], val [nnz]) copies on the device."""
        import torch
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lv_graph_csr(self.handle, ctypes.byref(n), ctypes.byref(nnz), None, None, None, _stream()))
        rp = torch.empty((n.value + 1,), device="cuda", dtype=torch.int32)
        col = torch.empty((nnz.value,), device="cuda", dtype=torch.int32)
        val = torch.empty((nnz.value,), device="cuda",
                          dtype=torch.bfloat16 if self.dtype == LV_BF16 else torch.float32)
        _check(lib().lv_graph_csr(self.handle, None, None, _ptr(rp), _ptr(col), _ptr(val), _stream()))
        return rp, col, val

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lv_graph_destroy(self.handle)
            self.handle = None

    __del__ = close

    def diffuse(self, g0, steps, scene=None, out=None):
        """Eq. (8): g0 [n] or [n, D] (f32 or bf16) -> g_steps, same dtype and shape."""
        import torch
        dt = LV_BF16 if g0.dtype == torch.bfloat16 else LV_F32
        D = 1 if g0.dim() == 1 else g0.shape[1]
        if out is None:
            out = torch.empty_like(g0)
        _check(lib().lv_diffuse(scene.handle if scene is not None else None, self.handle, _ptr(g0),
                                dt, D, steps, _ptr(out), _stream()))
        return out


def completion_record(c):
    """One finished request (a dict of Server.poll) as a JSON-ready dict: the
    per-request metrics (arrival, admission, start, done, D, views, bytes)."""
    return {k: c[k] for k in ("tag", "status", "batch_size", "t_submit", "t_admit", "t_start", "t_end",
                              "bytes", "D", "views")}


class Server:
    """lv_server: uplift requests admitted by memory budget, merged per scene
    into wide passes, several passes in flight (one HIP stream per worker)."""

    def __init__(self, budget=0, workers=2, max_sets=8, max_channels=1024, scratch=0):
        o = lv_server_opts(int(budget), workers, max_sets, max_channels, 0, int(scratch))
        h = ctypes.c_void_p()
        _check(lib().lv_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self._live = {}
        self._next = 0

    def submit(self, scene, cams, maps, dtype="f32", scales=None, out=None, wsum=None, tag=None):
        """maps: one [H, W, D] tensor per camera (channel slices of wider maps
        allowed).  Returns the tag; the tensors are kept alive until the
        request is polled."""
        import torch
        dt = _DTYPES[dtype]
        D = int(maps[0].shape[2])
        tab, stride = _slice_table(maps, dt, D)
        if out is None:
            out = torch.empty((scene.n, D), device="cuda", dtype=torch.float32)
        if wsum is None:
            wsum = torch.empty((scene.n,), device="cuda", dtype=torch.float32)
        if tag is None:
            tag = self._next
        self._next = max(self._next, tag + 1)
        ca = camera_array(cams)
        q = lv_request(scene.handle.value, ctypes.cast(ca, ctypes.c_void_p), len(cams),
                       ctypes.cast(tab, ctypes.c_void_p), stride, dt,
                       None if scales is None else scales.data_ptr(), D, out.data_ptr(),
                       wsum.data_ptr(), tag, _stream().value)
        _check(lib().lv_server_submit(self.handle, ctypes.byref(q)))
        self._live[tag] = (scene, list(maps), scales, out, wsum)
        return tag

    def poll(self, cap=4096):
        """Finished requests: dicts with tag, status, batch_size, times (s:
        submission, admission, start and end of the pass), admitted bytes, D,
        views and the outputs (features, weight sums).  completion_record()
        makes one JSON-ready line of a result."""
        buf = (lv_completion * cap)()
        n = ctypes.c_int32()
        _check(lib().lv_server_poll(self.handle, buf, cap, ctypes.byref(n)))
        res = []
        for c in buf[:n.value]:
            live = self._live.pop(c.tag, None)
            res.append({"tag": c.tag, "status": c.status, "batch_size": c.batch_size,
                        "t_submit": c.t_submit * 1e-9, "t_admit": c.t_admit * 1e-9,
                        "t_start": c.t_start * 1e-9, "t_end": c.t_end * 1e-9, "bytes": c.bytes,
                        "D": c.D, "views": c.views,
                        "out": live[3] if live else None, "wsum": live[4] if live else None})
        return res

    def drain(self):
        _check(lib().lv_server_drain(self.handle))

    def cancel(self, tag):
        """Cancel a waiting request: True if it was cancelled (it completes
        with status LV_ERR_CANCELLED), False if it is running or finished."""
        st = lib().lv_server_cancel(self.handle, tag)
        return st == 0

    def stats(self):
        st = lv_server_stats()
        _check(lib().lv_server_stats_get(self.handle, ctypes.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in lv_server_stats._fields_}

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lv_server_destroy(self.handle)
            self.handle = None

    __del__ = close


# ------------------------------------------------------------ device memory
_allocator = None  # keeps the registered ctypes callbacks alive


def set_allocator(alloc=None, free=None):
    """Route every device allocation of the library through Python callables
    alloc(bytes, stream) -> int pointer and free(ptr, bytes, stream); None,
    None restores hipMalloc / hipFree.  The library must hold no memory."""
    global _allocator
    if alloc is None:
        _check(lib().lv_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _allocator = None
        return
    a = ALLOC_FN(lambda nbytes, stream, ctx: alloc(int(nbytes), stream) or None)
    f = FREE_FN(lambda ptr, nbytes, stream, ctx: free(ptr, int(nbytes), stream))
    _check(lib().lv_set_allocator(a, f, None))
    _allocator = (a, f)


def use_torch_allocator():
    """Route the library's device allocations through torch's caching
    allocator (on the stream each allocation is made for)."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(max(nbytes, 1), torch.cuda.current_device(),
                                                  stream or 0)

    def free(ptr, nbytes, stream):
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(alloc, free)


def release_scratch(all_streams=True):
    """Free the scratch the library caches (this stream's, or every stream's
    and the buffers of destroyed scenes)."""
    _check(lib().lv_release_scratch(_stream() if not all_streams else None, 1 if all_streams else 0))


def memory_stats():
    """-> (bytes, allocations) of device memory the library holds."""
    b, n = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().lv_memory_stats(ctypes.byref(b), ctypes.byref(n)))
    return b.value, n.value
