"""Thin ctypes binding of libshapetrace.so (the C ABI in include/shapetrace.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of rendering and differentiation runs in the HIP kernels of
the library.  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SHAPETRACE_LIB selects another build of the same library (tuning variants);
# SHAPETRACE_SANITIZE=1 the host-sanitized build (build(sanitize=True))
LIB_PATH = os.environ.get("SHAPETRACE_LIB", os.path.join(
    _HERE, "libshapetrace_san.so" if os.environ.get("SHAPETRACE_SANITIZE", "") == "1" else "libshapetrace.so"))

ST_GRAD_INTERIOR = 1
ST_EDGE_PRIMARY = 2
ST_EDGE_SECONDARY = 4
ST_EDGE_SHADOW = 8
ST_EDGE_SECONDARY_INTERIOR = 64
ST_FORWARD_MEGAKERNEL = 16
ST_COUNT_WORK = 32
ST_ALL_GRADS = 15
ST_BACKWARD_RETRACE = 128
ST_EDGE_SECONDARY_HIERARCHY = 256
ST_ENV_SAMPLER_CDF = 0
ST_ENV_SAMPLER_ALIAS = 1
ST_BSDF_SAMPLER_HALFVECTOR = 0
ST_BSDF_SAMPLER_VNDF = 1

EXPORTED = ["st_render_opts_default", "st_scene_create", "st_scene_update", "st_scene_set_mesh_colors",
            "st_scene_mesh_colors_info", "st_scene_subdivide", "st_scene_set_env_sampler", "st_scene_env_alias_table", "st_scene_set_bsdf_sampler", "st_scene_edge_tree", "st_render", "st_render_noalloc", "st_render_backward",
            "st_render_batch", "st_autotune", "st_check_errors", "st_read_work", "st_scene_info", "st_scene_edges", "st_scene_lbvh",
            "st_trace_rays", "st_stream_copy", "st_profile_enable", "st_profile_read", "st_scene_destroy", "st_last_error",
            "st_version"]


class StCamera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("target", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fov_y_deg", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class StOpts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("edge_spp_ratio", ctypes.c_float), ("queue_capacity", ctypes.c_int64),
                ("debug_decision_hash", ctypes.c_void_p), ("debug_edge_hash", ctypes.c_void_p),
                ("debug_sample_radiance", ctypes.c_void_p), ("path_mask", ctypes.c_void_p),
                ("edge_mask", ctypes.c_void_p), ("max_workspace_bytes", ctypes.c_int64)]


class StError(RuntimeError):
    pass


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (no GPU needed) and declare every exported symbol."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise StError(f"{path} is missing: build it with __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(path)
    P, I32, U32, F32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_float
    L.st_render_opts_default.restype = StOpts
    L.st_scene_create.argtypes = [P, I32, P, I32, P, P, I32, P, I32, I32, U32, P, ctypes.POINTER(P)]
    L.st_scene_update.argtypes = [P, P, P, P]
    L.st_scene_set_mesh_colors.argtypes = [P, I32, P, P]
    L.st_scene_mesh_colors_info.argtypes = [P, P, P]
    L.st_scene_subdivide.argtypes = [P, P, P, P]
    L.st_scene_set_env_sampler.argtypes = [P, I32, P]
    L.st_scene_set_bsdf_sampler.argtypes = [P, I32, P]
    L.st_scene_edge_tree.argtypes = [P, P, P, P, P, P, P, P]
    L.st_scene_env_alias_table.argtypes = [P, P, P]
    L.st_render.argtypes = [P, P, I32, I32, I32, U32, ctypes.POINTER(StOpts), P, P]
    L.st_render_noalloc.argtypes = [P, P, I32, I32, I32, U32, ctypes.POINTER(StOpts), P, P]
    L.st_stream_copy.argtypes = [P, P, ctypes.c_int64, P]
    L.st_render_backward.argtypes = [P, P, I32, I32, I32, U32, ctypes.POINTER(StOpts), P, P, P, P]
    L.st_render_batch.argtypes = [P, I32, P, P, I32, I32, I32, U32, ctypes.POINTER(StOpts), P, P]
    L.st_check_errors.argtypes = [P, P]
    L.st_autotune.argtypes = [P, I32, P, P, I32, I32, I32, ctypes.c_char_p, P, P, P]
    L.st_scene_info.argtypes = [P, P]
    L.st_read_work.argtypes = [P, P, P]
    L.st_scene_edges.argtypes = [P, P, P]
    L.st_scene_lbvh.argtypes = [P, P, P, P, P, P]
    L.st_trace_rays.argtypes = [P, P, P, I32, F32, I32, P, P, P]
    L.st_profile_enable.argtypes = [ctypes.c_int]
    L.st_profile_read.argtypes = [ctypes.c_char_p, I32, P, P, I32]
    L.st_scene_destroy.argtypes = [P]
    L.st_last_error.restype = ctypes.c_char_p
    L.st_version.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise StError(f"shapetrace error {rc}: {load().st_last_error().decode()}")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA (HIP) tensors"
    return ctypes.c_void_p(t.data_ptr())


def make_cameras(cams) -> ctypes.Array:
    """cams: objects with eye, target, up, fov_y_deg, width, height."""
    arr = (StCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].eye[:] = [float(x) for x in c.eye]
        arr[i].target[:] = [float(x) for x in c.target]
        arr[i].up[:] = [float(x) for x in c.up]
        arr[i].fov_y_deg = float(c.fov_y_deg)
        arr[i].width = int(c.width)
        arr[i].height = int(c.height)
    return arr


def num_pixels(cams) -> int:
    return int(sum(int(c.width) * int(c.height) for c in cams))


def num_edge_samples(cams, spp: int, ratio: float, n_shadow_lights: int = 0) -> int:
    """Primary edge samples, followed by n_shadow_lights x as many point-light
    shadow-edge samples (ST_EDGE_SHADOW with the scene's light count)."""
    n = int(sum(round(ratio * int(c.width) * int(c.height) * spp) for c in cams))
    return n * (1 + int(n_shadow_lights))


def make_opts(flags=ST_ALL_GRADS, edge_ratio=1.0, queue_capacity=0, dbg_hash=None, dbg_edge_hash=None,
              dbg_radiance=None, path_mask=None, edge_mask=None, max_workspace_bytes=0) -> StOpts:
    o = StOpts()
    o.flags = flags
    o.edge_spp_ratio = edge_ratio
    o.queue_capacity = queue_capacity
    o.debug_decision_hash = _ptr(dbg_hash)
    o.debug_edge_hash = _ptr(dbg_edge_hash)
    o.debug_sample_radiance = _ptr(dbg_radiance)
    o.path_mask = _ptr(path_mask)
    o.edge_mask = _ptr(edge_mask)
    o.max_workspace_bytes = int(max_workspace_bytes)
    return o


class GPUScene:
    """One library scene (mesh, per-face materials, lights, environment map)."""

    def __init__(self, V, F, mat, lights=None, env=None, scene_id: int = 0):
        import torch
        dev = torch.device("cuda")
        L = load()
        self.V = torch.as_tensor(V, dtype=torch.float32, device=dev).contiguous()
        self.F = torch.as_tensor(F, dtype=torch.int32, device=dev).contiguous()
        self.mat = torch.as_tensor(mat, dtype=torch.float32, device=dev).contiguous()
        lt = None if lights is None or len(lights) == 0 else torch.as_tensor(lights, dtype=torch.float32,
                                                                              device=dev).contiguous()
        ev = None if env is None else torch.as_tensor(env, dtype=torch.float32, device=dev).contiguous()
        self.nv, self.nf = int(self.V.shape[0]), int(self.F.shape[0])
        nl = 0 if lt is None else int(lt.shape[0])
        he, we = (0, 0) if ev is None else (int(ev.shape[0]), int(ev.shape[1]))
        h = ctypes.c_void_p()
        _check(L.st_scene_create(_ptr(self.V), self.nv, _ptr(self.F), self.nf, _ptr(self.mat), _ptr(lt), nl,
                                 _ptr(ev), he, we, scene_id, _stream(), ctypes.byref(h)))
        self.h = h
        self.scene_id = scene_id
        self.version = 0          # bumped by every update()
        info = (ctypes.c_int64 * 6)()
        _check(L.st_scene_info(self.h, info))
        self.ne = int(info[2])
        self.he, self.we = int(info[4]), int(info[5])
        self.tex_res, self.ntex = 0, self.nf

    def subdivide(self):
        """1 -> 4 midpoint subdivision of the current mesh: (V [nv+ne,3], F [4nf,3]) device tensors."""
        import torch
        V = torch.empty((self.nv + self.ne, 3), dtype=torch.float32, device="cuda")
        F = torch.empty((4 * self.nf, 3), dtype=torch.int32, device="cuda")
        _check(load().st_scene_subdivide(self.h, _ptr(V), _ptr(F), _stream()))
        return V, F

    def set_mesh_colors(self, r: int, texels):
        """Materials as mesh colours of resolution r: texels [nf (r+1)(r+2)/2, 7] (Sec. 3.3)."""
        import torch
        n = self.nf * (r + 1) * (r + 2) // 2
        t = torch.as_tensor(texels, dtype=torch.float32, device="cuda").contiguous()
        if tuple(t.shape) != (n, 7):
            raise ValueError(f"texels must be [{n}, 7] at r = {r}")
        _check(load().st_scene_set_mesh_colors(self.h, int(r), _ptr(t), _stream()))
        self.mat = t
        rr, nt = ctypes.c_int32(), ctypes.c_int64()
        _check(load().st_scene_mesh_colors_info(self.h, ctypes.byref(rr), ctypes.byref(nt)))
        self.tex_res, self.ntex = int(rr.value), int(nt.value)

    def set_env_sampler(self, method: int):
        """ST_ENV_SAMPLER_CDF (default) or ST_ENV_SAMPLER_ALIAS for environment texels."""
        _check(load().st_scene_set_env_sampler(self.h, int(method), _stream()))

    def edge_tree(self):
        """(keys, child, parent, box, len, nbox) of the secondary-edge importance tree (device tensors)."""
        import torch
        n = self.ne
        keys = torch.empty(n, dtype=torch.int64, device="cuda")
        child = torch.empty((max(n - 1, 1), 2), dtype=torch.int32, device="cuda")
        parent = torch.empty(2 * n - 1, dtype=torch.int32, device="cuda")
        box = torch.empty((2 * n - 1, 6), dtype=torch.float32, device="cuda")
        ln = torch.empty(2 * n - 1, dtype=torch.float32, device="cuda")
        nbox = torch.empty((2 * n - 1, 6), dtype=torch.float32, device="cuda")
        _check(load().st_scene_edge_tree(self.h, _ptr(keys), _ptr(child), _ptr(parent), _ptr(box), _ptr(ln),
                                         _ptr(nbox), _stream()))
        return keys, child[:max(n - 1, 0)], parent, box, ln, nbox

    def set_bsdf_sampler(self, method: int):
        """ST_BSDF_SAMPLER_HALFVECTOR (default) or ST_BSDF_SAMPLER_VNDF for the specular lobe."""
        _check(load().st_scene_set_bsdf_sampler(self.h, int(method), _stream()))

    def env_alias_table(self):
        """(prob float64 [he*we], alias int32 [he*we]) of the built alias table."""
        n = self.he * self.we
        prob, alias = np.zeros(n), np.zeros(n, np.int32)
        _check(load().st_scene_env_alias_table(self.h, prob.ctypes.data, alias.ctypes.data))
        return prob, alias

    @classmethod
    def from_scene(cls, sc):
        return cls(sc.V, sc.F, sc.mat, sc.lights, sc.env, sc.scene_id)

    def close(self):
        if getattr(self, "h", None):
            load().st_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, V=None, mat=None):
        _check(load().st_scene_update(self.h, _ptr(V), _ptr(mat), _stream()))
        self.version += 1

    def render(self, cams, spp: int, bounces: int, seed: int = 0, out=None, flags: int = 0, queue_capacity: int = 0,
               debug_hash=None, debug_radiance=None, max_workspace_bytes: int = 0):
        import torch
        cam = make_cameras(cams)
        if out is None:
            out = torch.empty((num_pixels(cams), 3), dtype=torch.float32, device="cuda")
        o = make_opts(flags=flags, queue_capacity=queue_capacity, dbg_hash=debug_hash, dbg_radiance=debug_radiance,
                      max_workspace_bytes=max_workspace_bytes)
        _check(load().st_render(self.h, cam, len(cams), spp, bounces, seed, ctypes.byref(o), _ptr(out), _stream()))
        return out

    def render_noalloc(self, cams, spp: int, bounces: int, seed: int = 0, out=None, flags: int = 0,
                       queue_capacity: int = 0, debug_hash=None):
        """st_render_noalloc: the same image as render(), with every workspace in
        the library's static per-device scratch (no allocation; calls on one GPU
        must not overlap).  out must be given by callers that cannot allocate."""
        import torch
        cam = make_cameras(cams)
        if out is None:
            out = torch.empty((num_pixels(cams), 3), dtype=torch.float32, device="cuda")
        o = make_opts(flags=flags, queue_capacity=queue_capacity, dbg_hash=debug_hash)
        _check(load().st_render_noalloc(self.h, cam, len(cams), spp, bounces, seed, ctypes.byref(o), _ptr(out),
                                        _stream()))
        return out

    def backward(self, cams, spp: int, bounces: int, d_image, seed: int = 0, flags: int = ST_ALL_GRADS,
                 edge_ratio: float = 1.0, dV=None, dmat=None, path_mask=None, edge_mask=None, debug_hash=None,
                 debug_edge_hash=None, max_workspace_bytes: int = 0):
        import torch
        cam = make_cameras(cams)
        if dV is None:
            dV = torch.empty((self.nv, 3), dtype=torch.float32, device="cuda")
        if dmat is None:
            dmat = torch.empty((self.ntex, 7), dtype=torch.float32, device="cuda")
        o = make_opts(flags=flags, edge_ratio=edge_ratio, dbg_hash=debug_hash, dbg_edge_hash=debug_edge_hash,
                      path_mask=path_mask, edge_mask=edge_mask, max_workspace_bytes=max_workspace_bytes)
        d = d_image.contiguous()
        _check(load().st_render_backward(self.h, cam, len(cams), spp, bounces, seed, ctypes.byref(o), _ptr(d),
                                         _ptr(dV), _ptr(dmat), _stream()))
        return dV, dmat

    def check_errors(self):
        _check(load().st_check_errors(self.h, _stream()))

    WORK_KERNELS = ("k_extend", "k_shadow", "k_adjoint", "k_forward_mega", "k_trace_pair")

    def read_work(self):
        """{kernel: (node visits, triangle tests, rays)} counted by ST_COUNT_WORK calls since the last read."""
        out = (ctypes.c_uint64 * (3 * len(self.WORK_KERNELS)))()
        _check(load().st_read_work(self.h, out, _stream()))
        return {k: (int(out[3 * i]), int(out[3 * i + 1]), int(out[3 * i + 2])) for i, k in enumerate(self.WORK_KERNELS)}

    def edges(self):
        import torch
        out = torch.empty((self.ne, 4), dtype=torch.int32, device="cuda")
        _check(load().st_scene_edges(self.h, _ptr(out), _stream()))
        return out

    def lbvh(self):
        import torch
        n = self.nf
        keys = torch.empty(n, dtype=torch.int64, device="cuda")
        child = torch.empty((max(n - 1, 0), 2), dtype=torch.int32, device="cuda")
        parent = torch.empty(2 * n - 1, dtype=torch.int32, device="cuda")
        aabb = torch.empty((2 * n - 1, 6), dtype=torch.float32, device="cuda")
        _check(load().st_scene_lbvh(self.h, _ptr(keys), _ptr(child) if n > 1 else None, _ptr(parent), _ptr(aabb),
                                    _stream()))
        return keys, child, parent, aabb

    def trace(self, o, d, tmin: float = 1e-4, brute: bool = False):
        import torch
        n = int(o.shape[0])
        f = torch.empty(n, dtype=torch.int32, device="cuda")
        t = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(load().st_trace_rays(self.h, _ptr(o.contiguous()), _ptr(d.contiguous()), n, tmin, int(brute),
                                    _ptr(f), _ptr(t), _stream()))
        return f, t


def autotune(scenes: Sequence["GPUScene"], cams, spp: int, bounces: int, cam_scene=None, cache_path=None):
    """Pick the wavefront chunk size and traversal grid for this workload (see st_autotune)."""
    arr = (ctypes.c_void_p * len(scenes))(*[s.h.value for s in scenes])
    cs = None if cam_scene is None else (ctypes.c_int32 * len(cams))(*[int(x) for x in cam_scene])
    cap = ctypes.c_int64(0)
    grid = ctypes.c_int32(0)
    _check(load().st_autotune(arr, len(scenes), make_cameras(cams), cs, len(cams), spp, bounces,
                              None if cache_path is None else cache_path.encode(), ctypes.byref(cap),
                              ctypes.byref(grid), _stream()))
    return int(cap.value), int(grid.value)


def stream_copy(dst, src):
    """st_stream_copy of a whole contiguous tensor (same byte size, 16-byte multiple)."""
    n = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == n
    _check(load().st_stream_copy(_ptr(dst), _ptr(src), n, _stream()))


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Achievable HBM bandwidth (GB/s, read + write) of st_stream_copy on nbytes buffers."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream_copy(b, a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        stream_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert torch.equal(a[:1 << 20], b[:1 << 20])
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def profile_enable(on: bool = True):
    load().st_profile_enable(1 if on else 0)


def profile_read(max_kernels: int = 64):
    """{kernel name: (total ms, launches)} for the launches since the last read."""
    L = load()
    names = ctypes.create_string_buffer(1 << 16)
    ms = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_int32 * max_kernels)()
    n = L.st_profile_read(names, len(names), ms, cnt, max_kernels)
    if n < 0:
        _check(n)
    keys = names.value.decode().split("\n")[:n]
    return {k: (ms[i], cnt[i]) for i, k in enumerate(keys)}


def render_batch(scenes: Sequence[GPUScene], cams, cam_scene, spp: int, bounces: int, seed: int = 0, out=None,
                 flags: int = 0, queue_capacity: int = 0, debug_hash=None):
    import torch
    arr = (ctypes.c_void_p * len(scenes))(*[s.h.value for s in scenes])
    cs = (ctypes.c_int32 * len(cams))(*[int(x) for x in cam_scene])
    cam = make_cameras(cams)
    if out is None:
        out = torch.empty((num_pixels(cams), 3), dtype=torch.float32, device="cuda")
    o = make_opts(flags=flags, queue_capacity=queue_capacity, dbg_hash=debug_hash)
    _check(load().st_render_batch(arr, len(scenes), cam, cs, len(cams), spp, bounces, seed, ctypes.byref(o),
                                  _ptr(out), _stream()))
    return out
