"""Thin ctypes binding of libgsr (include/gsr.h).

Argument marshalling only: every step of rendering runs in the HIP library.
Device memory and streams come from PyTorch.  Importing this module does not
load the library; the first use does, and fails loudly when the in-tree
libgsr.so is missing (build it with ``python -m paper_2604_25459_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")

GSR_OK = 0
GSR_E_INVALID = -1
GSR_E_OOM = -2
GSR_E_DEVICE = -3
GSR_E_NOT_FOUND = -4
GSR_E_BUSY = -5
GSR_E_REJECTED = -6
GSR_E_OVERFLOW = -7
GSR_E_TIMEOUT = -8

STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
OBS_FORMAT = {"u8": 1, "f16": 2}
MEM_HOST, MEM_DEVICE = 0, 1


class Options(C.Structure):
    _fields_ = [("tile_size", C.c_int), ("images_per_thread", C.c_int), ("chunk_bytes", C.c_int64),
                ("cutoff", C.c_float), ("profile", C.c_int), ("graphs", C.c_int), ("overlap", C.c_int),
                ("sync_lists", C.c_int), ("list_cap", C.c_int), ("reserved", C.c_int * 3)]


class TuningDesc(C.Structure):
    _fields_ = [("tile_size", C.c_int), ("lds_batch", C.c_int), ("images_per_thread", C.c_int),
                ("persistent", C.c_int), ("chunk_images", C.c_int), ("ms", C.c_float),
                ("bin_schedule", C.c_int), ("reserved", C.c_int * 3)]


class SceneDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int), ("storage", C.c_int), ("mem_kind", C.c_int),
                ("n_bodies", C.c_int), ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p), ("body_offsets", C.c_void_p)]


class CameraDesc(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("near_plane", C.c_float), ("attach_body", C.c_int)]


class ObsDesc(C.Structure):
    _fields_ = [("format", C.c_int), ("reserved0", C.c_int), ("gain", C.c_void_p), ("contrast", C.c_void_p),
                ("brightness", C.c_void_p), ("out", C.c_void_p)]


class RenderDesc(C.Structure):
    _fields_ = [("scene_id", C.c_uint64), ("n_envs", C.c_int), ("n_cams", C.c_int), ("cams", C.c_void_p),
                ("viewmats", C.c_void_p), ("body_poses", C.c_void_p), ("bg", C.c_float * 3),
                ("out_rgb", C.c_void_p), ("out_depth", C.c_void_p), ("out_alpha", C.c_void_p),
                ("out_work", C.c_void_p), ("obs", C.c_void_p)]


class LidarDesc(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int), ("az0", C.c_float), ("az_step", C.c_float),
                ("elevations", C.c_void_p), ("near_range", C.c_float), ("attach_body", C.c_int),
                ("pattern", C.c_int), ("x0", C.c_float), ("y0", C.c_float), ("dx", C.c_float), ("dy", C.c_float),
                ("ray_az", C.c_void_p), ("ray_el", C.c_void_p)]


class LidarRenderDesc(C.Structure):
    _fields_ = [("scene_id", C.c_uint64), ("n_envs", C.c_int), ("n_lidars", C.c_int), ("lidars", C.c_void_p),
                ("viewmats", C.c_void_p), ("body_poses", C.c_void_p), ("out_range", C.c_void_p),
                ("out_hit", C.c_void_p)]


class BinsOut(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("keys", C.c_void_p), ("values", C.c_void_p), ("ranges", C.c_void_p),
                ("ranges_capacity", C.c_int64), ("n_pairs", C.c_int64), ("n_visible", C.c_int64),
                ("tiles_x", C.c_int32), ("tiles_y", C.c_int32), ("tile_base", C.c_int64), ("tile_size", C.c_int32),
                ("reserved0", C.c_int32)]


class ProjOut(C.Structure):
    _fields_ = [("n", C.c_int64), ("zkey", C.c_void_p), ("rect", C.c_void_p), ("rec", C.c_void_p)]


class ServerCfg(C.Structure):
    _fields_ = [("n_streams", C.c_int), ("max_batch_images", C.c_int), ("memory_budget", C.c_int64),
                ("reserved", C.c_int * 8)]


class ReqInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("n_images", C.c_int), ("batch_id", C.c_int64), ("batch_requests", C.c_int),
                ("batch_images", C.c_int), ("t_submit_us", C.c_int64), ("t_admit_us", C.c_int64),
                ("t_start_us", C.c_int64), ("t_complete_us", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64), ("pending", C.c_int64),
                ("batches", C.c_int64), ("images", C.c_int64), ("in_flight_bytes", C.c_int64),
                ("in_flight_bytes_max", C.c_int64), ("latency_p50_us", C.c_double), ("latency_p99_us", C.c_double),
                ("latency_mean_us", C.c_double), ("latency_max_us", C.c_double), ("mean_batch_requests", C.c_double)]


# name -> (restype, argtypes); every entry point declared in include/gsr.h
SIGNATURES = {
    "gsr_create": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p]),
    "gsr_destroy": (C.c_int, [C.c_void_p]),
    "gsr_trim": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsr_scene_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_scene_destroy": (C.c_int, [C.c_void_p, C.c_uint64]),
    "gsr_scene_info": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_render": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_render_plain": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_render_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_render_lidar": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_debug_bins": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "gsr_debug_project": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "gsr_stage_times": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int]),
    "gsr_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_tuning_get": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_tuning_set": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_tuning_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "gsr_tuning_load": (C.c_int, [C.c_void_p, C.c_char_p]),
    "gsr_server_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int64, C.c_void_p]),
    "gsr_server_stats": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsr_server_destroy": (C.c_int, [C.c_void_p]),
    "gsr_last_error": (C.c_char_p, []),
    "gsr_version": (C.c_char_p, []),
}

_lib = None


class GsrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgsr error {code}: {msg}")
        self.code = code


def load():
    """Load the in-tree libgsr.so (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2604_25459_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != GSR_OK:
        raise GsrError(rc, load().gsr_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near: float = 0.01
    attach_body: int = -1     # >= 0: the slot's viewmats are body -> camera offsets of that body


@dataclass
class Lidar:
    """A ray grid: ``height`` beams at ``elevations`` (radians, ascending) x
    ``width`` columns at azimuths az0 + (c + 0.5) az_step; sensor frame x
    forward, y left, z up."""
    width: int
    height: int
    az0: float
    az_step: float
    elevations: object          # sequence of height floats
    near_range: float = 0.05
    attach_body: int = -1


@dataclass
class LidarRays:
    """A non-repetitive scan as listed rays: ray k of the ``height`` x
    ``width`` rays at azimuth ``ray_az[k]`` (radians, [-pi, pi]) and
    elevation ``ray_el[k]`` (radians, (-pi/2, pi/2)), arrays of that shape
    (row-major); ranges and hits come back in the same order."""
    width: int
    height: int
    ray_az: object
    ray_el: object
    near_range: float = 0.05
    attach_body: int = -1
    pattern: int = 2
    az0: float = 0.0
    az_step: float = 0.0
    elevations: object = ()


@dataclass
class Observation:
    """Fused observation epilogue request: ``out`` receives u8 or f16 pixels
    ([pixels * 3], the layout of rgb); gain / contrast / brightness are
    optional CUDA float32 tensors [C * E]."""
    format: str
    out: object
    gain: object = None
    contrast: object = None
    brightness: object = None


class Renderer:
    """One libgsr context on a device."""

    def __init__(self, device: int = 0, tile_size: int = 16, images_per_thread: int = 16, chunk_bytes: int = 0,
                 cutoff: float = 0.0, profile: bool = False, graphs: bool = True, overlap: bool = True,
                 sync_lists: bool = False, list_cap: int = 0):
        lib = load()
        opt = Options(tile_size=tile_size, images_per_thread=images_per_thread, chunk_bytes=chunk_bytes,
                      cutoff=cutoff, profile=int(profile), graphs=0 if graphs else -1, overlap=0 if overlap else -1,
                      sync_lists=-1 if sync_lists else 0, list_cap=int(list_cap))
        h = C.c_void_p()
        _check(lib.gsr_create(device, C.byref(opt), C.byref(h)))
        self._h = h
        self.device = device
        self.tile_size = tile_size

    def close(self):
        if getattr(self, "_h", None):
            load().gsr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    STAGES = ("project", "depth_sort", "tile_count", "tile_scatter", "raster")

    def trim(self) -> int:
        """Release idle working memory (gsr_trim); returns the bytes freed on the device."""
        freed = C.c_int64(0)
        _check(load().gsr_trim(self._h, C.byref(freed)))
        return int(freed.value)

    def stage_times(self, reset: bool = True):
        """Device ms per stage accumulated since the last reset (profile=True)."""
        ms = np.zeros(10, np.float64)
        _check(load().gsr_stage_times(self._h, ms.ctypes.data, 10, int(reset)))
        out = dict(zip(self.STAGES, ms[:5].tolist()))
        out["raster_launches"] = int(ms[5])
        out["renders"] = int(ms[6])
        out["visible"] = int(ms[7])
        out["pairs"] = int(ms[8])
        out["row_entries"] = int(ms[9])
        return out

    # ---------------------------------------------------------- scenes
    def add_scene(self, means, scales, quats, opacities, sh, sh_degree: int, body_offsets, storage: str = "f32") -> int:
        """Host numpy float32 arrays (or CUDA tensors, all on one side)."""
        import torch
        dev = isinstance(means, torch.Tensor) and means.is_cuda
        if not dev:
            conv = lambda a: np.ascontiguousarray(a, dtype=np.float32)
            means, scales, quats, opacities, sh = map(conv, (means, scales, quats, opacities, sh))
        off = np.ascontiguousarray(body_offsets, dtype=np.int64)
        d = SceneDesc(n=int(means.shape[0]), sh_degree=int(sh_degree), storage=STORAGE[storage],
                      mem_kind=MEM_DEVICE if dev else MEM_HOST, n_bodies=int(off.shape[0]) - 1,
                      means=_ptr(means), scales=_ptr(scales), quats=_ptr(quats), opacities=_ptr(opacities),
                      sh=_ptr(sh), body_offsets=off.ctypes.data)
        sid = C.c_uint64()
        _check(load().gsr_scene_create(self._h, C.byref(d), C.byref(sid)))
        return int(sid.value)

    def add_synth_scene(self, scene, storage: str = "f32") -> int:
        return self.add_scene(scene.means, scene.scales, scene.quats, scene.opacities, scene.sh, scene.sh_degree,
                              scene.body_offsets, storage)

    def remove_scene(self, sid: int):
        _check(load().gsr_scene_destroy(self._h, sid))

    def scene_info(self, sid: int):
        n, b, by = C.c_int64(), C.c_int(), C.c_int64()
        _check(load().gsr_scene_info(self._h, sid, C.byref(n), C.byref(b), C.byref(by)))
        return int(n.value), int(b.value), int(by.value)

    # ---------------------------------------------------------- rendering
    @staticmethod
    def _cams(cams: Sequence) -> C.Array:
        arr = (CameraDesc * len(cams))()
        for k, c in enumerate(cams):
            arr[k] = CameraDesc(width=int(c.width), height=int(c.height), fx=c.fx, fy=c.fy, cx=c.cx, cy=c.cy,
                                near_plane=c.near, attach_body=int(getattr(c, "attach_body", -1)))
        return arr

    def _desc(self, sid, cams, viewmats, poses, bg, rgb=None, depth=None, alpha=None, work=None, obs=None):
        carr = self._cams(cams)
        d = RenderDesc(scene_id=sid, n_envs=int(viewmats.shape[1]), n_cams=len(cams), cams=C.addressof(carr),
                       viewmats=_ptr(viewmats), body_poses=_ptr(poses) if poses is not None and poses.numel() else None,
                       out_rgb=_ptr(rgb), out_depth=_ptr(depth), out_alpha=_ptr(alpha), out_work=_ptr(work))
        d.bg[0], d.bg[1], d.bg[2] = [float(x) for x in bg]
        keep = [carr]
        if obs is not None:
            od = ObsDesc(format=OBS_FORMAT[obs.format], gain=_ptr(obs.gain), contrast=_ptr(obs.contrast),
                         brightness=_ptr(obs.brightness), out=_ptr(obs.out))
            d.obs = C.addressof(od)
            keep.append(od)
        return d, keep

    def alloc_outputs(self, cams, n_envs: int, alpha: bool = False):
        import torch
        npix = sum(n_envs * c.width * c.height for c in cams)
        dev = torch.device("cuda", self.device)
        rgb = torch.empty(npix * 3, dtype=torch.float32, device=dev)
        depth = torch.empty(npix, dtype=torch.float32, device=dev)
        a = torch.empty(npix, dtype=torch.float32, device=dev) if alpha else None
        return rgb, depth, a

    @staticmethod
    def split(cams, n_envs: int, rgb, depth, alpha=None):
        """Per camera slot views: rgb [E, H, W, 3], depth [E, H, W]."""
        out, base = [], 0
        for c in cams:
            n = n_envs * c.width * c.height
            r = rgb[3 * base:3 * (base + n)].view(n_envs, c.height, c.width, 3)
            dd = depth[base:base + n].view(n_envs, c.height, c.width)
            aa = alpha[base:base + n].view(n_envs, c.height, c.width) if alpha is not None else None
            out.append((r, dd, aa))
            base += n
        return out

    def render_into(self, sid, cams, viewmats, poses, rgb, depth, alpha=None, bg=(0.0, 0.0, 0.0), plain=False,
                    stream=None, work=None, obs=None, noalloc=False):
        """viewmats: CUDA float32 [C, E, 3, 4]; poses: CUDA float32 [E, B, 7]; work: optional CUDA int32
        [pixels * 2] receiving (visited list entries, blended Gaussians) per pixel; obs: optional
        Observation (rgb may then be None); noalloc: gsr_render_noalloc (working memory in the
        library's fixed scratch)."""
        import torch
        d, carr = self._desc(sid, cams, viewmats, poses, bg, rgb, depth, alpha, work, obs)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        lib = load()
        fn = lib.gsr_render_noalloc if noalloc else lib.gsr_render_plain if plain else lib.gsr_render
        _check(fn(self._h, C.byref(d), C.c_void_p(st)))
        del carr

    def render(self, sid, cams, viewmats, poses, bg=(0.0, 0.0, 0.0), alpha=False, plain=False, stream=None):
        E = int(viewmats.shape[1])
        rgb, depth, a = self.alloc_outputs(cams, E, alpha)
        self.render_into(sid, cams, viewmats, poses, rgb, depth, a, bg, plain, stream)
        return self.split(cams, E, rgb, depth, a)

    # ---------------------------------------------------------- LiDAR
    def render_lidar_into(self, sid, lidars, viewmats, poses, out_range, out_hit=None, stream=None):
        """viewmats: CUDA float32 [L, E, 3, 4] world -> sensor (body -> sensor for attached slots);
        out_range / out_hit: CUDA float32 [sum over slots of E * H * W]."""
        import torch
        keep = []
        arr = (LidarDesc * len(lidars))()
        for k, l in enumerate(lidars):
            el = np.ascontiguousarray(np.asarray(l.elevations, np.float32))
            keep.append(el)
            ray_az = ray_el = None
            if int(getattr(l, "pattern", 0)) == 2:          # listed rays: [H * W] azimuths, elevations
                ray_az = np.ascontiguousarray(np.asarray(l.ray_az, np.float32).reshape(-1))
                ray_el = np.ascontiguousarray(np.asarray(l.ray_el, np.float32).reshape(-1))
                if ray_az.size != l.width * l.height or ray_el.size != l.width * l.height:
                    raise ValueError("ray_az / ray_el must hold width * height values")
                keep += [ray_az, ray_el]
            arr[k] = LidarDesc(width=int(l.width), height=int(l.height), az0=float(l.az0), az_step=float(l.az_step),
                               elevations=el.ctypes.data if el.size else None, near_range=float(l.near_range),
                               attach_body=int(l.attach_body), pattern=int(getattr(l, "pattern", 0)),
                               x0=float(getattr(l, "x0", 0.0)), y0=float(getattr(l, "y0", 0.0)),
                               dx=float(getattr(l, "dx", 0.0)), dy=float(getattr(l, "dy", 0.0)),
                               ray_az=ray_az.ctypes.data if ray_az is not None else None,
                               ray_el=ray_el.ctypes.data if ray_el is not None else None)
        d = LidarRenderDesc(scene_id=sid, n_envs=int(viewmats.shape[1]), n_lidars=len(lidars),
                            lidars=C.addressof(arr), viewmats=_ptr(viewmats),
                            body_poses=_ptr(poses) if poses is not None and poses.numel() else None,
                            out_range=_ptr(out_range), out_hit=_ptr(out_hit))
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(load().gsr_render_lidar(self._h, C.byref(d), C.c_void_p(st)))
        del keep, arr

    def render_lidar(self, sid, lidars, viewmats, poses, hit=True, stream=None):
        """Per slot: (range [E, H, W], hit [E, H, W] or None)."""
        import torch
        E = int(viewmats.shape[1])
        n = sum(E * l.width * l.height for l in lidars)
        dev = torch.device("cuda", self.device)
        rng = torch.empty(n, dtype=torch.float32, device=dev)
        h = torch.empty(n, dtype=torch.float32, device=dev) if hit else None
        self.render_lidar_into(sid, lidars, viewmats, poses, rng, h, stream)
        out, base = [], 0
        for l in lidars:
            m = E * l.width * l.height
            out.append((rng[base:base + m].view(E, l.height, l.width),
                        h[base:base + m].view(E, l.height, l.width) if h is not None else None))
            base += m
        return out

    # ---------------------------------------------------------- tuning
    TUNING_KEYS = ("tile_size", "lds_batch", "images_per_thread", "persistent", "chunk_images", "bin_schedule", "ms")

    def autotune(self, sid, cams, viewmats, poses, rgb, depth, alpha=None, stream=None) -> dict:
        import torch
        d, carr = self._desc(sid, cams, viewmats, poses, (0, 0, 0), rgb, depth, alpha)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        t = TuningDesc()
        _check(load().gsr_autotune(self._h, C.byref(d), C.c_void_p(st), C.byref(t)))
        return {k: getattr(t, k) for k in self.TUNING_KEYS}

    def tuning(self, sid, cams, viewmats, poses) -> dict:
        d, carr = self._desc(sid, cams, viewmats, poses, (0, 0, 0))
        t = TuningDesc()
        _check(load().gsr_tuning_get(self._h, C.byref(d), C.byref(t)))
        return {k: getattr(t, k) for k in self.TUNING_KEYS}

    def set_tuning(self, sid, cams, viewmats, poses, **kw):
        d, carr = self._desc(sid, cams, viewmats, poses, (0, 0, 0))
        cur = self.tuning(sid, cams, viewmats, poses)
        cur.update(kw)
        t = TuningDesc(**{k: cur[k] for k in self.TUNING_KEYS})
        _check(load().gsr_tuning_set(self._h, C.byref(d), C.byref(t)))

    def save_tuning(self, path: str):
        _check(load().gsr_tuning_save(self._h, path.encode()))

    def load_tuning(self, path: str):
        _check(load().gsr_tuning_load(self._h, path.encode()))

    # ---------------------------------------------------------- debug
    def debug_bins(self, sid, cams, viewmats, poses, image: int, capacity: int = 1 << 22):
        """Keys, ids and tile ranges of one image as gsr_render builds them
        (tuned launch parameters; ``tile_size`` reports the tile side used)."""
        d, carr = self._desc(sid, cams, viewmats, poses, (0, 0, 0))
        for _ in range(2):
            keys = np.empty(capacity, np.uint64)
            vals = np.empty(capacity, np.uint32)
            cam = cams[image // int(viewmats.shape[1])]
            T = ((cam.width + 7) // 8) * ((cam.height + 7) // 8)      # room for the smallest tile size
            ranges = np.empty((T, 2), np.uint32)
            o = BinsOut(capacity=capacity, keys=keys.ctypes.data, values=vals.ctypes.data, ranges=ranges.ctypes.data,
                        ranges_capacity=T)
            rc = load().gsr_debug_bins(self._h, C.byref(d), int(image), C.byref(o))
            if rc == GSR_E_INVALID and o.n_pairs > capacity:
                capacity = int(o.n_pairs)
                continue
            _check(rc)
            n = int(o.n_pairs)
            nt = int(o.tiles_x) * int(o.tiles_y)
            return dict(keys=keys[:n].copy(), values=vals[:n].copy(), ranges=ranges[:nt].astype(np.int64),
                        n_visible=int(o.n_visible), tiles_x=int(o.tiles_x), tiles_y=int(o.tiles_y),
                        tile_base=int(o.tile_base), tile_size=int(o.tile_size))
        raise GsrError(GSR_E_INVALID, "debug_bins capacity retry failed")

    def debug_project(self, sid, cams, viewmats, poses, image: int, n: int):
        d, carr = self._desc(sid, cams, viewmats, poses, (0, 0, 0))
        z = np.empty(n, np.uint32)
        rect = np.empty((n, 4), np.int32)
        rec = np.empty((n, 12), np.float32)
        o = ProjOut(n=n, zkey=z.ctypes.data, rect=rect.ctypes.data, rec=rec.ctypes.data)
        _check(load().gsr_debug_project(self._h, C.byref(d), int(image), C.byref(o)))
        return dict(zkey=z, rect=rect, rec=rec)


class Server:
    """Continuous-batching request server on a Renderer's context."""

    def __init__(self, renderer: Renderer, n_streams: int = 2, max_batch_images: int = 4096, memory_budget: int = 0):
        cfg = ServerCfg(n_streams=n_streams, max_batch_images=max_batch_images, memory_budget=memory_budget)
        h = C.c_void_p()
        _check(load().gsr_server_create(renderer._h, C.byref(cfg), C.byref(h)))
        self._h = h
        self._r = renderer
        self._keep = {}

    def submit(self, sid, cams, viewmats, poses, rgb, depth, alpha=None, bg=(0.0, 0.0, 0.0), obs=None) -> int:
        d, carr = self._r._desc(sid, cams, viewmats, poses, bg, rgb, depth, alpha, obs=obs)
        t = C.c_uint64()
        _check(load().gsr_submit(self._h, C.byref(d), C.byref(t)))
        self._keep[int(t.value)] = (viewmats, poses, rgb, depth, alpha, obs)
        return int(t.value)

    def wait(self, ticket: int, timeout_us: int = -1) -> dict:
        info = ReqInfo()
        rc = load().gsr_wait(self._h, C.c_uint64(ticket), C.c_int64(timeout_us), C.byref(info))
        if rc != GSR_E_TIMEOUT:
            self._keep.pop(ticket, None)
        _check(rc)
        return {k: getattr(info, k) for k, _ in ReqInfo._fields_}

    def stats(self) -> dict:
        st = Stats()
        _check(load().gsr_server_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().gsr_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_tensors(batch, device: int = 0):
    """CUDA tensors (viewmats [C,E,3,4], poses [E,B,7]) and camera list of a synth.Batch."""
    import torch
    dev = torch.device("cuda", device)
    vm = torch.from_numpy(np.ascontiguousarray(batch.viewmats, np.float32)).to(dev)
    poses = torch.from_numpy(np.ascontiguousarray(batch.poses, np.float32)).to(dev)
    cams = [Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.near, getattr(c, "attach_body", -1))
            for c in batch.cams]
    return cams, vm, poses
