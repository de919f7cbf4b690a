"""ctypes front end of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading
import zlib
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "alternatives.c"),
        os.path.join(_HERE, "view.c"), os.path.join(_HERE, "resample.c")]
_HDR = [os.path.join(_HERE, "oracle.h"), os.path.join(_HERE, "oracle_internal.h")]
_lock = threading.RLock()
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (strict IEEE: no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", _SO + ".tmp"] + _SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class _Params(C.Structure):
    _fields_ = [("width", C.c_int32), ("rows", C.c_int32), ("texel_m", C.c_double),
                ("radius_m", C.c_double), ("elev_rad", C.c_double), ("azim_rad", C.c_double),
                ("ang_radius_rad", C.c_double), ("max_len_m", C.c_double),
                ("n_prime0", C.c_int32), ("schedule", C.c_int32), ("n_segments", C.c_int32),
                ("mode", C.c_int32), ("uniform_step", C.c_double),
                ("uniform_tmax_m", C.c_double), ("n_prime_list", C.c_int32 * 16)]


TRACE_DTYPE = np.dtype([("seg", np.int32), ("n", np.int32), ("t", np.float64),
                        ("dh", np.float64), ("alpha", np.float64), ("base_i", np.int32),
                        ("base_j", np.int32), ("evals", np.int32), ("margin_lb", np.float64),
                        ("margin_dh", np.float64), ("margin_round", np.float64),
                        ("margin_seg", np.float64), ("margin_geo", np.float64),
                        ("margin_tap", np.float64)], align=True)


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("eye", C.c_double * 3),
                ("fwd", C.c_double * 3), ("right", C.c_double * 3), ("up", C.c_double * 3),
                ("step_m", C.c_double), ("far_m", C.c_double)]


class _ViewTol(C.Structure):
    _fields_ = [("eh_abs", C.c_double), ("eh_rel", C.c_double), ("ep_abs", C.c_double),
                ("ep_rel", C.c_double), ("max_samples", C.c_int64)]


class _Frame(C.Structure):
    _fields_ = [("width", C.c_int32), ("rows", C.c_int32), ("texel_m", C.c_double),
                ("centre", C.c_double * 3), ("ex", C.c_double * 3), ("ey", C.c_double * 3),
                ("origin_m", C.c_double * 2)]


VIEW_MAXADM = 8
VIEW_DTYPE = np.dtype([("n_hit", np.int32), ("n_adm", np.int32), ("adm", np.int32, VIEW_MAXADM),
                       ("adm_overflow", np.int32), ("status", np.int32), ("t_hit", np.float64),
                       ("qx", np.float64), ("qy", np.float64), ("f_prev", np.float64),
                       ("f_hit", np.float64), ("eps", np.float64), ("dqdt", np.float64)],
                      align=True)


def load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_SO) or any(
                os.path.getmtime(s) > os.path.getmtime(_SO) for s in _SRC + _HDR):
            build()
        lib = C.CDLL(_SO)
        P = C.POINTER
        lib.or_maxmip_levels.argtypes = [C.c_int32, C.c_int32]
        lib.or_maxmip_levels.restype = C.c_int32
        lib.or_maxmip_offset.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        lib.or_maxmip_offset.restype = C.c_int64
        lib.or_maxmip_floats.argtypes = [C.c_int32, C.c_int32]
        lib.or_maxmip_floats.restype = C.c_int64
        lib.or_ctx_create.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        lib.or_ctx_create.restype = C.c_void_p
        lib.or_ctx_destroy.argtypes = [C.c_void_p]
        lib.or_ctx_destroy.restype = None
        lib.or_ctx_copy_maxmip.argtypes = [C.c_void_p, C.c_void_p]
        lib.or_ctx_copy_maxmip.restype = None
        lib.or_shadow.argtypes = [C.c_void_p, P(_Params), C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_void_p, C.c_void_p]
        lib.or_shadow.restype = C.c_int32
        lib.or_shadow_points.argtypes = [C.c_void_p, P(_Params), C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_void_p, C.c_void_p]
        lib.or_shadow_points.restype = C.c_int32
        lib.or_alternatives.argtypes = [C.c_void_p, P(_Params), C.c_int64, C.c_double,
                                        C.c_double, C.c_double, C.c_double, C.c_void_p,
                                        C.c_int32]
        lib.or_alternatives.restype = C.c_int32
        lib.or_disc_fraction.argtypes = [C.c_double]
        lib.or_disc_fraction.restype = C.c_double
        lib.or_schedule.argtypes = [P(_Params), C.c_void_p, C.c_void_p, C.c_void_p]
        lib.or_schedule.restype = C.c_int32
        lib.or_ray_consts.argtypes = [C.c_void_p, P(_Params), C.c_int32, C.c_int32, C.c_void_p]
        lib.or_ray_consts.restype = None
        lib.or_probe.argtypes = [C.c_void_p, P(_Params), C.c_int32, C.c_int32, C.c_double,
                                 C.c_void_p]
        lib.or_probe.restype = None
        lib.or_path_cells.argtypes = [C.c_void_p, P(_Params), C.c_int32, C.c_int32, C.c_int32,
                                      C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_int32]
        lib.or_path_cells.restype = C.c_int32
        lib.or_view.argtypes = [C.c_void_p, C.c_double, C.c_double, P(_Camera), C.c_void_p,
                                C.c_int64, P(_ViewTol), C.c_void_p]
        lib.or_view.restype = C.c_int32
        lib.or_view_direction.argtypes = [P(_Camera), C.c_int32, C.c_int32, C.c_void_p]
        lib.or_view_direction.restype = None
        lib.or_view_probe.argtypes = [C.c_void_p, C.c_double, C.c_double, P(_Camera), C.c_int32,
                                      C.c_int32, C.c_double, C.c_void_p]
        lib.or_view_probe.restype = None
        lib.or_resample.argtypes = [C.c_void_p, P(_Frame), P(_Frame), C.c_double, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
        lib.or_resample.restype = C.c_int32
        lib.or_frame_source_coords.argtypes = [P(_Frame), P(_Frame), C.c_double, C.c_int32,
                                               C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.or_frame_source_coords.restype = None
        _lib = lib
        return lib


@dataclass
class Params:
    """Problem statement of one (tile, sun) pair; angles in radians, lengths in metres."""
    width: int
    rows: int
    texel_m: float
    radius_m: float
    elev: float
    azim: float
    ang_radius: float = math.radians(0.267)
    max_len_m: float = 0.0
    n_prime0: int = 5
    schedule: int = 0
    n_segments: int = 0
    mode: int = 0
    uniform_step: float = 1.0
    uniform_tmax_m: float = 0.0
    n_prime_list: tuple = ()

    def c(self) -> _Params:
        lst = (C.c_int32 * 16)(*[int(v) for v in self.n_prime_list][:16])
        return _Params(self.width, self.rows, self.texel_m, self.radius_m, self.elev, self.azim,
                       self.ang_radius, self.max_len_m, self.n_prime0, self.schedule,
                       self.n_segments, self.mode, self.uniform_step, self.uniform_tmax_m, lst)

    def replace(self, **kw) -> "Params":
        d = dict(self.__dict__)
        d.update(kw)
        return Params(**d)


class _Ctx:
    """Owns the oracle's maximum mipmap of one heightfield."""

    def __init__(self, h: np.ndarray):
        self.h = np.ascontiguousarray(h, dtype=np.float32)
        self.lib = load()
        rows, width = self.h.shape
        self.ptr = self.lib.or_ctx_create(self.h.ctypes.data, width, rows)
        if not self.ptr:
            raise MemoryError("oracle context")

    def __del__(self):
        if getattr(self, "ptr", None):
            self.lib.or_ctx_destroy(self.ptr)
            self.ptr = None


_ctx_cache: dict = {}


def _ctx(h: np.ndarray) -> _Ctx:
    """Context for h, reused while the array's address, shape and contents are unchanged."""
    key = (h.__array_interface__["data"][0], h.shape, zlib.crc32(memoryview(h).cast("B")))
    with _lock:
        c = _ctx_cache.get(key)
        if c is None:
            c = _Ctx(h)
            _ctx_cache.clear()
            _ctx_cache[key] = c
    return c


def maxmip_levels(width: int, rows: int) -> int:
    return load().or_maxmip_levels(width, rows)


def maxmip(h: np.ndarray) -> list:
    """Levels 1..L-1 of the maximum mipmap as a list of float32 arrays."""
    h = np.ascontiguousarray(h, dtype=np.float32)
    rows, width = h.shape
    lib = load()
    ctx = _ctx(h)
    total = lib.or_maxmip_floats(width, rows)
    flat = np.empty(max(total, 1), dtype=np.float32)
    lib.or_ctx_copy_maxmip(ctx.ptr, flat.ctypes.data)
    out = []
    w, r = width, rows
    for m in range(1, lib.or_maxmip_levels(width, rows)):
        w, r = (w + 1) // 2, (r + 1) // 2
        off = lib.or_maxmip_offset(width, rows, m)
        out.append(flat[off:off + w * r].reshape(r, w).copy())
    return out


def tap_bound(h: np.ndarray) -> list:
    """Tap-bound pyramid of h: [level 0, level 1, ...] as float32 arrays.

    A bilinear sample at continuous texel position q (texel i covers [i, i+1))
    reads the texels floor(q - 1/2) and floor(q - 1/2) + 1 per axis, clamped to
    the tile (Sec. 3.4 samples the terrain bilinearly).  For q anywhere in
    texel (x, y), or up to half a texel outside it, those taps lie in the 3 x 3
    block of texels around (x, y).  Level 0 therefore holds, per texel, the
    largest height of that block clipped to the tile; levels >= 1 are the
    maximum mipmap of level 0 (Sec. 3.2).  -0 is stored as +0.
    """
    h = np.ascontiguousarray(h, dtype=np.float32)
    rows, width = h.shape
    pad = np.full((rows + 2, width + 2), -np.inf, dtype=np.float32)
    pad[1:-1, 1:-1] = h
    d0 = np.full((rows, width), -np.inf, dtype=np.float32)
    for dy in (0, 1, 2):
        for dx in (0, 1, 2):
            d0 = np.maximum(d0, pad[dy:dy + rows, dx:dx + width])
    d0 = d0 + np.float32(0.0)  # -0 -> +0
    return [d0] + maxmip(d0)


def shadow(h: np.ndarray, p: Params, rays=None, trace: bool = False, _c=None):
    """Shadow factor s (float64) for all texels ([rows, width]) or the given linear indices."""
    h = np.ascontiguousarray(h, dtype=np.float32)
    rows, width = h.shape
    assert (p.width, p.rows) == (width, rows)
    lib = load()
    ctx = _c if _c is not None else _ctx(h)
    if rays is None:
        n = width * rows
        rp = None
    else:
        rays = np.ascontiguousarray(rays, dtype=np.int64)
        n = rays.size
        rp = rays.ctypes.data
    s = np.empty(n, dtype=np.float64)
    alpha = np.empty(n, dtype=np.float64)
    tr = np.empty(n, dtype=TRACE_DTYPE) if trace else None
    pc = p.c()
    rc = lib.or_shadow(ctx.ptr, C.byref(pc), rp, n, s.ctypes.data, alpha.ctypes.data,
                       tr.ctypes.data if trace else None)
    if rc != 0:
        raise ValueError(f"oracle rejected the problem ({rc})")
    if rays is None:
        s = s.reshape(rows, width)
        alpha = alpha.reshape(rows, width)
        if trace:
            tr = tr.reshape(rows, width)
    return (s, alpha, tr) if trace else (s, alpha)


def shadow_points(h: np.ndarray, p: Params, xy, trace: bool = False):
    """s (float64) for shadow rays from surface points xy[k] = (qx, qy) in
    continuous texel coordinates; the origin height is the bilinear terrain."""
    h = np.ascontiguousarray(h, dtype=np.float32)
    rows, width = h.shape
    assert (p.width, p.rows) == (width, rows)
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    n = xy.shape[0]
    s = np.empty(n, dtype=np.float64)
    alpha = np.empty(n, dtype=np.float64)
    tr = np.empty(n, dtype=TRACE_DTYPE) if trace else None
    pc = p.c()
    rc = load().or_shadow_points(_ctx(h).ptr, C.byref(pc), xy.ctypes.data, n, s.ctypes.data,
                                 alpha.ctypes.data, tr.ctypes.data if trace else None)
    if rc != 0:
        raise ValueError(f"oracle rejected the points ({rc})")
    return (s, alpha, tr) if trace else (s, alpha)


def shadow_threaded(h: np.ndarray, p: Params, rays=None, threads: int | None = None,
                    trace: bool = False):
    """Same as ``shadow`` over ray chunks on a thread pool (ctypes drops the GIL)."""
    h = np.ascontiguousarray(h, dtype=np.float32)
    rows, width = h.shape
    if rays is None:
        rays_all = np.arange(width * rows, dtype=np.int64)
    else:
        rays_all = np.ascontiguousarray(rays, dtype=np.int64)
    threads = threads or max(1, len(os.sched_getaffinity(0)))
    c = _ctx(h)  # one mipmap shared by every thread
    chunks = np.array_split(rays_all, max(1, threads * 4))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda r: shadow(h, p, r, trace=trace, _c=c), chunks))
    s = np.concatenate([q[0] for q in parts])
    a = np.concatenate([q[1] for q in parts])
    t = np.concatenate([q[2] for q in parts]) if trace else None
    if rays is None:
        s = s.reshape(rows, width)
        a = a.reshape(rows, width)
        if trace:
            t = t.reshape(rows, width)
    return (s, a, t) if trace else (s, a)


def alternatives(h: np.ndarray, p: Params, ray: int, eh_abs: float, eh_rel: float = 0.0,
                 et_abs: float = 0.0, et_rel: float = 0.0):
    """Angular clearances valid for one ray under near-ties; None if the branch cap hit.

    Height tolerance eh_abs + eh_rel*t (m), position tolerance et_abs + et_rel*t/delta
    (texels), t the ray length at the decision."""
    h = np.ascontiguousarray(h, dtype=np.float32)
    lib = load()
    ctx = _ctx(h)
    out = np.empty(256, dtype=np.float64)
    pc = p.c()
    n = lib.or_alternatives(ctx.ptr, C.byref(pc), int(ray), eh_abs, eh_rel, et_abs, et_rel,
                            out.ctypes.data, 256)
    if n == -2:
        raise ValueError("bad ray or mode")
    if n < 0:
        return None
    return out[:n].copy()


def disc_fraction(d: float) -> float:
    return load().or_disc_fraction(float(d))


def schedule(p: Params):
    """(m0 list, tau list, delta) of the segment schedule."""
    lib = load()
    m0 = np.zeros(64, dtype=np.int32)
    tau = np.zeros(65, dtype=np.float64)
    delta = C.c_double()
    pc = p.c()
    n = lib.or_schedule(C.byref(pc), m0.ctypes.data, tau.ctypes.data, C.byref(delta))
    return m0[:n].tolist(), tau[:n + 1].tolist(), delta.value


_CONST_NAMES = ["nx", "ny", "nz", "px", "py", "pz", "rho", "sp", "cp", "t_hmin", "texit",
                "Lx", "Ly", "Lz", "delta", "hp"]


def ray_consts(h: np.ndarray, p: Params, i: int, j: int) -> dict:
    h = np.ascontiguousarray(h, dtype=np.float32)
    ctx = _ctx(h)
    out = np.zeros(16, dtype=np.float64)
    pc = p.c()
    load().or_ray_consts(ctx.ptr, C.byref(pc), i, j, out.ctypes.data)
    return dict(zip(_CONST_NAMES, out.tolist()))


def probe(h: np.ndarray, p: Params, i: int, j: int, t: float) -> dict:
    h = np.ascontiguousarray(h, dtype=np.float32)
    ctx = _ctx(h)
    out = np.zeros(8, dtype=np.float64)
    pc = p.c()
    load().or_probe(ctx.ptr, C.byref(pc), i, j, float(t), out.ctypes.data)
    k = ["qx", "qy", "H", "h_bil", "dh", "alpha", "inside", "texit"]
    return dict(zip(k, out.tolist()))


def path_cells(h: np.ndarray, p: Params, i: int, j: int, level: int, ta: float, tb: float):
    h = np.ascontiguousarray(h, dtype=np.float32)
    ctx = _ctx(h)
    cells = np.zeros(64, dtype=np.int32)
    ts = np.zeros(64, dtype=np.float64)
    pc = p.c()
    n = load().or_path_cells(ctx.ptr, C.byref(pc), i, j, level, float(ta), float(tb),
                             cells.ctypes.data, ts.ctypes.data, 32)
    return [((int(cells[2 * k]), int(cells[2 * k + 1])), (float(ts[2 * k]), float(ts[2 * k + 1])))
            for k in range(n)]


@dataclass
class Camera:
    """Pinhole camera in the tile frame (metres; eye relative to the point where the
    tile's z axis meets the reference surface).  Pixel (px, py) looks along
    fwd + sx*right + sy*up, sx = 2(px+1/2)/width - 1, sy = 1 - 2(py+1/2)/height."""
    width: int
    height: int
    eye: tuple
    fwd: tuple
    right: tuple
    up: tuple
    step_m: float
    far_m: float = 0.0

    def c(self) -> _Camera:
        v3 = C.c_double * 3
        return _Camera(self.width, self.height, v3(*self.eye), v3(*self.fwd), v3(*self.right),
                       v3(*self.up), self.step_m, self.far_m)


@dataclass
class ViewTol:
    """Decision margins of the view oracle: heights eh_abs + eh_rel*(|eye|+t) plus the local
    slope times the position tolerance ep_abs + ep_rel*(|eye|+t) (metres)."""
    eh_abs: float = 0.0
    eh_rel: float = 0.0
    ep_abs: float = 0.0
    ep_rel: float = 0.0
    max_samples: int = 10_000_000

    def c(self) -> _ViewTol:
        return _ViewTol(self.eh_abs, self.eh_rel, self.ep_abs, self.ep_rel, self.max_samples)


def view(h: np.ndarray, radius_m: float, texel_m: float, cam: Camera, pixels=None,
         tol: ViewTol | None = None) -> np.ndarray:
    """First hits of view rays (VIEW_DTYPE per pixel; [height, width] without pixels)."""
    h = np.ascontiguousarray(h, dtype=np.float32)
    ctx = _ctx(h)
    tol = tol or ViewTol()
    if pixels is None:
        n = cam.width * cam.height
        pp = None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        n = pixels.shape[0]
        pp = pixels.ctypes.data
    out = np.zeros(n, dtype=VIEW_DTYPE)
    cc, tc = cam.c(), tol.c()
    rc = load().or_view(ctx.ptr, float(radius_m), float(texel_m), C.byref(cc), pp, n,
                        C.byref(tc), out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected the view ({rc})")
    return out.reshape(cam.height, cam.width) if pixels is None else out


def view_threaded(h: np.ndarray, radius_m: float, texel_m: float, cam: Camera,
                  tol: ViewTol | None = None, threads: int | None = None) -> np.ndarray:
    """``view`` over all pixels, in row chunks on a thread pool."""
    h = np.ascontiguousarray(h, dtype=np.float32)
    _ctx(h)
    threads = threads or max(1, len(os.sched_getaffinity(0)))
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    pix = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)
    chunks = np.array_split(pix, max(1, threads * 4))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda q: view(h, radius_m, texel_m, cam, q, tol), chunks))
    return np.concatenate(parts).reshape(cam.height, cam.width)


def view_direction(cam: Camera, px: int, py: int) -> np.ndarray:
    out = np.zeros(3, dtype=np.float64)
    cc = cam.c()
    load().or_view_direction(C.byref(cc), int(px), int(py), out.ctypes.data)
    return out


def view_probe(h: np.ndarray, radius_m: float, texel_m: float, cam: Camera, px: int, py: int,
               t: float) -> dict:
    h = np.ascontiguousarray(h, dtype=np.float32)
    out = np.zeros(6, dtype=np.float64)
    cc = cam.c()
    load().or_view_probe(_ctx(h).ptr, float(radius_m), float(texel_m), C.byref(cc), int(px),
                         int(py), float(t), out.ctypes.data)
    return dict(zip(["qx", "qy", "H", "terrain", "f", "defined"], out.tolist()))


@dataclass
class Frame:
    """Gnomonic tile frame: plane tangent at unit vector ``centre`` with unit axes ex (+column)
    and ey (+row), texel spacing texel_m in the plane, grid centre at plane coordinates
    ``origin``."""
    width: int
    rows: int
    texel_m: float
    centre: tuple
    ex: tuple
    ey: tuple
    origin: tuple = (0.0, 0.0)

    def c(self) -> _Frame:
        v3, v2 = C.c_double * 3, C.c_double * 2
        return _Frame(self.width, self.rows, self.texel_m, v3(*self.centre), v3(*self.ex),
                      v3(*self.ey), v2(*self.origin))


def resample(src: np.ndarray, fs: Frame, fd: Frame, radius_m: float, dst=None):
    """(dst float32, dst float64, covered bool, edge margin) of resampling src into fd."""
    src = np.ascontiguousarray(src, dtype=np.float32)
    assert src.shape == (fs.rows, fs.width)
    out = (np.full((fd.rows, fd.width), np.nan, dtype=np.float32) if dst is None
           else np.ascontiguousarray(dst, dtype=np.float32).copy())
    o64 = np.full((fd.rows, fd.width), np.nan)
    cov = np.zeros((fd.rows, fd.width), dtype=np.uint8)
    mar = np.zeros((fd.rows, fd.width))
    a, b = fs.c(), fd.c()
    rc = load().or_resample(src.ctypes.data, C.byref(a), C.byref(b), float(radius_m),
                            out.ctypes.data, o64.ctypes.data, cov.ctypes.data, mar.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the frames")
    return out, o64, cov.astype(bool), mar


def frame_source_coords(fs: Frame, fd: Frame, radius_m: float, i: int, j: int):
    qx, qy, fr = C.c_double(), C.c_double(), C.c_double()
    a, b = fs.c(), fd.c()
    load().or_frame_source_coords(C.byref(a), C.byref(b), float(radius_m), int(i), int(j),
                                  C.byref(qx), C.byref(qy), C.byref(fr))
    return qx.value, qy.value, fr.value
