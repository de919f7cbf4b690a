"""Python binding of libsoftshadow: argument marshalling around the C ABI.

Every step of the soft-shadow path runs in the HIP kernels; torch provides the
device buffers and the current stream.  Names follow include/softshadow.h.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from . import _lib as L

SUN_RADIUS_RAD = math.radians(0.267)


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_f32_2d(h: torch.Tensor, name: str = "h") -> torch.Tensor:
    if not isinstance(h, torch.Tensor) or h.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor [rows, width]")
    if not h.is_cuda or h.dtype != torch.float32 or not h.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return h


@dataclass
class Params:
    """Method parameters (ss_params)."""
    radius_m: float = 1737400.0
    max_len_m: float = 0.0
    n_prime0: int = 5
    schedule: int = L.SS_SCHED_GEOMETRIC
    n_segments: int = 0
    mode: int = L.SS_MODE_DP
    uniform_step: float = 1.0
    prune: int = 1
    ray_tile: int = 0
    n_prime_list: tuple = ()

    def c(self) -> L.SSParams:
        lst = (C.c_int32 * 16)(*[int(v) for v in self.n_prime_list][:16])
        return L.SSParams(float(self.radius_m), float(self.max_len_m), int(self.n_prime0),
                          int(self.schedule), int(self.n_segments), int(self.mode),
                          float(self.uniform_step), int(self.prune), int(self.ray_tile), lst)


def maxmip_levels(width: int, rows: int) -> int:
    return L.lib().ss_maxmip_levels(width, rows)


def maxmip_floats(width: int, rows: int) -> int:
    return L.lib().ss_maxmip_floats(width, rows)


def maxmip_level_offset(width: int, rows: int, level: int) -> int:
    return L.lib().ss_maxmip_level_offset(width, rows, level)


def maxmip(h: torch.Tensor, fuse_depth: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """Levels >= 1 of the maximum mipmap of h, packed (ss_maxmip_level_offset)."""
    _dev_f32_2d(h)
    rows, width = h.shape
    n = max(1, maxmip_floats(width, rows))
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=h.device)
    elif out.numel() < n or out.dtype != torch.float32 or not out.is_cuda:
        raise ValueError("out is too small or not float32 CUDA")
    L.check("ss_maxmip_build", L.lib().ss_maxmip_build(h.data_ptr(), width, rows, out.data_ptr(),
                                                       int(fuse_depth), _stream(h.device)))
    return out


def maxmip_unpack(mm: torch.Tensor, width: int, rows: int) -> list:
    """Views of levels 1..L-1 of a packed mipmap as [rows_m, width_m] tensors."""
    out = []
    w, r = width, rows
    for m in range(1, maxmip_levels(width, rows)):
        w, r = (w + 1) // 2, (r + 1) // 2
        off = maxmip_level_offset(width, rows, m)
        out.append(mm[off:off + w * r].view(r, w))
    return out


def bound_floats(width: int, rows: int) -> int:
    return L.lib().ss_bound_floats(width, rows)


def bound_level_offset(width: int, rows: int, level: int) -> int:
    return L.lib().ss_bound_level_offset(width, rows, level)


def bound_build(h: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Tap-bound pyramid of h (ss_bound_build), packed (ss_bound_level_offset)."""
    _dev_f32_2d(h)
    rows, width = h.shape
    n = max(1, bound_floats(width, rows))
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=h.device)
    elif out.numel() < n or out.dtype != torch.float32 or not out.is_cuda:
        raise ValueError("out is too small or not float32 CUDA")
    L.check("ss_bound_build", L.lib().ss_bound_build(h.data_ptr(), width, rows, out.data_ptr(),
                                                     _stream(h.device)))
    return out


def bound_unpack(b: torch.Tensor, width: int, rows: int) -> list:
    """Views of levels 0..L-1 of a packed tap-bound pyramid as [rows_m, width_m] tensors."""
    out = [b[:width * rows].view(rows, width)]
    w, r = width, rows
    for m in range(1, maxmip_levels(width, rows)):
        w, r = (w + 1) // 2, (r + 1) // 2
        off = bound_level_offset(width, rows, m)
        out.append(b[off:off + w * r].view(r, w))
    return out


def _tile(h: torch.Tensor, mm: torch.Tensor, texel_m: float, bound=None, window=None) -> L.SSTile:
    """window = (x0, y0, w, h): rays start only in that rectangle (ss_tile)."""
    rows, width = h.shape
    x0, y0, w, hh = (0, 0, 0, 0) if window is None else (int(v) for v in window)
    return L.SSTile(h.data_ptr(), mm.data_ptr(), width, rows, float(texel_m),
                    bound.data_ptr() if bound is not None else None, x0, y0, w, hh)


def _ray_shape(h: torch.Tensor, window) -> tuple:
    """Shape of the per-ray buffers: the window's, or the tile's."""
    if window is None:
        return tuple(h.shape)
    return (int(window[3]), int(window[2]))


def _check_ray_buf(t: torch.Tensor, h: torch.Tensor, window, dtype, name: str) -> None:
    if (not isinstance(t, torch.Tensor) or tuple(t.shape) != _ray_shape(h, window)
            or t.dtype != dtype or not t.is_contiguous() or t.device != h.device):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape "
                         f"{_ray_shape(h, window)} on {h.device}")


def _bound_for(h, params, bound):
    if bound is None and params.mode == L.SS_MODE_EXACT:
        bound = bound_build(h)
    return bound


def _sun(elev: float, azim: float, ang_radius: float) -> L.SSSun:
    return L.SSSun(float(elev), float(azim), float(ang_radius))


def shadow_cast(h: torch.Tensor, texel_m: float, elev: float, azim: float,
                ang_radius: float = SUN_RADIUS_RAD, params: Params | None = None,
                mm: torch.Tensor | None = None, out: torch.Tensor | None = None,
                bound: torch.Tensor | None = None, window=None) -> torch.Tensor:
    """Shadow factor s in [0, 1] for every texel of h, or of the ray window
    (x0, y0, w, h) (builds the mipmap if mm is None, and in the exact mode the
    tap-bound pyramid if bound is None)."""
    _dev_f32_2d(h)
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    if out is None:
        out = torch.empty(_ray_shape(h, window), dtype=torch.float32, device=h.device)
    _check_ray_buf(out, h, window, torch.float32, "out")
    t = _tile(h, mm, texel_m, bound, window)
    s = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_cast", L.lib().ss_shadow_cast(C.byref(t), C.byref(s), C.byref(p),
                                                     out.data_ptr(), _stream(h.device)))
    return out


def shadow_cast_counted(h, texel_m, elev, azim, ang_radius=SUN_RADIUS_RAD, params=None, mm=None,
                        out=None, bound=None, window=None):
    """(s, [lower-bound evaluations, bilinear samples]) of one forward launch."""
    _dev_f32_2d(h)
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    if out is None:
        out = torch.empty(_ray_shape(h, window), dtype=torch.float32, device=h.device)
    _check_ray_buf(out, h, window, torch.float32, "out")
    cnt = torch.zeros(2, dtype=torch.int64, device=h.device)
    t = _tile(h, mm, texel_m, bound, window)
    s = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_cast_counted",
            L.lib().ss_shadow_cast_counted(C.byref(t), C.byref(s), C.byref(p), out.data_ptr(),
                                           cnt.data_ptr(), _stream(h.device)))
    return out, cnt


def shadow_cast_backward(h, texel_m, elev, azim, grad_s, ang_radius=SUN_RADIUS_RAD, params=None,
                         mm=None, grad_h=None, grad_sun=None, bound=None, window=None):
    """Accumulates dL/dh (float32) and dL/d(elev, azim) (float64[2]) for upstream dL/ds."""
    _dev_f32_2d(h)
    _check_ray_buf(grad_s, h, window, torch.float32, "grad_s")
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    if grad_h is None:
        grad_h = torch.zeros_like(h)
    if grad_sun is None:
        grad_sun = torch.zeros(2, dtype=torch.float64, device=h.device)
    t = _tile(h, mm, texel_m, bound, window)
    s = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_cast_backward",
            L.lib().ss_shadow_cast_backward(C.byref(t), C.byref(s), C.byref(p),
                                            grad_s.data_ptr(), grad_h.data_ptr(),
                                            grad_sun.data_ptr(), _stream(h.device)))
    return grad_h, grad_sun


def shadow_cast_backward_penumbra(h, texel_m, elev, azim, s, grad_s, ang_radius=SUN_RADIUS_RAD,
                                  params=None, mm=None, grad_h=None, grad_sun=None, bound=None,
                                  window=None):
    """shadow_cast_backward given the forward's output s: rays at s = 0 or 1 (no derivative)
    are not replayed; same accumulation."""
    _dev_f32_2d(h)
    _check_ray_buf(grad_s, h, window, torch.float32, "grad_s")
    _check_ray_buf(s, h, window, torch.float32, "s")
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    if grad_h is None:
        grad_h = torch.zeros_like(h)
    if grad_sun is None:
        grad_sun = torch.zeros(2, dtype=torch.float64, device=h.device)
    t = _tile(h, mm, texel_m, bound, window)
    sn = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_cast_backward_penumbra",
            L.lib().ss_shadow_cast_backward_penumbra(C.byref(t), C.byref(sn), C.byref(p),
                                                     s.data_ptr(), grad_s.data_ptr(),
                                                     grad_h.data_ptr(), grad_sun.data_ptr(),
                                                     _stream(h.device)))
    return grad_h, grad_sun


def shadow_cast_save(h, texel_m, elev, azim, ang_radius=SUN_RADIUS_RAD, params=None, mm=None,
                     out=None, bound=None, sample=None, window=None):
    """(s, sample): s as shadow_cast, and each ray's deciding sample index (int32, -1 none)."""
    _dev_f32_2d(h)
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    if out is None:
        out = torch.empty(_ray_shape(h, window), dtype=torch.float32, device=h.device)
    if sample is None:
        sample = torch.empty(_ray_shape(h, window), dtype=torch.int32, device=h.device)
    _check_ray_buf(out, h, window, torch.float32, "out")
    _check_ray_buf(sample, h, window, torch.int32, "sample")
    t = _tile(h, mm, texel_m, bound, window)
    s = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_cast_save",
            L.lib().ss_shadow_cast_save(C.byref(t), C.byref(s), C.byref(p), out.data_ptr(),
                                        sample.data_ptr(), _stream(h.device)))
    return out, sample


def shadow_cast_backward_saved(h, texel_m, elev, azim, sample, grad_s, ang_radius=SUN_RADIUS_RAD,
                               params=None, mm=None, grad_h=None, grad_sun=None, bound=None,
                               window=None):
    """shadow_cast_backward from the record of shadow_cast_save (no replay)."""
    _dev_f32_2d(h)
    _check_ray_buf(grad_s, h, window, torch.float32, "grad_s")
    _check_ray_buf(sample, h, window, torch.int32, "sample")
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    if grad_h is None:
        grad_h = torch.zeros_like(h)
    if grad_sun is None:
        grad_sun = torch.zeros(2, dtype=torch.float64, device=h.device)
    t = _tile(h, mm, texel_m, bound, window)
    s = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_cast_backward_saved",
            L.lib().ss_shadow_cast_backward_saved(C.byref(t), C.byref(s), C.byref(p),
                                                  sample.data_ptr(), grad_s.data_ptr(),
                                                  grad_h.data_ptr(), grad_sun.data_ptr(),
                                                  _stream(h.device)))
    return grad_h, grad_sun


def shadow_points(h: torch.Tensor, texel_m: float, elev: float, azim: float, xy: torch.Tensor,
                  ang_radius: float = SUN_RADIUS_RAD, params: Params | None = None,
                  mm: torch.Tensor | None = None, out: torch.Tensor | None = None,
                  bound: torch.Tensor | None = None) -> torch.Tensor:
    """s at surface points xy [n, 2] (float32 CUDA, continuous texel coordinates)."""
    _dev_f32_2d(h)
    if (not isinstance(xy, torch.Tensor) or xy.dim() != 2 or xy.shape[1] != 2 or not xy.is_cuda
            or xy.dtype != torch.float32 or not xy.is_contiguous()):
        raise ValueError("xy must be a contiguous float32 CUDA tensor [n, 2]")
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    n = xy.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=h.device)
    t = _tile(h, mm, texel_m, bound)
    s = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_points",
            L.lib().ss_shadow_points(C.byref(t), C.byref(s), C.byref(p), xy.data_ptr(), n,
                                     out.data_ptr(), _stream(h.device)))
    return out


@dataclass
class Camera:
    """Pinhole camera in the tile frame (ss_camera): metres; the eye relative to the
    point where the tile's z axis meets the reference surface.  Pixel (px, py)
    looks along fwd + sx*right + sy*up, sx = 2(px+1/2)/width - 1,
    sy = 1 - 2(py+1/2)/height."""
    width: int
    height: int
    eye: tuple
    fwd: tuple
    right: tuple
    up: tuple
    step_m: float
    far_m: float = 0.0
    mode: int = L.SS_VIEW_HIER

    def c(self) -> L.SSCamera:
        v3 = C.c_double * 3
        return L.SSCamera(int(self.width), int(self.height), v3(*map(float, self.eye)),
                          v3(*map(float, self.fwd)), v3(*map(float, self.right)),
                          v3(*map(float, self.up)), float(self.step_m), float(self.far_m),
                          int(self.mode))


def view_cast(h: torch.Tensor, texel_m: float, cam: Camera, radius_m: float = 1737400.0,
              bound: torch.Tensor | None = None, steps: bool = False, out_t=None, out_xy=None):
    """First hits of the camera's view rays (ss_view_cast).

    Returns (t [H, W] float32, xy [H, W, 2] float32) and, with steps=True, the
    int32 [H, W, 2] counts (grid samples tested, pyramid cells visited)."""
    _dev_f32_2d(h)
    if bound is None:
        bound = bound_build(h)
    shape = (int(cam.height), int(cam.width))
    if out_t is None:
        out_t = torch.empty(shape, dtype=torch.float32, device=h.device)
    if out_xy is None:
        out_xy = torch.empty(shape + (2,), dtype=torch.float32, device=h.device)
    for t, sh, name in ((out_t, shape, "out_t"), (out_xy, shape + (2,), "out_xy")):
        if (tuple(t.shape) != sh or t.dtype != torch.float32 or not t.is_contiguous()
                or t.device != h.device):
            raise ValueError(f"{name} must be a contiguous float32 tensor of shape {sh}")
    st = torch.empty(shape + (2,), dtype=torch.int32, device=h.device) if steps else None
    rows, width = h.shape
    tile = L.SSTile(h.data_ptr(), None, width, rows, float(texel_m), bound.data_ptr(), 0, 0, 0, 0)
    cc = cam.c()
    L.check("ss_view_cast",
            L.lib().ss_view_cast(C.byref(tile), float(radius_m), C.byref(cc), out_t.data_ptr(),
                                 out_xy.data_ptr(), st.data_ptr() if steps else None,
                                 _stream(h.device)))
    return (out_t, out_xy, st) if steps else (out_t, out_xy)


def frame(h: torch.Tensor, texel_m: float, cam: Camera, elev: float, azim: float,
          ang_radius: float = SUN_RADIUS_RAD, params: Params | None = None,
          mm: torch.Tensor | None = None, bound: torch.Tensor | None = None):
    """One frame as Sec. 4 and 6.3 run it: view rays to the terrain, then a shadow ray
    from every visible point.  Returns (s [H, W], t [H, W], xy [H, W, 2]); pixels that
    see no terrain have s = NaN, t = +inf."""
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    if bound is None:
        bound = bound_build(h)
    t, xy = view_cast(h, texel_m, cam, params.radius_m, bound)
    s = shadow_points_image(h, texel_m, elev, azim, xy, ang_radius, params, mm, bound=bound)
    return s, t, xy


@dataclass
class Frame:
    """Gnomonic tile frame (ss_frame): plane tangent at unit vector ``centre`` (planet frame),
    unit axes ex (+column) and ey (+row), texel spacing texel_m in the plane, grid centre at
    plane coordinates ``origin`` (metres)."""
    width: int
    rows: int
    texel_m: float
    centre: tuple
    ex: tuple
    ey: tuple
    origin: tuple = (0.0, 0.0)

    def c(self) -> L.SSFrame:
        v3, v2 = C.c_double * 3, C.c_double * 2
        return L.SSFrame(int(self.width), int(self.rows), float(self.texel_m),
                         v3(*map(float, self.centre)), v3(*map(float, self.ex)),
                         v3(*map(float, self.ey)), v2(*map(float, self.origin)))


def resample(src: torch.Tensor, fs: Frame, dst: torch.Tensor, fd: Frame,
             radius_m: float = 1737400.0) -> torch.Tensor:
    """Writes src's heights into the texels of dst that fall inside src (ss_resample)."""
    _dev_f32_2d(src, "src")
    _dev_f32_2d(dst, "dst")
    if tuple(src.shape) != (fs.rows, fs.width) or tuple(dst.shape) != (fd.rows, fd.width):
        raise ValueError("tensor shapes must match their frames")
    a, b = fs.c(), fd.c()
    L.check("ss_resample", L.lib().ss_resample(src.data_ptr(), C.byref(a), dst.data_ptr(),
                                               C.byref(b), float(radius_m), _stream(dst.device)))
    return dst


def stitch(sources, fd: Frame, radius_m: float = 1737400.0, out: torch.Tensor | None = None,
           device=None) -> torch.Tensor:
    """One tile in frame fd from (heights, Frame) sources, later sources over earlier ones;
    texels no source covers stay NaN."""
    if out is None:
        dev = device if device is not None else sources[0][0].device
        out = torch.full((fd.rows, fd.width), float("nan"), dtype=torch.float32, device=dev)
    for h, f in sources:
        resample(h, f, out, fd, radius_m)
    return out


def shadow_points_image(h: torch.Tensor, texel_m: float, elev: float, azim: float,
                        xy: torch.Tensor, ang_radius: float = SUN_RADIUS_RAD,
                        params: Params | None = None, mm: torch.Tensor | None = None,
                        out: torch.Tensor | None = None,
                        bound: torch.Tensor | None = None) -> torch.Tensor:
    """s at an image of surface points xy [H, W, 2] (float32 CUDA, as view_cast returns it):
    shadow_points' values, shaded in 8 x 8 pixel tiles.  Returns [H, W]."""
    _dev_f32_2d(h)
    if (not isinstance(xy, torch.Tensor) or xy.dim() != 3 or xy.shape[2] != 2 or not xy.is_cuda
            or xy.dtype != torch.float32 or not xy.is_contiguous()):
        raise ValueError("xy must be a contiguous float32 CUDA tensor [H, W, 2]")
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    H, W = int(xy.shape[0]), int(xy.shape[1])
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=h.device)
    t = _tile(h, mm, texel_m, bound)
    s = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_points_image",
            L.lib().ss_shadow_points_image(C.byref(t), C.byref(s), C.byref(p), xy.data_ptr(), W, H,
                                           out.data_ptr(), _stream(h.device)))
    return out


def probe_gather_tiles(src: torch.Tensor, iters: int = 64, n_threads: int = 1 << 21,
                       out: torch.Tensor | None = None) -> torch.Tensor:
    """Coherent gather probe (ss_probe_gather_tiles): each wavefront reads 8 x 8 patches of the
    2-D float32 image src; returns the per-lane sums."""
    if (not src.is_cuda or src.dtype != torch.float32 or not src.is_contiguous()
            or src.dim() != 2):
        raise ValueError("src must be a contiguous 2-D float32 CUDA tensor")
    if out is None:
        out = torch.empty(n_threads, dtype=torch.float32, device=src.device)
    elif out.numel() < n_threads:
        raise ValueError("out is too small")
    L.check("ss_probe_gather_tiles",
            L.lib().ss_probe_gather_tiles(src.data_ptr(), int(src.shape[1]), int(src.shape[0]),
                                          int(iters), out.data_ptr(), int(n_threads),
                                          _stream(src.device)))
    return out


def probe_valu(iters: int = 4096, n_workgroups: int = 8192, device=None,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """FP32 VALU probe (ss_probe_valu): 32 * iters FMAs per lane over n_workgroups x 256 lanes;
    returns the per-lane sums."""
    n = int(n_workgroups) * 256
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=device or "cuda")
    elif out.numel() < n or not out.is_cuda or out.dtype != torch.float32:
        raise ValueError("out must be float32 CUDA with n_workgroups * 256 elements")
    L.check("ss_probe_valu", L.lib().ss_probe_valu(int(iters), int(n_workgroups), out.data_ptr(),
                                                   _stream(out.device)))
    return out


def probe_gather(src: torch.Tensor, window: int = 0, iters: int = 64, n_threads: int = 1 << 21,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """Memory-system gather probe (ss_probe_gather); returns the per-lane sums."""
    if not src.is_cuda or src.dtype != torch.float32 or not src.is_contiguous():
        raise ValueError("src must be a contiguous float32 CUDA tensor")
    if out is None:
        out = torch.empty(n_threads, dtype=torch.float32, device=src.device)
    elif out.numel() < n_threads:
        raise ValueError("out is too small")
    L.check("ss_probe_gather", L.lib().ss_probe_gather(src.data_ptr(), src.numel(), int(window),
                                                       int(iters), out.data_ptr(), int(n_threads),
                                                       _stream(src.device)))
    return out


class ShadowCast(torch.autograd.Function):
    """s = shadow(h, elev, azim) with the hand-written adjoint kernel as backward.

    By default the forward keeps only the heights, the max-mip, (exact mode)
    the tap-bound pyramid and its own output, and the backward recomputes the
    decisions of every ray whose s lies strictly inside (0, 1) (the others have
    no derivative; ss_shadow_cast_backward_penumbra) before applying the chain
    rule.  With record=True
    the forward also writes each ray's deciding sample (4 bytes per ray,
    ss_shadow_cast_save) and the backward reads it instead of replaying
    (ss_shadow_cast_backward_saved); both give the same gradient up to the order
    of the atomic sums.
    h: float32 CUDA [rows, width]; elev, azim: 0-d float64 tensors (CPU or CUDA).
    Gradients: dL/dh float32 (same device as h), dL/delev and dL/dazim float64.
    """

    @staticmethod
    def forward(ctx, h, elev, azim, texel_m, ang_radius, params, window=None, record=False):
        e = float(elev)
        a = float(azim)
        hd = h.detach().contiguous()
        mm = maxmip(hd)
        bound = _bound_for(hd, params, None)
        if record:
            s, sample = shadow_cast_save(hd, texel_m, e, a, ang_radius, params, mm=mm,
                                         bound=bound, window=window)
        else:
            s = shadow_cast(hd, texel_m, e, a, ang_radius, params, mm=mm, bound=bound,
                            window=window)
            sample = s  # the forward's values tell the backward which rays to replay
        ctx.save_for_backward(hd, mm, bound if bound is not None else hd.new_empty(0), sample)
        ctx.has_bound = bound is not None
        ctx.cfg = (texel_m, e, a, ang_radius, params, elev, azim, window, record)
        return s

    @staticmethod
    def backward(ctx, grad_s):
        hd, mm, bound, sample = ctx.saved_tensors
        texel_m, e, a, ang_radius, params, elev, azim, window, record = ctx.cfg
        bound = bound if ctx.has_bound else None
        g = grad_s.contiguous()
        if record:
            gh, gsun = shadow_cast_backward_saved(hd, texel_m, e, a, sample, g, ang_radius,
                                                  params, mm=mm, bound=bound, window=window)
        else:
            gh, gsun = shadow_cast_backward_penumbra(hd, texel_m, e, a, sample, g, ang_radius,
                                                     params, mm=mm, bound=bound, window=window)
        ge = gsun[0].to(elev.device) if isinstance(elev, torch.Tensor) else None
        ga = gsun[1].to(azim.device) if isinstance(azim, torch.Tensor) else None
        return gh, ge, ga, None, None, None, None, None


def shadow(h, elev, azim, texel_m, ang_radius=SUN_RADIUS_RAD, params: Params | None = None,
           window=None, record: bool = False):
    """Differentiable shadow factor (see ShadowCast); window = (x0, y0, w, h)
    limits the ray origins, the gradient still covers every height.  The
    backward recomputes the descent's decisions; record=True stores 4 bytes per
    ray in the forward instead."""
    params = params or Params()
    if not isinstance(elev, torch.Tensor):
        elev = torch.tensor(float(elev), dtype=torch.float64)
    if not isinstance(azim, torch.Tensor):
        azim = torch.tensor(float(azim), dtype=torch.float64)
    return ShadowCast.apply(h, elev, azim, texel_m, ang_radius, params, window, bool(record))


def shadow_points_backward(h: torch.Tensor, texel_m: float, elev: float, azim: float,
                           xy: torch.Tensor, grad_s: torch.Tensor,
                           ang_radius: float = SUN_RADIUS_RAD, params: Params | None = None,
                           mm: torch.Tensor | None = None, bound: torch.Tensor | None = None,
                           grad_h: torch.Tensor | None = None,
                           grad_sun: torch.Tensor | None = None):
    """Adjoint of shadow_points / shadow_points_image with the points held fixed
    (ss_shadow_points_backward).  xy: [n, 2] or an image [H, W, 2]; grad_s: n or [H, W]
    values.  Returns (dL/dh float32 [rows, width], dL/d(elev, azim) float64 [2]),
    accumulated into grad_h / grad_sun when given."""
    _dev_f32_2d(h)
    if (not isinstance(xy, torch.Tensor) or xy.dim() not in (2, 3) or xy.shape[-1] != 2
            or not xy.is_cuda or xy.dtype != torch.float32 or not xy.is_contiguous()):
        raise ValueError("xy must be a contiguous float32 CUDA tensor [n, 2] or [H, W, 2]")
    n = xy.numel() // 2
    width = int(xy.shape[1]) if xy.dim() == 3 else 0
    g = grad_s.contiguous()
    if g.numel() != n or g.dtype != torch.float32 or not g.is_cuda:
        raise ValueError("grad_s must be float32 CUDA with one value per point")
    params = params or Params()
    if mm is None:
        mm = maxmip(h)
    bound = _bound_for(h, params, bound)
    if grad_h is None:
        grad_h = torch.zeros_like(h)
    if grad_sun is None:
        grad_sun = torch.zeros(2, dtype=torch.float64, device=h.device)
    t = _tile(h, mm, texel_m, bound)
    s = _sun(elev, azim, ang_radius)
    p = params.c()
    L.check("ss_shadow_points_backward",
            L.lib().ss_shadow_points_backward(C.byref(t), C.byref(s), C.byref(p), xy.data_ptr(), n,
                                              width, g.data_ptr(), grad_h.data_ptr(),
                                              grad_sun.data_ptr(), _stream(h.device)))
    return grad_h, grad_sun


class ShadowPoints(torch.autograd.Function):
    """s at fixed surface points (a frame's view hits), differentiable in the heights and the
    sun direction: the forward is shadow_points (or shadow_points_image for [H, W, 2] points),
    the backward the points adjoint kernel.  The points themselves get no gradient."""

    @staticmethod
    def forward(ctx, h, elev, azim, xy, texel_m, ang_radius, params):
        e = float(elev)
        a = float(azim)
        hd = h.detach().contiguous()
        mm = maxmip(hd)
        bound = _bound_for(hd, params, None)
        if xy.dim() == 3:
            s = shadow_points_image(hd, texel_m, e, a, xy, ang_radius, params, mm, bound=bound)
        else:
            s = shadow_points(hd, texel_m, e, a, xy, ang_radius, params, mm, bound=bound)
        ctx.save_for_backward(hd, mm, bound if bound is not None else hd.new_empty(0), xy)
        ctx.has_bound = bound is not None
        ctx.cfg = (texel_m, e, a, ang_radius, params, elev, azim)
        return s

    @staticmethod
    def backward(ctx, grad_s):
        hd, mm, bound, xy = ctx.saved_tensors
        texel_m, e, a, ang_radius, params, elev, azim = ctx.cfg
        g = torch.nan_to_num(grad_s.contiguous(), nan=0.0)
        gh, gsun = shadow_points_backward(hd, texel_m, e, a, xy, g, ang_radius, params, mm=mm,
                                          bound=bound if ctx.has_bound else None)
        ge = gsun[0].to(elev.device) if isinstance(elev, torch.Tensor) else None
        ga = gsun[1].to(azim.device) if isinstance(azim, torch.Tensor) else None
        return gh, ge, ga, None, None, None, None


def shadow_at(h, elev, azim, xy, texel_m, ang_radius=SUN_RADIUS_RAD,
              params: Params | None = None):
    """Differentiable shadow factor at fixed surface points xy ([n, 2] or a frame's [H, W, 2]
    view hits; NaN points give NaN and no gradient)."""
    params = params or Params()
    if not isinstance(elev, torch.Tensor):
        elev = torch.tensor(float(elev), dtype=torch.float64)
    if not isinstance(azim, torch.Tensor):
        azim = torch.tensor(float(azim), dtype=torch.float64)
    return ShadowPoints.apply(h, elev, azim, xy, texel_m, ang_radius, params)


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------

def _batch_structs(heights, mms, texels, suns, windows=None, bounds=None):
    nt = len(heights)
    tiles = (L.SSTile * max(1, nt))()
    windows = windows or [None] * nt
    bounds = bounds or [None] * nt
    for k, (h, mm, tx) in enumerate(zip(heights, mms, texels)):
        _dev_f32_2d(h, f"heights[{k}]")
        tiles[k] = _tile(h, mm, tx, bounds[k], windows[k])
    ns = len(suns)
    ss = (L.SSSun * max(1, ns))()
    for k, sun in enumerate(suns):
        e, a = sun[0], sun[1]
        r = sun[2] if len(sun) > 2 else SUN_RADIUS_RAD
        ss[k] = _sun(e, a, r)
    return tiles, ss


def batched_workspace_bytes(n_tiles: int, n_suns: int) -> int:
    return L.lib().ss_batched_workspace_bytes(n_tiles, n_suns)


def _alloc_batch(heights, suns, outs, mms, windows=None, ws=None):
    dev = heights[0].device
    windows = windows or [None] * len(heights)
    if mms is None:
        mms = [torch.empty(max(1, maxmip_floats(h.shape[1], h.shape[0])), dtype=torch.float32,
                           device=dev) for h in heights]
    if outs is None:
        outs = [[torch.empty(_ray_shape(h, w), dtype=torch.float32, device=dev) for _ in suns]
                for h, w in zip(heights, windows)]
    ptrs = (C.c_void_p * max(1, len(heights) * len(suns)))()
    for t in range(len(heights)):
        for k in range(len(suns)):
            o = outs[t][k]
            _check_ray_buf(o, heights[t], windows[t], torch.float32, "out")
            ptrs[t * len(suns) + k] = o.data_ptr()
    need = max(256, batched_workspace_bytes(len(heights), len(suns)))
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    elif ws.dtype != torch.uint8 or ws.numel() < need or not ws.is_cuda or ws.data_ptr() % 256:
        raise ValueError(f"ws must be a 256-byte aligned uint8 CUDA tensor of >= {need} bytes")
    return mms, outs, ptrs, ws


def _bounds_for(heights, params, bounds):
    """Tap-bound buffers for the exact mode (the batched call fills them)."""
    if bounds is None and params.mode == L.SS_MODE_EXACT:
        bounds = [torch.empty(max(1, bound_floats(h.shape[1], h.shape[0])), dtype=torch.float32,
                              device=h.device) for h in heights]
    return bounds


def shadow_cast_batched(heights, texels, suns, params: Params | None = None, outs=None, mms=None,
                        windows=None, bounds=None, ws=None):
    """s for every (tile, sun): returns outs[t][k] (float32, shape of tile t or
    of its ray window).

    Builds every tile's mipmap (and, in the exact mode, its tap-bound pyramid
    into ``bounds``) and runs one launch over every ray block of every (tile, sun)
    (flat by default; SS_BATCH_FORM=persistent selects the persistent form).
    ``ws``: the workspace (uint8, batched_workspace_bytes), allocated if None.
    """
    params = params or Params()
    if len(heights) == 0 or len(suns) == 0:
        return [[] for _ in heights]
    mms, outs, ptrs, ws = _alloc_batch(heights, suns, outs, mms, windows, ws)
    bounds = _bounds_for(heights, params, bounds)
    tiles, ss = _batch_structs(heights, mms, texels, suns, windows, bounds)
    p = params.c()
    L.check("ss_shadow_cast_batched",
            L.lib().ss_shadow_cast_batched(tiles, len(heights), ss, len(suns), C.byref(p),
                                           ptrs, ws.data_ptr(), ws.numel(),
                                           _stream(heights[0].device)))
    return outs


class BatchedPlan:
    """Captured HIP graph of the batched call for fixed buffers (tuned at creation)."""

    def __init__(self, heights, texels, suns, params: Params | None = None, outs=None, mms=None,
                 windows=None, bounds=None):
        self.params = params or Params()
        self.heights = list(heights)
        self.mms, self.outs, self._ptrs, self.ws = _alloc_batch(self.heights, suns, outs, mms,
                                                                windows)
        self.bounds = _bounds_for(self.heights, self.params, bounds)
        self._tiles, self._suns = _batch_structs(self.heights, self.mms, texels, suns, windows,
                                                 self.bounds)
        self._p = self.params.c()
        handle = C.c_void_p()
        L.check("ss_batched_plan_create",
                L.lib().ss_batched_plan_create(self._tiles, len(self.heights), self._suns,
                                               len(suns), C.byref(self._p), self._ptrs,
                                               self.ws.data_ptr(), self.ws.numel(),
                                               _stream(self.heights[0].device), C.byref(handle)))
        self._h = handle

    def launch(self):
        L.check("ss_batched_plan_launch",
                L.lib().ss_batched_plan_launch(self._h, _stream(self.heights[0].device)))
        return self.outs

    def config(self):
        rt = C.c_int32()
        fd = C.c_int32()
        L.check("ss_batched_plan_config", L.lib().ss_batched_plan_config(self._h, C.byref(rt),
                                                                         C.byref(fd)))
        return int(rt.value), int(fd.value)

    def close(self):
        if getattr(self, "_h", None):
            L.lib().ss_batched_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
