"""MI355X (gfx950) Canny edge detector: Python binding of libcanny.so.

Each function marshals torch tensors (device memory, the current HIP stream)
into the C ABI declared in include/canny.h; every step of the operator runs
in the library's HIP kernels.  There is no CPU or PyTorch fallback: if the
library is missing or the device is not a gfx950, the call raises.

Operator (paper Section 2.2.1, Steps 1-4): noise filter -> Sobel gradient
strength and direction -> non-maximum suppression -> hysteresis with a low
and a high threshold.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import CannyError, check, lib

__all__ = [
    "canny_u8", "canny_u8_noalloc", "canny_log_u8", "canny_f32", "canny_f32_sector", "VideoStream", "hysteresis", "class_pitch", "u8_workspace_bytes", "f32_workspace_bytes",
    "BatchPlan", "mag_forward", "mag_backward", "CannyMagnitude", "canny_magnitude",
    "CannyError", "StageTiming",
]


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _check_image(img: torch.Tensor, dtype: torch.dtype, name: str = "img"):
    if not isinstance(img, torch.Tensor) or not img.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if img.dtype != dtype or img.dim() != 2:
        raise ValueError(f"{name} must be a 2-D {dtype} tensor, got {img.dtype} {tuple(img.shape)}")
    if img.stride(1) != 1 or img.stride(0) < img.shape[1]:
        raise ValueError(f"{name} rows must be contiguous (stride(1) == 1)")


def class_pitch(W: int) -> int:
    """Row pitch in bytes of the packed 2-bit class map."""
    return int(lib().canny_class_pitch(int(W)))


def u8_workspace_bytes(H: int, W: int) -> int:
    return int(lib().canny_u8_workspace_bytes(int(H), int(W)))


def f32_workspace_bytes(H: int, W: int) -> int:
    return int(lib().canny_f32_workspace_bytes(int(H), int(W)))


def _workspace(n: int, device, ws: Optional[torch.Tensor]) -> torch.Tensor:
    if ws is not None:
        if ws.numel() * ws.element_size() < n:
            raise ValueError("workspace too small")
        return ws
    return torch.empty(max(n, 1), dtype=torch.uint8, device=device)


def canny_u8(img: torch.Tensor, low: int = 40, high: int = 100, *, edges: Optional[torch.Tensor] = None,
             with_edges: bool = True, return_classes: bool = False,
             class_map: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None):
    """Integer Canny on a uint8 image (5x5 binomial blur, L1 strength, 4-sector
    direction).  Returns the uint8 edge map (255 / 0), and the packed class
    map (H x class_pitch(W) bytes) if ``return_classes``."""
    _check_image(img, torch.uint8)
    H, W = img.shape
    if with_edges and edges is None:
        edges = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    if return_classes and class_map is None:
        class_map = torch.empty((H, class_pitch(W)), dtype=torch.uint8, device=img.device)
    ws = _workspace(u8_workspace_bytes(H, W), img.device, workspace)
    st = lib().canny_u8(img.data_ptr(), img.stride(0), H, W, int(low), int(high),
                        _ptr(edges) if with_edges else None, edges.stride(0) if with_edges else 0,
                        _ptr(class_map), ws.data_ptr(), ws.numel() * ws.element_size(), _stream(img))
    check("canny_u8", st)
    if return_classes:
        return (edges if with_edges else None), class_map
    return edges


def canny_u8_noalloc(img: torch.Tensor, low: int = 40, high: int = 100, *, edges: torch.Tensor,
                     class_map: Optional[torch.Tensor] = None):
    """canny_u8 through the allocation-free entry point: the caller passes the
    output buffers; the workspace is the library's static device scratch
    (images needing more than CANNY_NOALLOC_SCRATCH_BYTES raise).  This
    function allocates nothing either."""
    _check_image(img, torch.uint8)
    H, W = img.shape
    st = lib().canny_u8_noalloc(img.data_ptr(), img.stride(0), H, W, int(low), int(high),
                                _ptr(edges), edges.stride(0) if edges is not None else 0,
                                _ptr(class_map), _stream(img))
    check("canny_u8_noalloc", st)
    return edges


def canny_log_u8(img: torch.Tensor, t: int = 10, *, edges: Optional[torch.Tensor] = None,
                 return_laplacian: bool = False):
    """Laplacian zero-crossing detector on a uint8 image: binomial blur,
    5-point Laplacian L, edges at sign changes of L between 4-neighbours with
    |L(p) - L(q)| >= t (on the pixel nearer the zero) and at zeros between
    opposite neighbours.  Returns the edge map (255 / 0), and L (int16) if
    ``return_laplacian``."""
    _check_image(img, torch.uint8)
    H, W = img.shape
    if edges is None:
        edges = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    lap = torch.empty((H, W), dtype=torch.int16, device=img.device) if return_laplacian else None
    st = lib().canny_log_u8(img.data_ptr(), img.stride(0), H, W, int(t), edges.data_ptr(),
                            edges.stride(0), _ptr(lap), W if lap is not None else 0, _stream(img))
    check("canny_log_u8", st)
    return (edges, lap) if return_laplacian else edges


def hysteresis(class_map: torch.Tensor, H: int, W: int, *, edges: Optional[torch.Tensor] = None,
               workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Step 4 connectivity alone on a packed class map (H x class_pitch(W))."""
    if not class_map.is_cuda or class_map.dtype != torch.uint8 or not class_map.is_contiguous():
        raise ValueError("class_map must be a contiguous CUDA uint8 tensor")
    if tuple(class_map.shape) != (H, class_pitch(W)):
        raise ValueError("class_map must have shape (H, class_pitch(W))")
    if edges is None:
        edges = torch.empty((H, W), dtype=torch.uint8, device=class_map.device)
    n = int(lib().canny_hysteresis_workspace_bytes(int(H), int(W)))
    ws = _workspace(n, class_map.device, workspace)
    st = lib().canny_hysteresis(class_map.data_ptr(), int(H), int(W), edges.data_ptr(), edges.stride(0),
                                ws.data_ptr(), ws.numel() * ws.element_size(), _stream(class_map))
    check("canny_hysteresis", st)
    return edges


def canny_f32(img: torch.Tensor, sigma: float = 1.4, radius: int = 3, low: float = 0.05,
              high: float = 0.15, relative: bool = True, *, edges: Optional[torch.Tensor] = None,
              with_edges: bool = True, return_classes: bool = False, return_magnitude: bool = False,
              return_max: bool = False, workspace: Optional[torch.Tensor] = None):
    """Float Canny on an fp32 image (sampled Gaussian, L2 strength, continuous
    direction suppression).  ``relative``: thresholds are fractions of the
    image's largest strength.  Returns edges, then optionally the class map,
    the fp32 strength map and a 1-element max tensor, in that order."""
    _check_image(img, torch.float32)
    H, W = img.shape
    dev = img.device
    if with_edges and edges is None:
        edges = torch.empty((H, W), dtype=torch.uint8, device=dev)
    cls = torch.empty((H, class_pitch(W)), dtype=torch.uint8, device=dev) if return_classes else None
    mag = torch.empty((H, W), dtype=torch.float32, device=dev) if return_magnitude else None
    mx = torch.empty((1,), dtype=torch.float32, device=dev) if return_max else None
    ws = _workspace(f32_workspace_bytes(H, W), dev, workspace)
    st = lib().canny_f32(img.data_ptr(), img.stride(0), H, W, float(sigma), int(radius), float(low),
                         float(high), int(bool(relative)), _ptr(edges) if with_edges else None,
                         edges.stride(0) if with_edges else 0, _ptr(cls), _ptr(mag), _ptr(mx),
                         ws.data_ptr(), ws.numel() * ws.element_size(), _stream(img))
    check("canny_f32", st)
    out = [edges if with_edges else None]
    if return_classes:
        out.append(cls)
    if return_magnitude:
        out.append(mag)
    if return_max:
        out.append(mx)
    return out[0] if len(out) == 1 else tuple(out)


def canny_f32_sector(img: torch.Tensor, sigma: float = 1.4, radius: int = 3, low: float = 20.0,
                     high: float = 60.0, *, edges: Optional[torch.Tensor] = None,
                     with_edges: bool = True, return_classes: bool = False,
                     return_magnitude: bool = False, workspace: Optional[torch.Tensor] = None):
    """Float Canny with the direction quantised to four sectors (suppression
    against the two 8-neighbours along it) and absolute thresholds.  Returns
    edges, then optionally the class map and the fp32 strength map."""
    _check_image(img, torch.float32)
    H, W = img.shape
    dev = img.device
    if with_edges and edges is None:
        edges = torch.empty((H, W), dtype=torch.uint8, device=dev)
    cls = torch.empty((H, class_pitch(W)), dtype=torch.uint8, device=dev) if return_classes else None
    mag = torch.empty((H, W), dtype=torch.float32, device=dev) if return_magnitude else None
    ws = _workspace(f32_workspace_bytes(H, W), dev, workspace)
    st = lib().canny_f32_sector(img.data_ptr(), img.stride(0), H, W, float(sigma), int(radius),
                                float(low), float(high), _ptr(edges) if with_edges else None,
                                edges.stride(0) if with_edges else 0, _ptr(cls), _ptr(mag),
                                ws.data_ptr(), ws.numel() * ws.element_size(), _stream(img))
    check("canny_f32_sector", st)
    out = [edges if with_edges else None]
    if return_classes:
        out.append(cls)
    if return_magnitude:
        out.append(mag)
    return out[0] if len(out) == 1 else tuple(out)


class VideoStream:
    """Streaming integer Canny over host frames of one size: uploads, detection
    and downloads of successive frames overlap on three HIP streams, with a
    ring of ``depth`` device slots.  See canny_video_create.  Frames and edge
    buffers are CPU uint8 tensors of shape (H, W) (pinned ones copy
    asynchronously) and must stay untouched until ``sync()``."""

    def __init__(self, H: int, W: int, low: int = 40, high: int = 100, depth: int = 3,
                 device=None):
        self.H, self.W = int(H), int(W)
        self.device = torch.device(device or "cuda")
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib().canny_video_create(self.H, self.W, int(low), int(high), int(depth),
                                          C.byref(handle))
        check("canny_video_create", st)
        self._h = handle

    def _host(self, t: torch.Tensor, name: str):
        if t.device.type != "cpu" or t.dtype != torch.uint8 or tuple(t.shape) != (self.H, self.W) \
                or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous CPU uint8 tensor of shape "
                             f"({self.H}, {self.W})")
        return t.data_ptr()

    def push(self, frame: torch.Tensor, edges: torch.Tensor) -> None:
        if not self._h:
            raise ValueError("video stream is closed")
        with torch.cuda.device(self.device):
            st = lib().canny_video_push(self._h, self._host(frame, "frame"),
                                        self._host(edges, "edges"))
        check("canny_video_push", st)

    def sync(self) -> None:
        if self._h:
            check("canny_video_sync", lib().canny_video_sync(self._h))

    def close(self) -> None:
        if self._h:
            lib().canny_video_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Batched integer Canny over images of uneven sizes: one flat launch per
    phase, replayed from a recorded HIP graph.  See canny_batch_plan_create."""

    def __init__(self, shapes: Sequence[Sequence[int]], low: int = 40, high: int = 100,
                 autotune: bool = False, device=None):
        self.shapes = [(int(h), int(w)) for h, w in shapes]
        self.device = torch.device(device or "cuda")
        n = len(self.shapes)
        Hs = (C.c_int32 * n)(*[h for h, _ in self.shapes])
        Ws = (C.c_int32 * n)(*[w for _, w in self.shapes])
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib().canny_batch_plan_create(n, C.cast(Hs, C.c_void_p), C.cast(Ws, C.c_void_p),
                                               int(low), int(high), int(bool(autotune)),
                                               C.byref(handle))
        check("canny_batch_plan_create", st)
        self._h = handle
        self.workspace_bytes = int(lib().canny_batch_workspace_bytes(self._h))
        self._ws = None

    def info(self):
        a, b = C.c_int32(), C.c_int32()
        check("canny_batch_plan_info", lib().canny_batch_plan_info(self._h, C.byref(a), C.byref(b)))
        return {"fwd_rows": a.value, "hyst_rows": b.value}

    def run(self, images: Sequence[torch.Tensor], edges: Optional[Sequence[torch.Tensor]] = None,
            workspace: Optional[torch.Tensor] = None) -> List[torch.Tensor]:
        n = len(self.shapes)
        if len(images) != n:
            raise ValueError(f"expected {n} images")
        for k, (img, (h, w)) in enumerate(zip(images, self.shapes)):
            _check_image(img, torch.uint8, f"images[{k}]")
            if tuple(img.shape) != (h, w):
                raise ValueError(f"images[{k}] has shape {tuple(img.shape)}, plan expects {(h, w)}")
        if edges is None:
            edges = [torch.empty((h, w), dtype=torch.uint8, device=self.device) for h, w in self.shapes]
        if workspace is None:
            if self._ws is None:
                self._ws = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=self.device)
            workspace = self._ws
        ip = (C.c_void_p * n)(*[t.data_ptr() for t in images])
        ep = (C.c_void_p * n)(*[t.data_ptr() for t in edges])
        ipt = (C.c_int64 * n)(*[t.stride(0) for t in images])
        ept = (C.c_int64 * n)(*[t.stride(0) for t in edges])
        st = lib().canny_batch(self._h, C.cast(ip, C.c_void_p), C.cast(ipt, C.c_void_p),
                               C.cast(ep, C.c_void_p), C.cast(ept, C.c_void_p), workspace.data_ptr(),
                               workspace.numel(), _stream(images[0]))
        check("canny_batch", st)
        return list(edges)

    def close(self):
        if getattr(self, "_h", None):
            lib().canny_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_stack(t: torch.Tensor, name: str):
    if not t.is_cuda or t.dtype != torch.float32 or t.dim() != 3 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA float32 [N, H, W] tensor")


def mag_forward(I: torch.Tensor, sigma: torch.Tensor, radius: int = 9) -> torch.Tensor:
    """M = |Sobel * G_sigma * I| per image; I [N,H,W] fp32, sigma [N] fp32."""
    _check_stack(I, "I")
    N, H, W = I.shape
    sigma = sigma.contiguous()
    if sigma.dtype != torch.float32 or sigma.numel() != N or sigma.device != I.device:
        raise ValueError("sigma must be a float32 tensor of N values on I's device")
    M = torch.empty_like(I)
    st = lib().canny_mag_forward(I.data_ptr(), sigma.data_ptr(), N, H, W, int(radius), M.data_ptr(),
                                 _stream(I))
    check("canny_mag_forward", st)
    return M


def mag_backward(I: torch.Tensor, sigma: torch.Tensor, dM: torch.Tensor, radius: int = 9):
    """(dL/dI, dL/dsigma) of mag_forward given dL/dM."""
    _check_stack(I, "I")
    dM = dM.contiguous()
    _check_stack(dM, "dM")
    N, H, W = I.shape
    sigma = sigma.contiguous()
    dI = torch.empty_like(I)
    ds = torch.empty((N,), dtype=torch.float32, device=I.device)
    nws = int(lib().canny_mag_backward_workspace_bytes(N, H, W, int(radius)))
    ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=I.device)
    st = lib().canny_mag_backward(I.data_ptr(), sigma.data_ptr(), dM.data_ptr(), N, H, W, int(radius),
                                  dI.data_ptr(), ds.data_ptr(), ws.data_ptr(), nws, _stream(I))
    check("canny_mag_backward", st)
    return dI, ds


class CannyMagnitude(torch.autograd.Function):
    """Differentiable front end M(I, sigma) = |Sobel * G_sigma * I|.  Saves I
    and sigma only; the backward recomputes the blur in the adjoint kernel."""

    @staticmethod
    def forward(ctx, I, sigma, radius: int = 9):
        ctx.radius = int(radius)
        ctx.save_for_backward(I, sigma)
        return mag_forward(I.detach().contiguous(), sigma.detach().contiguous(), ctx.radius)

    @staticmethod
    def backward(ctx, gM):
        I, sigma = ctx.saved_tensors
        dI, ds = mag_backward(I.detach().contiguous(), sigma.detach().contiguous(), gM, ctx.radius)
        return (dI if ctx.needs_input_grad[0] else None,
                ds if ctx.needs_input_grad[1] else None, None)


def canny_magnitude(I: torch.Tensor, sigma: torch.Tensor, radius: int = 9) -> torch.Tensor:
    return CannyMagnitude.apply(I, sigma, radius)


class StageTiming:
    """Context manager over canny_timing_begin / _read / _end: while open,
    every library call records HIP events around each stage it runs (first
    ``capacity`` launches per stage).  ``read(stage)`` returns (total ms,
    launches) for a stage name of ``STAGES``."""

    STAGES = _lib.STAGES

    def __init__(self, capacity: int = 1024):
        self.capacity = int(capacity)

    def __enter__(self):
        check("canny_timing_begin", lib().canny_timing_begin(self.capacity))
        return self

    def read(self, stage: str):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        check("canny_timing_read", lib().canny_timing_read(self.STAGES[stage], C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def __exit__(self, *exc):
        lib().canny_timing_end()
        return False
