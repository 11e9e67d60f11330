"""PyTorch-facing calls of the shiftable bilateral filter.

PyTorch provides device memory and the current stream; every arithmetic step
runs in libbsk's HIP kernels through the C ABI (include/bsk.h).  Tensors must
be 2-D, contiguous and on the GPU.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence, Tuple

import torch

from . import _lib

__all__ = ["bilateral", "nlm2", "spatial_filter", "spatial_sigma_for", "bilateral_train", "bilateral_backward",
           "bilateral_batched", "order_for", "plan_info", "poly_order_for", "poly_plan_info", "autotune",
           "batched_shape", "autotune_batched", "tune_cache_load", "tune_cache_save", "tune_cache_clear",
           "BilateralFunction", "ShiftableBilateral", "release"]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_image(t: torch.Tensor, name: str, dtype=torch.float32, stack: bool = False):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor (libbsk runs only on the GPU)")
    if t.dim() != 2 and not (stack and t.dim() == 3):
        want = "2-D (H, W) or 3-D (B, H, W)" if stack else "2-D (H, W)"
        raise ValueError(f"{name} must be {want}, got shape {tuple(t.shape)}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _options(N=None, precision="fp32", weight_eps=0.0, kahan=False, block=0, strip_h=0, order_chunk=0,
             spatial_sigma=None, spatial_N=None, range_kernel="cos"):
    o = _lib.Options()
    if range_kernel not in _lib.RANGE_KERNELS:
        raise ValueError(f"range_kernel must be one of {sorted(_lib.RANGE_KERNELS)}")
    o.range_kernel = _lib.RANGE_KERNELS[range_kernel]
    if spatial_sigma is not None:
        o.spatial_sigma = float(spatial_sigma)
        o.spatial_N = -1 if spatial_N is None else int(spatial_N)
    elif spatial_N:
        raise ValueError("spatial_N needs spatial_sigma")
    if N is None:
        o.order_mode = 0
        o.N = 0
    else:
        o.order_mode = 1
        o.N = int(N)
    o.precision = _lib.PRECISIONS[precision]
    o.weight_eps = float(weight_eps)
    o.kahan = 1 if kahan else 0
    o.block = int(block)
    o.strip_h = int(strip_h)
    o.order_chunk = int(order_chunk)
    return o


def order_for(sigma_r: float, T: float = 255.0) -> int:
    """N_0: smallest order making the kernel non-negative and unimodal on [-T, T]."""
    n = _lib.load().bsk_order_for(float(sigma_r), float(T))
    if n < 0:
        _lib.check(_lib.BSK_EINVAL)
    return n


def plan_info(N: int, eps: float = 0.0):
    """(folded orders kept, dropped unfolded weight mass) for order N and threshold eps."""
    K = ctypes.c_int(0)
    d = ctypes.c_double(0.0)
    _lib.check(_lib.load().bsk_plan_info(int(N), float(eps), ctypes.byref(K), ctypes.byref(d)))
    return K.value, d.value


def poly_order_for(sigma_r: float, T: float = 255.0) -> int:
    """N_p = ceil(T^2 / (2 sigma_r^2)): smallest order making the polynomial kernel
    non-negative and unimodal on [-T, T]."""
    n = _lib.load().bsk_poly_order_for(float(sigma_r), float(T))
    if n < 0:
        _lib.check(_lib.BSK_EINVAL)
    return n


def poly_plan_info(sigma_r: float, T: float = 255.0, N: Optional[int] = None, eps: float = 0.0):
    """(Chebyshev coefficients kept, bound on the dropped part of the normalised kernel) of the
    polynomial range kernel; the filter box-sums one channel more than the coefficients kept."""
    K = ctypes.c_int(0)
    b = ctypes.c_double(0.0)
    _lib.check(_lib.load().bsk_poly_plan_info(-1 if N is None else int(N), float(sigma_r), float(T), float(eps),
                                              ctypes.byref(K), ctypes.byref(b)))
    return K.value, b.value


def bilateral(img: torch.Tensor, radius: int, sigma_r: float, T: float = 255.0, N: Optional[int] = None,
              precision: str = "fp32", weight_eps: float = 0.0, kahan: bool = False, block: int = 0,
              strip_h: int = 0, order_chunk: int = 0, out: Optional[torch.Tensor] = None,
              spatial_sigma: Optional[float] = None, spatial_N: Optional[int] = None,
              range_kernel: str = "cos") -> torch.Tensor:
    """Bilateral filter on the (2r+1)^2 window with the range kernel cos^N(t / (sigma_r sqrt N)).

    range_kernel: "cos" (the raised cosine above) or "poly", the polynomial kernel
    (1 - t^2 / (2 N sigma_r^2))^N (Section 3's p_N in the scaling of eq. (5); N None selects
    N_p(sigma_r, T); precision "fp32" or "fp64"; weight_eps > 0 truncates its Chebyshev
    expansion; box spatial kernel only).

    precision: "fp32" (default); "bf16", "fp16" or "i16" (precision form: the cos/sin stack
    quantised to bfloat16, float16 or 16-bit fixed point, FP32 sums); "fp64" (img float64).
    N: None selects N_0(sigma_r, T).  weight_eps > 0 drops binomial weights below it.
    spatial_sigma: None for the box spatial kernel; otherwise the separable spatial kernel
    w(dy) w(dx), w(d) = cos^Ns(d / (spatial_sigma sqrt Ns)) (Algorithm 2 with M = (Ns+1)^2),
    Ns = spatial_N, or the smallest order unimodal on the window when None (at most 6).
    block, strip_h, order_chunk: launch shape (0 = tuned or automatic).
    """
    dt = torch.float64 if precision == "fp64" else torch.float32
    _check_image(img, "img", dt)
    if out is None:
        out = torch.empty_like(img)
    else:
        _check_image(out, "out", dt)
        if out.shape != img.shape:
            raise ValueError("out has the wrong shape")
    H, W = img.shape
    opt = _options(N, precision, weight_eps, kahan, block, strip_h, order_chunk, spatial_sigma, spatial_N,
                   range_kernel)
    with torch.cuda.device(img.device):
        _lib.check(_lib.load().bilateral_shiftable_ex(
            ctypes.c_void_p(img.data_ptr()), H, W, int(radius), float(sigma_r), float(T),
            ctypes.c_void_p(out.data_ptr()), ctypes.byref(opt), _stream()))
    return out


def nlm2(img: torch.Tensor, radius: int, sigma_1: float, sigma_2: float, offset=(0, 1), T: float = 255.0,
         N1: Optional[int] = None, N2: Optional[int] = None, weight_eps: float = 0.0, block: int = 0,
         strip_h: int = 0, order_chunk: int = 0, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Two-pixel-patch non-local means (Section 5 with p = 2): the patches {x, x + offset} are
    compared through cos^N1(t1 / (sigma_1 sqrt N1)) cos^N2(t2 / (sigma_2 sqrt N2)) over the
    (2r+1)^2 window.  offset = (rows, columns); N1, N2 None select N_0 of each factor."""
    _check_image(img, "img")
    if out is None:
        out = torch.empty_like(img)
    else:
        _check_image(out, "out")
        if out.shape != img.shape:
            raise ValueError("out has the wrong shape")
    H, W = img.shape
    opt = _options(None, "fp32", weight_eps, False, block, strip_h, order_chunk)
    uy, ux = (int(v) for v in offset)
    with torch.cuda.device(img.device):
        _lib.check(_lib.load().bilateral_shiftable_nlm2(
            ctypes.c_void_p(img.data_ptr()), H, W, int(radius), float(sigma_1), float(sigma_2),
            -1 if N1 is None else int(N1), -1 if N2 is None else int(N2), uy, ux, float(T),
            ctypes.c_void_p(out.data_ptr()), ctypes.byref(opt), _stream()))
    return out


def spatial_filter(img: torch.Tensor, radius: int, spatial_sigma: float, spatial_N: Optional[int] = None,
                   out: Optional[torch.Tensor] = None, block: int = 0, strip_h: int = 0) -> torch.Tensor:
    """Algorithm 1: the normalised linear filter sum_y w(y - x) f(y) / sum_y w(y - x) over the
    (2r+1)^2 window with the separable raised-cosine spatial kernel (the range order N = 0)."""
    return bilateral(img, radius, 1.0, 1.0, N=0, out=out, block=block, strip_h=strip_h,
                     spatial_sigma=spatial_sigma, spatial_N=spatial_N)


def spatial_sigma_for(T_s: float, Ns: int) -> float:
    """spatial_sigma giving the paper's q_Ns(t) = cos^Ns(pi t / (2 T_s)) (Section 3)."""
    return 2.0 * float(T_s) / (math.pi * math.sqrt(int(Ns)))


def bilateral_train(img: torch.Tensor, radius: int, sigma_r: float, T: float = 255.0, N: Optional[int] = None):
    """(out, saved): the filter output and the planes the adjoint needs, saved = (Q, E1, E2).

    img (H, W) gives saved of shape (3, H, W); a stack (B, H, W) of images filtered with the
    same parameters runs as one launch and gives saved of shape (B, 3, H, W)."""
    _check_image(img, "img", stack=True)
    H, W = img.shape[-2:]
    B = img.shape[0] if img.dim() == 3 else 1
    out = torch.empty_like(img)
    saved = torch.empty((*img.shape[:-2], 3, H, W), dtype=torch.float32, device=img.device)
    opt = _options(N)
    lib = _lib.load()
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    with torch.cuda.device(img.device):
        if img.dim() == 2:
            _lib.check(lib.bilateral_shiftable_train(p(img), H, W, int(radius), float(sigma_r), float(T),
                                                     ctypes.byref(opt), p(out), p(saved), _stream()))
        else:
            _lib.check(lib.bilateral_shiftable_train_stack(p(img), B, H, W, int(radius), float(sigma_r), float(T),
                                                           ctypes.byref(opt), p(out), p(saved), _stream()))
    return out, saved


def bilateral_backward(img: torch.Tensor, grad_out: torch.Tensor, radius: int, sigma_r: float, T: float = 255.0,
                       N: Optional[int] = None, out: Optional[torch.Tensor] = None,
                       saved: Optional[torch.Tensor] = None, need_img: bool = True, need_sigma: bool = True):
    """(dL/dimg or None, dL/dsigma_r as a 0-d tensor or None).

    For a stack img (B, H, W) (one launch), dL/dsigma_r is summed over the stack."""
    _check_image(img, "img", stack=True)
    _check_image(grad_out, "grad_out", stack=True)
    if grad_out.shape != img.shape:
        raise ValueError("grad_out must have the shape of img")
    H, W = img.shape[-2:]
    B = img.shape[0] if img.dim() == 3 else 1
    if (out is None) != (saved is None):
        raise ValueError("give both out and saved, or neither")
    if out is not None:
        _check_image(out, "out", stack=True)
        if out.shape != img.shape:
            raise ValueError("out must have the shape of img")
        if (saved.shape != (*img.shape[:-2], 3, H, W) or not saved.is_contiguous()
                or saved.dtype != torch.float32):
            raise ValueError("saved must be a contiguous float32 tensor of shape (3, H, W), or (B, 3, H, W) "
                             "for a stack")
    gi = torch.empty_like(img) if need_img else None
    gs = torch.empty((), dtype=torch.float32, device=img.device) if need_sigma else None
    opt = _options(N)
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    lib = _lib.load()
    with torch.cuda.device(img.device):
        if img.dim() == 2:
            _lib.check(lib.bilateral_shiftable_backward(
                p(img), p(grad_out), p(out), p(saved), H, W, int(radius), float(sigma_r), float(T),
                ctypes.byref(opt), p(gi), p(gs), _stream()))
        else:
            _lib.check(lib.bilateral_shiftable_backward_stack(
                p(img), p(grad_out), p(out), p(saved), B, H, W, int(radius), float(sigma_r), float(T),
                ctypes.byref(opt), p(gi), p(gs), _stream()))
    return gi, gs


def _batch_descs(imgs, outs, radii, sigmas, Ns):
    B = len(imgs)
    descs = (_lib.ImageDesc * B)()
    for b, (x, o) in enumerate(zip(imgs, outs)):
        _check_image(x, f"imgs[{b}]")
        _check_image(o, f"outs[{b}]")
        descs[b].img = x.data_ptr()
        descs[b].out = o.data_ptr()
        descs[b].H, descs[b].W = x.shape
        descs[b].radius = int(radii[b])
        descs[b].sigma_r = float(sigmas[b])
        descs[b].N = -1 if Ns is None or Ns[b] is None else int(Ns[b])
    return descs


def bilateral_batched(imgs: Sequence[torch.Tensor], radii: Sequence[int], sigmas: Sequence[float],
                      T: float = 255.0, Ns: Optional[Sequence[int]] = None, outs=None,
                      graph_key: Optional[int] = None, strip_h: int = 0, block: int = 0, order_chunk: int = 0):
    """Filters many images (any sizes, radii, sigma_r) in one persistent launch.

    With graph_key set, the first call captures the launch into a HIP graph on the
    current (non-default) stream and later calls with the same key replay it.
    block, strip_h and order_chunk left at 0 take the tuned (bsk_autotune_batched)
    or default launch shape."""
    B = len(imgs)
    if outs is None:
        outs = [torch.empty_like(x) for x in imgs]
    descs = _batch_descs(imgs, outs, radii, sigmas, Ns)
    opt = _options(strip_h=strip_h, block=block, order_chunk=order_chunk)
    lib = _lib.load()
    with torch.cuda.device(imgs[0].device):
        if graph_key is None:
            _lib.check(lib.bilateral_shiftable_batched(descs, B, float(T), ctypes.byref(opt), _stream()))
        else:
            _lib.check(lib.bilateral_shiftable_batched_graph(descs, B, float(T), ctypes.byref(opt), int(graph_key),
                                                             _stream()))
    return outs


def batched_shape(shapes: Sequence[Tuple[int, int]], radii: Sequence[int], sigmas: Sequence[float],
                  T: float = 255.0, Ns: Optional[Sequence[int]] = None, strip_h: int = 0, block: int = 0,
                  order_chunk: int = 0):
    """The launch shape the batched entry points would use for images of these (H, W):
    (lanes per workgroup, [rows per unit], [orders per pass]).  Host-side planning only:
    the descriptors carry placeholder addresses that nothing reads."""
    B = len(shapes)
    descs = (_lib.ImageDesc * B)()
    for b, (h, w) in enumerate(shapes):
        # disjoint placeholder ranges, far apart, never dereferenced
        descs[b].img = (2 * b + 1) << 36
        descs[b].out = (2 * b + 2) << 36
        descs[b].H, descs[b].W = int(h), int(w)
        descs[b].radius = int(radii[b])
        descs[b].sigma_r = float(sigmas[b])
        descs[b].N = -1 if Ns is None or Ns[b] is None else int(Ns[b])
    opt = _options(strip_h=strip_h, block=block, order_chunk=order_chunk)
    blk = ctypes.c_int(0)
    rows = (ctypes.c_int * B)()
    chunk = (ctypes.c_int * B)()
    _lib.check(_lib.load().bsk_batched_shape(descs, B, float(T), ctypes.byref(opt), ctypes.byref(blk), rows, chunk))
    return blk.value, list(rows), list(chunk)


def autotune_batched(imgs: Sequence[torch.Tensor], radii: Sequence[int], sigmas: Sequence[float], T: float = 255.0,
                     Ns: Optional[Sequence[int]] = None, outs=None, path: Optional[str] = None):
    """Times launch shapes of the batched kernel on these images, per (radius bucket, order
    bucket), and stores the fastest for later batched calls; returns (block, ms)."""
    if outs is None:
        outs = [torch.empty_like(x) for x in imgs]
    descs = _batch_descs(imgs, outs, radii, sigmas, Ns)
    opt = _options()
    blk, ms = ctypes.c_int(0), ctypes.c_double(0)
    with torch.cuda.device(imgs[0].device):
        _lib.check(_lib.load().bsk_autotune_batched(descs, len(imgs), float(T), ctypes.byref(opt),
                                                    path.encode() if path else None, _stream(), ctypes.byref(blk),
                                                    ctypes.byref(ms)))
    return blk.value, ms.value


def tune_cache_load(path: str):
    _lib.check(_lib.load().bsk_tune_cache_load(path.encode()))


def tune_cache_save(path: str):
    _lib.check(_lib.load().bsk_tune_cache_save(path.encode()))


def tune_cache_clear():
    _lib.check(_lib.load().bsk_tune_cache_clear())


def autotune(img: torch.Tensor, radius: int, sigma_r: float, T: float = 255.0, N: Optional[int] = None,
             precision: str = "fp32", weight_eps: float = 0.0, kahan: bool = False, path: Optional[str] = None):
    """Times the launch shapes for this request and caches the fastest; returns (block, rows, chunk, ms)."""
    dt = torch.float64 if precision == "fp64" else torch.float32
    _check_image(img, "img", dt)
    out = torch.empty_like(img)
    H, W = img.shape
    opt = _options(N, precision, weight_eps, kahan)
    b, s, k, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
    with torch.cuda.device(img.device):
        _lib.check(_lib.load().bsk_autotune(
            ctypes.c_void_p(img.data_ptr()), H, W, int(radius), float(sigma_r), float(T),
            ctypes.c_void_p(out.data_ptr()), ctypes.byref(opt), path.encode() if path else None, _stream(),
            ctypes.byref(b), ctypes.byref(s), ctypes.byref(k), ctypes.byref(ms)))
    return b.value, s.value, k.value, ms.value


def release():
    _lib.check(_lib.load().bsk_release())


class BilateralFunction(torch.autograd.Function):
    """Autograd wrapper: forward saves (out, Q, E1, E2); backward runs the adjoint kernel.

    sigma_r is a 0-d tensor (learnable); the order N stays fixed (an integer)."""

    @staticmethod
    def forward(ctx, img, sigma_r, radius: int, T: float, N: int):
        s = float(sigma_r.detach())
        out, saved = bilateral_train(img.detach(), radius, s, T, N)
        ctx.save_for_backward(img, out, saved)
        ctx.params = (radius, s, T, N)
        ctx.sigma_dtype = sigma_r.dtype
        return out

    @staticmethod
    def backward(ctx, grad_out):
        img, out, saved = ctx.saved_tensors
        radius, s, T, N = ctx.params
        need_img, need_sigma = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gi, gs = bilateral_backward(img, grad_out.contiguous(), radius, s, T, N, out=out, saved=saved,
                                    need_img=need_img, need_sigma=need_sigma)
        if gs is not None:
            gs = gs.to(ctx.sigma_dtype)
        return gi, gs, None, None, None


class ShiftableBilateral(torch.nn.Module):
    """Bilateral filter layer with a learnable range scale sigma_r and a fixed order N."""

    def __init__(self, radius: int, sigma_r: float, T: float = 255.0, N: Optional[int] = None):
        super().__init__()
        self.radius = int(radius)
        self.T = float(T)
        self.N = int(N) if N is not None else order_for(sigma_r, T)
        self.sigma_r = torch.nn.Parameter(torch.tensor(float(sigma_r)))

    def forward(self, img: torch.Tensor) -> torch.Tensor:
        """img (H, W), or (..., H, W): the leading dimensions form one stack, filtered by one
        training-forward launch (and one adjoint launch in the backward pass)."""
        if img.dim() == 2:
            return BilateralFunction.apply(img, self.sigma_r, self.radius, self.T, self.N)
        x = img.reshape(-1, *img.shape[-2:]).contiguous()
        return BilateralFunction.apply(x, self.sigma_r, self.radius, self.T, self.N).reshape(img.shape)
