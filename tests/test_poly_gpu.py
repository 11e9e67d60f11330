"""Parity of the HIP polynomial-range-kernel path (Section 3's p_N in the scaling of eq. (5))
against the FP64 oracle, through the C ABI.

Tolerances: FP32 1e-4 T and FP64 1e-9 T (T = 255), max-abs over every compared pixel.  With
truncation the bound of the dropped Chebyshev coefficients is added per pixel:
|d out| <= b |B| T / (Q - b |B|) with b the plan's bound, |B| the window size and Q the
oracle's normaliser (the normalised kernel moves by at most b on [-1, 1], and T / 2 maps
the normalised values back).
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1107_4617_amd import _lib, bilateral, poly_order_for, poly_plan_info
from paper_1107_4617_amd import filter as F
from paper_1107_4617_amd import workloads as wl

pytestmark = pytest.mark.gpu

T = 255.0
TOL32 = 1e-4 * T
TOL64 = 1e-9 * T


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)


def _run(f, r, sigma_r, N=None, dtype=np.float32, **kw):
    x = torch.from_numpy(np.ascontiguousarray(f, dtype=dtype)).cuda()
    prec = "fp64" if dtype == np.float64 else "fp32"
    y = bilateral(x, r, sigma_r, T, N=N, precision=prec, range_kernel="poly", **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


# (shape, r, sigma_r, N, block); N None is N_p(sigma_r, T)
CASES = [
    ((64, 80), 3, 30.0, None, 0),        # N = 37: 75 coefficients, 3 passes of 16 pairs
    ((50, 70), 5, 60.0, None, 0),        # N = 10: one pass
    ((41, 300), 7, 15.0, None, 0),       # N = 145: 291 coefficients, 10 passes
    ((90, 61), 6, 40.0, 21, 0),          # odd order above N_p = 21
    ((57, 299), 20, 30.0, 60, 0),        # order above N_p
    ((33, 47), 4, 200.0, 1, 0),          # N = N_p = 1: a quadratic kernel
    ((180, 400), 100, 80.0, None, 0),    # 512-lane strips
    ((40, 520), 12, 30.0, None, 512),
    ((37, 1100), 300, 50.0, None, 0),    # 1024-lane strips
    ((1, 333), 4, 30.0, None, 0),        # one row
    ((301, 1), 4, 30.0, None, 0),        # one column
    ((5, 6), 10, 30.0, None, 0),         # window larger than the image
    ((23, 29), 0, 30.0, None, 0),        # r = 0: identity
    ((44, 52), 5, 30.0, 0, 0),           # N = 0: the box mean
]


@pytest.mark.parametrize("shape,r,sigma_r,N,block", CASES)
def test_poly_matches_oracle_fp32(shape, r, sigma_r, N, block):
    f = wl.rect_image(*shape, seed=11 + r)
    out = _run(f, r, sigma_r, N, block=block)
    Nn = poly_order_for(sigma_r, T) if N is None else N
    ref = oracle.bilateral_poly(f, r, sigma_r, Nn)
    err = np.abs(out - ref)
    assert np.max(err) <= TOL32, (np.max(err), np.unravel_index(np.argmax(err), err.shape))


@pytest.mark.parametrize("r", [3, 5, 8, 10, 16, 20, 25, 32])
@pytest.mark.parametrize("sigma_r,eps", [(30.0, 0.0),    # 75 coefficients: three passes of 16 pairs
                                         (60.0, 0.0),    # N = 10: one pass
                                         (30.0, 1e-7)])  # 26 coefficients: one pass
def test_poly_compile_time_radius_kernels(r, sigma_r, eps):
    """The radii with their own polynomial kernels (walkers hand out box sums), over two
    strips and several segments, with one pass and with several."""
    f = wl.rect_image(60, 300, seed=7 * r + int(sigma_r), n_rect=8)
    out = _run(f, r, sigma_r, weight_eps=eps, strip_h=19)
    Nn = poly_order_for(sigma_r, T)
    ref, _, Q = oracle.bilateral_poly(f, r, sigma_r, Nn, return_pq=True)
    bound = 0.0
    if eps > 0:
        # the truncated expansion's own bound, as in test_poly_truncated_within_bound
        _, b = poly_plan_info(sigma_r, T, eps=eps)
        nwin = (2 * r + 1) ** 2
        bound = b * nwin * T / (Q - b * nwin)
    assert np.all(np.abs(out - ref) <= TOL32 + bound)


@pytest.mark.parametrize("shape,r,sigma_r,N", [((64, 80), 3, 30.0, None), ((41, 300), 7, 15.0, None),
                                               ((90, 61), 6, 40.0, 21), ((37, 700), 200, 50.0, None),
                                               ((44, 52), 5, 30.0, 0)])
def test_poly_matches_oracle_fp64(shape, r, sigma_r, N):
    f = wl.smooth_image(*shape, seed=3).astype(np.float64)
    out = _run(f, r, sigma_r, N, dtype=np.float64)
    Nn = poly_order_for(sigma_r, T) if N is None else N
    ref = oracle.bilateral_poly(f, r, sigma_r, Nn)
    assert np.max(np.abs(out - ref)) <= TOL64


@pytest.mark.parametrize("sigma_r,eps", [(30.0, 1e-7), (15.0, 1e-7), (30.0, 1e-5)])
def test_poly_truncated_within_bound(sigma_r, eps):
    f = wl.rect_image(70, 90, seed=4)
    r = 6
    out = _run(f, r, sigma_r, weight_eps=eps)
    N = poly_order_for(sigma_r, T)
    ref, _, Q = oracle.bilateral_poly(f, r, sigma_r, N, return_pq=True)
    K, b = poly_plan_info(sigma_r, T, eps=eps)
    assert K < 2 * N + 1 and 0 < b <= eps
    nwin = (2 * r + 1) ** 2
    bound = b * nwin * T / (Q - b * nwin)
    assert np.all(np.abs(out - ref) <= TOL32 + bound)


@pytest.mark.parametrize("kc", [8, 16, 24])
def test_poly_every_pass_size(kc):
    """38 channel pairs (N = 37) in passes of 8, 16 or 24 pairs (5, 3 or 2 passes) at a radius
    with its own kernels."""
    f = wl.rect_image(60, 200, seed=6)
    a = _run(f, 5, 30.0, order_chunk=kc)
    ref = oracle.bilateral_poly(f, 5, 30.0, 37)
    assert np.max(np.abs(a - ref)) <= TOL32


def test_poly_24_pair_pass_needs_its_radii():
    """The 24-pair pass exists at the polynomial kernel's compile-time radii only."""
    f = wl.rect_image(30, 200, seed=6)
    with pytest.raises(_lib.BskError, match="EINVAL"):
        _run(f, 6, 30.0, order_chunk=24)


def test_poly_offset_data():
    """Values far from zero: the workgroup midrange recentres them (the span is still T)."""
    f = wl.rect_image(48, 300, seed=9).astype(np.float64) + 1000.0
    out = _run(f.astype(np.float32), 5, 30.0)
    ref = oracle.bilateral_poly(f.astype(np.float32), 5, 30.0, 37)
    assert np.max(np.abs(out - ref)) <= TOL32


def test_poly_deterministic():
    f = wl.rect_image(120, 330, seed=8)
    assert np.array_equal(_run(f, 5, 30.0), _run(f, 5, 30.0))


def test_poly_pitch():
    f = wl.rect_image(45, 70, seed=13)
    base = torch.zeros((45, 96), dtype=torch.float32, device="cuda")
    base[:, :70] = torch.from_numpy(f).cuda()
    outp = torch.full((45, 128), -7.0, dtype=torch.float32, device="cuda")
    o = F._options(range_kernel="poly")
    o.pitch_in, o.pitch_out = 96, 128
    _lib.check(_lib.load().bilateral_shiftable_ex(ctypes.c_void_p(base.data_ptr()), 45, 70, 4, 30.0, T,
                                                  ctypes.c_void_p(outp.data_ptr()), ctypes.byref(o), F._stream()))
    torch.cuda.synchronize()
    got = outp.cpu().numpy()
    ref = oracle.bilateral_poly(f, 4, 30.0, 37)
    assert np.max(np.abs(got[:, :70] - ref)) <= TOL32
    assert np.all(got[:, 70:] == -7.0)


@pytest.mark.parametrize("eps", [0.0, 1e-7])
def test_poly_rect4096_sampled(eps):
    """The 4096x4096 rect image, r = 20, sigma_r = 30 (N_p = 37), in the default launch shape;
    the oracle at sampled pixels (random, borders, strip and segment edges)."""
    f = wl.rect_image(4096, 4096, seed=2)
    out = _run(f, 20, 30.0, weight_eps=eps)
    rng = np.random.default_rng(21)
    idx = np.unique(np.concatenate([rng.integers(0, 4096 * 4096, 3000),
                                    rng.integers(0, 4096, 300),
                                    4095 * 4096 + rng.integers(0, 4096, 300),
                                    rng.integers(0, 4096, 300) * 4096 + 215,
                                    rng.integers(0, 4096, 300) * 4096 + 216]))
    ref = oracle.bilateral_poly_at(f, idx, 20, 30.0, 37)
    tol = TOL32
    if eps > 0:
        _, b = poly_plan_info(30.0, T, eps=eps)
        tol += b * 41 * 41 * T   # Q >= 1 (the centre pixel's own weight is 1)
    assert np.max(np.abs(out.ravel()[idx] - ref)) <= tol


def test_coefficient_table_survives_batched_multipass_calls():
    """The polynomial kernel keeps its coefficient table in a workspace buffer of the stream
    and re-uploads it only when the plan or the buffer changes.  Batched calls with a
    multi-pass image (their accumulator planes live in a workspace buffer of the same stream)
    interleaved with two identical polynomial calls must leave it intact (regression: the two
    once shared a buffer, and the second polynomial call read accumulator data as its
    recurrence rows)."""
    from paper_1107_4617_amd import bilateral_batched
    f = wl.rect_image(64, 80, seed=7)
    x = torch.from_numpy(f).cuda()
    bimg = [torch.from_numpy(wl.gradient_image(300, 257, 9)).cuda()]
    # sigma_r = 12: N_0 = 183, 92 folded orders, several 16-order passes
    bilateral_batched(bimg, [5], [12.0], T)
    y1 = bilateral(x, 4, 30.0, T, range_kernel="poly").clone()
    bilateral_batched(bimg, [5], [12.0], T)
    y2 = bilateral(x, 4, 30.0, T, range_kernel="poly")
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    ref = oracle.bilateral_poly(f, 4, 30.0, poly_order_for(30.0, T))
    assert np.max(np.abs(y2.cpu().numpy() - ref)) <= TOL32
