"""Parity of the HIP spatial-kernel path (Algorithm 2 with M = (Ns+1)^2 spatial basis
functions, and Algorithm 1 as its N = 0 case) against the FP64 oracle, through the C ABI.

Tolerance: the FP32 bound of the box path, 1e-4 T (T = 255), max-abs over every compared
pixel.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1107_4617_amd import _lib, bilateral, spatial_filter, spatial_sigma_for
from paper_1107_4617_amd import filter as F
from paper_1107_4617_amd import workloads as wl

pytestmark = pytest.mark.gpu

T = 255.0
TOL32 = 1e-4 * T


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)


def _run(f, r, sigma_r, N, sigma_s, Ns, **kw):
    x = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
    y = bilateral(x, r, sigma_r, T, N=N, spatial_sigma=sigma_s, spatial_N=Ns, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


# (shape, r, N, sigma_r, Ns, sigma_s, block)
CASES = [
    ((64, 80), 3, 30, 30.0, 2, 2.25, 0),        # q_2 spatial kernel, N = 30 range kernel
    ((50, 70), 5, 4, 100.0, 2, spatial_sigma_for(5, 2), 0),   # the paper's M x N = 3^2 x 5
    ((41, 300), 7, 30, 30.0, 1, 6.0, 0),        # odd order: no zero frequency
    ((90, 61), 6, 17, 40.0, 3, 2.6, 0),
    ((33, 47), 4, 30, 30.0, 4, 1.5, 0),
    ((70, 90), 9, 7, 70.0, 5, 3.2, 0),
    ((37, 45), 8, 2, 120.0, 6, 2.6, 0),         # three frequencies with the zero one
    ((57, 299), 20, 43, 25.0, 2, 9.0, 0),       # multi-pass (22 orders, 4 per pass)
    ((180, 400), 150, 8, 80.0, 2, 70.0, 0),     # 512-lane strips
    ((40, 520), 12, 30, 30.0, 2, 5.0, 512),
    ((1, 333), 4, 30, 30.0, 2, 2.0, 0),         # one row
    ((301, 1), 4, 30, 30.0, 2, 2.0, 0),         # one column
    ((5, 6), 10, 30, 30.0, 3, 4.0, 0),          # window larger than the image
    ((23, 29), 0, 30, 30.0, 2, 1.0, 0),         # r = 0: identity
]


@pytest.mark.parametrize("shape,r,N,sigma_r,Ns,sigma_s,block", CASES)
def test_spatial_matches_oracle(shape, r, N, sigma_r, Ns, sigma_s, block):
    f = wl.rect_image(*shape, seed=3 + r + Ns)
    out = _run(f, r, sigma_r, N, sigma_s, Ns, block=block)
    ref = oracle.bilateral_sp(f, r, sigma_r, N, sigma_s, Ns)
    err = np.abs(out - ref)
    assert np.max(err) <= TOL32, (np.max(err), np.unravel_index(np.argmax(err), err.shape))


@pytest.mark.parametrize("r", [3, 5, 8, 10, 16, 20, 25, 32])
@pytest.mark.parametrize("N,sigma_r", [(30, 30.0),   # 16 orders: four passes of 4
                                       (0, 1.0)])    # Algorithm 1: one order, the small pass
def test_q2_compile_time_radius_kernels(r, N, sigma_r):
    """The q_2 spatial kernel at the radii with compile-time-radius kernels (walkers hand out
    box sums of all three basis rows), over two strips and several segments."""
    f = wl.rect_image(60, 300, seed=5 * r + N, n_rect=8)
    s_s = spatial_sigma_for(r, 2)
    out = _run(f, r, sigma_r, N, s_s, 2, strip_h=23)
    ref = oracle.bilateral_sp(f, r, sigma_r, N, s_s, 2)
    assert np.max(np.abs(out - ref)) <= TOL32


@pytest.mark.parametrize("r,sigma_s,Ns", [(3, 1.5, 2), (10, 4.0, 4), (6, 3.0, 1)])
def test_algorithm1_linear_filter(r, sigma_s, Ns):
    """Algorithm 1 (the range kernel is 1): the normalised separable linear filter."""
    f = wl.smooth_image(96, 130, seed=1)
    x = torch.from_numpy(f).cuda()
    out = spatial_filter(x, r, sigma_s, Ns).cpu().numpy().astype(np.float64)
    ref = oracle.bilateral_sp(f, r, 1.0, 0, sigma_s, Ns)
    assert np.max(np.abs(out - ref)) <= TOL32


def test_order_zero_is_the_box_path():
    f = wl.rect_image(70, 90, seed=4)
    box = _run(f, 6, 30.0, 30, None, None)
    sp0 = _run(f, 6, 30.0, 30, 3.0, 0)
    assert np.array_equal(box, sp0)


def test_automatic_spatial_order():
    """spatial_N = None picks the smallest order unimodal on the window, ceil((2r/(pi s))^2)."""
    f = wl.rect_image(60, 77, seed=6)
    r, sigma_s = 7, 3.5
    Ns = max(1, math.ceil((2 * r / (math.pi * sigma_s)) ** 2))
    assert Ns == 2
    out = _run(f, r, 30.0, 30, sigma_s, None)
    ref = oracle.bilateral_sp(f, r, 30.0, 30, sigma_s, Ns)
    assert np.max(np.abs(out - ref)) <= TOL32


def test_spatial_deterministic():
    f = wl.rect_image(120, 330, seed=8)
    a = _run(f, 5, 30.0, 30, 2.25, 2)
    b = _run(f, 5, 30.0, 30, 2.25, 2)
    assert np.array_equal(a, b)


def test_spatial_large_image_sampled():
    """2048x2048 rect image, r=5, the q_2 kernel of the paper's timed instance (T_s = 5),
    N = 30, in the default launch shape; oracle at sampled pixels (random, borders,
    strip edges), where the absolute phases nu_j x and nu_j y are largest."""
    f = wl.rect_image(2048, 2048, seed=2)
    sigma_s = spatial_sigma_for(5, 2)
    out = _run(f, 5, 30.0, 30, sigma_s, 2)
    rng = np.random.default_rng(12)
    idx = np.unique(np.concatenate([rng.integers(0, 2048 * 2048, 3000),
                                    2047 * 2048 + rng.integers(0, 2048, 200),
                                    rng.integers(0, 2048, 200) * 2048 + 2047]))
    ref = oracle.bilateral_sp_at(f, idx, 5, 30.0, 30, sigma_s, 2)
    assert np.max(np.abs(out.ravel()[idx] - ref)) <= TOL32


def _rect4096_samples(seed):
    rng = np.random.default_rng(seed)
    n = 4096
    return np.unique(np.concatenate([rng.integers(0, n * n, 2000),          # interior
                                     (n - 1) * n + rng.integers(0, n, 150),  # last row
                                     rng.integers(0, n, 150) * n + n - 1,    # last column
                                     rng.integers(0, n, 150) * n + 215,      # strip edges (216 columns)
                                     rng.integers(0, n, 150) * n + 216]))


def test_spatial_rect4096_sampled():
    """The separable q_2 kernel (M = 9) at the workload bench.py times: 4096x4096 rect, r = 20,
    sigma_r = 30, N = 30, sigma_s = spatial_sigma_for(20, 2), in the default launch shape."""
    f = wl.rect_image(4096, 4096, seed=2)
    sigma_s = spatial_sigma_for(20, 2)
    out = _run(f, 20, 30.0, 30, sigma_s, 2)
    idx = _rect4096_samples(31)
    ref = oracle.bilateral_sp_at(f, idx, 20, 30.0, 30, sigma_s, 2)
    assert np.max(np.abs(out.ravel()[idx] - ref)) <= TOL32


def test_algorithm1_rect4096_sampled():
    """Algorithm 1 with the same q_2 kernel on the same 4096x4096 image, as bench.py times it."""
    f = wl.rect_image(4096, 4096, seed=2)
    sigma_s = spatial_sigma_for(20, 2)
    x = torch.from_numpy(f).cuda()
    out = spatial_filter(x, 20, sigma_s, 2).cpu().numpy().astype(np.float64)
    idx = _rect4096_samples(32)
    ref = oracle.bilateral_sp_at(f, idx, 20, 1.0, 0, sigma_s, 2)
    assert np.max(np.abs(out.ravel()[idx] - ref)) <= TOL32


def test_spatial_pitch():
    """Row pitches larger than the width: the spatial path reads and writes through them."""
    f = wl.rect_image(45, 70, seed=13)
    base = torch.zeros((45, 96), dtype=torch.float32, device="cuda")
    base[:, :70] = torch.from_numpy(f).cuda()
    outp = torch.full((45, 128), -7.0, dtype=torch.float32, device="cuda")
    o = F._options(30, spatial_sigma=2.5, spatial_N=2)
    o.pitch_in, o.pitch_out = 96, 128
    _lib.check(_lib.load().bilateral_shiftable_ex(ctypes.c_void_p(base.data_ptr()), 45, 70, 4, 30.0, T,
                                                  ctypes.c_void_p(outp.data_ptr()), ctypes.byref(o), F._stream()))
    torch.cuda.synchronize()
    got = outp.cpu().numpy()
    ref = oracle.bilateral_sp(f, 4, 30.0, 30, 2.5, 2)
    assert np.max(np.abs(got[:, :70] - ref)) <= TOL32
    assert np.all(got[:, 70:] == -7.0)
