"""Parity of the HIP two-pixel-patch non-local means (Section 5 with p = 2) against the FP64
oracle, through the C ABI.

Tolerance: the FP32 bound of the box path, 1e-4 T (T = 255), max-abs over every compared pixel.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1107_4617_amd import _lib, bilateral, nlm2, order_for
from paper_1107_4617_amd import filter as F
from paper_1107_4617_amd import workloads as wl

pytestmark = pytest.mark.gpu

T = 255.0
TOL32 = 1e-4 * T


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)


def _run(f, r, s1, s2, off, N1=None, N2=None, **kw):
    x = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
    y = nlm2(x, r, s1, s2, off, T, N1=N1, N2=N2, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def _orders(s1, s2, N1, N2):
    return (order_for(s1, T) if N1 is None else N1), (order_for(s2, T) if N2 is None else N2)


# (shape, r, sigma_1, sigma_2, offset, N1, N2, kw)
CASES = [
    ((64, 80), 3, 60.0, 60.0, (0, 1), None, None, {}),            # N = 8 each: 9 groups of 5 orders
    ((50, 70), 5, 45.0, 70.0, (1, 0), None, None, {}),
    ((41, 120), 7, 30.0, 60.0, (-2, 3), None, None, {}),          # 31 first-pixel terms
    ((57, 99), 4, 60.0, 40.0, (0, -1), 9, 25, {}),                # odd first order, 13 folded second
    ((40, 90), 6, 60.0, 60.0, (3, 3), None, None, {"order_chunk": 16}),
    ((40, 90), 6, 60.0, 60.0, (3, 3), None, None, {"order_chunk": 8}),
    ((45, 77), 4, 60.0, 60.0, (0, 1), 8, 14, {}),                 # packed, 2 groups of 8 per pass, ragged last
    ((45, 77), 4, 60.0, 60.0, (1, -1), 5, 45, {"order_chunk": 16}),  # 23 folded: a term spans two passes
    ((38, 70), 5, 60.0, 60.0, (0, 1), 12, 5, {}),                 # packed, 5 groups of 3 per pass
    ((60, 600), 100, 60.0, 60.0, (0, 2), None, None, {}),         # 512-lane strips
    ((30, 1100), 300, 80.0, 80.0, (1, 1), None, None, {}),        # 1024-lane strips
    ((1, 200), 4, 60.0, 60.0, (0, 1), None, None, {}),            # one row
    ((150, 1), 4, 60.0, 60.0, (1, 0), None, None, {}),            # one column
    ((5, 6), 10, 60.0, 60.0, (4, 7), None, None, {}),             # window and offset beyond the image
    ((23, 29), 0, 60.0, 60.0, (0, 1), None, None, {}),            # r = 0: identity
    ((33, 47), 4, 60.0, 60.0, (0, 1), 0, None, {}),               # N1 = 0
    ((33, 47), 4, 60.0, 60.0, (0, 1), 8, 0, {}),                  # N2 = 0: the bilateral filter
]


@pytest.mark.parametrize("shape,r,s1,s2,off,N1,N2,kw", CASES)
def test_nlm2_matches_oracle(shape, r, s1, s2, off, N1, N2, kw):
    f = wl.rect_image(*shape, seed=31 + r)
    out = _run(f, r, s1, s2, off, N1, N2, **kw)
    n1, n2 = _orders(s1, s2, N1, N2)
    ref = oracle.nlm2(f, r, s1, n1, s2, n2, off)
    err = np.abs(out - ref)
    assert np.max(err) <= TOL32, (np.max(err), np.unravel_index(np.argmax(err), err.shape))


@pytest.mark.parametrize("r", [8, 20, 32])
@pytest.mark.parametrize("N2", [2, 8, 14, 30])   # packed 8, 3 and 2 groups per pass; unpacked
def test_nlm2_compile_time_radius_kernels(r, N2):
    """The radii with their own patch kernels (the walkers hand out weighted box sums), packed
    and unpacked, over two strips and several segments."""
    f = wl.rect_image(40, 300, seed=7 * r + N2)
    out = _run(f, r, 60.0, 60.0, (1, -1), 8, N2, strip_h=13)
    ref = oracle.nlm2(f, r, 60.0, 8, 60.0, N2, (1, -1))
    assert np.max(np.abs(out - ref)) <= TOL32


def test_nlm2_second_order_zero_matches_bilateral_path():
    """N2 = 0 is the bilateral filter: the two HIP paths agree to FP32 rounding."""
    f = wl.rect_image(70, 90, seed=4)
    x = torch.from_numpy(f).cuda()
    a = nlm2(x, 5, 30.0, 50.0, (0, 1), T, N1=30, N2=0)
    b = bilateral(x, 5, 30.0, T, N=30)
    torch.cuda.synchronize()
    assert float((a - b).abs().max()) <= TOL32


def test_nlm2_truncated():
    """weight_eps drops small binomial weights of either factor; the change of the kernel is
    bounded by the dropped mass of both factors, as for the bilateral filter's truncation."""
    f = wl.rect_image(60, 80, seed=5)
    r = 5
    out = _run(f, r, 30.0, 40.0, (0, 1), weight_eps=1e-7)
    ref, _, Q = oracle.nlm2(f, r, 30.0, 30, 40.0, 17, (0, 1), return_pq=True)
    _, d1 = oracle.trunc_terms(30, 1e-7)
    _, d2 = oracle.trunc_terms(17, 1e-7)
    b = d1 + d2
    nwin = (2 * r + 1) ** 2
    assert np.all(np.abs(out - ref) <= TOL32 + b * nwin * T / (Q - b * nwin))


def test_nlm2_deterministic_and_pitch():
    f = wl.rect_image(45, 70, seed=13)
    a = _run(f, 4, 60.0, 60.0, (1, 2))
    assert np.array_equal(a, _run(f, 4, 60.0, 60.0, (1, 2)))
    base = torch.zeros((45, 96), dtype=torch.float32, device="cuda")
    base[:, :70] = torch.from_numpy(f).cuda()
    outp = torch.full((45, 128), -7.0, dtype=torch.float32, device="cuda")
    o = F._options()
    o.pitch_in, o.pitch_out = 96, 128
    _lib.check(_lib.load().bilateral_shiftable_nlm2(ctypes.c_void_p(base.data_ptr()), 45, 70, 4, 60.0, 60.0, -1,
                                                    -1, 1, 2, T, ctypes.c_void_p(outp.data_ptr()), ctypes.byref(o),
                                                    F._stream()))
    torch.cuda.synchronize()
    got = outp.cpu().numpy()
    assert np.max(np.abs(got[:, :70] - a)) <= 1e-3
    assert np.all(got[:, 70:] == -7.0)


def test_nlm2_rect4096_sampled():
    """4096x4096 rect image, r = 20, sigma_1 = sigma_2 = 60 (N = 8 each), offset (0, 1), in the
    default launch shape; the oracle at sampled pixels, strip edges and borders included."""
    f = wl.rect_image(4096, 4096, seed=2)
    out = _run(f, 20, 60.0, 60.0, (0, 1))
    rng = np.random.default_rng(22)
    idx = np.unique(np.concatenate([rng.integers(0, 4096 * 4096, 2000),
                                    4095 * 4096 + rng.integers(0, 4096, 200),
                                    rng.integers(0, 4096, 200) * 4096 + 4095,
                                    rng.integers(0, 4096, 200) * 4096 + 215]))
    ref = oracle.nlm2_at(f, idx, 20, 60.0, 8, 60.0, 8, (0, 1))
    assert np.max(np.abs(out.ravel()[idx] - ref)) <= TOL32
