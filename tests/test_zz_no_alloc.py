"""The allocation-free forward (bilateral_shiftable_noalloc) against bilateral_shiftable_ex,
through the C ABI: the same kernels and launch shapes, with the multi-pass accumulators in
the library's fixed scratch array instead of the per-stream workspace, so the outputs must
agree bit for bit.  Two calls in a row, the second on a smaller image, check that nothing
left in the shared array by the first call leaks into the second."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1107_4617_amd import _lib
from paper_1107_4617_amd import workloads as wl

pytestmark = pytest.mark.gpu
T = 255.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)


def _opt(N, precision=_lib.BSK_FP32, eps=0.0, kahan=0):
    o = _lib.Options()
    o.order_mode, o.N = 1, int(N)
    o.precision = precision
    o.weight_eps = eps
    o.kahan = kahan
    return o


def _call(name, x, r, sigma, opt):
    lib = _lib.load()
    y = torch.full_like(x, float("nan"))
    H, W = x.shape
    st = getattr(lib, name)(ctypes.c_void_p(x.data_ptr()), H, W, r, float(sigma), T,
                            ctypes.c_void_p(y.data_ptr()), ctypes.byref(opt),
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st)
    torch.cuda.synchronize()
    return y


# (H, W, radius, sigma_r, N, precision, eps, kahan): multi-pass requests (several
# passes keep partial accumulators in the scratch array), then a smaller one
CASES = [
    [(300, 517, 9, 15.0, 117, _lib.BSK_FP32, 0.0, 0), (97, 130, 4, 20.0, 66, _lib.BSK_FP32, 0.0, 0)],
    [(256, 300, 6, 25.0, 43, _lib.BSK_I16, 1e-7, 1), (64, 90, 3, 12.0, 183, _lib.BSK_BF16, 1e-7, 0)],
    [(180, 211, 5, 25.0, 43, _lib.BSK_FP64, 0.0, 0), (40, 33, 2, 30.0, 30, _lib.BSK_FP64, 0.0, 0)],
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_matches_ex_on_two_calls(case):
    for (H, W, r, sigma, N, prec, eps, kahan) in CASES[case]:
        print(f"noalloc case {case}: {H}x{W} r={r} sigma={sigma} N={N} prec={prec}", flush=True)
        f = wl.rect_image(H, W, seed=H + W)
        dt = torch.float64 if prec == _lib.BSK_FP64 else torch.float32
        x = torch.from_numpy(f).to(device="cuda", dtype=dt)
        o = _opt(N, prec, eps, kahan)
        a = _call("bilateral_shiftable_noalloc", x, r, sigma, o)
        b = _call("bilateral_shiftable_ex", x, r, sigma, o)
        assert torch.equal(a, b)
        if prec in (_lib.BSK_FP32, _lib.BSK_FP64) and eps == 0.0:
            ref = oracle.bilateral(f, r, sigma, N)
            tol = 1e-9 * T if prec == _lib.BSK_FP64 else 1e-4 * T
            assert np.max(np.abs(a.cpu().numpy() - ref)) <= tol


def test_noalloc_rejects_requests_beyond_its_scratch():
    """Two FP32 planes of 4096 x 4096 fill the 128 MiB array; one more row is refused before
    anything is queued, and the output is left untouched."""
    lib = _lib.load()
    H, W = 4097, 4096
    x = torch.zeros((H, W), device="cuda")
    y = torch.full_like(x, 7.0)
    o = _opt(117)
    st = lib.bilateral_shiftable_noalloc(ctypes.c_void_p(x.data_ptr()), H, W, 5, 15.0, T,
                                         ctypes.c_void_p(y.data_ptr()), ctypes.byref(o), None)
    assert st == _lib.BSK_ENOMEM
    assert b"scratch" in lib.bsk_last_error()
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    o.spatial_N, o.spatial_sigma = 2, 3.0
    st = lib.bilateral_shiftable_noalloc(ctypes.c_void_p(x.data_ptr()), 64, 64, 5, 15.0, T,
                                         ctypes.c_void_p(y.data_ptr()), ctypes.byref(o), None)
    assert st == _lib.BSK_EUNSUPPORTED
