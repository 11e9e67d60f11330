"""Host-side tests of libbsk (no GPU needed): exports, planning, argument validation."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1107_4617_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _header_functions():
    src = open(os.path.join(ROOT, "include", "bsk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol(lib):
    names = _header_functions()
    assert "bilateral_shiftable" in names and "bilateral_shiftable_batched" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(_lib.EXPORTS)


def test_version(lib):
    assert b"gfx950" in lib.bsk_version()


@pytest.mark.parametrize("sigma,expect", [(30.0, 30), (25.0, 43), (15.0, 118), (10.0, 264), (60.0, 8)])
def test_order_for(lib, sigma, expect):
    assert lib.bsk_order_for(sigma, 255.0) == expect


def test_order_for_rejects_bad_input(lib):
    assert lib.bsk_order_for(0.0, 255.0) == -1
    assert lib.bsk_order_for(float("nan"), 255.0) == -1
    assert lib.bsk_order_for(30.0, -1.0) == -1


@pytest.mark.parametrize("N,eps", [(0, 0.0), (1, 0.0), (2, 0.0), (30, 0.0), (30, 1e-7), (117, 1e-7), (264, 1e-7),
                                   (43, 1e-4), (117, 0.0), (511, 0.0)])
def test_plan_counts_match_exact_binomials(lib, N, eps):
    """Folded orders kept and dropped mass against exact integer binomials."""
    K = ctypes.c_int(0)
    d = ctypes.c_double(0.0)
    assert lib.bsk_plan_info(N, eps, ctypes.byref(K), ctypes.byref(d)) == 0
    w = [math.comb(N, n) / 2 ** N for n in range(N + 1)]
    kept = [n for n in range(N + 1) if not (eps > 0 and w[n] < eps)]
    folded = len([n for n in kept if 2 * n <= N])   # one folded order per pair (and the centre)
    assert K.value == folded
    drop = math.fsum(w[n] for n in range(N + 1) if eps > 0 and w[n] < eps)
    assert abs(d.value - drop) <= 1e-12 * max(drop, 1e-300) + 1e-300
    assert abs(lib.bsk_truncation_error(N, eps) - drop) <= 1e-12 * max(drop, 1e-300) + 1e-300


def test_truncation_table():
    from paper_1107_4617_amd import plan_info
    for N, K, eps in [(117, 28, 1.283e-7), (30, 14, 5.8e-8), (264, 42, 2.6e-7)]:
        k, d = plan_info(N, 1e-7)
        assert k == K and abs(d - eps) / eps < 0.01


def _call_ex(lib, img=1, H=8, W=8, r=2, s=30.0, T=255.0, out=2, opt=None):
    o = opt if opt is not None else _lib.Options()
    return lib.bilateral_shiftable_ex(ctypes.c_void_p(img), H, W, r, s, T, ctypes.c_void_p(out),
                                      ctypes.byref(o), None)


def test_argument_errors(lib):
    E = _lib.BSK_EINVAL
    big = 1 << 40
    assert _call_ex(lib, img=0) == E
    assert _call_ex(lib, out=0) == E
    assert _call_ex(lib, img=big, out=big) == E        # img == out
    assert _call_ex(lib, img=big, out=big + 8) == E    # overlapping rows
    assert b"overlap" in lib.bsk_last_error()
    assert _call_ex(lib, H=0) == E
    assert _call_ex(lib, W=-3) == E
    assert _call_ex(lib, r=-1) == E
    assert _call_ex(lib, s=0.0) == E
    assert _call_ex(lib, s=float("nan")) == E
    assert _call_ex(lib, s=float("inf")) == E
    assert _call_ex(lib, T=0.0) == E
    assert b"T must be" in lib.bsk_last_error()
    o = _lib.Options()
    o.order_mode = 1
    o.N = -2
    assert _call_ex(lib, opt=o) == E
    o = _lib.Options()
    o.precision = 9
    assert _call_ex(lib, opt=o) == E
    o = _lib.Options()
    o.weight_eps = -1.0
    assert _call_ex(lib, opt=o) == E
    o = _lib.Options()
    o.pitch_in = 3
    assert _call_ex(lib, opt=o) == E
    o = _lib.Options()
    o.block = 300
    assert _call_ex(lib, opt=o) == E
    o = _lib.Options()
    o.order_mode = 2
    assert _call_ex(lib, opt=o) == E


def test_range_and_unsupported_errors(lib):
    o = _lib.Options()
    o.order_mode = 1
    o.N = 2000          # 1001 folded orders > BSK_MAX_ORDERS
    assert _call_ex(lib, img=1 << 40, out=1 << 41, opt=o) == _lib.BSK_ERANGE
    o.weight_eps = 1e-7  # truncation brings it back under the limit
    K = ctypes.c_int(0)
    lib.bsk_plan_info(2000, 1e-7, ctypes.byref(K), None)
    assert K.value <= 256
    assert _call_ex(lib, img=1 << 40, out=1 << 41, H=2000, W=2000, r=600) == _lib.BSK_EUNSUPPORTED
    o = _lib.Options()
    o.block = 256
    assert _call_ex(lib, img=1 << 40, out=1 << 41, H=300, W=300, r=200, opt=o) == _lib.BSK_EUNSUPPORTED


def test_train_and_backward_validation(lib):
    o = _lib.Options()
    vp = ctypes.c_void_p
    assert lib.bilateral_shiftable_train(None, 8, 8, 2, 30.0, 255.0, ctypes.byref(o), vp(1), vp(2), None) == -1
    o.precision = _lib.BSK_BF16
    assert lib.bilateral_shiftable_train(vp(1 << 40), 8, 8, 2, 30.0, 255.0, ctypes.byref(o), vp(1 << 41),
                                         vp(1 << 42), None) == _lib.BSK_EUNSUPPORTED
    o = _lib.Options()
    # out given without saved
    assert lib.bilateral_shiftable_backward(vp(1 << 40), vp(1 << 41), vp(1 << 42), None, 8, 8, 2, 30.0, 255.0,
                                            ctypes.byref(o), vp(1 << 43), None, None) == -1
    # nothing requested: no work, success
    assert lib.bilateral_shiftable_backward(vp(1 << 40), vp(1 << 41), None, None, 8, 8, 2, 30.0, 255.0,
                                            ctypes.byref(o), None, None, None) == 0


def test_batched_validation(lib):
    d = (_lib.ImageDesc * 2)()
    for b in range(2):
        d[b].img = (1 << 40) + b * (1 << 30)
        d[b].out = (1 << 41) + b * (1 << 30)
        d[b].H, d[b].W, d[b].radius, d[b].sigma_r, d[b].N = 16, 16, 2, 30.0, -1
    o = _lib.Options()
    d[1].sigma_r = -1.0
    assert lib.bilateral_shiftable_batched(d, 2, 255.0, ctypes.byref(o), None) == -1
    d[1].sigma_r = 30.0
    d[0].out = d[0].img
    assert lib.bilateral_shiftable_batched(d, 2, 255.0, ctypes.byref(o), None) == -1
    assert lib.bilateral_shiftable_batched(d, 0, 255.0, ctypes.byref(o), None) == -1
    assert lib.bilateral_shiftable_batched_graph(d, 2, 255.0, ctypes.byref(o), 7, None) == -1  # default stream


def test_workspace_limit_reports_enomem(lib):
    """A multi-pass request (N = 117: 59 folded orders, several passes) keeps two planes of
    partial accumulators in a library workspace.  Under a workspace cap smaller than that
    the call fails with BSK_ENOMEM before anything is queued (so fake device pointers are
    never touched), and lifting the cap restores the default."""
    big, big2 = 1 << 40, 1 << 41
    o = _lib.Options()
    o.order_mode, o.N = 1, 117
    try:
        assert lib.bsk_set_workspace_limit(1 << 20) == _lib.BSK_OK
        assert _call_ex(lib, img=big, out=big2, H=1024, W=1024, r=5, s=15.0, opt=o) == _lib.BSK_ENOMEM
        assert b"limit" in lib.bsk_last_error()
        # the training forward (five planes) and the batched path are capped alike
        o32 = _lib.Options()
        o32.order_mode, o32.N = 1, 117
        out = ctypes.c_void_p(big2)
        saved = ctypes.c_void_p(big2 + (1 << 32))
        assert lib.bilateral_shiftable_train(ctypes.c_void_p(big), 1024, 1024, 5, 15.0, 255.0,
                                             ctypes.byref(o32), out, saved, None) == _lib.BSK_ENOMEM
        d = (_lib.ImageDesc * 1)()
        d[0].img, d[0].out = big, big2
        d[0].H, d[0].W, d[0].radius, d[0].sigma_r, d[0].N = 1024, 1024, 5, 15.0, 117
        assert lib.bilateral_shiftable_batched(d, 1, 255.0, ctypes.byref(_lib.Options()), None) == _lib.BSK_ENOMEM
        assert lib.bsk_set_workspace_limit(-1) == _lib.BSK_EINVAL
    finally:
        assert lib.bsk_set_workspace_limit(0) == _lib.BSK_OK


def _no_device():
    import torch
    return torch.cuda.device_count() == 0


@pytest.mark.skipif(not _no_device(), reason="checks the no-device error path; a GPU is present")
def test_no_device_reports_hip_error(lib):
    assert _call_ex(lib, img=1 << 40, out=1 << 41) == _lib.BSK_EHIP
    assert len(lib.bsk_last_error()) > 0


def test_python_layer_rejects_cpu_tensors():
    import torch
    from paper_1107_4617_amd import bilateral
    with pytest.raises(TypeError):
        bilateral(torch.zeros(4, 4), 1, 30.0)


def test_spatial_kernel_errors(lib):
    """Separable spatial kernel options: invalid values, orders above 6, and the entry points
    and shapes that do not run it."""
    big, big2 = 1 << 40, 1 << 41

    def opt(Ns, sigma, **kw):
        o = _lib.Options()
        o.spatial_N = Ns
        o.spatial_sigma = sigma
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    assert _call_ex(lib, img=big, out=big2, opt=opt(2, 0.0)) == _lib.BSK_EINVAL
    assert _call_ex(lib, img=big, out=big2, opt=opt(2, float("nan"))) == _lib.BSK_EINVAL
    assert _call_ex(lib, img=big, out=big2, opt=opt(-2, 2.0)) == _lib.BSK_EINVAL
    assert _call_ex(lib, img=big, out=big2, opt=opt(7, 2.0)) == _lib.BSK_ERANGE
    # automatic order: ceil((2 r / (pi sigma_s))^2) = 163 > 6
    assert _call_ex(lib, img=big, out=big2, r=10, opt=opt(-1, 0.5)) == _lib.BSK_ERANGE
    assert b"spatial order" in lib.bsk_last_error()
    assert _call_ex(lib, img=big, out=big2, opt=opt(2, 2.0, precision=_lib.BSK_BF16)) == _lib.BSK_EUNSUPPORTED
    assert _call_ex(lib, img=big, out=big2, opt=opt(2, 2.0, kahan=1)) == _lib.BSK_EUNSUPPORTED
    assert _call_ex(lib, img=big, out=big2, opt=opt(2, 2.0, precision=3)) == _lib.BSK_EUNSUPPORTED
    assert _call_ex(lib, img=big, out=big2, opt=opt(2, 2.0, block=1024)) == _lib.BSK_EUNSUPPORTED
    # three frequencies need 256-lane strips: radius 200 leaves none
    assert _call_ex(lib, img=big, out=big2, H=500, W=500, r=200, opt=opt(5, 90.0)) == _lib.BSK_EUNSUPPORTED
    assert _call_ex(lib, img=big, out=big2, opt=opt(2, 2.0, order_chunk=8)) == _lib.BSK_EINVAL
    vp = ctypes.c_void_p
    o = opt(2, 2.0)
    assert lib.bilateral_shiftable_train(vp(big), 8, 8, 2, 30.0, 255.0, ctypes.byref(o), vp(big2), vp(1 << 42),
                                         None) == _lib.BSK_EUNSUPPORTED
    assert lib.bilateral_shiftable_backward(vp(big), vp(big2), None, None, 8, 8, 2, 30.0, 255.0, ctypes.byref(o),
                                            vp(1 << 43), None, None) == _lib.BSK_EUNSUPPORTED
    d = (_lib.ImageDesc * 1)()
    d[0].img, d[0].out, d[0].H, d[0].W, d[0].radius, d[0].sigma_r, d[0].N = big, big2, 8, 8, 2, 30.0, -1
    assert lib.bilateral_shiftable_batched(d, 1, 255.0, ctypes.byref(o), None) == _lib.BSK_EUNSUPPORTED


# ------------------------------------------------ polynomial range kernel ----
@pytest.mark.parametrize("sigma,expect", [(30.0, 37), (60.0, 10), (15.0, 145), (255.0, 1)])
def test_poly_order_for(lib, sigma, expect):
    assert lib.bsk_poly_order_for(sigma, 255.0) == expect
    assert lib.bsk_poly_order_for(0.0, 255.0) == -1


def _cheb_coef_max(N, sigma, T, grid=257):
    """max over centres c in [-1, 1] of |d_k(c)|, the Chebyshev coefficients of
    (1 - (x - c)^2 / a^2)^N, a = sqrt(2N) sigma / (T / 2), by repeated series products."""
    from numpy.polynomial import chebyshev as C
    a2 = 2.0 * N * (sigma / (0.5 * T)) ** 2
    best = np.zeros(2 * N + 1)
    for c in np.linspace(-1.0, 1.0, grid):
        h = np.array([1.0 - (c * c + 0.5) / a2, 2.0 * c / a2, -0.5 / a2])   # h in the T_k basis
        d = np.array([1.0])
        for _ in range(N):
            d = C.chebmul(d, h)
        best = np.maximum(best, np.abs(d))
    return best


@pytest.mark.parametrize("N,sigma,eps", [(37, 30.0, 1e-7), (10, 60.0, 1e-7), (37, 30.0, 1e-4), (60, 30.0, 1e-7),
                                         (5, 100.0, 0.0)])
def test_poly_plan_truncation(lib, N, sigma, eps):
    """Kept coefficient count and dropped bound against an independent FP64 expansion (series
    products, not the library's recurrence)."""
    K = ctypes.c_int(0)
    b = ctypes.c_double(0.0)
    assert lib.bsk_poly_plan_info(N, sigma, 255.0, eps, ctypes.byref(K), ctypes.byref(b)) == _lib.BSK_OK
    mx = _cheb_coef_max(N, sigma, 255.0)
    if eps == 0.0:
        assert K.value == 2 * N + 1 and b.value == 0.0
        return
    tail = mx[K.value:].sum()
    assert tail <= eps * (1 + 1e-6)
    assert mx[K.value - 1:].sum() > eps * (1 - 1e-6)
    assert abs(b.value - tail) <= 1e-6 * eps


def test_poly_plan_info_errors(lib):
    K = ctypes.c_int(0)
    b = ctypes.c_double(0.0)
    assert lib.bsk_poly_plan_info(5000, 30.0, 255.0, 0.0, ctypes.byref(K), ctypes.byref(b)) == _lib.BSK_ERANGE
    assert lib.bsk_poly_plan_info(-1, 2.0, 255.0, 0.0, ctypes.byref(K), ctypes.byref(b)) == _lib.BSK_ERANGE
    assert lib.bsk_poly_plan_info(10, -1.0, 255.0, 0.0, None, None) == _lib.BSK_EINVAL
    assert lib.bsk_poly_plan_info(10, 30.0, 255.0, -1.0, None, None) == _lib.BSK_EINVAL
    assert lib.bsk_poly_plan_info(0, 30.0, 255.0, 0.0, ctypes.byref(K), None) == _lib.BSK_OK and K.value == 1


def test_poly_kernel_errors(lib):
    """Requests the polynomial range kernel does not run are refused before any launch."""
    big, big2 = 1 << 40, 1 << 41

    def opt(**kw):
        o = _lib.Options()
        o.range_kernel = _lib.BSK_RANGE_POLY
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    bad = _lib.Options()
    bad.range_kernel = 7
    assert _call_ex(lib, img=big, out=big2, opt=bad) == _lib.BSK_EINVAL
    assert _call_ex(lib, img=big, out=big2, opt=opt(precision=_lib.BSK_BF16)) == _lib.BSK_EUNSUPPORTED
    assert _call_ex(lib, img=big, out=big2, opt=opt(precision=_lib.BSK_I16)) == _lib.BSK_EUNSUPPORTED
    assert _call_ex(lib, img=big, out=big2, opt=opt(kahan=1)) == _lib.BSK_EUNSUPPORTED
    assert _call_ex(lib, img=big, out=big2, opt=opt(spatial_N=2, spatial_sigma=2.0)) == _lib.BSK_EUNSUPPORTED
    assert _call_ex(lib, img=big, out=big2, opt=opt(order_mode=1, N=4097)) == _lib.BSK_ERANGE
    assert _call_ex(lib, img=big, out=big2, s=2.0, opt=opt()) == _lib.BSK_ERANGE     # N_p = 8129
    assert _call_ex(lib, img=big, out=big2, opt=opt(order_chunk=5)) == _lib.BSK_EINVAL
    vp = ctypes.c_void_p
    o = opt()
    assert lib.bilateral_shiftable_train(vp(big), 8, 8, 2, 30.0, 255.0, ctypes.byref(o), vp(big2), vp(1 << 42),
                                         None) == _lib.BSK_EUNSUPPORTED
    assert lib.bilateral_shiftable_backward(vp(big), vp(big2), None, None, 8, 8, 2, 30.0, 255.0, ctypes.byref(o),
                                            vp(1 << 43), None, None) == _lib.BSK_EUNSUPPORTED
    d = (_lib.ImageDesc * 1)()
    d[0].img, d[0].out, d[0].H, d[0].W, d[0].radius, d[0].sigma_r, d[0].N = big, big2, 8, 8, 2, 30.0, -1
    assert lib.bilateral_shiftable_batched(d, 1, 255.0, ctypes.byref(o), None) == _lib.BSK_EUNSUPPORTED


def test_missing_library_fails_loudly(monkeypatch):
    """Without libbsk.so the binding raises; there is no fallback implementation."""
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libbsk.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _lib.load()


def test_nlm2_errors(lib):
    """Two-pixel-patch argument checks, refused before any launch."""
    vp = ctypes.c_void_p
    big, big2 = 1 << 40, 1 << 41

    def call(s1=60.0, s2=60.0, N1=-1, N2=-1, img=big, out=big2, opt=None, T=255.0):
        o = opt if opt is not None else _lib.Options()
        return lib.bilateral_shiftable_nlm2(vp(img), 8, 8, 2, s1, s2, N1, N2, 0, 1, T, vp(out), ctypes.byref(o),
                                            None)

    assert call(img=0) == _lib.BSK_EINVAL
    assert call(s2=0.0) == _lib.BSK_EINVAL
    assert call(s1=float("nan")) == _lib.BSK_EINVAL
    assert call(N1=1001) == _lib.BSK_ERANGE
    assert call(s1=0.5, s2=0.5) == _lib.BSK_ERANGE     # automatic orders beyond 1000
    o = _lib.Options()
    o.order_mode = 1
    assert call(opt=o) == _lib.BSK_EINVAL
    for field, value in (("precision", _lib.BSK_BF16), ("kahan", 1), ("range_kernel", _lib.BSK_RANGE_POLY)):
        o = _lib.Options()
        setattr(o, field, value)
        assert call(opt=o) == _lib.BSK_EUNSUPPORTED, field
    o = _lib.Options()
    o.spatial_N, o.spatial_sigma = 2, 2.0
    assert call(opt=o) == _lib.BSK_EUNSUPPORTED
    o = _lib.Options()
    o.order_chunk = 5
    assert call(opt=o) == _lib.BSK_EINVAL
    # 31 x 16 folded orders fit; orders 1000 x 1000 do not
    assert call(N1=1000, N2=1000) == _lib.BSK_ERANGE
    o = _lib.Options()
    o.weight_eps = 0.9   # above every binomial weight of N = 8: nothing would be left
    assert call(opt=o) == _lib.BSK_EINVAL


def test_weight_eps_dropping_every_order_is_refused(lib):
    """A weight_eps above the central binomial weight would leave no order (the filter 0/0):
    refused before any launch, by the single-image and the batched entry points."""
    vp = ctypes.c_void_p
    o = _lib.Options()
    o.order_mode, o.N, o.weight_eps = 1, 30, 0.5      # the central weight of N = 30 is 0.144
    assert lib.bilateral_shiftable_ex(vp(1 << 40), 8, 8, 2, 30.0, 255.0, vp(1 << 41), ctypes.byref(o),
                                      None) == _lib.BSK_EINVAL
    d = _lib.ImageDesc()
    d.img, d.out, d.H, d.W, d.radius, d.sigma_r, d.N = 1 << 40, 1 << 41, 8, 8, 2, 30.0, 30
    assert lib.bilateral_shiftable_batched(ctypes.byref(d), 1, 255.0, ctypes.byref(o), None) == _lib.BSK_EINVAL
    k = ctypes.c_int()                                 # 0.14 keeps only the central order (0.135 next)
    assert lib.bsk_plan_info(30, 0.14, ctypes.byref(k), None) == _lib.BSK_OK and k.value == 1


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU; --gpus above 1 exits with a message before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
