"""Forward parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (max-abs over compared pixels): FP64 path 1e-9 T, FP32 path 1e-4 T,
BF16/FP16 precision form 2e-3 T, with T = 255 the range bound.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1107_4617_amd import bilateral, order_for, plan_info
from paper_1107_4617_amd import workloads as wl

pytestmark = pytest.mark.gpu

T = 255.0
TOL32 = 1e-4 * T
TOL64 = 1e-9 * T
TOL16 = 2e-3 * T


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)


def _gpu_filter(f, r, s, N=None, **kw):
    dt = torch.float64 if kw.get("precision") == "fp64" else torch.float32
    x = torch.from_numpy(np.ascontiguousarray(f)).to(dtype=dt, device="cuda")
    y = bilateral(x, r, s, T, N=N, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def _sample_idx(H, W, n, seed, extra_rows=(), extra_cols=()):
    rng = np.random.default_rng(seed)
    idx = set(rng.integers(0, H * W, n).tolist())
    rows = {0, 1, H - 2, H - 1, *[x for x in extra_rows if 0 <= x < H]}
    cols = {0, 1, W - 2, W - 1, *[x for x in extra_cols if 0 <= x < W]}
    for i in rows:
        for j in rng.integers(0, W, 64):
            idx.add(i * W + int(j))
    for j in cols:
        for i in rng.integers(0, H, 64):
            idx.add(int(i) * W + j)
    return np.array(sorted(idx), dtype=np.int64)


def test_smooth256_fp64_and_fp32():
    """256x256 smooth+noise image, r=5, sigma_r=30, N=30; full-image comparison."""
    f = wl.smooth_image(256, 256, 1)
    ref = oracle.bilateral(f, 5, 30.0, 30)
    out64 = _gpu_filter(f.astype(np.float64), 5, 30.0, N=30, precision="fp64")
    assert np.max(np.abs(out64 - ref)) <= TOL64
    out32 = _gpu_filter(f, 5, 30.0, N=30)
    err = np.max(np.abs(out32 - ref))
    assert err <= TOL32, err


@pytest.mark.parametrize("shape,r,N,sigma,block", [
    ((70, 300), 8, 31, 30.0, 0),       # odd N, 16 orders: the one-pass FP64 kernel
    ((150, 500), 12, 30, 30.0, 0),     # even N, 16 orders, one pass over several strips and segments
    ((70, 300), 8, 7, 70.0, 0),        # odd N, one pass (4 orders padded to 16)
    ((60, 90), 6, 8, 60.0, 0),         # even N, one pass
    ((129, 257), 20, 43, 25.0, 256),   # 22 orders: three passes of 8 orders
    ((80, 600), 70, 30, 30.0, 512),    # 512-lane strips
])
def test_fp64_matches_oracle(shape, r, N, sigma, block):
    """The FP64 path (transforms, sums and recombination in FP64) against the oracle to 1e-9 T."""
    f = wl.rect_image(*shape, seed=7 + r)
    ref = oracle.bilateral(f, r, sigma, N)
    out = _gpu_filter(f.astype(np.float64), r, sigma, N=N, precision="fp64", block=block)
    assert np.max(np.abs(out - ref)) <= TOL64


@pytest.mark.parametrize("shape,r,N,sigma,block,strip_h", [
    ((1, 1), 3, 30, 30.0, 0, 0),
    ((1, 37), 4, 30, 30.0, 0, 0),
    ((41, 1), 4, 30, 30.0, 0, 0),
    ((7, 300), 9, 30, 30.0, 0, 0),          # H < 2r+1
    ((300, 500), 7, 30, 30.0, 256, 16),     # many strips and segments, ragged tails
    ((129, 257), 20, 30, 30.0, 256, 33),
    ((64, 64), 200, 30, 30.0, 0, 0),        # radius beyond the image: whole-image windows
    ((50, 70), 0, 30, 30.0, 0, 0),          # r = 0: identity
    ((60, 90), 6, 0, 30.0, 0, 0),           # N = 0: box mean
    ((60, 90), 6, 1, 200.0, 0, 0),          # N = 1 (N_0 = 1 at sigma_r = 200)
    ((60, 90), 6, 7, 70.0, 0, 0),           # odd N (N_0 = 6 at sigma_r = 70)
    ((60, 90), 6, 2, 120.0, 0, 0),          # N = 2
    ((70, 300), 8, 31, 30.0, 0, 0),         # odd N filling one 16-order pass
    ((70, 300), 8, 29, 30.0, 256, 0),       # odd N, 15 orders in a 16-order pass
    ((80, 600), 70, 30, 30.0, 512, 20),     # 512-lane strips
    ((90, 300), 6, 20, 36.0, 256, 0),       # 11 orders, one 12-order pass (N_0 = 20 at sigma_r = 36)
    ((90, 300), 6, 43, 25.0, 256, 0),       # 22 orders, two 12-order passes
    ((40, 1100), 200, 30, 30.0, 1024, 0),   # 1024-lane strips
    ((12, 1100), 500, 30, 30.0, 0, 0),      # the largest clamped radius (BSK_MAX_RADIUS)
    # compile-time-radius kernels on images smaller than their window
    ((1, 1), 20, 30, 30.0, 0, 0),
    ((3, 50), 32, 30, 30.0, 0, 0),
    ((60, 2), 16, 43, 25.0, 0, 0),          # two 12-order passes
    ((33, 217), 20, 30, 30.0, 0, 5),        # one column past a full strip, 5-row segments
])
def test_shapes_and_edge_cases(shape, r, N, sigma, block, strip_h):
    """Orders at or above N_0(sigma_r, 255), where the kernel is a valid (non-negative) kernel."""
    f = wl.random_image(*shape, seed=sum(shape) + r)
    ref = oracle.bilateral(f, r, sigma, N)
    out = _gpu_filter(f, r, sigma, N=N, block=block, strip_h=strip_h)
    assert np.max(np.abs(out - ref)) <= TOL32


# Radii on both sides of the walker-chunk multiples (the box width 2r + 1 against 17,
# 34 and 51 positions: r = 8, 16/17, 24/25) and in each of the four compiled parts.
CT_RADII = [1, 2, 3, 5, 7, 8, 10, 13, 16, 17, 20, 24, 25, 31, 32]


@pytest.mark.parametrize("r", CT_RADII)
@pytest.mark.parametrize("N,sigma", [(30, 30.0),    # 16 orders, even N: the full pass
                                     (31, 30.0),    # 16 orders, odd N
                                     (7, 70.0)])    # 4 orders, odd N: the half pass
def test_compile_time_radius_kernels(r, N, sigma):
    """The radii with their own one-pass kernels (the walkers hand out box sums): several
    strips and segments with ragged tails, both start modes and both pass sizes."""
    f = wl.rect_image(150, 700, seed=r + N, n_rect=12)
    ref = oracle.bilateral(f, r, sigma, N)
    out = _gpu_filter(f, r, sigma, N=N, strip_h=37)
    assert np.max(np.abs(out - ref)) <= TOL32


@pytest.mark.parametrize("r", range(1, 65))
def test_every_compile_time_radius(r):
    """Every radius from 1 to 64 has its own forward kernel: the headline's order count on
    a small image with two or more strips and ragged segments."""
    f = wl.rect_image(70, 330, seed=100 + r, n_rect=8)
    ref = oracle.bilateral(f, r, 30.0, 30)
    out = _gpu_filter(f, r, 30.0, N=30, strip_h=23)
    assert np.max(np.abs(out - ref)) <= TOL32


@pytest.mark.parametrize("r", CT_RADII)
@pytest.mark.parametrize("N,sigma", [(20, 36.0),    # 11 orders: one 12-order pass
                                     (43, 25.0),    # 22 orders: two 12-order passes
                                     (117, 15.0)])  # 59 orders: four 16-order passes
def test_compile_time_radius_kernels_multi_pass(r, N, sigma):
    """The compile-time-radius kernels with the 12-order pass and with several passes
    (run-time start mode, partial accumulators in the workspace)."""
    f = wl.rect_image(80, 460, seed=3 * r + N, n_rect=10)
    ref = oracle.bilateral(f, r, sigma, N)
    out = _gpu_filter(f, r, sigma, N=N, strip_h=29)
    assert np.max(np.abs(out - ref)) <= TOL32


@pytest.mark.parametrize("r,kc", [(7, 8), (7, 12), (7, 16), (7, 20), (7, 24), (50, 20), (50, 24),
                                  (70, 8), (70, 12), (70, 16)])
def test_every_pass_size(kc, r):
    """30 folded orders (N = 59) in passes of 8, 12, 16, 20 or 24 orders (4, 3, 2, 2 or 2
    passes, the last one padded) against the oracle: every pass size of the compile-time
    radius 7, the large ones at the forward-only compile-time radius 50, and those of the
    run-time radius 70 (256-lane strips)."""
    f = wl.rect_image(100, 300, seed=59, n_rect=10)
    ref = oracle.bilateral(f, r, 22.0, 59)
    out = _gpu_filter(f, r, 22.0, N=59, block=256, order_chunk=kc)
    assert np.max(np.abs(out - ref)) <= TOL32


@pytest.mark.parametrize("r", [5, 70])
def test_many_orders(r):
    """sigma_r = 10 (N_0 = 264, 133 folded orders): six 24-order passes at the compile-time
    radius 5, nine 16-order ones at the run-time radius 70."""
    f = wl.rect_image(48, 300, seed=264 + r, n_rect=8)
    N = order_for(10.0, T)
    ref = oracle.bilateral(f, r, 10.0, N)
    out = _gpu_filter(f, r, 10.0, strip_h=17, block=256)
    assert np.max(np.abs(out - ref)) <= TOL32


@pytest.mark.parametrize("kc", [20, 24])
def test_large_passes_need_a_compile_time_radius(kc):
    """The 20- and 24-order passes exist at the compile-time radii (1 to 64) only; elsewhere
    the request is rejected before any launch."""
    from paper_1107_4617_amd._lib import BskError

    f = wl.rect_image(40, 300, seed=1, n_rect=4)
    with pytest.raises(BskError, match="EINVAL"):
        _gpu_filter(f, 70, 22.0, N=59, block=256, order_chunk=kc)


@pytest.mark.parametrize("r,N", [(20, 43), (20, 44), (31, 43), (2, 44)])
def test_one_pass_of_24(r, N):
    """22 or 23 folded orders: the automatic choice is one 24-order pass with the start mode
    as a constant (odd and even N)."""
    f = wl.rect_image(90, 330, seed=N + r, n_rect=10)
    ref = oracle.bilateral(f, r, 25.0, N)
    out = _gpu_filter(f, r, 25.0, N=N)
    assert np.max(np.abs(out - ref)) <= TOL32


def test_autotune_applies_its_shape(tmp_path):
    """bsk_autotune times the single-image launch shapes (lanes, rows, every pass size),
    caches the fastest, and a later call with automatic options runs exactly that shape:
    bit for bit the output of the call that names it, within the oracle bound."""
    from paper_1107_4617_amd import autotune, tune_cache_clear

    tune_cache_clear()
    try:
        f = wl.rect_image(96, 500, seed=5, n_rect=10)
        x = torch.from_numpy(f).cuda()
        b, rows, kc, ms = autotune(x, 6, 12.0, T, path=str(tmp_path / "tune.jsonl"))
        assert b in (256, 512, 1024) and rows > 0 and kc > 0 and ms > 0
        auto = bilateral(x, 6, 12.0, T)
        named = bilateral(x, 6, 12.0, T, block=b, strip_h=rows, order_chunk=kc)
        torch.cuda.synchronize()
        assert torch.equal(auto, named)
        ref = oracle.bilateral(f, 6, 12.0, order_for(12.0, T))
        assert np.max(np.abs(auto.cpu().numpy() - ref)) <= TOL32
    finally:
        tune_cache_clear()


def test_radius_zero_is_exact_identity():
    f = wl.random_image(33, 45, 3)
    out = _gpu_filter(f, 0, 30.0, N=30)
    assert np.max(np.abs(out - f)) <= 2e-5 * T


def test_constant_image_is_fixed():
    f = np.full((70, 90), 137.25, np.float32)
    out = _gpu_filter(f, 8, 30.0, N=30)
    assert np.max(np.abs(out - 137.25)) <= 1e-5 * T


@pytest.mark.parametrize("N", [117, 264])
def test_multi_pass_orders(N):
    """More folded orders than one pass holds (N=117: 59 orders; N=264: 133)."""
    sigma = 15.0 if N == 117 else 10.0
    f = wl.rect_image(96, 200, seed=N, n_rect=12)
    ref = oracle.bilateral(f, 6, sigma, N)
    out = _gpu_filter(f, 6, sigma, N=N)
    assert np.max(np.abs(out - ref)) <= TOL32


def test_pitch():
    f = wl.random_image(40, 60, 5)
    big = np.zeros((40, 80), np.float32)
    big[:, :60] = f
    x = torch.from_numpy(big).cuda()
    y = torch.full((40, 96), -7.0, device="cuda")
    from paper_1107_4617_amd import _lib
    import ctypes
    o = _lib.Options()
    o.pitch_in, o.pitch_out = 80, 96
    _lib.check(_lib.load().bilateral_shiftable_ex(ctypes.c_void_p(x.data_ptr()), 40, 60, 4, 30.0, T,
                                                  ctypes.c_void_p(y.data_ptr()), ctypes.byref(o), None))
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    ref = oracle.bilateral(f, 4, 30.0, 30)
    assert np.max(np.abs(y[:, :60] - ref)) <= TOL32
    assert np.all(y[:, 60:] == -7.0)


def test_sync_entry_point():
    from paper_1107_4617_amd import _lib
    import ctypes
    f = wl.random_image(50, 77, 6)
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    _lib.check(_lib.load().bilateral_shiftable(ctypes.c_void_p(x.data_ptr()), 50, 77, 3, 30.0, T,
                                               ctypes.c_void_p(y.data_ptr())))
    ref = oracle.bilateral(f, 3, 30.0, order_for(30.0, T))
    assert np.max(np.abs(y.cpu().numpy() - ref)) <= TOL32


def test_deterministic():
    f = wl.rect_image(300, 400, seed=9)
    a = _gpu_filter(f, 11, 30.0)
    b = _gpu_filter(f, 11, 30.0)
    assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def rect4096():
    """The headline input and its exact FP64 oracle result on every pixel (about 15 s on
    16 host cores)."""
    f = wl.rect_image(4096, 4096, seed=2)
    return f, oracle.bilateral(f, 20, 30.0, 30)


def test_rect4096_r20_full_image(rect4096):
    """Full-size 4096x4096 rect image, r=20, sigma_r=30, N=30, in the launch shape the
    benchmark uses, against the oracle on every pixel (strip and segment edges included)."""
    f, ref = rect4096
    out = _gpu_filter(f, 20, 30.0, N=30)
    err = np.abs(out - ref)
    assert np.max(err) <= TOL32, np.max(err)


def test_rect4096_r20_sampled():
    """The same launch against the oracle's per-pixel entry point at sampled pixels
    (random, borders, strip edges): both oracle entry points and the kernel agree."""
    f = wl.rect_image(4096, 4096, seed=2)
    out = _gpu_filter(f, 20, 30.0, N=30)
    Wt = 256 - 40
    cols = [k * Wt + d for k in range(1, 4096 // Wt + 1) for d in (-1, 0)]
    idx = _sample_idx(4096, 4096, 3000, 22, extra_cols=cols)
    ref = oracle.bilateral_at(f, idx, 20, 30.0, 30)
    err = np.abs(out.ravel()[idx] - ref)
    assert np.max(err) <= TOL32, np.max(err)


# Which 16-bit stacks meet 2e-3 T at their worst pixels.  A 16-bit stack perturbs the kernel by
# about one rounding unit u per order, so the output moves by roughly u sqrt(|B|) |f_y - out| / Q:
# it is largest where few neighbours resemble the pixel and the normaliser Q is small.  The
# Q15 stack (u = 2^-15 on [-1, 1]) meets the tolerance at the headline workload; the float16
# (u = 2^-11 relative) and bfloat16 (2^-8) stacks do not, and at 8192^2, r = 32, sigma_r = 15
# (|B| = 4225, normalisers down to ~1) none does.  The failing forms are strict xfails: the
# day one of them passes, the test says so.
PRECISION_FORMS = [(p, k) for p in ("i16", "fp16", "bf16") for k in (False, True)]
MEETS_4096 = {("i16", False): True, ("i16", True): True, ("fp16", False): False, ("fp16", True): False,
              ("bf16", False): False, ("bf16", True): False}
MEETS_8192 = {key: False for key in PRECISION_FORMS}


def _worst(err, n):
    """Flat indices of the n largest entries of err."""
    flat = err.ravel()
    return np.argpartition(flat, -n)[-n:]


def _form_param(prec, kahan, meets):
    marks = [] if meets[(prec, kahan)] else [pytest.mark.xfail(
        strict=True, reason=f"{prec} stack{' + Kahan' if kahan else ''}: max error above 2e-3 T where the "
                            "normaliser is small (quantisation of the stack, not the sums)")]
    return pytest.param(prec, kahan, marks=marks, id=f"{prec}{'-kahan' if kahan else ''}")


@pytest.mark.parametrize("prec,kahan", [_form_param(p, k, MEETS_4096) for p, k in PRECISION_FORMS])
def test_precision_form_rect4096_worst_pixels(rect4096, prec, kahan):
    """Headline workload (4096^2, r=20, sigma_r=30, N=30) with the stack held in 16 bits and
    weights below 1e-7 dropped (14 of 16 folded orders): every pixel against the exact oracle,
    and the 2000 pixels where the form departs most from the FP32 path plus 800 random ones
    against the oracle's truncated kernel, all at 2e-3 T."""
    f, ref = rect4096
    out32 = _gpu_filter(f, 20, 30.0, N=30)
    out = _gpu_filter(f, 20, 30.0, N=30, precision=prec, weight_eps=1e-7, kahan=kahan)
    err_exact = float(np.max(np.abs(out - ref)))
    idx = np.union1d(_worst(np.abs(out - out32), 2000), _sample_idx(4096, 4096, 800, 44))
    ref_t = oracle.bilateral_at(f, idx, 20, 30.0, 30, eps=1e-7, truncated=True)
    err_t = float(np.max(np.abs(out.ravel()[idx] - ref_t)))
    print(f"{prec} kahan={kahan} 4096^2: max vs exact oracle {err_exact:.4g}, vs truncated oracle at "
          f"the worst pixels {err_t:.4g}", flush=True)
    assert err_exact <= TOL16 and err_t <= TOL16, (err_exact, err_t)


@pytest.fixture(scope="module")
def rect8192():
    f = wl.rect_image(8192, 8192, seed=3)
    return f, _gpu_filter(f, 32, 15.0, N=117)


def test_rect8192_r32_fp32_and_truncation(rect8192):
    """8192^2, r=32, sigma_r=15, N=117: the FP32 path against the exact oracle at sampled
    pixels, and truncation at 1e-7 (28 of 59 folded orders) moving the exact result by far
    less than the tolerance."""
    f, out32 = rect8192
    K, eps = plan_info(117, 1e-7)
    assert K == 28 and abs(eps - 1.283e-7) < 1e-9
    idx = _sample_idx(8192, 8192, 600, 33)
    ref = oracle.bilateral_at(f, idx, 32, 15.0, 117)
    ref_t = oracle.bilateral_at(f, idx, 32, 15.0, 117, eps=1e-7, truncated=True)
    assert np.max(np.abs(ref - ref_t)) <= 1e-3
    assert np.max(np.abs(out32.ravel()[idx] - ref)) <= TOL32


@pytest.mark.parametrize("prec,kahan", [_form_param(p, k, MEETS_8192) for p, k in PRECISION_FORMS])
def test_rect8192_r32_precision_form_worst_pixels(rect8192, prec, kahan):
    """The precision form's own workload (8192^2, r=32, sigma_r=15, N=117, weights below 1e-7
    dropped): the 2000 pixels where the 16-bit form departs most from the FP32 path, plus 600
    random and border pixels, against the oracle's truncated kernel at 2e-3 T."""
    f, out32 = rect8192
    out = _gpu_filter(f, 32, 15.0, N=117, precision=prec, weight_eps=1e-7, kahan=kahan)
    d32 = float(np.max(np.abs(out - out32)))
    idx = np.union1d(_worst(np.abs(out - out32), 2000), _sample_idx(8192, 8192, 600, 33))
    ref_t = oracle.bilateral_at(f, idx, 32, 15.0, 117, eps=1e-7, truncated=True)
    err = float(np.max(np.abs(out.ravel()[idx] - ref_t)))
    print(f"{prec} kahan={kahan} 8192^2: max vs FP32 {d32:.4g}, vs truncated oracle at the worst "
          f"pixels {err:.4g}", flush=True)
    assert err <= TOL16, err


def test_fp64_rect4096_sampled():
    """The FP64 path at the headline workload, as bench.py times it; oracle at sampled pixels."""
    f = wl.rect_image(4096, 4096, seed=2)
    out = _gpu_filter(f.astype(np.float64), 20, 30.0, N=30, precision="fp64")
    rng = np.random.default_rng(33)
    idx = np.unique(np.concatenate([rng.integers(0, 4096 * 4096, 1500),
                                    4095 * 4096 + rng.integers(0, 4096, 100),
                                    rng.integers(0, 4096, 100) * 4096 + 215]))
    ref = oracle.bilateral_at(f, idx, 20, 30.0, 30)
    assert np.max(np.abs(out.ravel()[idx] - ref)) <= TOL64


