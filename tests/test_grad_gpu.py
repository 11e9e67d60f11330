"""Adjoint (d/d image, d/d sigma_r) of the HIP path against the FP64 oracle gradient.

Tolerances: dL/dimg within 1e-3 of max |dL/dimg| (max-abs), dL/dsigma_r within
1e-3 relative; the oracle gradient itself is pinned to central differences in
the CPU tests.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1107_4617_amd import ShiftableBilateral, bilateral_backward, bilateral_train
from paper_1107_4617_amd import workloads as wl

pytestmark = pytest.mark.gpu
T = 255.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("shape,r,sigma,N,seed", [((40, 56), 3, 25.0, 43, 1), ((33, 70), 5, 30.0, 30, 2),
                                                  ((64, 64), 10, 25.0, 43, 3), ((20, 300), 7, 40.0, 17, 4)])
def test_adjoint_matches_oracle(shape, r, sigma, N, seed):
    f = wl.rect_image(*shape, seed=seed, n_rect=6)
    g = np.random.default_rng(seed).normal(size=shape)
    gf_ref, gs_ref, u_ref = oracle.bilateral_grad(f.astype(np.float64), g, r, sigma, N)
    x = _cuda(f)
    out, saved = bilateral_train(x, r, sigma, T, N)
    assert np.max(np.abs(out.cpu().numpy() - u_ref)) <= 1e-4 * T
    _, _, Q = oracle.bilateral(f, r, sigma, N, return_pq=True)
    assert np.max(np.abs(saved[0].cpu().numpy() - Q) / Q) <= 1e-4
    gi, gs = bilateral_backward(x, _cuda(g), r, sigma, T, N, out=out, saved=saved)
    torch.cuda.synchronize()
    scale = np.max(np.abs(gf_ref))
    assert np.max(np.abs(gi.cpu().numpy() - gf_ref)) <= 1e-3 * scale
    assert abs(float(gs) - gs_ref) <= 1e-3 * abs(gs_ref)
    # recompute path (no saved state) gives the same numbers
    gi2, gs2 = bilateral_backward(x, _cuda(g), r, sigma, T, N)
    torch.cuda.synchronize()
    assert torch.equal(gi, gi2) and torch.equal(gs, gs2)


def test_denoise_crop_against_oracle_and_differences():
    """Centre 32x32 crop of the first 1024x1024 denoising image (r=10, sigma_r=25, N=43),
    treated as a standalone image; loss = mean((u - target)^2)."""
    noisy, target = wl.denoise_pair(0)
    c0 = 512 - 16
    f = noisy[c0:c0 + 32, c0:c0 + 32].astype(np.float64)
    tg = target[c0:c0 + 32, c0:c0 + 32].astype(np.float64)
    r, s, N = 10, 25.0, 43
    u = oracle.bilateral(f, r, s, N)
    gbar = 2.0 * (u - tg) / u.size
    gf_ref, gs_ref, _ = oracle.bilateral_grad(f, gbar, r, s, N)

    def loss(ff, ss):
        return float(np.mean((oracle.bilateral(ff, r, ss, N) - tg) ** 2))

    h = 1e-3
    fd_s = (loss(f, s + h) - loss(f, s - h)) / (2 * h)
    assert abs(gs_ref - fd_s) <= 1e-6 * abs(fd_s)
    x = _cuda(f)
    layer = ShiftableBilateral(r, s, T, N).cuda()
    xr = x.clone().requires_grad_(True)
    out = layer(xr)
    L = torch.mean((out - _cuda(tg)) ** 2)
    L.backward()
    torch.cuda.synchronize()
    scale = np.max(np.abs(gf_ref))
    assert np.max(np.abs(xr.grad.cpu().numpy() - gf_ref)) <= 1e-3 * scale
    assert abs(float(layer.sigma_r.grad) - gs_ref) <= 1e-3 * abs(gs_ref)


def test_denoise_256_crop():
    noisy, _ = wl.denoise_pair(1)
    f = noisy[300:556, 200:456]
    g = np.random.default_rng(7).normal(size=f.shape)
    gf_ref, gs_ref, _ = oracle.bilateral_grad(f.astype(np.float64), g, 10, 25.0, 43)
    gi, gs = bilateral_backward(_cuda(f), _cuda(g), 10, 25.0, T, 43)
    torch.cuda.synchronize()
    assert np.max(np.abs(gi.cpu().numpy() - gf_ref)) <= 1e-3 * np.max(np.abs(gf_ref))
    assert abs(float(gs) - gs_ref) <= 1e-3 * abs(gs_ref)


def test_rect4096_adjoint_sampled():
    """Training forward and adjoint at the headline workload (4096x4096 rect, r = 20, sigma_r = 30,
    N = 30) in the launch shapes bench.py times.  dL/dimg at a pixel z depends on f and gbar only
    within distance 2r of z, so the oracle gradient of a crop holding that neighbourhood (cut at
    the image's own edges) equals the full image's at z."""
    n, r, s, N = 4096, 20, 30.0, 30
    f = wl.rect_image(n, n, seed=2)
    g = np.random.default_rng(9).normal(size=(n, n)).astype(np.float32)
    x = _cuda(f)
    out, saved = bilateral_train(x, r, s, T, N)
    gi, _ = bilateral_backward(x, _cuda(g), r, s, T, N, out=out, saved=saved)
    torch.cuda.synchronize()
    gi = gi.cpu().numpy()
    rng = np.random.default_rng(10)
    pts = [(int(a), int(b)) for a, b in rng.integers(0, n, (20, 2))]
    pts += [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0), (int(rng.integers(0, n)), 215),
            (int(rng.integers(0, n)), 216), (51, int(rng.integers(0, n))), (52, int(rng.integers(0, n)))]
    got, ref = [], []
    m = 2 * r + 1
    for i, j in pts:
        i0, i1, j0, j1 = max(0, i - m), min(n, i + m + 1), max(0, j - m), min(n, j + m + 1)
        gf, _, _ = oracle.bilateral_grad(f[i0:i1, j0:j1].astype(np.float64), g[i0:i1, j0:j1].astype(np.float64),
                                         r, s, N)
        ref.append(gf[i - i0, j - j0])
        got.append(gi[i, j])
    ref, got = np.array(ref), np.array(got)
    assert np.max(np.abs(got - ref)) <= 1e-3 * np.max(np.abs(ref))


# Radii on both sides of the walker-chunk multiples, in each compiled part up to 32, and above
# 32 (compile-time training forward, run-time-radius adjoint).
CT_RADII = [1, 2, 3, 5, 7, 8, 10, 13, 16, 17, 20, 24, 25, 31, 32, 40, 57, 64]


@pytest.mark.parametrize("r", CT_RADII)
@pytest.mark.parametrize("N,sigma", [(30, 30.0),    # 16 orders, even N: two training passes of 8, one adjoint pass of 16
                                     (31, 30.0),    # 16 orders, odd N
                                     (43, 25.0),    # 22 orders, odd N: three training passes, one adjoint pass of 24
                                     (42, 25.0),    # 22 orders, even N
                                     (7, 70.0),     # 4 orders, odd N: one training pass, the adjoint's half pass
                                     (8, 70.0)])    # 5 orders, even N
def test_compile_time_radius_gradients(r, N, sigma):
    """The radii with their own training-forward and adjoint kernels (the walkers hand out box
    sums), across two strips and several segments: output, saved normaliser and both gradients
    against the oracle."""
    f = wl.rect_image(40, 260, seed=r + N, n_rect=8)
    g = np.random.default_rng(r + N).normal(size=f.shape)
    gf_ref, gs_ref, u_ref = oracle.bilateral_grad(f.astype(np.float64), g, r, sigma, N)
    x = _cuda(f)
    out, saved = bilateral_train(x, r, sigma, T, N)
    assert np.max(np.abs(out.cpu().numpy() - u_ref)) <= 1e-4 * T
    gi, gs = bilateral_backward(x, _cuda(g), r, sigma, T, N, out=out, saved=saved)
    torch.cuda.synchronize()
    assert np.max(np.abs(gi.cpu().numpy() - gf_ref)) <= 1e-3 * np.max(np.abs(gf_ref))
    assert abs(float(gs) - gs_ref) <= 1e-3 * abs(gs_ref)


@pytest.mark.parametrize("r", [0, 70])
@pytest.mark.parametrize("N,sigma", [(30, 30.0), (31, 30.0), (43, 25.0), (42, 25.0), (7, 70.0)])
def test_run_time_radius_gradients(r, N, sigma):
    """Radii without compile-time-radius kernels: 0 (256-lane strips: the one-pass 16- and
    24-order adjoints with the start mode as a constant, both modes, and the half pass) and
    70 (512-lane strips), against the oracle."""
    f = wl.rect_image(36, 300, seed=7 * r + N, n_rect=8)
    g = np.random.default_rng(r + 2 * N).normal(size=f.shape)
    gf_ref, gs_ref, u_ref = oracle.bilateral_grad(f.astype(np.float64), g, r, sigma, N)
    x = _cuda(f)
    out, saved = bilateral_train(x, r, sigma, T, N)
    assert np.max(np.abs(out.cpu().numpy() - u_ref)) <= 1e-4 * T
    gi, gs = bilateral_backward(x, _cuda(g), r, sigma, T, N, out=out, saved=saved)
    torch.cuda.synchronize()
    assert np.max(np.abs(gi.cpu().numpy() - gf_ref)) <= 1e-3 * max(np.max(np.abs(gf_ref)), 1e-12)
    if r == 0:
        # the exact sigma_r gradient is 0, and the kernel's is the FP32 rounding of
        # C (g S) - S (g C) summed over the image
        return
    # The sigma_r gradient sums g(x) du(x)/dsigma_r, terms of both signs: bounded by 1e-3 of
    # it plus 1e-5 of the sum of the terms' sizes (from central differences of the oracle),
    # which covers sums that nearly cancel.
    h = 1e-3 * sigma
    du = (oracle.bilateral(f, r, sigma + h, N) - oracle.bilateral(f, r, sigma - h, N)) / (2 * h)
    size = float(np.sum(np.abs(g) * np.abs(du)))
    assert abs(float(gs) - gs_ref) <= 1e-3 * abs(gs_ref) + 1e-5 * size


@pytest.mark.parametrize("shape,r", [((1, 1), 20), ((5, 40), 32), ((50, 3), 10)])
def test_compile_time_radius_gradients_small_images(shape, r):
    """Compile-time-radius training forward and adjoint on images smaller than the window."""
    f = wl.rect_image(*shape, seed=sum(shape) + r, n_rect=3)
    g = np.random.default_rng(r).normal(size=f.shape)
    gf_ref, gs_ref, u_ref = oracle.bilateral_grad(f.astype(np.float64), g, r, 25.0, 43)
    x = _cuda(f)
    out, saved = bilateral_train(x, r, 25.0, T, 43)
    assert np.max(np.abs(out.cpu().numpy() - u_ref)) <= 1e-4 * T
    gi, gs = bilateral_backward(x, _cuda(g), r, 25.0, T, 43, out=out, saved=saved)
    torch.cuda.synchronize()
    assert np.max(np.abs(gi.cpu().numpy() - gf_ref)) <= 1e-3 * max(np.max(np.abs(gf_ref)), 1e-12)
    assert abs(float(gs) - gs_ref) <= 1e-3 * abs(gs_ref) + 1e-9


@pytest.mark.parametrize("N,sigma", [(117, 15.0), (90, 17.0)])
def test_multi_pass_adjoint(N, sigma):
    """Several passes in both training forward and adjoint: N = 117 (59 folded orders,
    adjoint passes of 16) and N = 90 (46 orders, two adjoint passes of 24)."""
    f = wl.rect_image(48, 80, seed=11, n_rect=8)
    g = np.random.default_rng(11).normal(size=f.shape)
    gf_ref, gs_ref, _ = oracle.bilateral_grad(f.astype(np.float64), g, 4, sigma, N)
    gi, gs = bilateral_backward(_cuda(f), _cuda(g), 4, sigma, T, N)
    torch.cuda.synchronize()
    assert np.max(np.abs(gi.cpu().numpy() - gf_ref)) <= 1e-3 * np.max(np.abs(gf_ref))
    assert abs(float(gs) - gs_ref) <= 1e-3 * abs(gs_ref)


def test_adjoint_deterministic():
    f = wl.rect_image(200, 300, seed=12)
    g = np.random.default_rng(12).normal(size=f.shape)
    a = bilateral_backward(_cuda(f), _cuda(g), 9, 25.0, T, 43)
    b = bilateral_backward(_cuda(f), _cuda(g), 9, 25.0, T, 43)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_stack_matches_single_images_and_oracle():
    """A stack of images in one training-forward launch and one adjoint launch: each image's
    output, saved planes and image gradient agree with the single-image calls (the launch
    shape, hence the summation order, differs), dL/dsigma_r is the sum of the single-image
    ones, and image 1 matches the FP64 oracle gradient."""
    B, H, W, r, sigma, N = 5, 48, 72, 4, 25.0, 43
    fs = np.stack([wl.rect_image(H, W, seed=30 + b, n_rect=6) for b in range(B)])
    gs_np = np.random.default_rng(30).normal(size=(B, H, W))
    x = _cuda(fs)
    g = _cuda(gs_np)
    out, saved = bilateral_train(x, r, sigma, T, N)
    assert out.shape == (B, H, W) and saved.shape == (B, 3, H, W)
    gi, gsig = bilateral_backward(x, g, r, sigma, T, N, out=out, saved=saved)
    torch.cuda.synchronize()
    gsum = 0.0
    for b in range(B):
        o1, s1 = bilateral_train(x[b].contiguous(), r, sigma, T, N)
        gi1, gs1 = bilateral_backward(x[b].contiguous(), g[b].contiguous(), r, sigma, T, N, out=o1, saved=s1)
        torch.cuda.synchronize()
        assert float((out[b] - o1).abs().max()) <= 5e-4
        for p in range(3):
            ref = s1[p].abs().max()
            assert float((saved[b, p] - s1[p]).abs().max()) <= 1e-5 * float(ref) + 1e-6, (b, p)
        assert float((gi[b] - gi1).abs().max()) <= 1e-4 * float(gi1.abs().max()), b
        gsum += float(gs1)
    assert abs(float(gsig) - gsum) <= 1e-4 * abs(gsum)
    gf_ref, _, _ = oracle.bilateral_grad(fs[1].astype(np.float64), gs_np[1], r, sigma, N)
    assert np.max(np.abs(gi[1].cpu().numpy() - gf_ref)) <= 1e-3 * np.max(np.abs(gf_ref))
    # the recompute path (no saved state) over the stack gives the same numbers
    gi2, gsig2 = bilateral_backward(x, g, r, sigma, T, N)
    torch.cuda.synchronize()
    assert torch.equal(gi, gi2) and torch.equal(gsig, gsig2)


def test_layer_runs_a_stack_in_one_launch_pair():
    """ShiftableBilateral on a (B, H, W) batch: gradients equal those of the stacked calls."""
    B, H, W = 3, 40, 40
    fs = np.stack([wl.rect_image(H, W, seed=40 + b, n_rect=5) for b in range(B)])
    layer = ShiftableBilateral(3, 25.0, T, 43).cuda()
    x = _cuda(fs).requires_grad_(True)
    w = _cuda(np.random.default_rng(40).normal(size=(B, H, W)))
    (layer(x) * w).sum().backward()
    torch.cuda.synchronize()
    out, saved = bilateral_train(_cuda(fs), 3, 25.0, T, 43)
    gi, gs = bilateral_backward(_cuda(fs), w, 3, 25.0, T, 43, out=out, saved=saved)
    torch.cuda.synchronize()
    assert torch.equal(x.grad, gi) and float(layer.sigma_r.grad) == float(gs)
