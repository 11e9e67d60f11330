"""Constant-time bilateral filtering with shiftable kernels on MI355X (gfx950).

K. N. Chaudhury, "Constant-time filtering using shiftable kernels": Algorithm 2
with a box spatial window (or the separable raised-cosine spatial kernel, and
Algorithm 1 as its range-free case) and the raised-cosine range kernel
cos^N(t / (sigma_r sqrt N)) or the polynomial one (1 - t^2 / (2 N sigma_r^2))^N, computed
by fused HIP kernels (libbsk.so) behind a
C ABI (include/bsk.h).  The torch-facing calls live in `filter`; importing this
package does not touch the GPU.
"""
from .filter import (BilateralFunction, ShiftableBilateral, autotune, autotune_batched,  # noqa: F401
                     batched_shape, bilateral, bilateral_backward, bilateral_batched, bilateral_train, nlm2,
                     order_for, plan_info, poly_order_for, poly_plan_info, release, spatial_filter,
                     spatial_sigma_for, tune_cache_clear, tune_cache_load, tune_cache_save)

__version__ = "0.1.0"
