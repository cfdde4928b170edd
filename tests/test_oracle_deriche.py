"""Pins for the gradient front-end oracle (oracle/deriche.py) against closed
forms that do not use its recursions: the impulse responses of the two
kernels written out, direct convolution with edge-replicated signals, the
unit sum and unit ramp response, separability, transposition, and the
float32 decision staying within rounding of the float64 reference."""
import math

import numpy as np
import pytest

from oracle import deriche
from paper_1603_09180_amd import synth

ALPHAS = [0.5, 1.0, 2.0]


def kernels(alpha, L):
    """f(n) and g(n) for |n| <= L, from their closed forms."""
    a = float(np.float32(alpha))
    r = math.exp(-a)
    n = np.arange(-L, L + 1, dtype=np.float64)
    k = (1 - r) ** 2 / (1 + 2 * a * r - r * r)
    c = (1 - r) ** 3 / (2 * r * (1 + r))
    return n, k * (a * np.abs(n) + 1) * r ** np.abs(n), -c * n * r ** np.abs(n)


def direct(x, kern, L):
    """Convolution sum_m kern(m) x(n - m) with x extended by its edge values."""
    xe = np.concatenate([np.full(L, x[0]), x, np.full(L, x[-1])]).astype(np.float64)
    out = np.zeros(len(x))
    for idx, m in enumerate(range(-L, L + 1)):
        out += kern[idx] * xe[L - m: L - m + len(x)]
    return out


@pytest.mark.parametrize("alpha", ALPHAS)
def test_impulse_responses(alpha):
    N = 301
    x = np.zeros(N)
    x[150] = 1.0
    n, f, g = kernels(alpha, 150)
    assert np.allclose(deriche.smooth_1d(x, alpha), f, rtol=0, atol=1e-13)
    assert np.allclose(deriche.deriv_1d(x, alpha), g, rtol=0, atol=1e-13)
    assert abs(f.sum() - 1) < 1e-12          # unit sum
    assert abs(-(g * n).sum() - 1) < 1e-12   # unit ramp response


@pytest.mark.parametrize("alpha", ALPHAS)
def test_constant_and_ramp(alpha):
    x = np.full(64, 37.0)
    assert np.allclose(deriche.smooth_1d(x, alpha), 37.0, rtol=0, atol=1e-11)
    assert np.allclose(deriche.deriv_1d(x, alpha), 0.0, rtol=0, atol=1e-11)
    ramp = np.arange(401, dtype=np.float64) * 3.0
    mid = slice(150, 251)
    assert np.allclose(deriche.deriv_1d(ramp, alpha)[mid], 3.0, rtol=0, atol=1e-9)
    assert np.allclose(deriche.smooth_1d(ramp, alpha)[mid], ramp[mid], rtol=0, atol=1e-9)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_recursions_equal_direct_convolution_with_replicated_edges(alpha):
    rng = np.random.default_rng(7)
    L = int(math.ceil(45 / float(np.float32(alpha))))
    n, f, g = kernels(alpha, L)
    for N in (1, 2, 3, 17, 100):
        x = rng.uniform(0, 255, size=N)
        assert np.allclose(deriche.smooth_1d(x, alpha), direct(x, f, L), rtol=0, atol=1e-9), N
        assert np.allclose(deriche.deriv_1d(x, alpha), direct(x, g, L), rtol=0, atol=1e-9), N


def test_gradient_is_separable_convolution():
    rng = np.random.default_rng(8)
    alpha = 1.0
    F = rng.integers(0, 256, size=(23, 31)).astype(np.uint8)
    L = 50
    n, f, g = kernels(alpha, L)
    A = np.stack([direct(F[:, j].astype(float), f, L) for j in range(F.shape[1])], axis=1)
    B = np.stack([direct(F[:, j].astype(float), g, L) for j in range(F.shape[1])], axis=1)
    gx = np.stack([direct(A[i], g, L) for i in range(F.shape[0])])
    gy = np.stack([direct(B[i], f, L) for i in range(F.shape[0])])
    ox, oy, om = deriche.gradient(F, alpha)
    assert np.allclose(ox, gx, rtol=0, atol=1e-9)
    assert np.allclose(oy, gy, rtol=0, atol=1e-9)
    assert np.allclose(om, np.hypot(gx, gy), rtol=0, atol=1e-9)


def test_transpose_swaps_components_and_columns_only_image():
    rng = np.random.default_rng(9)
    F = rng.integers(0, 256, size=(19, 27)).astype(np.float64)
    gx, gy, m = deriche.gradient(F, 0.8)
    tx, ty, tm = deriche.gradient(F.T, 0.8)
    assert np.allclose(tx, gy.T, atol=1e-9) and np.allclose(ty, gx.T, atol=1e-9)
    # an image that varies along j only has no i-derivative
    G = np.tile(rng.uniform(0, 200, size=27), (19, 1))
    gx, gy, m = deriche.gradient(G, 0.8)
    assert np.allclose(gy, 0.0, atol=1e-9)
    assert np.allclose(gx, np.tile(deriche.deriv_1d(G[0], 0.8), (19, 1)), atol=1e-9)


def test_float32_decision_close_to_float64():
    rng = np.random.default_rng(10)
    F = rng.integers(0, 256, size=(64, 80)).astype(np.uint8)
    _, _, m64 = deriche.gradient(F, 1.0)
    _, _, m32 = deriche.gradient(F, 1.0, np.float32)
    assert m32.dtype == np.float32
    assert np.max(np.abs(m32 - m64)) <= 1e-5 * np.max(m64)
    q = deriche.gradient_image(F, 1.0, 2.0)
    want = np.minimum(np.rint(m64 * 2.0), 255)
    # equal except where m64 * gain lies within float32 rounding of a half
    close = np.abs(np.abs(m64 * 2.0 - np.floor(m64 * 2.0)) - 0.5) < 1e-3
    assert np.all((q == want) | close)
    assert q.dtype == np.uint8
    q16 = deriche.gradient_image(F, 1.0, 600.0, np.uint16)
    assert q16.dtype == np.uint16 and q16.max() <= 65535


def test_quantize_rounds_half_to_even_and_clamps():
    m = np.array([0.0, 0.5, 1.5, 2.5, 254.4, 254.5, 300.0], np.float32)
    assert deriche.quantize(m, 1.0).tolist() == [0, 0, 2, 2, 254, 254, 255]


def test_quantize_reference_margins():
    """The float64 decision of D5 and its distance from the rounding
    boundaries, on hand-picked values (gain 1): rint halves go to even, the
    clamp at the top has no boundary."""
    mag = np.array([0.0, 0.2, 0.5, 1.5, 2.49, 254.6, 255.4, 255.5, 300.0])
    q, margin = deriche.quantize_reference(mag, 1.0, np.uint8)
    assert q.tolist() == [0, 0, 0, 2, 2, 255, 255, 255, 255]
    assert np.allclose(margin[:7], [0.5, 0.3, 0.0, 0.0, 0.01, 0.1, 0.1])
    assert margin[7] == 0.0 and np.isinf(margin[8])
    q16, _ = deriche.quantize_reference(np.array([70000.0, 12.5]), 1.0, np.uint16)
    assert q16.tolist() == [65535, 12]


def test_float32_decision_differs_only_near_boundaries():
    """The float32 gradient image differs from the float64 decision only
    where the float64 value sits within the stated tolerance of a rounding
    boundary (the bound the GPU test applies)."""
    F = synth.gen_blobs(120, 90, 3)
    _, _, m64 = deriche.gradient(F, 1.0)
    q32 = deriche.gradient_image(F, 1.0, 12.0)
    q64, margin = deriche.quantize_reference(m64, 12.0)
    scale = max(float(m64.max()), float(F.max()), 1.0)
    tol = 2e-5 * scale * 12.0 + 2.0 ** -23 * (m64 * 12.0 + 1.0)
    diff = q32.astype(int) - q64.astype(int)
    assert np.all((diff == 0) | (margin <= tol))
    assert np.abs(diff).max() <= 1
