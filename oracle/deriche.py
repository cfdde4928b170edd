"""Oracle of the gradient front-end (test infrastructure only).

The paper's illustration (Fig. 1) thins a gradient image obtained with the
Deriche gradient operator; the operator itself is defined in Deriche's own
work, not in the paper, so this module restates the published recursive
filters with the readings below.  Only the test-suite and the benchmark's
CPU-baseline leg may import it; it shares no code with the HIP library.

Readings (none of them is fixed by the paper):
  D1  smoothing kernel f(n) = k (a|n| + 1) r^|n|, r = exp(-a), with k making
      sum_n f(n) = 1, i.e. k = (1 - r)^2 / (1 + 2 a r - r^2);
  D2  derivative kernel g(n) = -c n r^|n| with c making the response to the
      unit ramp x(n) = n equal 1, i.e. c = (1 - r)^3 / (2 r (1 + r));
  D3  separable 2-D gradient: gx = g along columns (j) of f along rows (i),
      gy = g along i of f along j; magnitude sqrt(gx^2 + gy^2);
  D4  signals are extended beyond the image by their edge values; the
      recursions start from the steady state of that constant extension;
  D5  the stored gradient is q = min(top, rint(magnitude * gain)) with
      rint rounding half to even, top = 255 (u8) or 65535 (u16); this
      decision is taken in float32, the kernel's precision.

Each 1-D filter is the sum of a causal and an anticausal second-order
recursion obtained from the z-transforms of the two halves of its kernel:
  f, causal:      y+(n) = a0 x(n) + a1 x(n-1) + b1 y+(n-1) + b2 y+(n-2)
  f, anticausal:  y-(n) = a2 x(n+1) + a3 x(n+2) + b1 y-(n+1) + b2 y-(n+2)
  g, causal:      y+(n) = d1 x(n-1) + b1 y+(n-1) + b2 y+(n-2)
  g, anticausal:  y-(n) = d2 x(n+1) + b1 y-(n+1) + b2 y-(n+2)
with a0 = k, a1 = k (a - 1) r, a2 = k (a + 1) r, a3 = -k r^2, d1 = -c r,
d2 = c r, b1 = 2 r, b2 = -r^2.  In float32 mode every product and sum is
rounded to float32 in the association order written above (left to right).
That mode serves the CPU baseline (the cost of the pipeline on the host);
no test takes it as a reference for the kernels, which compute short
columns in segments and so round differently: the tests hold them to the
float64 mode within a stated tolerance.
"""
from __future__ import annotations

import math

import numpy as np


def coefficients(alpha: float) -> dict:
    """Filter coefficients (float64) for smoothing parameter alpha > 0;
    alpha is first rounded to float32, the type the library takes."""
    a = float(np.float32(alpha))
    if not a > 0.0:
        raise ValueError("alpha must be positive")
    r = math.exp(-a)
    k = (1.0 - r) ** 2 / (1.0 + 2.0 * a * r - r * r)
    c = (1.0 - r) ** 3 / (2.0 * r * (1.0 + r))
    co = {"alpha": a, "r": r, "k": k, "c": c,
          "a0": k, "a1": k * (a - 1.0) * r, "a2": k * (a + 1.0) * r, "a3": -k * r * r,
          "d1": -c * r, "d2": c * r, "b1": 2.0 * r, "b2": -r * r}
    den = 1.0 - co["b1"] - co["b2"]
    # steady states of the four recursions for a constant input of 1
    co["s_plus"] = (co["a0"] + co["a1"]) / den
    co["s_minus"] = (co["a2"] + co["a3"]) / den
    co["d_plus"] = co["d1"] / den
    co["d_minus"] = co["d2"] / den
    return co


ORDER = ("a0", "a1", "a2", "a3", "d1", "d2", "b1", "b2", "s_plus", "s_minus", "d_plus",
         "d_minus")


def _cast(co, dt):
    return {k: dt(v) for k, v in co.items()}


def _filter(X, axis, co, dt, kind):
    """One 1-D filter (kind "smooth" or "deriv") along `axis` of a 2-D array,
    every line independently, in arithmetic type dt."""
    X = np.moveaxis(np.asarray(X, dtype=dt), axis, 0)
    n = X.shape[0]
    c = _cast(co, dt)
    out = np.empty_like(X)
    if n == 0:
        return np.moveaxis(out, 0, axis)
    # causal part, stored in out
    x_prev = X[0]
    if kind == "smooth":
        y1 = c["s_plus"] * X[0]
    else:
        y1 = c["d_plus"] * X[0]
    y2 = y1
    for i in range(n):
        if kind == "smooth":
            y = ((c["a0"] * X[i] + c["a1"] * x_prev) + c["b1"] * y1) + c["b2"] * y2
        else:
            y = (c["d1"] * x_prev + c["b1"] * y1) + c["b2"] * y2
        out[i] = y
        x_prev = X[i]
        y2, y1 = y1, y
    # anticausal part, added
    x1 = X[n - 1]
    x2 = X[n - 1]
    if kind == "smooth":
        y1 = c["s_minus"] * X[n - 1]
    else:
        y1 = c["d_minus"] * X[n - 1]
    y2 = y1
    for i in range(n - 1, -1, -1):
        if kind == "smooth":
            y = ((c["a2"] * x1 + c["a3"] * x2) + c["b1"] * y1) + c["b2"] * y2
        else:
            y = (c["d2"] * x1 + c["b1"] * y1) + c["b2"] * y2
        out[i] = out[i] + y
        x2, x1 = x1, X[i]
        y2, y1 = y1, y
    return np.moveaxis(out, 0, axis)


def smooth_1d(x, alpha, dtype=np.float64):
    """Smoothing filter f applied to a 1-D signal."""
    x = np.asarray(x)
    return _filter(x[:, None], 0, coefficients(alpha), dtype, "smooth")[:, 0]


def deriv_1d(x, alpha, dtype=np.float64):
    """Derivative filter g applied to a 1-D signal."""
    x = np.asarray(x)
    return _filter(x[:, None], 0, coefficients(alpha), dtype, "deriv")[:, 0]


def gradient(F, alpha, dtype=np.float64):
    """(gx, gy, magnitude) of image F (rows i, columns j) in arithmetic dt:
    A = f along i, B = g along i, then gx = g along j of A, gy = f along j
    of B (the order the kernels use)."""
    co = coefficients(alpha)
    F = np.asarray(F)
    A = _filter(F, 0, co, dtype, "smooth")
    B = _filter(F, 0, co, dtype, "deriv")
    gx = _filter(A, 1, co, dtype, "deriv")
    gy = _filter(B, 1, co, dtype, "smooth")
    mag = np.sqrt(gx * gx + gy * gy)
    return gx, gy, mag


def quantize(mag32, gain, out_dtype=np.uint8):
    """D5: min(top, rint(magnitude * gain)) in float32."""
    top = np.iinfo(out_dtype).max
    v = np.asarray(mag32, np.float32) * np.float32(gain)
    q = np.rint(v)
    return np.minimum(q, np.float32(top)).astype(out_dtype)


def quantize_reference(mag64, gain, out_dtype=np.uint8):
    """D5 in float64: (q, margin) with q = min(top, rint(magnitude * gain))
    and margin the distance of magnitude * gain from the nearest rounding
    boundary (a half-integer at or below top + 1/2; infinity where the value
    is clamped to top).  A stored value computed in lower precision may differ
    from q only where its error exceeds the margin."""
    top = np.iinfo(out_dtype).max
    v = np.asarray(mag64, np.float64) * float(gain)
    q = np.minimum(np.rint(v), float(top)).astype(out_dtype)
    margin = np.abs(v - np.floor(v) - 0.5)
    margin = np.where(v > top + 0.5, np.inf, margin)
    return q, margin


def gradient_image(F, alpha, gain, out_dtype=np.uint8):
    """The stored gradient image (float32 arithmetic, D5)."""
    _, _, mag = gradient(F, alpha, np.float32)
    return quantize(mag, gain, out_dtype)
