"""GPU parity of the gradient front-end (the Deriche gradient the paper thins
in Fig. 1) and of the whole front-end + lambda-skeleton pipeline, through the
C ABI, against the float64 oracle only.

The float32 magnitude must stay within the tolerance derived below of the
float64 reference.  The stored u8/u16 gradient must equal the float64
decision min(top, rint(magnitude * gain)) everywhere except where the
float64 value lies within that tolerance (times the gain) of a rounding
boundary: there a float32 computation may legitimately land on the other
side, by one level, and such pixels are counted and reported.  The
pipeline's thinned image must equal the oracle's skeleton of the GPU's own
gradient image, so the thinning parity does not depend on how the gradient
was rounded.

Tolerance against float64: each of the four recursions (two per pass) rounds
about 8 times per sample and its feedback part amplifies an error at most
1 / (1 - r)^2 (sum of |impulse response| of the poles at r); with alpha >=
0.5 that is <= 6.5, so 4 * 8 * 6.5 * 2^-24 * (signal scale) stays below
2e-5 of the largest magnitude (plus the same of the input range for
near-zero magnitudes).  The product by the gain adds one float32 rounding
(2^-24 relative) to the stored value's error.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import deriche
from paper_1603_09180_amd import synth, thin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_gradient(F, alpha, gain, out_dtype):
    src = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    tdt = torch.uint8 if out_dtype == np.uint8 else torch.uint16
    dst = torch.empty(F.shape, dtype=tdt, device="cuda")
    mag = torch.empty(F.shape, dtype=torch.float32, device="cuda")
    with thin.Context() as ctx:
        ctx.gradient(src, dst, alpha, gain, magnitude=mag)
    torch.cuda.synchronize()
    return dst.cpu().numpy(), mag.cpu().numpy()


TOL = 2e-5


def check_quantized(got, m64, gain, out_dtype, tol_mag):
    """The stored gradient against the float64 decision; returns the number
    of pixels that sit within the tolerance of a rounding boundary and
    differ from it (by one level)."""
    q64, margin = deriche.quantize_reference(m64, gain, out_dtype)
    tol_q = tol_mag * gain + 2.0 ** -23 * (np.abs(m64) * gain + 1.0)
    diff = got.astype(np.int64) - q64.astype(np.int64)
    off = np.argwhere((diff != 0) & (margin > tol_q))
    assert off.size == 0, (f"{len(off)} stored values differ from the float64 decision away from "
                           f"a rounding boundary, first {off[:4].tolist()}")
    assert np.abs(diff).max(initial=0) <= 1
    return int(np.count_nonzero(diff))


def check(F, alpha, gain, out_dtype):
    got, mag = gpu_gradient(F, alpha, gain, out_dtype)
    _, _, m64 = deriche.gradient(F, alpha)
    scale = max(float(np.max(m64)) if m64.size else 0.0, float(np.max(F)) if F.size else 0.0, 1.0)
    err = np.max(np.abs(mag.astype(np.float64) - m64), initial=0.0)
    assert err <= TOL * scale, f"float magnitude off by {err} (scale {scale})"
    flips = check_quantized(got, m64, gain, out_dtype, TOL * scale)
    if flips:
        say(f"  {flips} of {got.size} stored values sit within the tolerance of a rounding "
            "boundary and took the other side")
    return flips


CASES = [((1, 1), np.uint8), ((1, 9), np.uint8), ((9, 1), np.uint16), ((2, 2), np.uint8),
         ((3, 5), np.uint16), ((64, 80), np.uint8), ((200, 131), np.uint16), ((257, 300), np.uint8),
         ((512, 512), np.uint8),
         # lines longer than the segmented passes take (1024 samples) run one
         # chain per thread; 1024 itself is 16 full segments
         ((1500, 40), np.uint8), ((30, 1300), np.uint16), ((1024, 65), np.uint8),
         ((65, 1025), np.uint8)]


@pytest.mark.parametrize("shape,dt", CASES, ids=lambda c: str(c))
@pytest.mark.parametrize("alpha", [0.5, 1.0, 2.0])
def test_matches_oracle(shape, dt, alpha):
    F = synth.gen_blobs(shape[0], shape[1], 31 + shape[0], dt)
    gain = 12.0 if dt == np.uint8 else 12.0 / 257.0   # the same scale for both input types
    say("case gradient", shape, np.dtype(dt).name, alpha)
    check(F, alpha, gain, np.uint8)
    check(F, alpha, gain * 200.0, np.uint16)


def test_pitched_views_and_in_place():
    big = synth.gen_blobs(90, 160, 5)
    F = big[:, 20:140].copy()
    src_big = torch.from_numpy(big.copy()).cuda()
    dst_big = torch.zeros((90, 200), dtype=torch.uint8, device="cuda")
    say("case gradient pitched")
    with thin.Context() as ctx:
        ctx.gradient(src_big[:, 20:140], dst_big[:, 30:150], 1.0, 12.0)
        torch.cuda.synchronize()
        out = dst_big.cpu().numpy()
        _, _, m64 = deriche.gradient(F, 1.0)
        scale = max(float(np.max(m64)), float(np.max(F)), 1.0)
        check_quantized(out[:, 30:150], m64, 12.0, np.uint8, TOL * scale)
        assert not out[:, :30].any() and not out[:, 150:].any()
        # a contiguous source gives the same bytes, and so does dst = src
        want, _ = gpu_gradient(F, 1.0, 12.0, np.uint8)
        assert np.array_equal(out[:, 30:150], want)
        t = torch.from_numpy(F.copy()).cuda()
        ctx.gradient(t, t, 1.0, 12.0)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), want)


def test_bad_arguments():
    t = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    with thin.Context() as ctx:
        for alpha, gain in ((0.0, 1.0), (-1.0, 1.0), (1.0, -1.0), (float("nan"), 1.0)):
            with pytest.raises(thin.ThinError):
                ctx.gradient(t, t, alpha, gain)
        ctx.gradient(t[:0], t[:0], 1.0, 1.0)       # empty: nothing to do


@pytest.mark.parametrize("adj", [0, 1])
def test_pipeline_gradient_then_skeleton(adj):
    """Fig. 1's pipeline: gradient of a gray image, then its lambda-skeleton
    (lambda = 10), all on the GPU.  The gradient is checked against the
    float64 oracle; the skeleton against the oracle's skeleton of the GPU's
    own gradient image."""
    F = synth.gen_blobs(300, 260, 77)
    say("case gradient pipeline adj", adj)
    src = torch.from_numpy(F).cuda()
    G = torch.empty_like(src)
    with thin.Context() as ctx:
        ctx.gradient(src, G, 1.0, 12.0)
        torch.cuda.synchronize()
        g_gpu = G.cpu().numpy()
        st = ctx.run(G, 10, adj, op="skeleton")
    torch.cuda.synchronize()
    _, _, m64 = deriche.gradient(F, 1.0)
    scale = max(float(np.max(m64)), float(np.max(F)), 1.0)
    check_quantized(g_gpu, m64, 12.0, np.uint8, TOL * scale)
    ref = oracle.sweep_dirty(g_gpu, 10, adj, op="skeleton")
    assert np.array_equal(G.cpu().numpy(), ref.image)
    assert (st.passes, st.lowerings) == (ref.passes, ref.lowerings)
    assert ref.lowerings > 0
