"""Pins for the oracle's whole loop (lower lambda-destructible points until
stability, sections 2.1-2.2), checked against what the method fixes rather
than against the oracle itself:

  * lambda = 0: every threshold section and its complement keep their
    components one-to-one (the operator preserves topology), no destructible
    point remains, the result is idempotent, pointwise lower, takes only
    values of the input, and the read-only frame is kept;
  * lambda > 0: no lambda-destructible point remains, sections may split but
    never lose a component, complement components may only merge;
  * value-map equivariance (shift, strictly increasing maps at lambda = 0,
    the u8 -> u16 scaling by 257);
  * the binary special case: a simply connected set thins to one point;
  * lowering one parity class in any order equals raster order (the
    argument that makes the sweep deterministic);
  * the dirty-pixel variant and the paper's minimal-value queue order.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle.sections import homotopic_sections, section_counts
from paper_1603_09180_amd import synth

ADJS = ["8,4", "4,8"]


def _small_images(seed, n, max_side=14, levels=6):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        h = int(rng.integers(3, max_side + 1))
        w = int(rng.integers(3, max_side + 1))
        if rng.random() < 0.5:
            F = rng.integers(0, levels, size=(h, w))
        else:
            F = synth.gen_blobs(h, w, int(rng.integers(1 << 30)), nblobs=3, sigma=(1.0, 4.0),
                                noise=8.0).astype(np.int64) // 32
        yield F.astype(np.int64)


def _frame(F):
    return np.concatenate([F[0], F[-1], F[:, 0], F[:, -1]])


@pytest.mark.parametrize("adj", ADJS)
def test_lambda0_preserves_topology(adj):
    for F in _small_images(21 if adj == "8,4" else 22, 120):
        r = oracle.sweep(F, 0, adj)
        G = r.image.astype(np.int64)
        assert homotopic_sections(F, G, adj), F.tolist()
        assert oracle.count_destructible(G, 0, adj) == (0, 0)
        assert np.all(G <= F)
        assert set(np.unique(G)) <= set(np.unique(F))
        assert np.array_equal(_frame(G), _frame(F))
        again = oracle.sweep(G, 0, adj)
        assert np.array_equal(again.image, G) and again.passes == 1 and again.lowerings == 0


@pytest.mark.parametrize("adj", ADJS)
@pytest.mark.parametrize("lam", [1, 2, 3, 10])
def test_lambda_positive_invariants(adj, lam):
    for F in _small_images(31 + lam, 60):
        r = oracle.sweep(F, lam, adj)
        G = r.image.astype(np.int64)
        ld, _ = oracle.count_destructible(G, lam, adj)
        assert ld == 0
        assert np.all(G <= F)
        assert set(np.unique(G)) <= set(np.unique(F))
        assert np.array_equal(_frame(G), _frame(F))
        levels = sorted(set(np.unique(F).tolist()) | {int(F.max()) + 1})
        cf = section_counts(F, adj, levels)
        cg = section_counts(G, adj, levels)
        for k in levels:
            assert cg[k][0] >= cf[k][0], (k, F.tolist())   # sections split, never vanish
            assert cg[k][1] <= cf[k][1], (k, F.tolist())   # complements only merge


@pytest.mark.parametrize("adj", ADJS)
def test_shift_equivariance(adj):
    for F in _small_images(41, 40):
        for lam in (0, 3):
            a = oracle.sweep(F, lam, adj)
            b = oracle.sweep(F + 1000, lam, adj)
            assert np.array_equal(b.image, a.image + 1000)
            assert (a.passes, a.lowerings) == (b.passes, b.lowerings)


@pytest.mark.parametrize("adj", ADJS)
def test_increasing_map_equivariance_lambda0(adj):
    rng = np.random.default_rng(42)
    for F in _small_images(43, 40, levels=8):
        g = np.cumsum(rng.integers(1, 50, size=int(F.max()) + 1))   # strictly increasing
        a = oracle.sweep(F, 0, adj)
        b = oracle.sweep(g[F], 0, adj)
        assert np.array_equal(b.image, g[a.image])
        assert (a.passes, a.lowerings) == (b.passes, b.lowerings)


@pytest.mark.parametrize("adj", ADJS)
def test_u8_to_u16_scaling(adj):
    for seed in range(6):
        F = synth.gen_blobs(24, 31, 100 + seed)
        for lam in (0, 5, 20):
            a = oracle.sweep(F, lam, adj)
            b = oracle.sweep(F.astype(np.uint16) * 257, lam * 257, adj)
            assert b.image.dtype == np.uint16
            assert np.array_equal(b.image, a.image.astype(np.uint16) * 257)
            assert (a.passes, a.lowerings) == (b.passes, b.lowerings)


def _simply_connected_set(rng, h, w):
    """A random 8-connected set with a 4-connected complement, away from the
    image frame (binary thinning's textbook input)."""
    while True:
        f = ndimage.gaussian_filter(rng.standard_normal((h, w)), sigma=rng.uniform(1.0, 2.5))
        X = f > np.quantile(f, rng.uniform(0.4, 0.8))
        X[0, :] = X[-1, :] = X[:, 0] = X[:, -1] = False
        X[1, :] = X[-2, :] = X[:, 1] = X[:, -2] = False
        lab, n = ndimage.label(X, structure=np.ones((3, 3)))
        if n == 0:
            continue
        sizes = ndimage.sum(np.ones_like(lab), lab, index=range(1, n + 1))
        X = lab == (1 + int(np.argmax(sizes)))
        X = ndimage.binary_fill_holes(X, structure=np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]]))
        _, nc = ndimage.label(~X, structure=np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]]))
        _, nx = ndimage.label(X, structure=np.ones((3, 3)))
        if nx == 1 and nc == 1 and X.sum() >= 2:
            return X


def test_binary_simply_connected_thins_to_one_point():
    """A finite simply connected set with more than one point always has a
    simple point, so lambda = 0 thinning of F in {0, M} stops at one point."""
    rng = np.random.default_rng(51)
    for _ in range(40):
        X = _simply_connected_set(rng, int(rng.integers(8, 30)), int(rng.integers(8, 30)))
        F = X.astype(np.int64) * 200
        r = oracle.sweep(F, 0, "8,4")
        assert int((r.image == 200).sum()) == 1
        assert int((r.image > 0).sum()) == 1


def test_binary_set_with_holes_keeps_them():
    X = np.zeros((16, 16), bool)
    X[3:13, 3:13] = True
    X[5:7, 5:7] = False
    X[9:11, 8:11] = False
    F = X.astype(np.int64) * 9
    G = oracle.sweep(F, 0, "8,4").image
    _, nx = ndimage.label(G > 0, structure=np.ones((3, 3)))
    _, nc = ndimage.label(G == 0, structure=np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]]))
    assert nx == 1 and nc == 3
    assert oracle.count_destructible(G, 0, "8,4") == (0, 0)


@pytest.mark.parametrize("adj", ADJS)
def test_any_order_within_a_parity_class(adj):
    rng = np.random.default_rng(61)
    for F in _small_images(62, 30, max_side=20):
        for lam in (0, 4):
            a = oracle.sweep(F, lam, adj)
            b = oracle.sweep_ordered(F, lam, adj, rng.permutation(F.size))
            assert np.array_equal(a.image, b.image)
            assert (a.passes, a.lowerings) == (b.passes, b.lowerings)


@pytest.mark.parametrize("adj", ADJS)
def test_dirty_equals_plain(adj):
    for F in _small_images(71, 150, max_side=24):
        for lam in (0, 2, 7):
            a = oracle.sweep(F, lam, adj)
            b = oracle.sweep_dirty(F, lam, adj)
            assert np.array_equal(a.image, b.image)
            assert (a.passes, a.lowerings) == (b.passes, b.lowerings)
            assert b.examinations <= (F.shape[0] - 2) * (F.shape[1] - 2) * a.passes


def test_dirty_equals_plain_ten_thousand_images():
    """10^4 seeded small images, each with its own lambda (0..40) and
    pairing: the dirty-pixel sweep gives the plain sweep's image, passes and
    lowerings, and never examines more than the plain sweep does."""
    rng = np.random.default_rng(2026)
    for k, F in enumerate(_small_images(91, 10_000, max_side=18, levels=12)):
        lam = int(rng.integers(0, 41))
        adj = ADJS[k & 1]
        a = oracle.sweep(F, lam, adj)
        b = oracle.sweep_dirty(F, lam, adj)
        assert np.array_equal(a.image, b.image), k
        assert (a.passes, a.lowerings) == (b.passes, b.lowerings), k
        assert b.examinations <= (F.shape[0] - 2) * (F.shape[1] - 2) * a.passes


def test_dirty_equals_plain_on_workloads():
    """The two sweeps agree on the single-image workloads: the 128x128 blob
    image (lambda 0) directly, and the 512x512 ridge image (lambda 20) through
    the stored digest of the dirty sweep's result (the plain sweep takes
    about half a minute there)."""
    import hashlib
    import json
    import os

    job = synth.blobs_128()
    F = job.image()
    a = oracle.sweep(F, job.lam, job.adj)
    b = oracle.sweep_dirty(F, job.lam, job.adj)
    assert np.array_equal(a.image, b.image)
    assert (a.passes, a.lowerings) == (b.passes, b.lowerings)
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "full_size.json")))["ridges_512"]
    job = synth.ridges_512()
    F = job.image()
    if hashlib.sha256(F.tobytes()).hexdigest() != g["input_sha256"]:
        pytest.skip("the generator does not reproduce the stored ridge image here")
    a = oracle.sweep(F, job.lam, job.adj)
    assert hashlib.sha256(np.ascontiguousarray(a.image).tobytes()).hexdigest() == g["output_sha256"]
    assert (a.passes, a.lowerings) == (g["passes"], g["lowerings"])


@pytest.mark.parametrize("adj", ADJS)
def test_queue_order_invariants(adj):
    """The paper's own order (section 2.2: lower a point of minimal value,
    re-examine its eight neighbours) reaches a different but equally valid
    fixed point; compare invariants, not pixels."""
    for F in _small_images(81, 60):
        q = oracle.queue(F, 0, adj)
        G = q.image.astype(np.int64)
        assert homotopic_sections(F, G, adj)
        assert oracle.count_destructible(G, 0, adj) == (0, 0)
        s = oracle.sweep(F, 0, adj)
        levels = sorted(section_counts(F, adj))
        # Both orders keep the section counts of F at every level.
        assert section_counts(G, adj, levels) == section_counts(F, adj, levels)
        assert section_counts(s.image, adj, levels) == section_counts(F, adj, levels)
        for lam in (3,):
            q = oracle.queue(F, lam, adj)
            assert oracle.count_destructible(q.image, lam, adj)[0] == 0
            assert np.all(q.image <= F)


def test_pass_count_convention():
    F = np.full((6, 7), 3, np.int64)
    r = oracle.sweep(F, 0)
    assert (r.passes, r.lowerings) == (1, 0)
    # One line end to remove at a time: a 1-pixel bright segment shrinks.
    F = np.zeros((5, 9), np.int64)
    F[2, 2:7] = 9
    r = oracle.sweep(F, 0)
    assert int((r.image == 9).sum()) == 1 and r.passes >= 2
    assert r.lowerings == 4


@pytest.mark.parametrize("shape", [(0, 0), (1, 5), (2, 9), (7, 2), (3, 1)])
def test_degenerate_sizes_unchanged(shape):
    F = np.arange(int(np.prod(shape)), dtype=np.int64).reshape(shape) % 7
    r = oracle.sweep(F, 0)
    assert np.array_equal(r.image, F) and r.passes == 0 and r.lowerings == 0
    r = oracle.sweep_dirty(F, 0)
    assert np.array_equal(r.image, F) and r.passes == 0


def test_pass_cap_and_resume():
    """The state after a whole pass is a complete checkpoint: stopping at a
    pass cap and running again gives the uncapped result."""
    F = synth.gen_blobs(40, 40, 9)
    full = oracle.sweep(F, 0)
    assert full.passes > 4
    part = oracle.sweep(F, 0, max_passes=3)
    assert part.limited and part.passes == 3
    rest = oracle.sweep(part.image, 0)
    assert np.array_equal(rest.image, full.image)
    assert part.lowerings + rest.lowerings == full.lowerings
    assert part.passes + rest.passes == full.passes
    exact = oracle.sweep(F, 0, max_passes=full.passes)
    assert not exact.limited and np.array_equal(exact.image, full.image)
