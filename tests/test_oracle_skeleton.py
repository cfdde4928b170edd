"""Pins for the oracle's lambda-skeleton (section 2.2's algorithm box: lower a
point that is lambda-deletable and not lambda-end to alpha- until stability;
section 2.1 for peaks, end points and their lambda forms).

Expected values come from the definitions, worked out by hand for shapes
whose fate they fix, not from the oracle:

  * 3x3 characterisation over all 256 upper masks: a peak (T+ = 0) has no
    n-neighbour in Gamma+ and is never lambda-destructible (its lower set is
    one counted component); an end point has exactly one upper n-neighbour
    and T+ = 1; the contrast thresholds of the peak and lambda-end clauses;
  * a lone peak of contrast d disappears exactly when lambda >= d;
  * a one-pixel line (straight, diagonal, or with a diagonal spur, which
    leaves its end one upper 4-neighbour) of contrast d is kept whole when
    lambda < d (interior points are 2-divergent with both lower components at
    contrast d, ends are lambda-end points), and vanishes when lambda >= d;
    lambda-leveling instead erodes a straight line from its ends to one point;
  * a T whose branch has contrast <= lambda and whose bar stays above lambda
    against both the background and the branch loses exactly its branch;
  * a 1-pixel cross is stable at lambda = 0 (its centre's lower corners are
    not counted under (8,4), its arms are 2-divergent, its tips are ends);
  * any image whose frame holds its minimum b is flattened to b when lambda
    is at least its value range: the top-left pixel of a component of the
    highest level is always a peak, destructible or divergent;
  * lambda = 0 preserves the topology of every section (the operator lowers
    only destructible points then), the result is a fixed point, idempotent,
    pointwise lower, valued in the input's values, frame untouched;
  * lambda > 0: fixed point, complements of sections only merge;
  * value-map equivariance, any order inside a parity class, dirty = plain,
    and the paper's minimal-value queue order, as for lambda-leveling.
"""
import numpy as np
import pytest

import oracle
from oracle.sections import homotopic_sections, section_counts
from paper_1603_09180_amd import synth

ADJS = ["8,4", "4,8"]
SK = oracle.OP_SKELETON
LV = oracle.OP_LEVELING
N_MASK = {"8,4": 0xFF, "4,8": 0x55}   # ring positions (E, NE, N, ..., SE) that are n-neighbours


def _patch_from_mask(u, hi=9, lo=1, v=5):
    ring = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]
    assert oracle.ring_offsets() == ring
    P = np.full((3, 3), v, np.int64)
    for p, (di, dj) in enumerate(ring):
        P[1 + di, 1 + dj] = hi if (u >> p) & 1 else lo
    return P


@pytest.mark.parametrize("adj", ADJS)
def test_peak_and_end_over_all_masks(adj):
    for u in range(256):
        P = _patch_from_mask(u)              # contrast v - alpha- = 5 - 1 = 4 when u != 255
        pt = oracle.classify_patch(P, adj, 0)
        upper_n = bin(u & N_MASK[adj]).count("1")
        assert pt.peak == (upper_n == 0), u
        assert pt.end == (upper_n == 1), u
        if pt.peak:
            assert pt.tminus == 1 and not pt.lambda_destructible, u
        if pt.end:
            assert pt.tplus == 1, u
        for lam in (0, 3, 4, 9):
            q = oracle.classify_patch(P, adj, lam)
            contrast_ok = u != 255 and 4 <= lam
            assert q.lambda_end == (q.end and not contrast_ok), (u, lam)
            assert q.lambda_deletable == (q.lambda_destructible or (q.peak and contrast_ok))
            assert q.skeleton == (q.lambda_deletable and not q.lambda_end)


def _canvas(h=15, w=17, b=10):
    return np.full((h, w), b, np.int64)


@pytest.mark.parametrize("adj", ADJS)
def test_lone_peak(adj):
    F = _canvas()
    F[7, 8] = 10 + 6
    for lam in (0, 5):
        r = oracle.sweep(F, lam, adj, op=SK)
        assert np.array_equal(r.image, F) and (r.passes, r.lowerings) == (1, 0)
    for lam in (6, 100):
        r = oracle.sweep(F, lam, adj, op=SK)
        assert np.array_equal(r.image, _canvas()) and (r.passes, r.lowerings) == (2, 1)
    # Lambda-leveling never lowers a peak.
    r = oracle.sweep(F, 1000, adj, op=LV)
    assert np.array_equal(r.image, F)


def _lines():
    F = _canvas(20, 24)
    out = []
    G = F.copy()
    G[9, 4:19] = 40                        # horizontal
    out.append(("h", G))
    G = F.copy()
    G[3:17, 11] = 40                       # vertical
    out.append(("v", G))
    G = F.copy()
    for t in range(12):                    # diagonal (8-connected only)
        G[4 + t, 5 + t] = 40
    out.append(("d", G))
    G = F.copy()
    G[9, 4:19] = 40                        # horizontal with a diagonal spur at one end: under
    G[8, 3] = 40                           # (4,8) the end keeps one upper 4-neighbour
    out.append(("spur", G))
    return out


@pytest.mark.parametrize("adj", ADJS)
def test_line_kept_below_its_contrast(adj):
    for name, F in _lines():
        for lam in (0, 10, 29):
            r = oracle.sweep(F, lam, adj, op=SK)
            assert np.array_equal(r.image, F), (name, lam)
            assert (r.passes, r.lowerings) == (1, 0)


@pytest.mark.parametrize("adj", ADJS)
def test_line_vanishes_at_its_contrast(adj):
    for name, F in _lines():
        for lam in (30, 31, 500):
            r = oracle.sweep(F, lam, adj, op=SK)
            assert np.array_equal(r.image, np.full_like(F, 10)), (name, lam)
            assert r.lowerings == int((F == 40).sum())


@pytest.mark.parametrize("adj", ADJS)
def test_leveling_erodes_a_straight_line_to_one_point(adj):
    for name, F in _lines()[:2]:
        G = oracle.sweep(F, 29, adj, op=LV).image
        assert int((G == 40).sum()) == 1 and int((G == 10).sum()) == F.size - 1, name
        assert F[G == 40].item() == 40


@pytest.mark.parametrize("adj", ADJS)
def test_t_junction_loses_its_low_branch(adj):
    b, D, d, lam = 10, 110, 30, 30         # branch contrast d <= lam < D - d < D
    F = _canvas(20, 21, b)
    F[5, 3:18] = b + D                      # bar
    F[6:15, 10] = b + d                     # branch hanging from the bar's middle
    want = _canvas(20, 21, b)
    want[5, 3:18] = b + D
    r = oracle.sweep(F, lam, adj, op=SK)
    assert np.array_equal(r.image, want)
    assert r.lowerings == 9
    # With lambda below the branch's contrast the whole T is kept.
    r = oracle.sweep(F, d - 1, adj, op=SK)
    assert np.array_equal(r.image, F)


def test_cross_is_stable_at_lambda0():
    F = _canvas(17, 17, 0)
    F[8, 2:15] = 200
    F[2:15, 8] = 200
    r = oracle.sweep(F, 0, "8,4", op=SK)
    assert np.array_equal(r.image, F) and r.lowerings == 0
    # lambda-leveling erodes the arms back to one pixel
    G = oracle.sweep(F, 0, "8,4", op=LV).image
    assert int((G == 200).sum()) == 1


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
def test_flattens_when_lambda_covers_the_range(adj):
    rng = np.random.default_rng(5)
    for F in _small_images(91, 80, max_side=18, levels=9):
        b = int(F.min())
        F = F.copy()
        F[0, :] = F[-1, :] = F[:, 0] = F[:, -1] = b
        rng_range = int(F.max()) - b
        lam = rng_range + int(rng.integers(0, 3))
        r = oracle.sweep(F, lam, adj, op=SK)
        assert np.all(r.image == b), F.tolist()


@pytest.mark.parametrize("adj", ADJS)
def test_lambda0_preserves_topology(adj):
    for F in _small_images(101 if adj == "8,4" else 102, 120):
        r = oracle.sweep(F, 0, adj, op=SK)
        G = r.image.astype(np.int64)
        assert homotopic_sections(F, G, adj), F.tolist()
        assert oracle.count_lowerable(G, 0, adj, op=SK) == 0
        assert np.all(G <= F)
        assert set(np.unique(G)) <= set(np.unique(F))
        assert np.array_equal(_frame(G), _frame(F))
        again = oracle.sweep(G, 0, adj, op=SK)
        assert np.array_equal(again.image, G) and again.passes == 1 and again.lowerings == 0


@pytest.mark.parametrize("adj", ADJS)
@pytest.mark.parametrize("lam", [1, 2, 3, 10])
def test_lambda_positive_invariants(adj, lam):
    for F in _small_images(111 + lam, 60):
        G = oracle.sweep(F, lam, adj, op=SK).image.astype(np.int64)
        assert oracle.count_lowerable(G, lam, adj, op=SK) == 0
        assert np.all(G <= F)
        assert set(np.unique(G)) <= set(np.unique(F))
        assert np.array_equal(_frame(G), _frame(F))
        levels = sorted(set(np.unique(F).tolist()) | {int(F.max()) + 1})
        cf = section_counts(F, adj, levels)
        cg = section_counts(G, adj, levels)
        for k in levels:
            assert cg[k][1] <= cf[k][1], (k, F.tolist())   # complements only merge


@pytest.mark.parametrize("adj", ADJS)
def test_equivariance(adj):
    rng = np.random.default_rng(121)
    for F in _small_images(122, 40, levels=8):
        for lam in (0, 3):
            a = oracle.sweep(F, lam, adj, op=SK)
            b = oracle.sweep(F + 1000, lam, adj, op=SK)
            assert np.array_equal(b.image, a.image + 1000)
            assert (a.passes, a.lowerings) == (b.passes, b.lowerings)
        g = np.cumsum(rng.integers(1, 50, size=int(F.max()) + 1))   # strictly increasing
        a = oracle.sweep(F, 0, adj, op=SK)
        b = oracle.sweep(g[F], 0, adj, op=SK)
        assert np.array_equal(b.image, g[a.image])
    for seed in range(4):
        F = synth.gen_blobs(24, 31, 130 + seed)
        for lam in (0, 5, 20):
            a = oracle.sweep(F, lam, adj, op=SK)
            b = oracle.sweep(F.astype(np.uint16) * 257, lam * 257, adj, op=SK)
            assert np.array_equal(b.image, a.image.astype(np.uint16) * 257)
            assert (a.passes, a.lowerings) == (b.passes, b.lowerings)


@pytest.mark.parametrize("adj", ADJS)
def test_order_dirty_and_queue(adj):
    rng = np.random.default_rng(141)
    for F in _small_images(142, 60, max_side=20):
        for lam in (0, 2, 7):
            a = oracle.sweep(F, lam, adj, op=SK)
            b = oracle.sweep_ordered(F, lam, adj, rng.permutation(F.size), op=SK)
            c = oracle.sweep_dirty(F, lam, adj, op=SK)
            assert np.array_equal(a.image, b.image) and np.array_equal(a.image, c.image)
            assert (a.passes, a.lowerings) == (b.passes, b.lowerings) == (c.passes, c.lowerings)
        q = oracle.queue(F, 0, adj, op=SK).image.astype(np.int64)
        assert homotopic_sections(F, q, adj)
        assert oracle.count_lowerable(q, 0, adj, op=SK) == 0


def test_workload_dirty_equals_plain():
    job = synth.ridges_512()
    F = job.image()[:160, :200]
    a = oracle.sweep(F, 10, job.adj, op=SK)
    b = oracle.sweep_dirty(F, 10, job.adj, op=SK)
    assert np.array_equal(a.image, b.image) and (a.passes, a.lowerings) == (b.passes, b.lowerings)
    assert a.lowerings > 0
