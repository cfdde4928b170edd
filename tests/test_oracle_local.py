"""Pins for the oracle's local (3x3) characterisation of a point.

Each test checks the oracle against something other than itself:
  * hand-worked neighbourhoods derived from the definitions of section 2.1
    (tests/golden/neighbourhoods.txt);
  * the Yokoi-Toriwaki-Fukumura connectivity numbers, a closed form for the
    binary connectivity numbers and simple points in 2-D;
  * global topology: lowering a point to alpha- keeps every threshold section
    and its complement homotopic exactly when the point is destructible
    (simple for F_k, section 2.1), checked by whole-image labelling;
  * the limits of the lambda clause (lambda = 0 and lambda above the value
    range), which do not depend on how the paper's F-(c) is read.
"""
import os

import numpy as np
import pytest

import oracle
from oracle.sections import homotopic_sections

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "neighbourhoods.txt")

# The test's own coordinates of the 8 neighbours, in the order E, NE, N, NW,
# W, SW, S, SE (row offset, column offset); rows grow downward.
OWN_RING = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]


def _load_golden():
    recs = []
    lines = [ln.rstrip("\n") for ln in open(GOLDEN)]
    i = 0
    while i < len(lines):
        ln = lines[i].split("#", 1)[0].strip()
        if not ln:
            i += 1
            continue
        head, vals = ln.split("|")
        name, adj, lam = head.split()
        tp, tm, d, ld, am = [int(v) for v in vals.split()]
        patch = np.array([[int(v) for v in lines[i + r].split()] for r in (1, 2, 3)])
        recs.append((name, adj, int(lam), tp, tm, bool(d), bool(ld), am, patch))
        i += 4
    return recs


GOLDEN_RECORDS = _load_golden()


def test_golden_file_parsed():
    assert len(GOLDEN_RECORDS) >= 20


@pytest.mark.parametrize("rec", GOLDEN_RECORDS, ids=lambda r: f"{r[0]}-{r[1]}-l{r[2]}")
def test_hand_worked_neighbourhoods(rec):
    name, adj, lam, tp, tm, d, ld, am, patch = rec
    pt = oracle.classify_patch(patch, adj, lam)
    assert (pt.tplus, pt.tminus) == (tp, tm)
    assert pt.destructible == d
    assert pt.lambda_destructible == ld
    assert pt.alpha_minus == am
    # The same decision through the whole-image path (the C code reads the 3x3
    # from image coordinates itself): a 3x3 image has one interior pixel.
    n_ld, n_d = oracle.count_destructible(patch, lam, adj)
    assert (n_ld, n_d) == (int(ld), int(d))
    # And one pass of the sweep lowers it to alpha- exactly when it is
    # lambda-destructible (later passes may lower it again).
    r = oracle.sweep(patch, lam, adj, max_passes=1)
    if ld:
        assert r.image[1, 1] == am and r.lowerings == 1
    else:
        assert np.array_equal(r.image, patch) and r.passes == 1 and r.lowerings == 0


def test_ring_is_the_eight_neighbours():
    offs = oracle.ring_offsets()
    assert sorted(offs) == sorted(OWN_RING)


# ---------------------------------------------------------------- Yokoi pins


def _bits(mask):
    return [(mask >> p) & 1 for p in range(8)]


def _yokoi_sum(b):
    """Sum over the 4-neighbours k of b_k - b_k b_{k+1} b_{k+2} (indices mod 8),
    in the order E, NE, N, ...; for b the set's bits this is the Yokoi
    4-connectivity number, for b the complement's bits the 8-number."""
    return sum(b[k] - b[k] * b[(k + 1) % 8] * b[(k + 2) % 8] for k in (0, 2, 4, 6))


def _closed_form(mask, adj):
    """(T+, T--, simple) of a binary neighbourhood, U = bits of `mask`,
    from the Yokoi sums and 2-D duality (degenerate cases by hand)."""
    u = _bits(mask)
    lo = [1 - v for v in u]
    evens_in_u = all(u[k] for k in (0, 2, 4, 6))
    evens_in_l = all(lo[k] for k in (0, 2, 4, 6))
    if adj == "8,4":
        # T-- = 4-components of L holding a 4-neighbour of x.
        tminus = 1 if mask == 0 else _yokoi_sum(lo)
        # T+ = 8-components of U: by duality the 4-gaps of L, except when U
        # holds every 4-neighbour (one component) or is empty.
        tplus = 0 if mask == 0 else (1 if evens_in_u else _yokoi_sum(lo))
        simple = _yokoi_sum(lo) == 1          # Yokoi 8-connectivity number = 1
    else:
        tplus = 1 if mask == 0xFF else _yokoi_sum(u)
        tminus = 0 if mask == 0xFF else (1 if evens_in_l else _yokoi_sum(u))
        simple = _yokoi_sum(u) == 1           # Yokoi 4-connectivity number = 1
    return tplus, tminus, simple


def _patch_from_mask(mask, inside=7, outside=2, centre=7):
    p = np.full((3, 3), outside, dtype=np.int64)
    p[1, 1] = centre
    for bit, (di, dj) in enumerate(OWN_RING):
        if (mask >> bit) & 1:
            p[1 + di, 1 + dj] = inside
    return p


@pytest.mark.parametrize("adj", ["8,4", "4,8"])
def test_yokoi_closed_form_all_masks(adj):
    n_simple = 0
    for mask in range(256):
        patch = _patch_from_mask(mask)
        tp, tm, simple = _closed_form(mask, adj)
        pt = oracle.classify_patch(patch, adj, 0)
        assert (pt.tplus, pt.tminus) == (tp, tm), (adj, mask)
        assert pt.destructible == simple, (adj, mask)
        _, n_d = oracle.count_destructible(patch, 0, adj)
        assert n_d == int(simple), (adj, mask)
        n_simple += simple
    # Complementing the neighbourhood and swapping (8,4) with (4,8) maps
    # simple configurations onto simple configurations.
    assert n_simple == sum(_closed_form(m ^ 0xFF, "4,8" if adj == "8,4" else "8,4")[2]
                           for m in range(256))


def test_divergent_points_keep_an_upper_component():
    """A k-divergent point (k >= 2) always has T+ >= 1 (by the 2-D duality
    T+ = T-- away from the degenerate cases), so lowering it never deletes a
    component of its section."""
    for adj in ("8,4", "4,8"):
        for mask in range(256):
            tp, tm, _ = _closed_form(mask, adj)
            pt = oracle.classify_patch(_patch_from_mask(mask), adj, 0)
            if pt.tminus >= 2:
                assert pt.tplus >= 1 and tp == pt.tplus


# ------------------------------------------------------- topology (global) pins


def _homotopy_cases(seed, n_images, shape=(6, 6), levels=4):
    rng = np.random.default_rng(seed)
    for _ in range(n_images):
        F = rng.integers(0, levels, size=shape).astype(np.int64)
        yield F


@pytest.mark.parametrize("adj", ["8,4", "4,8"])
def test_destructible_iff_lowering_preserves_section_topology(adj):
    """Section 2.1: x is destructible when it is simple for F_k, k = F(x);
    lowering a simple point to alpha- keeps the components of every section
    and of its complement (and 2-D non-simple points always change one)."""
    checked = 0
    seen = {True: 0, False: 0}
    for F in _homotopy_cases(11 if adj == "8,4" else 12, 140):
        h, w = F.shape
        for i in range(1, h - 1):
            for j in range(1, w - 1):
                pt = oracle.classify_patch(F[i - 1:i + 2, j - 1:j + 2], adj, 0)
                if pt.alpha_minus == F[i, j]:
                    continue  # no lower neighbour: lowering is the identity
                G = F.copy()
                G[i, j] = pt.alpha_minus
                keeps = homotopic_sections(F, G, adj)
                assert keeps == pt.destructible, (adj, F.tolist(), i, j)
                seen[keeps] += 1
                checked += 1
    assert checked > 1000 and seen[True] > 100 and seen[False] > 100


def test_lowering_below_alpha_minus_can_break_topology():
    """alpha- is the highest lower value: lowering a destructible point any
    further than alpha- can change a section's topology (here the point
    becomes a new complement component at level 5), so the target matters."""
    F = np.array([[9, 9, 9, 9, 9],
                  [9, 1, 9, 9, 9],
                  [9, 9, 9, 5, 9],
                  [9, 9, 9, 9, 9]], dtype=np.int64)
    # The centre (2, 2) has lower neighbour 5 only via (2, 3) and 1 via (1, 1).
    pt = oracle.classify_patch(F[1:4, 1:4], "8,4", 0)
    assert pt.alpha_minus == 5
    G = F.copy()
    G[2, 2] = pt.alpha_minus
    assert homotopic_sections(F, G, "8,4") == pt.destructible
    G2 = F.copy()
    G2[2, 2] = 1
    assert not homotopic_sections(F, G2, "8,4")


# ---------------------------------------------------------- lambda clause pins


@pytest.mark.parametrize("adj", ["8,4", "4,8"])
def test_lambda_zero_is_destructible(adj):
    rng = np.random.default_rng(5)
    for _ in range(3000):
        p = rng.integers(0, 6, size=(3, 3))
        pt = oracle.classify_patch(p, adj, 0)
        assert pt.lambda_destructible == pt.destructible


@pytest.mark.parametrize("adj", ["8,4", "4,8"])
def test_lambda_above_range_is_destructible_or_divergent(adj):
    """With lambda at or above every contrast, all k lower components
    qualify, so lambda-destructible <=> destructible or k >= 2."""
    rng = np.random.default_rng(6)
    for lam in (65535, 2**32 - 1):
        for _ in range(3000):
            p = rng.integers(0, 65536, size=(3, 3))
            if rng.random() < 0.5:
                p = rng.integers(0, 4, size=(3, 3)) * 20000
            pt = oracle.classify_patch(p, adj, lam)
            assert pt.lambda_destructible == (pt.destructible or pt.tminus >= 2)


@pytest.mark.parametrize("adj", ["8,4", "4,8"])
def test_lambda_monotone(adj):
    """More contrast allowed never makes a point less lambda-destructible."""
    rng = np.random.default_rng(7)
    for _ in range(2000):
        p = rng.integers(0, 40, size=(3, 3))
        prev = False
        for lam in (0, 1, 2, 3, 5, 8, 13, 21, 40):
            cur = oracle.classify_patch(p, adj, lam).lambda_destructible
            assert cur or not prev
            prev = cur


@pytest.mark.parametrize("adj", ["8,4", "4,8"])
def test_connectivity_numbers_by_labelling(adj):
    """T+ and T-- of every upper mask against scipy's labelling of the 3x3
    neighbourhood (components of the ring subset under n or n', counted when
    they hold a pixel n- or n'-adjacent to the centre; the centre itself
    belongs to neither set), a method independent of the oracle's ring
    flood fill.  The destructible masks are also counted: 116 per pairing."""
    from scipy import ndimage
    s8 = np.ones((3, 3), bool)
    s4 = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], bool)
    sn, sbar = (s8, s4) if adj == "8,4" else (s4, s8)
    near = {"n": sn.copy(), "nbar": sbar.copy()}
    for k in near.values():
        k[1, 1] = False
    ring = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]
    n_destr = 0
    for u in range(256):
        upper = np.zeros((3, 3), bool)
        for p, (di, dj) in enumerate(ring):
            upper[1 + di, 1 + dj] = bool((u >> p) & 1)
        lower = ~upper
        lower[1, 1] = False

        def counted(mask, struct, touch):
            lab, n = ndimage.label(mask, structure=struct)
            return len({int(lab[i, j]) for i in range(3) for j in range(3)
                        if touch[i, j] and lab[i, j] > 0})

        tplus = counted(upper, sn, near["n"])
        tminus = counted(lower, sbar, near["nbar"])
        patch = np.where(upper, 9, 1)
        patch[1, 1] = 5
        pt = oracle.classify_patch(patch, adj, 0)
        assert (pt.tplus, pt.tminus) == (tplus, tminus), u
        n_destr += tplus == 1 and tminus == 1
    assert n_destr == 116
