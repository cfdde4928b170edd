"""Brute-force topology of threshold sections (test infrastructure only).

For an image F and adjacency pair (n, n') the section F_k = {x : F(x) >= k} is
labelled with n-adjacency and its complement with n'-adjacency (section 2.1 of
the paper).  Labelling uses scipy.ndimage.label on the whole image domain; it
shares nothing with the oracle's ring flood fill, so it can check what the
oracle's local predicates claim about global topology.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

_S8 = np.ones((3, 3), dtype=bool)
_S4 = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], dtype=bool)


def _structs(adj):
    if adj in (0, "8,4", (8, 4)):
        return _S8, _S4
    if adj in (1, "4,8", (4, 8)):
        return _S4, _S8
    raise ValueError(adj)


def section_labels(F, k, adj):
    """(labels of F_k under n, count, labels of complement under n', count)."""
    sn, sbar = _structs(adj)
    sec = np.asarray(F) >= k
    lab, nlab = ndimage.label(sec, structure=sn)
    labc, nlabc = ndimage.label(~sec, structure=sbar)
    return lab, nlab, labc, nlabc


def section_counts(F, adj, levels=None):
    """{k: (#C_n(F_k), #C_n'(complement of F_k))} for every relevant level.

    Counts can change only at levels k that are values of F (plus one past
    the maximum), so those are enough; `levels` overrides the set."""
    F = np.asarray(F)
    if levels is None:
        vals = np.unique(F)
        levels = list(vals.tolist()) + [int(vals.max()) + 1] if vals.size else []
    out = {}
    for k in levels:
        _, n1, _, n2 = section_labels(F, k, adj)
        out[int(k)] = (n1, n2)
    return out


def homotopic_sections(F, G, adj):
    """True when G <= F and, at every level k, the inclusion G_k in F_k maps
    the components of G_k one-to-one onto those of F_k, and the inclusion of
    the complement of F_k in the complement of G_k maps components one-to-one
    onto the complement components of G_k.  Levels are all values of F and G."""
    F = np.asarray(F).astype(np.int64)
    G = np.asarray(G).astype(np.int64)
    if F.shape != G.shape or np.any(G > F):
        return False
    levels = np.union1d(np.unique(F), np.unique(G))
    levels = list(levels.tolist()) + [int(max(F.max(), G.max())) + 1]
    for k in levels:
        lf, nf, lfc, nfc = section_labels(F, k, adj)
        lg, ng, lgc, ngc = section_labels(G, k, adj)
        if nf != ng or nfc != ngc:
            return False
        # G_k is inside F_k: each G component lies in one F component; the
        # map must be a bijection.
        if ng:
            pairs = np.unique(np.stack([lg[lg > 0], lf[lg > 0]]), axis=1)
            if pairs.shape[1] != ng or np.unique(pairs[1]).size != nf:
                return False
        # complement of F_k is inside complement of G_k.
        if nfc:
            pairs = np.unique(np.stack([lfc[lfc > 0], lgc[lfc > 0]]), axis=1)
            if pairs.shape[1] != nfc or np.unique(pairs[1]).size != ngc:
                return False
    return True
