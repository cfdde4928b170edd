"""Host-side checks of the C-ABI library (no GPU needed, no kernel launched):
the library loads and exports every call include/thin.h declares, argument
validation rejects bad calls, and the connectivity table the kernels index
agrees with the oracle's flood-fill characterisation for every mask."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1603_09180_amd import thin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thin.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(thin_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(thin.LIB_PATH):
        from paper_1603_09180_amd import build
        build.build()
    return thin.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert names == sorted(thin.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(thin.ThinError):
        thin._lib_saved = thin._lib
        try:
            thin._lib = None
            thin.load_library(str(tmp_path / "nope.so"))
        finally:
            thin._lib = thin._lib_saved


def test_null_context_and_bad_arguments(lib):
    st = thin.thin_stats()
    assert lib.thin_run(None, None, 4, 4, 1, 0, 0, ctypes.byref(st)) == thin.THIN_EINVAL
    assert lib.thin_run_batch(None, None, 0, None) == thin.THIN_EINVAL
    assert lib.thin_destroy(None) == thin.THIN_OK
    assert lib.thin_last_error(None) == b""
    h = ctypes.c_void_p()
    assert lib.thin_create(None, None) == thin.THIN_EINVAL
    cfg = thin.thin_config()
    cfg.engine = 7
    assert lib.thin_create(ctypes.byref(h), ctypes.byref(cfg)) == thin.THIN_EINVAL
    cfg = thin.thin_config()
    cfg.tile = 32            # tile without steps_per_round
    assert lib.thin_create(ctypes.byref(h), ctypes.byref(cfg)) == thin.THIN_EINVAL
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.thin_strerror(code)
    assert lib.thin_topology_table(2, 0, None, 512) == thin.THIN_EINVAL
    buf = (ctypes.c_uint32 * 512)()
    assert lib.thin_topology_table(0, 2, buf, 512) == thin.THIN_EINVAL
    assert lib.thin_skeleton(None, None, 4, 4, 1, 0, 0, ctypes.byref(st)) == thin.THIN_EINVAL


OWN_RING = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]


@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("adj", [0, 1])
def test_table_matches_oracle_characterisation(lib, adj, op):
    table = thin.thin_topology_table(adj, op)
    for mask in range(256):
        flags, comps = table[mask]
        # Patch: ring neighbour p is upper (200) when bit p is set, else a
        # distinct lower value 10 + p; the centre is 100.
        patch = np.full((3, 3), 0, np.int64)
        patch[1, 1] = 100
        for p, (di, dj) in enumerate(OWN_RING):
            patch[1 + di, 1 + dj] = 200 if (mask >> p) & 1 else 10 + p
        pt = oracle.classify_patch(patch, adj, 0)
        assert (flags & 1) == int(pt.destructible), mask
        # peak and end bits only in the skeleton's tables
        assert (flags >> 1) & 1 == (int(pt.peak) if op else 0), mask
        assert (flags >> 2) & 1 == (int(pt.end) if op else 0), mask
        assert flags & 0xF808 == 0, mask
        assert (flags >> 4) & 7 == pt.tminus, mask
        assert (flags >> 8) & 7 == pt.tplus, mask
        masks = [(comps >> (8 * c)) & 0xFF for c in range(4)]
        got = sorted(max(10 + p for p in range(8) if (m >> p) & 1) for m in masks[:pt.tminus])
        assert all(m == 0 for m in masks[pt.tminus:]), mask
        assert all(m & mask == 0 for m in masks), mask          # components lie in L
        assert got == sorted(pt.comp_max), mask


def test_table_destructible_bit_is_the_yokoi_number():
    """The table's destructible bit against a closed form: the
    Yokoi-Toriwaki-Fukumura connectivity number of the upper mask (over the
    ring's 4-neighbour positions, on L for (8,4), on U for (4,8)) equals 1
    exactly for the destructible masks."""
    for adj in (thin.THIN_ADJ_8_4, thin.THIN_ADJ_4_8):
        table = thin.thin_topology_table(adj)
        for m, (flags, _) in enumerate(table):
            b = [((m >> p) & 1) ^ (1 if adj == thin.THIN_ADJ_8_4 else 0) for p in range(8)]
            n = sum(b[k] - b[k] * b[(k + 1) % 8] * b[(k + 2) % 8] for k in (0, 2, 4, 6))
            assert (flags & 1) == (1 if n == 1 else 0), (adj, m)


@pytest.mark.parametrize("alpha", [0.3, 1.0, 2.5])
def test_gradient_coefficients_match_the_oracle(lib, alpha):
    """The library's float32 filter coefficients equal the oracle's
    float64 ones rounded to float32 (the gradient kernels and the oracle's
    float32 mode start from the same numbers)."""
    from oracle import deriche
    got = thin.thin_gradient_coefficients(alpha)
    co = deriche.coefficients(alpha)
    want = [float(np.float32(co[k])) for k in deriche.ORDER]
    assert got == want


def test_gradient_argument_checks(lib):
    out = (ctypes.c_float * 12)()
    assert lib.thin_gradient_coefficients(0.0, out, 12) == thin.THIN_EINVAL
    assert lib.thin_gradient_coefficients(1.0, out, 11) == thin.THIN_EINVAL
    assert lib.thin_gradient(None, None, 4, 4, 4, 1, 1.0, 1.0, None, 4, 1, None) == thin.THIN_EINVAL
