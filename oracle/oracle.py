"""ctypes wrapper around the C oracle (test infrastructure only).

Every function takes and returns numpy arrays; images of dtype uint8 or uint16
are widened to int32 for the C code (the paper's F maps pixels to integers,
section 2.1) and narrowed back on return.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

ADJ_8_4 = 0
ADJ_4_8 = 1

# Operators (section 2.2): the lambda-leveling type set (lambda-destructible
# points) and the lambda-skeleton's (lambda-deletable and not lambda-end).
OP_LEVELING = 0
OP_SKELETON = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "thin_oracle.c")
_LIB = os.path.join(_HERE, "libthin_oracle.so")

_OK, _EINVAL, _ENOMEM, _ELIMIT = 0, -1, -2, -4


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, one thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Point(ctypes.Structure):
    _fields_ = [
        ("tplus", ctypes.c_int32),
        ("tminus", ctypes.c_int32),
        ("destructible", ctypes.c_int32),
        ("lambda_destr", ctypes.c_int32),
        ("alpha_minus", ctypes.c_int64),
        ("comp_max", ctypes.c_int64 * 4),
        ("qualifying", ctypes.c_int32),
        ("peak", ctypes.c_int32),
        ("end", ctypes.c_int32),
        ("lambda_deletable", ctypes.c_int32),
        ("lambda_end", ctypes.c_int32),
        ("skeleton", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_classify.argtypes = [i64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.POINTER(_Point)]
        lib.oracle_classify.restype = None
        img = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32,
               ctypes.c_int32]  # F, h, w, lambda, adjacency, op
        lib.oracle_sweep.argtypes = img + [ctypes.c_uint64, u64p, u64p]
        lib.oracle_sweep.restype = ctypes.c_int
        lib.oracle_sweep_ordered.argtypes = img + [i64p, u64p, u64p]
        lib.oracle_sweep_ordered.restype = ctypes.c_int
        lib.oracle_sweep_dirty.argtypes = img + [u64p, u64p, u64p]
        lib.oracle_sweep_dirty.restype = ctypes.c_int
        lib.oracle_queue.argtypes = img + [u64p, u64p]
        lib.oracle_queue.restype = ctypes.c_int
        lib.oracle_count_lowerable.argtypes = img + [u64p]
        lib.oracle_count_lowerable.restype = ctypes.c_int
        lib.oracle_count_destructible.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.c_uint32, ctypes.c_int32, u64p, u64p]
        lib.oracle_count_destructible.restype = ctypes.c_int
        lib.oracle_ring_offsets.argtypes = [i32p, i32p]
        lib.oracle_ring_offsets.restype = None
        _lib = lib
    return _lib


def _adj_code(adj) -> int:
    if adj in (ADJ_8_4, "8,4", (8, 4)):
        return ADJ_8_4
    if adj in (ADJ_4_8, "4,8", (4, 8)):
        return ADJ_4_8
    raise ValueError(f"unknown adjacency {adj!r}")


def _op_code(op) -> int:
    if op in (OP_LEVELING, "leveling"):
        return OP_LEVELING
    if op in (OP_SKELETON, "skeleton"):
        return OP_SKELETON
    raise ValueError(f"unknown operator {op!r}")


def _widen(F: np.ndarray) -> np.ndarray:
    F = np.asarray(F)
    if F.ndim != 2:
        raise ValueError("image must be 2-D")
    return np.array(F, dtype=np.int32, order="C", copy=True)


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


@dataclass
class SweepResult:
    image: np.ndarray
    passes: int
    lowerings: int
    examinations: int | None = None
    limited: bool = False


@dataclass
class Point:
    tplus: int
    tminus: int
    destructible: bool
    lambda_destructible: bool
    alpha_minus: int
    comp_max: list
    qualifying: int
    peak: bool
    end: bool
    lambda_deletable: bool
    lambda_end: bool
    skeleton: bool


def ring_offsets():
    """The 8-ring order used by the oracle: E, NE, N, NW, W, SW, S, SE."""
    lib = _load()
    di = np.zeros(8, np.int32)
    dj = np.zeros(8, np.int32)
    lib.oracle_ring_offsets(_ptr(di, ctypes.c_int32), _ptr(dj, ctypes.c_int32))
    return list(zip(di.tolist(), dj.tolist()))


def classify(neighbours, centre: int, adj=ADJ_8_4, lam: int = 0) -> Point:
    """Characterise a point from its 8 neighbour values (ring order E..SE)."""
    lib = _load()
    nb = np.ascontiguousarray(np.asarray(neighbours, dtype=np.int64).reshape(8))
    out = _Point()
    lib.oracle_classify(_ptr(nb, ctypes.c_int64), int(centre), _adj_code(adj),
                        ctypes.c_uint32(int(lam)), ctypes.byref(out))
    k = out.tminus
    return Point(out.tplus, out.tminus, bool(out.destructible), bool(out.lambda_destr),
                 int(out.alpha_minus), [int(out.comp_max[i]) for i in range(min(k, 4))],
                 out.qualifying, bool(out.peak), bool(out.end), bool(out.lambda_deletable),
                 bool(out.lambda_end), bool(out.skeleton))


def classify_patch(patch, adj=ADJ_8_4, lam: int = 0) -> Point:
    """Characterise the centre of a 3x3 array."""
    p = np.asarray(patch)
    nb = [p[1 + di, 1 + dj] for di, dj in ring_offsets()]
    return classify(nb, int(p[1, 1]), adj, lam)


def _check(rc: int, what: str):
    if rc == _EINVAL:
        raise OracleError(f"{what}: invalid argument")
    if rc == _ENOMEM:
        raise OracleError(f"{what}: out of memory")


def sweep(F, lam: int, adj=ADJ_8_4, max_passes: int = 0, op=OP_LEVELING) -> SweepResult:
    """ORACLE-SWEEP: four parity classes per pass, raster order, to stability."""
    lib = _load()
    src = np.asarray(F)
    a = _widen(src)
    p = ctypes.c_uint64()
    lo = ctypes.c_uint64()
    rc = lib.oracle_sweep(_ptr(a, ctypes.c_int32), a.shape[0], a.shape[1],
                          ctypes.c_uint32(int(lam)), _adj_code(adj), _op_code(op), max_passes,
                          ctypes.byref(p), ctypes.byref(lo))
    _check(rc, "oracle_sweep")
    return SweepResult(a.astype(src.dtype, copy=False), p.value, lo.value,
                       limited=(rc == _ELIMIT))


def sweep_ordered(F, lam: int, adj, order, op=OP_LEVELING) -> SweepResult:
    """Sweep with an arbitrary visiting order inside each parity class."""
    lib = _load()
    src = np.asarray(F)
    a = _widen(src)
    order = np.ascontiguousarray(np.asarray(order, dtype=np.int64))
    if order.size != a.size:
        raise ValueError("order must be a permutation of all pixel indices")
    p = ctypes.c_uint64()
    lo = ctypes.c_uint64()
    rc = lib.oracle_sweep_ordered(_ptr(a, ctypes.c_int32), a.shape[0], a.shape[1],
                                  ctypes.c_uint32(int(lam)), _adj_code(adj), _op_code(op),
                                  _ptr(order, ctypes.c_int64), ctypes.byref(p), ctypes.byref(lo))
    _check(rc, "oracle_sweep_ordered")
    return SweepResult(a.astype(src.dtype, copy=False), p.value, lo.value)


def sweep_dirty(F, lam: int, adj=ADJ_8_4, op=OP_LEVELING) -> SweepResult:
    """ORACLE-SWEEP-DIRTY: same output, re-examining only pixels whose 3x3 changed."""
    lib = _load()
    src = np.asarray(F)
    a = _widen(src)
    p = ctypes.c_uint64()
    lo = ctypes.c_uint64()
    ex = ctypes.c_uint64()
    rc = lib.oracle_sweep_dirty(_ptr(a, ctypes.c_int32), a.shape[0], a.shape[1],
                                ctypes.c_uint32(int(lam)), _adj_code(adj), _op_code(op),
                                ctypes.byref(p), ctypes.byref(lo), ctypes.byref(ex))
    _check(rc, "oracle_sweep_dirty")
    return SweepResult(a.astype(src.dtype, copy=False), p.value, lo.value, ex.value)


def queue(F, lam: int, adj=ADJ_8_4, op=OP_LEVELING) -> SweepResult:
    """ORACLE-QUEUE: the paper's minimal-value order (section 2.2).  passes=0."""
    lib = _load()
    src = np.asarray(F)
    a = _widen(src)
    lo = ctypes.c_uint64()
    pops = ctypes.c_uint64()
    rc = lib.oracle_queue(_ptr(a, ctypes.c_int32), a.shape[0], a.shape[1],
                          ctypes.c_uint32(int(lam)), _adj_code(adj), _op_code(op),
                          ctypes.byref(lo), ctypes.byref(pops))
    _check(rc, "oracle_queue")
    return SweepResult(a.astype(src.dtype, copy=False), 0, lo.value, pops.value)


def count_destructible(F, lam: int, adj=ADJ_8_4):
    """(lambda-destructible count, destructible count) over interior pixels."""
    lib = _load()
    a = _widen(F)
    ld = ctypes.c_uint64()
    d = ctypes.c_uint64()
    rc = lib.oracle_count_destructible(_ptr(a, ctypes.c_int32), a.shape[0], a.shape[1],
                                       ctypes.c_uint32(int(lam)), _adj_code(adj),
                                       ctypes.byref(ld), ctypes.byref(d))
    _check(rc, "oracle_count_destructible")
    return ld.value, d.value


def count_lowerable(F, lam: int, adj=ADJ_8_4, op=OP_LEVELING) -> int:
    """Interior pixels that operator op would lower (0 for a stable image)."""
    lib = _load()
    a = _widen(F)
    c = ctypes.c_uint64()
    rc = lib.oracle_count_lowerable(_ptr(a, ctypes.c_int32), a.shape[0], a.shape[1],
                                    ctypes.c_uint32(int(lam)), _adj_code(adj), _op_code(op),
                                    ctypes.byref(c))
    _check(rc, "oracle_count_lowerable")
    return c.value
