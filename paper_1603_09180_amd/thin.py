"""ctypes binding of libthin.so (include/thin.h).

The functions named like the C calls (thin_create, thin_run, ...) only
marshal arguments; every step of the lambda-leveling loop and of the
lambda-skeleton runs in the HIP library.  torch is used for device memory and streams only.  If the library
has not been built the binding raises ThinError: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libthin.so")

THIN_OK, THIN_EINVAL, THIN_ENOMEM, THIN_EDEVICE, THIN_ELIMIT, THIN_EBUSY = 0, -1, -2, -3, -4, -5
THIN_U8, THIN_U16 = 1, 2
THIN_ADJ_8_4, THIN_ADJ_4_8 = 0, 1
THIN_OP_LEVELING, THIN_OP_SKELETON = 0, 1
THIN_ENGINE_AUTO, THIN_ENGINE_TILED, THIN_ENGINE_STEP, THIN_ENGINE_COOP = 0, 1, 2, 4
THIN_ENGINE_WORKLIST = 5
THIN_FLAG_PROFILE = 1
THIN_FLAG_GRAPH = 2
THIN_FLAG_TAIL = 4

EXPORTED = [
    "thin_create", "thin_run", "thin_run_noalloc", "thin_skeleton", "thin_run_batch", "thin_serve_admit",
    "thin_serve_step",
    "thin_destroy", "thin_strerror", "thin_last_error", "thin_profile", "thin_topology_table",
    "thin_autotune", "thin_gradient", "thin_gradient_coefficients",
]


class ThinError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class thin_config(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("engine", ctypes.c_int32),
        ("hip_stream", ctypes.c_void_p),
        ("max_device_bytes", ctypes.c_uint64),
        ("max_passes", ctypes.c_uint64),
        ("tile", ctypes.c_int32),
        ("steps_per_round", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("threads", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("tune_cache", ctypes.c_char_p),
    ]


class thin_profile_info(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_uint64),
        ("kernel_ms", ctypes.c_double),
        ("tile_rounds", ctypes.c_uint64),
    ]


class thin_stats(ctypes.Structure):
    _fields_ = [
        ("passes", ctypes.c_uint64),
        ("lowerings", ctypes.c_uint64),
        ("tile_rounds", ctypes.c_uint64),
        ("converged", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("examinations", ctypes.c_uint64),
    ]


class thin_image(ctypes.Structure):
    _fields_ = [
        ("image", ctypes.c_void_p),
        ("h", ctypes.c_int64),
        ("w", ctypes.c_int64),
        ("pitch_elems", ctypes.c_int64),
        ("dtype", ctypes.c_int32),
        ("lambda_", ctypes.c_uint32),
        ("adjacency", ctypes.c_int32),
        ("op", ctypes.c_int32),
    ]


def _np_struct(cls):
    import numpy as np

    names, formats, offsets = [], [], []
    for name, ctype in cls._fields_:
        names.append(name)
        formats.append(np.dtype(ctype))
        offsets.append(getattr(cls, name).offset)
    return np.dtype({"names": names, "formats": formats, "offsets": offsets,
                     "itemsize": ctypes.sizeof(cls)})


_IMAGE_NP = _np_struct(thin_image)
_STATS_NP = _np_struct(thin_stats)


class thin_tune_result(ctypes.Structure):
    _fields_ = [
        ("tile_h", ctypes.c_int32),
        ("tile_w", ctypes.c_int32),
        ("steps_per_round", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("ms", ctypes.c_double),
        ("default_ms", ctypes.c_double),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libthin.so and declares the C signatures.  Raises ThinError
    when the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ThinError(THIN_EDEVICE, f"{path} is missing: build it with "
                                      "`python -m paper_1603_09180_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.thin_create.argtypes = [P(ctypes.c_void_p), P(thin_config)]
    lib.thin_create.restype = ctypes.c_int
    lib.thin_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                             ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32, P(thin_stats)]
    lib.thin_run.restype = ctypes.c_int
    lib.thin_run_noalloc.argtypes = lib.thin_run.argtypes
    lib.thin_run_noalloc.restype = ctypes.c_int
    lib.thin_skeleton.argtypes = lib.thin_run.argtypes
    lib.thin_skeleton.restype = ctypes.c_int
    lib.thin_run_batch.argtypes = [ctypes.c_void_p, P(thin_image), ctypes.c_int32, P(thin_stats)]
    lib.thin_run_batch.restype = ctypes.c_int
    lib.thin_serve_admit.argtypes = [ctypes.c_void_p, P(thin_image), ctypes.c_uint64]
    lib.thin_serve_admit.restype = ctypes.c_int
    lib.thin_serve_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_uint64),
                                    P(thin_stats), ctypes.c_int32, P(ctypes.c_int32),
                                    P(ctypes.c_int32)]
    lib.thin_serve_step.restype = ctypes.c_int
    lib.thin_destroy.argtypes = [ctypes.c_void_p]
    lib.thin_destroy.restype = ctypes.c_int
    lib.thin_strerror.argtypes = [ctypes.c_int]
    lib.thin_strerror.restype = ctypes.c_char_p
    lib.thin_last_error.argtypes = [ctypes.c_void_p]
    lib.thin_last_error.restype = ctypes.c_char_p
    lib.thin_profile.argtypes = [ctypes.c_void_p, P(thin_profile_info), ctypes.c_int32]
    lib.thin_profile.restype = ctypes.c_int
    lib.thin_topology_table.argtypes = [ctypes.c_int32, ctypes.c_int32, P(ctypes.c_uint32),
                                        ctypes.c_int32]
    lib.thin_topology_table.restype = ctypes.c_int
    lib.thin_autotune.argtypes = [ctypes.c_void_p, P(thin_image), ctypes.c_int32, ctypes.c_int32,
                                  P(thin_tune_result)]
    lib.thin_autotune.restype = ctypes.c_int
    lib.thin_gradient.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, P(ctypes.c_float)]
    lib.thin_gradient.restype = ctypes.c_int
    lib.thin_gradient_coefficients.argtypes = [ctypes.c_float, P(ctypes.c_float), ctypes.c_int32]
    lib.thin_gradient_coefficients.restype = ctypes.c_int
    _lib = lib
    return lib


# ----------------------------------------------------------- C-named wrappers


def thin_create(cfg: thin_config | None = None) -> ctypes.c_void_p:
    lib = load_library()
    h = ctypes.c_void_p()
    rc = lib.thin_create(ctypes.byref(h), ctypes.byref(cfg) if cfg is not None else None)
    if rc != THIN_OK:
        raise ThinError(rc, "thin_create: " + thin_strerror(rc))
    return h


def thin_run(ctx, image_ptr: int, h: int, w: int, dtype: int, lam: int, adjacency: int,
             stats: thin_stats | None = None) -> int:
    return load_library().thin_run(ctx, ctypes.c_void_p(image_ptr), h, w, dtype,
                                   ctypes.c_uint32(lam), adjacency,
                                   ctypes.byref(stats) if stats is not None else None)


def thin_run_noalloc(ctx, image_ptr: int, h: int, w: int, dtype: int, lam: int, adjacency: int,
                     stats: thin_stats | None = None) -> int:
    return load_library().thin_run_noalloc(ctx, ctypes.c_void_p(image_ptr), h, w, dtype,
                                           ctypes.c_uint32(lam), adjacency,
                                           ctypes.byref(stats) if stats is not None else None)


def thin_skeleton(ctx, image_ptr: int, h: int, w: int, dtype: int, lam: int, adjacency: int,
                  stats: thin_stats | None = None) -> int:
    return load_library().thin_skeleton(ctx, ctypes.c_void_p(image_ptr), h, w, dtype,
                                        ctypes.c_uint32(lam), adjacency,
                                        ctypes.byref(stats) if stats is not None else None)


def thin_run_batch(ctx, images, n: int, stats=None) -> int:
    return load_library().thin_run_batch(ctx, images, n, stats)


def thin_serve_admit(ctx, image: thin_image, tag: int) -> int:
    return load_library().thin_serve_admit(ctx, ctypes.byref(image), ctypes.c_uint64(tag))


def thin_serve_step(ctx, rounds: int, done_tags, done_stats, cap: int, n_done, n_resident) -> int:
    return load_library().thin_serve_step(ctx, rounds, done_tags, done_stats, cap, n_done,
                                          n_resident)


def thin_destroy(ctx) -> int:
    return load_library().thin_destroy(ctx)


def thin_strerror(code: int) -> str:
    return load_library().thin_strerror(code).decode()


def thin_last_error(ctx) -> str:
    return load_library().thin_last_error(ctx).decode()


def thin_profile(ctx, reset: bool = False) -> thin_profile_info:
    info = thin_profile_info()
    rc = load_library().thin_profile(ctx, ctypes.byref(info), 1 if reset else 0)
    if rc != THIN_OK:
        raise ThinError(rc, "thin_profile")
    return info


def thin_topology_table(adjacency: int, op: int = THIN_OP_LEVELING):
    """The connectivity table the kernels use: a list of 256 (flags, comps)."""
    lib = load_library()
    buf = (ctypes.c_uint32 * 512)()
    rc = lib.thin_topology_table(adjacency, op, buf, 512)
    if rc != THIN_OK:
        raise ThinError(rc, "thin_topology_table")
    return [(buf[2 * m], buf[2 * m + 1]) for m in range(256)]


def thin_gradient_coefficients(alpha: float):
    """The 12 float32 coefficients thin_gradient uses (see include/thin.h)."""
    buf = (ctypes.c_float * 12)()
    rc = load_library().thin_gradient_coefficients(ctypes.c_float(alpha), buf, 12)
    if rc != THIN_OK:
        raise ThinError(rc, "thin_gradient_coefficients")
    return [float(buf[i]) for i in range(12)]


# ------------------------------------------------------- tensor-level helpers


@dataclass
class Stats:
    passes: int
    lowerings: int
    tile_rounds: int
    converged: bool
    examinations: int = 0

    @staticmethod
    def of(s: thin_stats) -> "Stats":
        return Stats(int(s.passes), int(s.lowerings), int(s.tile_rounds), bool(s.converged),
                     int(s.examinations))


def _adj_code(adj) -> int:
    if adj in (THIN_ADJ_8_4, "8,4", (8, 4)):
        return THIN_ADJ_8_4
    if adj in (THIN_ADJ_4_8, "4,8", (4, 8)):
        return THIN_ADJ_4_8
    raise ValueError(f"unknown adjacency {adj!r}")


def _op_code(op) -> int:
    if op in (THIN_OP_LEVELING, "leveling"):
        return THIN_OP_LEVELING
    if op in (THIN_OP_SKELETON, "skeleton"):
        return THIN_OP_SKELETON
    raise ValueError(f"unknown operator {op!r}")


def _dtype_code(t) -> int:
    import torch

    if t.dtype == torch.uint8:
        return THIN_U8
    if t.dtype == torch.uint16:
        return THIN_U16
    raise ValueError(f"unsupported dtype {t.dtype}")


def describe(t, lam: int, adj, op="leveling") -> thin_image:
    """thin_image for a 2-D uint8/uint16 CUDA tensor with unit column stride;
    op is "leveling" (lambda-leveling) or "skeleton" (lambda-skeleton)."""
    if t.dim() != 2 or not t.is_cuda:
        raise ValueError("expected a 2-D tensor on the GPU")
    if t.numel() and t.stride(1) != 1:
        raise ValueError("columns must be contiguous")
    im = thin_image()
    im.image = t.data_ptr() if t.numel() else None
    im.h, im.w = int(t.shape[0]), int(t.shape[1])
    im.pitch_elems = int(t.stride(0)) if t.numel() else int(t.shape[1])
    im.dtype = _dtype_code(t)
    im.lambda_ = int(lam)
    im.adjacency = _adj_code(adj)
    im.op = _op_code(op)
    return im


def _describe_many(tensors, lams, adjs, ops):
    """The thin_image array of a batch as one numpy buffer with thin_image's
    layout: the same checks and fields as describe(), built as tuples and
    converted at once (a ctypes structure per image costs microseconds, which
    for batches of hundreds of small images is a visible share of a call)."""
    import numpy as np
    import torch

    dt_code = {torch.uint8: THIN_U8, torch.uint16: THIN_U16}
    adj_memo, op_memo = {}, {}
    rows = []
    for t, lam, adj, op in zip(tensors, lams, adjs, ops):
        shape = t.shape
        if len(shape) != 2 or not t.is_cuda:
            raise ValueError("expected a 2-D tensor on the GPU")
        h, w = int(shape[0]), int(shape[1])
        stride = t.stride()
        n = h * w
        if n and stride[1] != 1:
            raise ValueError("columns must be contiguous")
        code = dt_code.get(t.dtype)
        if code is None:
            raise ValueError(f"unsupported dtype {t.dtype}")
        a = adj_memo.get(adj) if isinstance(adj, (int, str)) else None
        if a is None:
            a = _adj_code(adj)
            if isinstance(adj, (int, str)):
                adj_memo[adj] = a
        o = op_memo.get(op) if isinstance(op, (int, str)) else None
        if o is None:
            o = _op_code(op)
            if isinstance(op, (int, str)):
                op_memo[op] = o
        lam = int(lam) & 0xFFFFFFFF  # as the uint32 field of describe() takes it
        rows.append((t.data_ptr() if n else 0, h, w, int(stride[0]) if n else w, code, lam, a, o))
    return np.array(rows, dtype=_IMAGE_NP) if rows else np.zeros(1, dtype=_IMAGE_NP)


def _stats_many(st, n):
    import numpy as np

    a = np.frombuffer(st, dtype=_STATS_NP, count=n)
    return [Stats(p, lo, tr, bool(c), e) for p, lo, tr, c, _, e in a.tolist()]


class Context:
    """Owns a thin_ctx bound to a device and a stream (torch's current stream
    of that device when not given)."""

    def __init__(self, device: int = 0, stream=None, engine: int = THIN_ENGINE_AUTO,
                 max_device_bytes: int = 0, max_passes: int = 0, tile: int = 0,
                 steps_per_round: int = 0, profile: bool = False, graph: bool = False,
                 threads: int = 0, variant: int = 0, tune_cache: str | None = None,
                 tail: bool = False):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(device)
        cfg = thin_config()
        cfg.device = device
        cfg.engine = engine
        cfg.hip_stream = stream.cuda_stream or None
        cfg.max_device_bytes = max_device_bytes
        cfg.max_passes = max_passes
        cfg.tile = tile
        cfg.steps_per_round = steps_per_round
        cfg.threads = threads
        cfg.variant = variant
        cfg.flags = ((THIN_FLAG_PROFILE if profile else 0) | (THIN_FLAG_GRAPH if graph else 0)
                     | (THIN_FLAG_TAIL if tail else 0))
        cfg.tune_cache = tune_cache.encode() if tune_cache else None
        self.device = device
        self.stream = stream
        self.handle = thin_create(cfg)
        self._serve_bufs = None

    def close(self):
        if self.handle:
            thin_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str, allow_limit: bool = False):
        if rc == THIN_OK or (allow_limit and rc == THIN_ELIMIT):
            return
        raise ThinError(rc, f"{what}: {thin_strerror(rc)}: {thin_last_error(self.handle)}")

    def profile(self, reset: bool = False) -> thin_profile_info:
        return thin_profile(self.handle, reset)

    def run(self, t, lam: int, adj="8,4", allow_limit: bool = False, op="leveling") -> Stats:
        """Thins one device tensor in place; returns its statistics."""
        im = describe(t, lam, adj, op)
        st = thin_stats()
        rc = load_library().thin_run_batch(self.handle, ctypes.byref(im), 1, ctypes.byref(st))
        self._check(rc, "thin_run", allow_limit)
        return Stats.of(st)

    def run_batch(self, tensors, lams, adjs, allow_limit: bool = False, ops=None):
        n = len(tensors)
        if not (len(lams) == len(adjs) == n and (ops is None or len(ops) == n)):
            raise ValueError("tensors, lams, adjs and ops differ in length")
        ops = ops if ops is not None else ["leveling"] * n
        arr = _describe_many(tensors, lams, adjs, ops)
        st = (thin_stats * max(n, 1))()
        rc = thin_run_batch(self.handle, arr.ctypes.data_as(ctypes.POINTER(thin_image)), n, st)
        self._check(rc, "thin_run_batch", allow_limit)
        return _stats_many(st, n)

    def autotune(self, tensors, lams, adjs, reps: int = 2, ops=None) -> dict:
        """Times every compiled tile shape on copies of these images and makes
        the fastest this context's choice for work lists of their size class."""
        n = len(tensors)
        ops = ops if ops is not None else ["leveling"] * n
        arr = (thin_image * max(n, 1))()
        for i, (t, lam, adj, op) in enumerate(zip(tensors, lams, adjs, ops)):
            arr[i] = describe(t, lam, adj, op)
        res = thin_tune_result()
        rc = load_library().thin_autotune(self.handle, arr, n, reps, ctypes.byref(res))
        self._check(rc, "thin_autotune")
        return {"tile": (res.tile_h, res.tile_w), "steps_per_round": res.steps_per_round,
                "threads": res.threads, "variant": res.variant, "candidates": res.candidates,
                "ms": res.ms, "default_ms": res.default_ms}

    def gradient(self, src, dst, alpha: float = 1.0, gain: float = 1.0, magnitude=None):
        """Deriche gradient of device tensor `src` into `dst` (same shape,
        uint8 or uint16); `magnitude`, when given, is a float32 tensor of the
        same shape that receives the unquantised magnitude."""
        for t in (src, dst):
            if t.dim() != 2 or not t.is_cuda or (t.numel() and t.stride(1) != 1):
                raise ValueError("expected 2-D GPU tensors with contiguous columns")
        if tuple(src.shape) != tuple(dst.shape):
            raise ValueError("src and dst shapes differ")
        mptr = None
        if magnitude is not None:
            import torch
            if (magnitude.dtype != torch.float32 or not magnitude.is_contiguous()
                    or tuple(magnitude.shape) != tuple(src.shape) or not magnitude.is_cuda):
                raise ValueError("magnitude must be a contiguous float32 GPU tensor of src's shape")
            mptr = ctypes.cast(ctypes.c_void_p(magnitude.data_ptr()), ctypes.POINTER(ctypes.c_float))
        h, w = int(src.shape[0]), int(src.shape[1])
        rc = load_library().thin_gradient(
            self.handle, ctypes.c_void_p(src.data_ptr() if src.numel() else None), h, w,
            int(src.stride(0)) if src.numel() else w, _dtype_code(src), ctypes.c_float(alpha),
            ctypes.c_float(gain), ctypes.c_void_p(dst.data_ptr() if dst.numel() else None),
            int(dst.stride(0)) if dst.numel() else w, _dtype_code(dst), mptr)
        self._check(rc, "thin_gradient")

    # ---------------------------------------------------------- serving

    def serve_admit(self, t, lam: int, adj="8,4", tag: int = 0, op="leveling") -> bool:
        """Makes device tensor `t` resident for serving under `tag`; False
        when the serving budget is full (nothing admitted)."""
        im = describe(t, lam, adj, op)
        rc = thin_serve_admit(self.handle, im, tag)
        if rc == THIN_EBUSY:
            return False
        self._check(rc, "thin_serve_admit")
        return True

    def serve_step(self, rounds: int, cap: int = 4096):
        """Runs `rounds` rounds over the resident images; returns
        ([(tag, Stats), ...] of the retired ones, number still resident)."""
        if self._serve_bufs is None or len(self._serve_bufs[0]) < cap:
            self._serve_bufs = ((ctypes.c_uint64 * cap)(), (thin_stats * cap)())
        tags, sts = self._serve_bufs
        n_done = ctypes.c_int32(0)
        n_res = ctypes.c_int32(0)
        rc = thin_serve_step(self.handle, rounds, tags, sts, cap, ctypes.byref(n_done),
                             ctypes.byref(n_res))
        self._check(rc, "thin_serve_step")
        return [(int(tags[i]), Stats.of(sts[i])) for i in range(n_done.value)], n_res.value


def run(t, lam: int, adj="8,4", op="leveling", **kw) -> Stats:
    """One-shot convenience: thin device tensor `t` in place."""
    with Context(device=t.device.index or 0, **kw) as ctx:
        return ctx.run(t, lam, adj, op=op)
