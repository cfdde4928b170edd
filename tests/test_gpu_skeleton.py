"""GPU parity of the lambda-skeleton (lower the lambda-deletable, not
lambda-end points until stability; the algorithm box of section 2.2) against
the oracle, bit for bit (image, pass count, lowering count), through the C
ABI: every engine, every compiled tile shape, both dtypes and adjacencies,
lambda from 0 to 2^32-1, ragged and degenerate sizes, batches that mix the
two operators, graph replays and serving.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1603_09180_amd import synth, thin
from test_gpu_parity import ALL_SHAPES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SK = "skeleton"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_skel(F, lam, adj, **kw):
    t = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    with thin.Context(**kw) as ctx:
        st = ctx.run(t, lam, adj, op=SK, allow_limit=bool(kw.get("max_passes")))
    torch.cuda.synchronize()
    return t.cpu().numpy(), st


def assert_same(F, lam, adj, got, st, ref=None, op=SK):
    if ref is None:
        ref = oracle.sweep_dirty(F, lam, adj, op=op)
    bad = np.argwhere(got != ref.image)
    assert bad.size == 0, f"{len(bad)} pixels differ, first at {bad[:5].tolist()}"
    assert (st.passes, st.lowerings) == (ref.passes, ref.lowerings)
    assert st.converged


ENGINES = [thin.THIN_ENGINE_COOP, thin.THIN_ENGINE_TILED, thin.THIN_ENGINE_STEP]


@pytest.mark.parametrize("engine", ENGINES)
def test_engines(engine):
    R = synth.ridges_512().image()[:200, :230].copy()
    B = synth.gen_blobs(131, 97, 17, np.uint16, nblobs=9, sigma=(2.0, 10.0))
    for F, lam, adj in ((R, 10, 0), (R, 0, 1), (B, 900, 1), (B, 0, 0)):
        say("case skeleton engine", engine, F.shape, lam, adj)
        got, st = gpu_skel(F, lam, adj, engine=engine)
        assert_same(F, lam, adj, got, st)


def test_c_entry_point():
    """thin_skeleton itself (the Python helper goes through thin_run_batch)."""
    F = synth.ridges_512().image()[:150, :170].copy()
    t = torch.from_numpy(F).cuda()
    st = thin.thin_stats()
    say("case thin_skeleton")
    with thin.Context() as ctx:
        torch.cuda.synchronize()
        rc = thin.thin_skeleton(ctx.handle, t.data_ptr(), F.shape[0], F.shape[1], thin.THIN_U8,
                                10, thin.THIN_ADJ_8_4, st)
        assert rc == thin.THIN_OK
    assert_same(F, 10, 0, t.cpu().numpy(), thin.Stats.of(st))


def _fuzz_cases():
    rng = np.random.default_rng(4242)
    sides = [3, 4, 5, 7, 31, 32, 33, 63, 64, 65, 97, 129, 200, 257]
    lams = [0, 1, 5, 10, 20, 50, 500, 2**32 - 1]
    cases = []
    for k in range(32):
        h = int(rng.choice(sides))
        w = int(rng.choice(sides))
        dt = np.uint8 if k % 2 == 0 else np.uint16
        adj = int(rng.integers(0, 2))
        lam = int(rng.choice(lams))
        ridges = k % 4 == 0 and min(h, w) >= 16
        cases.append((k, h, w, dt, adj, lam, ridges))
    return cases


@pytest.mark.parametrize("case", _fuzz_cases(), ids=lambda c: "c%d_%dx%d_%s_a%d_l%d%s" % (
    c[0], c[1], c[2], np.dtype(c[3]).name, c[4], c[5], "_r" if c[6] else ""))
def test_fuzz(case):
    k, h, w, dt, adj, lam, ridges = case
    if ridges:
        F = synth.gen_ridges(h, w, 8000 + k, dt)
    else:
        F = synth.gen_blobs(h, w, 8000 + k, dt, nblobs=6, sigma=(2.0, 12.0), noise=12.0)
    say("case skeleton fuzz", case)
    got, st = gpu_skel(F, lam, adj)
    assert_same(F, lam, adj, got, st)


_REF = {}


def _ref(key, F, lam, adj):
    if key not in _REF:
        _REF[key] = oracle.sweep_dirty(F, lam, adj, op=SK)
    return _REF[key]


@pytest.mark.parametrize("shape", ALL_SHAPES)
def test_every_compiled_shape(shape, monkeypatch):
    monkeypatch.setenv("THIN_TILE_SHAPE", shape)
    R = synth.ridges_512().image()[:260, :300].copy()
    B = synth.gen_blobs(150, 201, 77, np.uint16, nblobs=10, sigma=(3.0, 20.0))
    say("case skeleton compiled shape", shape)
    got, st = gpu_skel(R, 10, 0)
    assert_same(R, 10, 0, got, st, _ref("r", R, 10, 0))
    got, st = gpu_skel(B, 600, 1)
    assert_same(B, 600, 1, got, st, _ref("b", B, 600, 1))


def _mixed_items(seed, n):
    rng = np.random.default_rng(seed)
    items = []
    for i in range(n):
        h, w = (int(x) for x in rng.integers(3, 200, size=2))
        dt = np.uint16 if i % 3 == 0 else np.uint8
        if i % 4 == 1 and min(h, w) >= 16:
            F = synth.gen_ridges(h, w, seed * 100 + i, dt)
        else:
            F = synth.gen_blobs(h, w, seed * 100 + i, dt, sigma=(2.0, 10.0))
        lam = int(rng.choice([0, 5, 10, 20, 50])) * (257 if dt == np.uint16 else 1)
        items.append((F, lam, i % 2, SK if i % 2 == 0 or i % 5 == 0 else "leveling"))
    return items


def _check_items(items, outs, sts):
    for (F, lam, adj, op), out, st in zip(items, outs, sts):
        if min(F.shape) < 3:
            assert np.array_equal(out, F) and st.passes == 0
            continue
        assert_same(F, lam, adj, out, st, op=op)


@pytest.mark.parametrize("engine", ENGINES[:2])
def test_batch_mixing_operators(engine):
    items = _mixed_items(31, 18)
    ts = [torch.from_numpy(F.copy()).cuda() for F, _, _, _ in items]
    say("case skeleton batch mixing operators, engine", engine)
    with thin.Context(engine=engine) as ctx:
        sts = ctx.run_batch(ts, [x[1] for x in items], [x[2] for x in items],
                            ops=[x[3] for x in items])
    _check_items(items, [t.cpu().numpy() for t in ts], sts)


@pytest.mark.parametrize("variant", [3, 4])
def test_mixed_dtype_and_operator_batch_bit_flag_variants(variant):
    items = _mixed_items(37, 12)
    ts = [torch.from_numpy(F.copy()).cuda() for F, _, _, _ in items]
    say("case skeleton mixed batch variant", variant)
    with thin.Context(tile=64, steps_per_round=16, threads=256, variant=variant) as ctx:
        sts = ctx.run_batch(ts, [x[1] for x in items], [x[2] for x in items],
                            ops=[x[3] for x in items])
    _check_items(items, [t.cpu().numpy() for t in ts], sts)


def test_graph_mode():
    R = synth.ridges_512().image()[:200, :300].copy()
    ref = oracle.sweep_dirty(R, 10, 0, op=SK)
    with thin.Context(graph=True) as ctx:
        for rep in range(2):
            say("case skeleton graph rep", rep)
            t = torch.from_numpy(R.copy()).cuda()
            st = ctx.run(t, 10, 0, op=SK)
            torch.cuda.synchronize()
            assert_same(R, 10, 0, t.cpu().numpy(), st, ref)


def test_closed_form_shapes():
    """A line above lambda is kept, a T loses its low branch, a lone peak at
    lambda vanishes (the oracle's pins), at image sizes spanning tiles."""
    F = np.full((150, 170), 10, np.uint8)
    F[40, 5:160] = 140                      # line, contrast 130
    F[41:120, 80] = 40                      # branch, contrast 30
    F[100, 20] = 60                         # lone peak, contrast 50
    for adj in (0, 1):
        say("case skeleton closed forms adj", adj)
        got, st = gpu_skel(F, 50, adj)
        want = np.full_like(F, 10)
        want[40, 5:160] = 140
        assert np.array_equal(got, want)
        assert st.lowerings == 79 + 1
        got, st = gpu_skel(F, 29, adj)
        assert np.array_equal(got, F) and st.lowerings == 0


def test_pass_cap_then_resume():
    R = synth.ridges_512().image()[:120, :140].copy()
    full = oracle.sweep(R, 10, 0, op=SK)
    part = oracle.sweep(R, 10, 0, max_passes=4, op=SK)
    assert part.limited
    say("case skeleton pass cap")
    t = torch.from_numpy(R.copy()).cuda()
    with thin.Context(max_passes=4) as ctx:
        st = ctx.run(t, 10, 0, op=SK, allow_limit=True)
        assert not st.converged and st.passes == 4 and st.lowerings == part.lowerings
    assert np.array_equal(t.cpu().numpy(), part.image)
    with thin.Context() as ctx:
        st = ctx.run(t, 10, 0, op=SK)
    assert np.array_equal(t.cpu().numpy(), full.image)
    assert st.lowerings + part.lowerings == full.lowerings


def test_serving_mixes_operators():
    items = _mixed_items(43, 16)
    ts = [torch.from_numpy(F.copy()).cuda() for F, _, _, _ in items]
    stats = {}
    say("case skeleton serving")
    with thin.Context() as ctx:
        nxt = 0
        while len(stats) < len(items):
            for _ in range(3):
                if nxt < len(items):
                    F, lam, adj, op = items[nxt]
                    assert ctx.serve_admit(ts[nxt], lam, adj, tag=nxt, op=op)
                    nxt += 1
            done, _ = ctx.serve_step(2)
            stats.update(done)
    torch.cuda.synchronize()
    _check_items(items, [t.cpu().numpy() for t in ts], [stats[i] for i in range(len(items))])


def test_bad_operator_is_rejected():
    t = torch.zeros((16, 16), dtype=torch.uint8, device="cuda")
    im = thin.describe(t, 0, 0)
    im.op = 2
    st = thin.thin_stats()
    with thin.Context() as ctx:
        rc = thin.thin_run_batch(ctx.handle, ctypes.byref(im), 1, ctypes.byref(st))
        assert rc == thin.THIN_EINVAL
        assert thin.thin_serve_admit(ctx.handle, im, 1) == thin.THIN_EINVAL
