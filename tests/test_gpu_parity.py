"""GPU parity: the HIP path against the CPU oracle, bit for bit (image, pass
count and lowering count), through the C ABI.

Sizes are chosen so the oracle finishes in seconds while still spanning
several tiles with ragged right and bottom edges; the degenerate sizes, both
dtypes, both adjacency pairs and lambda from 0 to 2^32-1 are covered.  The
oracle side uses ORACLE-SWEEP-DIRTY, which the CPU suite pins equal to the
plain sweep.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1603_09180_amd import synth, thin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(32, 32, 8), (32, 32, 16), (64, 64, 16), (64, 64, 32)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_thin(F, lam, adj, **kw):
    t = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    with thin.Context(**kw) as ctx:
        st = ctx.run(t, lam, adj, allow_limit=bool(kw.get("max_passes")))
    torch.cuda.synchronize()
    return t.cpu().numpy(), st


def assert_same(F, lam, adj, got, st, ref=None):
    if ref is None:
        ref = oracle.sweep_dirty(F, lam, adj)
    bad = np.argwhere(got != ref.image)
    assert bad.size == 0, f"{len(bad)} pixels differ, first at {bad[:5].tolist()}"
    assert (st.passes, st.lowerings) == (ref.passes, ref.lowerings)
    assert st.converged


ENGINES = [thin.THIN_ENGINE_COOP, thin.THIN_ENGINE_TILED, thin.THIN_ENGINE_STEP]


@pytest.mark.parametrize("engine", ENGINES)
def test_blobs_128_lambda0(engine):
    job = synth.blobs_128()
    F = job.image()
    say("case blobs_128 engine", engine)
    got, st = gpu_thin(F, job.lam, job.adj, engine=engine)
    assert_same(F, job.lam, job.adj, got, st)


@pytest.mark.parametrize("engine", ENGINES[:2])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "t%dk%d" % (s[0], s[2]))
def test_blobs_128_every_tile_shape(shape, engine):
    job = synth.blobs_128()
    F = job.image()
    say("case blobs_128 shape", shape, "engine", engine)
    got, st = gpu_thin(F, job.lam, job.adj, tile=shape[0], steps_per_round=shape[2], engine=engine)
    assert_same(F, job.lam, job.adj, got, st)


@pytest.mark.parametrize("engine", ENGINES[:2])
def test_ridges_512_lambda20(engine):
    job = synth.ridges_512()
    F = job.image()
    say("case ridges_512 engine", engine)
    got, st = gpu_thin(F, job.lam, job.adj, engine=engine)
    assert_same(F, job.lam, job.adj, got, st)


def _fuzz_cases():
    rng = np.random.default_rng(2024)
    sides = [3, 4, 5, 7, 31, 32, 33, 63, 64, 65, 96, 97, 129, 200, 257, 300]
    lams = [0, 1, 5, 20, 50, 500, 2**32 - 1]
    cases = []
    for k in range(48):
        h = int(rng.choice(sides))
        w = int(rng.choice(sides))
        dt = np.uint8 if k % 2 == 0 else np.uint16
        adj = int(rng.integers(0, 2))
        lam = int(rng.choice(lams))
        if dt == np.uint8 and lam == 500:
            lam = 50
        cases.append((k, h, w, dt, adj, lam))
    return cases


@pytest.mark.parametrize("case", _fuzz_cases(), ids=lambda c: "c%d_%dx%d_%s_a%d_l%d" % (
    c[0], c[1], c[2], np.dtype(c[3]).name, c[4], c[5]))
def test_fuzz(case):
    k, h, w, dt, adj, lam = case
    F = synth.gen_blobs(h, w, 7000 + k, dt, nblobs=6, sigma=(2.0, 12.0), noise=12.0)
    say("case fuzz", case)
    got, st = gpu_thin(F, lam, adj)
    assert_same(F, lam, adj, got, st)


# Every compiled (tile height, width, halo, threads, residency variant) shape:
# variant 0 keeps per-pixel flags in LDS, 1 seeds them from the previous
# round, 2 keeps 4x4 windows in registers, 3 keeps one flag bit per candidate
# and examines dense lists, 4 seeds those bits from the previous round.
ALL_SHAPES = ["16,16,8,256,0", "32,32,8,256,0", "32,32,8,512,0", "32,32,16,256,0",
              "32,32,16,512,0", "32,32,16,1024,0", "32,32,16,1024,1", "48,48,16,512,0",
              "64,64,8,512,0", "64,64,8,1024,0", "64,64,16,256,0", "64,64,16,512,0",
              "64,64,16,1024,0", "64,64,16,1024,1", "64,64,32,512,0", "64,64,32,1024,0",
              "128,128,16,512,0", "128,128,16,512,1", "64,64,16,512,1",
              "16,16,8,256,2", "16,16,16,576,2", "16,16,16,256,2", "24,24,12,576,2",
              "16,16,16,576,0", "32,32,8,256,2", "32,32,16,256,2", "32,32,16,512,2",
              "32,32,16,1024,2", "32,32,32,1024,2", "64,64,16,512,2", "64,64,16,1024,2",
              "64,64,32,1024,2",
              "32,32,16,256,3", "32,32,16,512,3", "64,64,16,512,3", "64,64,16,512,4",
              "64,64,16,256,3", "64,64,16,256,4", "128,128,16,256,4",
              "64,64,32,512,3", "64,64,32,512,4", "128,128,16,512,3", "128,128,16,512,4",
              "128,128,32,512,4", "128,128,8,512,4", "128,128,24,512,4"]


@pytest.mark.parametrize("shape", ALL_SHAPES)
def test_every_compiled_shape(shape, monkeypatch):
    monkeypatch.setenv("THIN_TILE_SHAPE", shape)
    F = synth.gen_blobs(150, 201, 77, np.uint16, nblobs=10, sigma=(3.0, 20.0))
    say("case compiled shape", shape)
    got, st = gpu_thin(F, 500, 1)
    assert_same(F, 500, 1, got, st)
    job = synth.ridges_512()
    R = job.image()[:300, :260].copy()
    got, st = gpu_thin(R, 20, 0)
    assert_same(R, 20, 0, got, st)


def test_schedule_invariance_u16_4_8():
    """Tile shape, halo width and engine change the schedule, never the bytes."""
    F = synth.gen_blobs(150, 201, 77, np.uint16, nblobs=10, sigma=(3.0, 20.0))
    ref = oracle.sweep_dirty(F, 500, 1)
    for engine in ENGINES[:2]:
        for shape in SHAPES:
            say("case invariance shape", shape, "engine", engine)
            got, st = gpu_thin(F, 500, 1, tile=shape[0], steps_per_round=shape[2], engine=engine)
            assert_same(F, 500, 1, got, st, ref)
    got, st = gpu_thin(F, 500, 1, engine=thin.THIN_ENGINE_STEP)
    assert_same(F, 500, 1, got, st, ref)


def test_batch_equals_oracle_per_image():
    rng = np.random.default_rng(9)
    Fs, lams, adjs = [], [], []
    for i in range(14):
        h, w = int(rng.integers(3, 180)), int(rng.integers(3, 180))
        dt = np.uint8 if i % 3 else np.uint16
        Fs.append(synth.gen_blobs(h, w, 9100 + i, dt, sigma=(2.0, 10.0)))
        lams.append(int(rng.choice([0, 5, 20, 50])) * (257 if dt == np.uint16 else 1))
        adjs.append(i % 2)
    Fs.append(np.zeros((2, 50), np.uint8))      # no interior
    lams.append(0)
    adjs.append(0)
    ts = [torch.from_numpy(F).cuda() for F in Fs]
    say("case batch of", len(ts))
    with thin.Context() as ctx:
        sts = ctx.run_batch(ts, lams, adjs)
    torch.cuda.synchronize()
    for F, t, lam, adj, st in zip(Fs, ts, lams, adjs, sts):
        if min(F.shape) < 3:
            assert np.array_equal(t.cpu().numpy(), F) and st.passes == 0
            continue
        assert_same(F, lam, adj, t.cpu().numpy(), st)


@pytest.mark.parametrize("engine", ENGINES)
def test_pass_cap_then_resume(engine):
    F = synth.gen_blobs(90, 70, 123)
    full = oracle.sweep(F, 0)
    part = oracle.sweep(F, 0, max_passes=3)
    assert part.limited
    say("case pass cap engine", engine)
    t = torch.from_numpy(F.copy()).cuda()
    with thin.Context(max_passes=3, engine=engine) as ctx:
        st = ctx.run(t, 0, 0, allow_limit=True)
        assert not st.converged and st.passes == 3 and st.lowerings == part.lowerings
        assert np.array_equal(t.cpu().numpy(), part.image)
    with thin.Context() as ctx:
        st = ctx.run(t, 0, 0)
    assert np.array_equal(t.cpu().numpy(), full.image)
    assert st.lowerings + part.lowerings == full.lowerings


def test_pitched_view_leaves_margin_untouched():
    big = synth.gen_blobs(80, 140, 5)
    F = big[:, 10:110].copy()
    t_big = torch.from_numpy(big.copy()).cuda()
    view = t_big[:, 10:110]
    assert view.stride(0) == 140
    say("case pitched")
    with thin.Context() as ctx:
        st = ctx.run(view, 0, 0)
    out = t_big.cpu().numpy()
    assert np.array_equal(out[:, :10], big[:, :10]) and np.array_equal(out[:, 110:], big[:, 110:])
    assert_same(F, 0, 0, out[:, 10:110], st)


@pytest.mark.parametrize("shape", [(0, 0), (1, 40), (2, 2), (40, 2), (3, 3)])
def test_degenerate_sizes(shape):
    F = (np.arange(int(np.prod(shape)), dtype=np.uint8).reshape(shape) * 37) % 251
    say("case degenerate", shape)
    with thin.Context() as ctx:
        t = torch.from_numpy(F.copy()).cuda()
        st = ctx.run(t, 0, 0)
    ref = oracle.sweep(F, 0)
    assert np.array_equal(t.cpu().numpy(), ref.image)
    assert st.passes == ref.passes and st.lowerings == ref.lowerings


@pytest.mark.skip(reason="persistent engine removed: one launch ran past its time guards "
                         "without finishing and the cause is not established")
def test_persistent_engine_blobs_128():
    job = synth.blobs_128()
    F = job.image()
    got, st = gpu_thin(F, job.lam, job.adj, engine=3)
    assert_same(F, job.lam, job.adj, got, st)


def test_persistent_engine_reports_disabled():
    """Engine 3 (the removed persistent work-queue engine) is refused at
    thin_create."""
    with pytest.raises(thin.ThinError):
        thin.Context(engine=3)


def test_graph_mode_matches_oracle():
    """Chunks of rounds replayed as HIP graphs: same bytes, passes and lowerings."""
    cases = [(synth.blobs_128().image(), 0, 0), (synth.ridges_512().image()[:200, :300].copy(), 20, 0),
             (synth.gen_blobs(150, 201, 77, np.uint16, nblobs=10, sigma=(3.0, 20.0)), 500, 1)]
    with thin.Context(graph=True) as ctx:
        for rep in range(2):  # the second pass replays cached graphs
            for F, lam, adj in cases:
                say("case graph", F.shape, lam, adj, "rep", rep)
                t = torch.from_numpy(F.copy()).cuda()
                st = ctx.run(t, lam, adj)
                torch.cuda.synchronize()
                assert_same(F, lam, adj, t.cpu().numpy(), st)
        Fs = [synth.gen_blobs(64 + 37 * i, 90 + 23 * i, 300 + i) for i in range(12)]
        ts = [torch.from_numpy(F.copy()).cuda() for F in Fs]
        sts = ctx.run_batch(ts, [5] * 12, [0] * 12)
        for F, t, st in zip(Fs, ts, sts):
            assert_same(F, 5, 0, t.cpu().numpy(), st)


def test_graph_cache_tells_calls_apart():
    """Replayed graphs are keyed by everything the recorded launches bake in:
    a one-image call followed by a two-image batch with the same tile count,
    and a u8 then a u16 image of the same size on a bit-flag shape (one
    launch per pixel type), each checked against the oracle."""
    one = synth.gen_blobs(64, 128, 901, nblobs=6, sigma=(2.0, 8.0))
    pair = [synth.gen_blobs(64, 64, 902 + i, nblobs=6, sigma=(2.0, 8.0)) for i in range(2)]
    say("case graph key: image counts")
    with thin.Context(graph=True) as ctx:
        for rep in range(2):
            t = torch.from_numpy(one.copy()).cuda()
            st = ctx.run(t, 5, 0)
            assert_same(one, 5, 0, t.cpu().numpy(), st)
            ts = [torch.from_numpy(F.copy()).cuda() for F in pair]
            sts = ctx.run_batch(ts, [5, 5], [0, 0])
            for F, t, st in zip(pair, ts, sts):
                assert_same(F, 5, 0, t.cpu().numpy(), st)
    u8 = synth.gen_blobs(256, 256, 903, np.uint8, nblobs=10, sigma=(3.0, 12.0))
    u16 = synth.gen_blobs(256, 256, 904, np.uint16, nblobs=10, sigma=(3.0, 12.0))
    say("case graph key: pixel types")
    with thin.Context(graph=True, tile=64, steps_per_round=16, threads=256, variant=3) as ctx:
        for rep in range(2):
            for F, lam in ((u8, 20), (u16, 300)):
                t = torch.from_numpy(F.copy()).cuda()
                st = ctx.run(t, lam, 0)
                assert_same(F, lam, 0, t.cpu().numpy(), st)


def test_graph_mode_with_tile_queues_and_both_pixel_types():
    """Graph replays of a call with per-round tile queues and one launch per
    pixel type per round (each drawing its tiles from its own counter):
    every image equals the same call without graphs, and a sample the
    oracle."""
    rng = np.random.default_rng(67)
    Fs = []
    for i in range(200):
        h, w = (int(x) for x in rng.integers(150, 520, size=2))
        Fs.append(synth.gen_blobs(h, w, 6700 + i, np.uint16 if i % 3 == 0 else np.uint8,
                                  nblobs=10, sigma=(3.0, 14.0)))
    lams = [int(x) for x in rng.choice([0, 5, 20, 50], size=len(Fs))]
    adjs = [i % 2 for i in range(len(Fs))]
    kw = dict(tile=64, steps_per_round=16, threads=256, variant=4)
    say("case graph with tile queues")
    plain = [torch.from_numpy(F.copy()).cuda() for F in Fs]
    with thin.Context(**kw) as ctx:
        ref_sts = ctx.run_batch(plain, lams, adjs)
    with thin.Context(graph=True, **kw) as ctx:
        for rep in range(2):  # the second call replays cached graphs
            ts = [torch.from_numpy(F.copy()).cuda() for F in Fs]
            sts = ctx.run_batch(ts, lams, adjs)
            for i in range(len(Fs)):
                assert torch.equal(ts[i], plain[i]), (rep, i)
                assert (sts[i].passes, sts[i].lowerings) == (ref_sts[i].passes,
                                                             ref_sts[i].lowerings), (rep, i)
    for i in range(0, len(Fs), 25):
        assert_same(Fs[i], lams[i], adjs[i], plain[i].cpu().numpy(), ref_sts[i])


def test_autotune_leaves_inputs_and_results_unchanged():
    Fs = [synth.gen_blobs(80 + 40 * i, 120 + 30 * i, 500 + i, np.uint16 if i % 2 else np.uint8)
          for i in range(6)]
    lams = [0, 5, 20, 50, 0, 300]
    adjs = [0, 1, 0, 1, 0, 1]
    ts = [torch.from_numpy(F.copy()).cuda() for F in Fs]
    say("case autotune")
    with thin.Context() as ctx:
        res = ctx.autotune(ts, lams, adjs, reps=2)
        torch.cuda.synchronize()
        for F, t in zip(Fs, ts):
            assert np.array_equal(t.cpu().numpy(), F)
        assert res["candidates"] > 1 and res["ms"] > 0 and res["default_ms"] > 0
        assert res["steps_per_round"] in (8, 12, 16, 24, 32) and res["threads"] in (256, 512, 576, 1024)
        sts = ctx.run_batch(ts, lams, adjs)
    for F, t, st, lam, adj in zip(Fs, ts, sts, lams, adjs):
        assert_same(F, lam, adj, t.cpu().numpy(), st)


def test_tune_cache_round_trip(tmp_path):
    """thin_autotune records its choice in the tune cache under the device's
    architecture and size class; a context created on that file runs with the
    recorded shape (its tile residencies equal a run with that shape forced)
    and lines of another architecture are ignored."""
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    F = synth.gen_blobs(300, 200, 4321, np.uint8, nblobs=8, sigma=(3.0, 10.0))
    t = torch.from_numpy(F.copy()).cuda()
    path = str(tmp_path / "tune.txt")
    say("case tune cache")
    with thin.Context(tune_cache=path) as ctx:
        ctx.autotune([t], [5], [0], reps=1)
    lines = open(path).read().split("\n")
    mine = [l for l in lines if l.startswith(arch + " ")]
    assert len(mine) == 1 and mine[0].split()[1:3] == ["15", "15"]
    # a hand-written entry for this size class, plus one for another architecture
    with open(path, "w") as f:
        f.write("gfx000 15 15 32 32 8 256 0 1.0\n")
        f.write(f"{arch} 15 15 64 64 16 256 3 1.0\n")
    def run(**kw):
        u = torch.from_numpy(F.copy()).cuda()
        with thin.Context(**kw) as c:
            st = c.run(u, 5, 0)
        return u.cpu().numpy(), st
    got, st = run(tune_cache=path)
    want, st_forced = run(tile=64, steps_per_round=16, threads=256, variant=3)
    _, st_default = run()
    assert np.array_equal(got, want)
    assert st.tile_rounds == st_forced.tile_rounds != st_default.tile_rounds
    assert_same(F, 5, 0, got, st)


@pytest.mark.parametrize("variant", [3, 4])
@pytest.mark.parametrize("engine", ENGINES[:2])
def test_mixed_dtype_batch_bit_flag_variants(variant, engine):
    """The bit-flag variants keep a u8 or u16 LDS tile per launch: a batch of
    both pixel types runs as two launches per round (one cooperative launch
    falls back to the flag variant)."""
    Fs = [synth.gen_blobs(70 + 29 * i, 90 + 17 * i, 800 + i, np.uint16 if i % 3 == 0 else np.uint8,
                          nblobs=8, sigma=(2.0, 10.0)) for i in range(9)]
    lams = [0, 7, 300, 20, 0, 2000, 50, 3, 0]
    adjs = [i % 2 for i in range(9)]
    ts = [torch.from_numpy(F.copy()).cuda() for F in Fs]
    say("case mixed dtypes variant", variant, "engine", engine)
    with thin.Context(tile=64, steps_per_round=16, threads=256, variant=variant,
                      engine=engine) as ctx:
        sts = ctx.run_batch(ts, lams, adjs)
    for F, t, st, lam, adj in zip(Fs, ts, sts, lams, adjs):
        assert_same(F, lam, adj, t.cpu().numpy(), st)


@pytest.mark.parametrize("shape", ["32,32,16,256,0", "32,32,16,1024,2", "64,64,16,256,4"])
def test_work_lists_match_full_scans(shape, monkeypatch):
    """A batch with many more tiles than blocks runs on per-round tile queues
    (round 0 visits every tile, later rounds the tiles queued by the round
    before); each image must equal its own run, where every tile is scanned
    every round, and a sample the oracle."""
    monkeypatch.setenv("THIN_TILE_SHAPE", shape)
    rng = np.random.default_rng(61)
    Fs = []
    for i in range(120):
        h, w = (int(x) for x in rng.integers(150, 520, size=2))
        Fs.append(synth.gen_blobs(h, w, 6100 + i, np.uint16 if i % 5 == 0 else np.uint8,
                                  nblobs=10, sigma=(3.0, 14.0)))
    lams = [int(x) for x in rng.choice([0, 5, 20, 50], size=len(Fs))]
    adjs = [i % 2 for i in range(len(Fs))]
    say("case work lists", shape)
    batch = [torch.from_numpy(F.copy()).cuda() for F in Fs]
    with thin.Context() as ctx:
        sts = ctx.run_batch(batch, lams, adjs)
        for i, F in enumerate(Fs):
            t = torch.from_numpy(F.copy()).cuda()
            st = ctx.run(t, lams[i], adjs[i])
            assert torch.equal(t, batch[i]), i
            assert (st.passes, st.lowerings) == (sts[i].passes, sts[i].lowerings), i
    for i in range(0, len(Fs), 15):
        assert_same(Fs[i], lams[i], adjs[i], batch[i].cpu().numpy(), sts[i])


@pytest.mark.parametrize("mode", ["default", "queues"])
@pytest.mark.parametrize("seed", [81, 82, 83])
def test_random_mixed_batches(seed, mode):
    """Random batches: both pixel types, both operators, random lambda and
    pairing, some images as pitched views of wider buffers; every image
    against the oracle.  "default": sides log-uniform in 3..1100 (a few
    megapixels: the 128x128 bit-flag tiles, tiny and partial tiles next to
    full ones); "queues": 180 images with sides in 40..700 on 64x64 bit-flag
    tiles, enough tiles for per-round tile queues and the per-launch tile
    counters."""
    rng = np.random.default_rng(seed)
    n, lo, hi = (90, 3, 1100) if mode == "default" else (180, 40, 700)
    kw = {} if mode == "default" else dict(tile=64, steps_per_round=16, threads=512, variant=4)
    Fs, ts, lams, adjs, ops = [], [], [], [], []
    for i in range(n):
        h, w = (int(round(np.exp(x))) for x in rng.uniform(np.log(lo), np.log(hi), size=2))
        dt = np.uint16 if rng.random() < 0.3 else np.uint8
        F = synth.gen_blobs(h, w, seed * 1000 + i, dt, nblobs=8, sigma=(2.0, 12.0))
        lam = int(rng.choice([0, 3, 20, 60]))
        if dt == np.uint16:
            lam *= 257
        Fs.append(F)
        lams.append(lam)
        adjs.append(int(rng.integers(0, 2)))
        ops.append("skeleton" if rng.random() < 0.3 else "leveling")
        if rng.random() < 0.3:
            pad = int(rng.integers(1, 9))
            big = torch.zeros((h, w + pad), dtype=torch.uint8 if dt == np.uint8 else torch.uint16,
                              device="cuda")
            big[:, :w] = torch.from_numpy(F.copy()).cuda()
            ts.append(big[:, :w])
        else:
            ts.append(torch.from_numpy(F.copy()).cuda())
    say("case random batch seed", seed, mode, "pixels", sum(F.size for F in Fs))
    with thin.Context(**kw) as ctx:
        sts = ctx.run_batch(ts, lams, adjs, ops=ops)
    torch.cuda.synchronize()
    for i in range(n):
        ref = oracle.sweep_dirty(Fs[i], lams[i], adjs[i], op=ops[i])
        assert_same(Fs[i], lams[i], adjs[i], ts[i].cpu().numpy(), sts[i], ref)


def test_c_thin_run_entry_point():
    """thin_run itself (Context.run goes through thin_run_batch)."""
    F = synth.gen_blobs(97, 131, 4242, np.uint16, nblobs=8, sigma=(2.0, 9.0))
    t = torch.from_numpy(F.copy()).cuda()
    st = thin.thin_stats()
    say("case thin_run entry")
    with thin.Context() as ctx:
        torch.cuda.synchronize()
        rc = thin.thin_run(ctx.handle, t.data_ptr(), F.shape[0], F.shape[1], thin.THIN_U16,
                           300, thin.THIN_ADJ_4_8, st)
        assert rc == thin.THIN_OK
    assert_same(F, 300, 1, t.cpu().numpy(), thin.Stats.of(st))


@pytest.mark.parametrize("shape", [(3, 70001), (70001, 3), (5, 40003), (40003, 4), (2049, 7)])
def test_extreme_aspect_ratios(shape):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    F = rng.integers(0, 40, size=shape).astype(np.uint8)
    say("case aspect", shape)
    got, st = gpu_thin(F, 5, 0)
    assert_same(F, 5, 0, got, st)
