"""GPU parity of the pixel work-list engine (the re-examination rule of
section 2.2 as explicit per-class candidate lists) through the C ABI.

Started with every interior candidate pending, the engine examines exactly
the candidates the oracle's dirty-pixel sweep examines, so besides the image,
the pass count and the lowering count, its examination count must equal the
oracle's.  The tiled engine hands a single small image's convergence tail to
the same kernel; those runs must stay bit-exact (their examination count is
larger: the hand-over starts from every candidate near a pixel changed in the
last round).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1603_09180_amd import synth, thin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WL = thin.THIN_ENGINE_WORKLIST


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_thin(F, lam, adj, op="leveling", **kw):
    t = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    with thin.Context(**kw) as ctx:
        st = ctx.run(t, lam, adj, op=op, allow_limit=bool(kw.get("max_passes")))
    torch.cuda.synchronize()
    return t.cpu().numpy(), st


def check(F, lam, adj, got, st, op="leveling", exams=True):
    ref = oracle.sweep_dirty(F, lam, adj, op=op)
    bad = np.argwhere(got != ref.image)
    assert bad.size == 0, f"{len(bad)} pixels differ, first at {bad[:5].tolist()}"
    assert (st.passes, st.lowerings, st.converged) == (ref.passes, ref.lowerings, True)
    if exams:
        assert st.examinations == ref.examinations
    else:
        assert st.examinations >= ref.examinations


@pytest.mark.parametrize("name,make", [("blobs_128", synth.blobs_128),
                                       ("ridges_512", synth.ridges_512),
                                       ("skeleton_512", synth.skeleton_512)])
def test_examinations_equal_the_oracle(name, make):
    job = make()
    F = job.image()
    say("case worklist", name)
    got, st = gpu_thin(F, job.lam, job.adj, op=job.op, engine=WL)
    check(F, job.lam, job.adj, got, st, op=job.op)


def _cases():
    rng = np.random.default_rng(808)
    sides = [3, 4, 5, 9, 33, 64, 65, 127, 200, 257]
    out = []
    for k in range(24):
        h, w = int(rng.choice(sides)), int(rng.choice(sides))
        dt = np.uint8 if k % 2 == 0 else np.uint16
        lam = int(rng.choice([0, 1, 5, 20, 50, 500, 2**32 - 1]))
        if dt == np.uint8 and lam == 500:
            lam = 50
        out.append((k, h, w, dt, k % 4 // 2, lam, "skeleton" if k % 3 == 0 else "leveling"))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: "c%d_%dx%d_%s_a%d_l%d_%s" % (
    c[0], c[1], c[2], np.dtype(c[3]).name, c[4], c[5], c[6][:4]))
def test_fuzz(case):
    k, h, w, dt, adj, lam, op = case
    F = synth.gen_blobs(h, w, 8100 + k, dt, nblobs=6, sigma=(2.0, 12.0), noise=12.0)
    say("case worklist fuzz", case)
    got, st = gpu_thin(F, lam, adj, op=op, engine=WL)
    check(F, lam, adj, got, st, op=op)


def test_pending_bitmaps_in_global_memory():
    """An image whose pending bitmaps do not fit LDS (above 512x512)."""
    F = synth.gen_blobs(1100, 1000, 8201, np.uint8, nblobs=12, sigma=(3.0, 16.0))
    say("case worklist global bitmaps")
    got, st = gpu_thin(F, 20, 0, engine=WL)
    check(F, 20, 0, got, st)


def test_batch_one_block_per_image():
    Fs = [synth.gen_blobs(60 + 41 * i, 90 + 17 * i, 8300 + i, np.uint16 if i % 3 == 0 else np.uint8,
                          nblobs=8, sigma=(2.0, 10.0)) for i in range(9)]
    Fs.append(synth.gen_blobs(700, 800, 8310, np.uint16, nblobs=12))   # global bitmaps
    lams = [0, 7, 300, 20, 0, 2000, 50, 3, 0, 400]
    adjs = [i % 2 for i in range(len(Fs))]
    ts = [torch.from_numpy(F.copy()).cuda() for F in Fs]
    say("case worklist batch")
    with thin.Context(engine=WL) as ctx:
        sts = ctx.run_batch(ts, lams, adjs)
    for F, t, st, lam, adj in zip(Fs, ts, sts, lams, adjs):
        check(F, lam, adj, t.cpu().numpy(), st)


def test_pass_cap():
    job = synth.blobs_128()
    F = job.image()
    say("case worklist pass cap")
    got, st = gpu_thin(F, job.lam, job.adj, engine=WL, max_passes=3)
    ref = oracle.sweep(F, job.lam, job.adj, max_passes=3)
    assert np.array_equal(got, ref.image)
    assert not st.converged and st.passes == 3 and st.lowerings == ref.lowerings


@pytest.mark.parametrize("rate", ["0", "1e12"])
def test_tiled_tail_hand_over(rate, monkeypatch):
    """The tiled engine with the tail hand-over on (THIN_FLAG_TAIL) and its
    threshold at 0 (never) and huge (at the second counter read-back):
    bit-exact either way, with and without a pass cap."""
    monkeypatch.setenv("THIN_TAIL_RATE", rate)
    cases = [(synth.ridges_512().image(), 20, 0, "leveling"),
             (synth.ridges_512().image()[:300, :257].copy(), 10, 0, "skeleton"),
             (synth.gen_blobs(333, 190, 8401, np.uint16, nblobs=10, sigma=(3.0, 20.0)), 500, 1,
              "leveling"),
             (synth.blobs_128().image(), 0, 1, "leveling")]
    for F, lam, adj, op in cases:
        say("case tail hand-over rate", rate, F.shape, lam, adj, op)
        got, st = gpu_thin(F, lam, adj, op=op, tail=True)
        check(F, lam, adj, got, st, op=op, exams=False)
    F, lam, adj, _ = cases[0]
    got, st = gpu_thin(F, lam, adj, max_passes=40, tail=True)
    ref = oracle.sweep(F, lam, adj, max_passes=40)
    assert np.array_equal(got, ref.image) and st.passes == 40 and not st.converged
