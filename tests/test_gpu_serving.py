"""GPU serving (continuous batching) through the C ABI: every image comes out
bit-identical to the oracle and to a run of the same image alone, whether it
was served alone, joined a running batch between rounds, waited for room in
the serving budget, or stopped at a pass cap.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1603_09180_amd import serve, synth, thin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mix(seed=77, n=24):
    """Images of mixed sizes, dtypes, lambdas and adjacencies."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        kind = i % 4
        if kind == 0:
            F = synth.random_small(seed * 100 + i, max_side=60)
        elif kind == 1:
            h, w = (int(x) for x in rng.integers(40, 200, size=2))
            F = synth.gen_blobs(h, w, seed * 100 + i, synth.U16)
        elif kind == 2:
            h, w = (int(x) for x in rng.integers(40, 260, size=2))
            F = synth.gen_ridges(h, w, seed * 100 + i)
        else:
            h, w = (int(x) for x in rng.integers(3, 120, size=2))
            F = synth.gen_blobs(h, w, seed * 100 + i, sigma=3.0)
        lam = int(rng.choice([0, 5, 20, 50, 4000]))
        adj = int(rng.integers(0, 2))
        out.append((F, lam, adj))
    return out


def _serve_all(items, ctx, rounds=1, stagger=3):
    """Admits the items a few at a time between steps; returns outputs and
    stats by index."""
    tensors = [torch.from_numpy(F.copy()).cuda() for F, _, _ in items]
    stats = {}
    nxt = 0
    resident = 0
    while len(stats) < len(items):
        for _ in range(stagger):
            if nxt < len(items):
                F, lam, adj = items[nxt]
                assert ctx.serve_admit(tensors[nxt], lam, adj, tag=1000 + nxt)
                nxt += 1
        done, resident = ctx.serve_step(rounds)
        for tag, st in done:
            assert tag - 1000 not in stats
            stats[tag - 1000] = st
    assert resident == 0
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in tensors], stats


def _check_oracle(items, outs, stats):
    for i, (F, lam, adj) in enumerate(items):
        ref = oracle.sweep_dirty(F, lam, adj)
        bad = np.argwhere(outs[i] != ref.image)
        assert bad.size == 0, f"item {i} {F.shape}: {len(bad)} pixels differ"
        if min(F.shape) >= 3:
            assert (stats[i].passes, stats[i].lowerings) == (ref.passes, ref.lowerings), i
        else:
            assert stats[i].passes == 0
        assert stats[i].converged


@pytest.mark.parametrize("rounds", [1, 3])
def test_mix_matches_oracle_and_alone(rounds):
    items = _mix()
    say("case serving mix rounds", rounds)
    with thin.Context() as ctx:
        outs, stats = _serve_all(items, ctx, rounds=rounds)
    _check_oracle(items, outs, stats)
    # Each image served alone, then run alone through thin_run: same bits.
    with thin.Context() as ctx:
        for i, (F, lam, adj) in enumerate(items[:8]):
            t = torch.from_numpy(F.copy()).cuda()
            assert ctx.serve_admit(t, lam, adj, tag=i)
            while True:
                done, res = ctx.serve_step(rounds)
                if done:
                    break
            assert done[0][0] == i and res == 0
            assert np.array_equal(t.cpu().numpy(), outs[i])
            assert (done[0][1].passes, done[0][1].lowerings) == (stats[i].passes,
                                                                  stats[i].lowerings)
            t2 = torch.from_numpy(F.copy()).cuda()
            st = ctx.run(t2, lam, adj)
            assert np.array_equal(t2.cpu().numpy(), outs[i])
            assert (st.passes, st.lowerings) == (stats[i].passes, stats[i].lowerings)


def test_budget_refuses_then_admits():
    # 6 MiB budget: twins get about 4 MiB (the rest holds per-slot counters
    # and tile state), so three 1 MiB images always fit and eight never do.
    F = [synth.gen_blobs(1024, 1024, 900 + i) for i in range(8)]
    say("case serving budget")
    with thin.Context() as ref_ctx:
        want = []
        for f in F:
            t = torch.from_numpy(f.copy()).cuda()
            st = ref_ctx.run(t, 0, 0)
            want.append((t.cpu().numpy(), st))
    tensors = [torch.from_numpy(f.copy()).cuda() for f in F]
    with thin.Context(max_device_bytes=6 << 20) as ctx:
        admitted = [ctx.serve_admit(t, 0, 0, tag=i) for i, t in enumerate(tensors)]
        assert admitted[:3] == [True, True, True] and not all(admitted)
        assert admitted == sorted(admitted, reverse=True)  # refused from the first miss on
        waiting = [i for i, ok in enumerate(admitted) if not ok]
        finished = {}
        while len(finished) < len(F):
            while waiting and ctx.serve_admit(tensors[waiting[0]], 0, 0, tag=waiting[0]):
                waiting.pop(0)
            done, _ = ctx.serve_step(2)
            finished.update(done)
    for i in range(len(F)):
        assert np.array_equal(tensors[i].cpu().numpy(), want[i][0]), i
        assert (finished[i].passes, finished[i].lowerings) == (want[i][1].passes,
                                                                want[i][1].lowerings)


def test_budget_too_small_is_an_error():
    t = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with thin.Context(max_device_bytes=1 << 20) as ctx:
        with pytest.raises(thin.ThinError):
            ctx.serve_admit(t, 0, 0, tag=1)


def test_pass_cap_and_degenerate():
    F = synth.gen_blobs(90, 70, 123)
    part = oracle.sweep(F, 0, max_passes=3)
    assert part.limited
    small = (np.arange(10, dtype=np.uint8).reshape(2, 5) * 29)
    say("case serving pass cap")
    t = torch.from_numpy(F.copy()).cuda()
    ts = torch.from_numpy(small.copy()).cuda()
    with thin.Context(max_passes=3) as ctx:
        assert ctx.serve_admit(t, 0, 0, tag=7)
        assert ctx.serve_admit(ts, 0, 0, tag=8)
        got = {}
        for _ in range(10):
            done, res = ctx.serve_step(1)
            got.update(done)
            if res == 0:
                break
    assert set(got) == {7, 8}
    assert not got[7].converged and got[7].passes == 3 and got[7].lowerings == part.lowerings
    assert np.array_equal(t.cpu().numpy(), part.image)
    assert got[8].converged and got[8].passes == 0
    assert np.array_equal(ts.cpu().numpy(), small)


def test_replay_poisson_arrivals():
    items = _mix(seed=91, n=40)
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(1.0 / 4000.0, size=len(items)))
    reqs = [serve.Request(tag=i, image=torch.from_numpy(F.copy()).cuda(), lam=lam, adj=adj,
                          arrival=float(a))
            for i, ((F, lam, adj), a) in enumerate(zip(items, arrivals))]
    say("case serving replay")
    with thin.Context() as ctx:
        rep = serve.replay(ctx, reqs, rounds_per_step=2)
    torch.cuda.synchronize()
    assert rep.images == len(items) and len(rep.latencies_s) == len(items)
    assert (rep.latencies_s > 0).all()
    outs = [r.image.cpu().numpy() for r in reqs]
    _check_oracle(items, outs, rep.stats)


def test_replay_from_host_memory():
    """Requests in pinned host memory: copied in on a second stream when they
    arrive, copied back as they retire; every host result equals the oracle,
    and a large u8 and u16 image ride along with the small ones."""
    items = _mix(seed=93, n=30)
    items.append((synth.gen_blobs(1500, 1100, 9301, synth.U8), 20, 0))
    items.append((synth.gen_blobs(1200, 900, 9302, synth.U16), 300, 0))
    rng = np.random.default_rng(6)
    arrivals = np.cumsum(rng.exponential(1.0 / 3000.0, size=len(items)))
    reqs = []
    for i, ((F, lam, adj), a) in enumerate(zip(items, arrivals)):
        host = torch.from_numpy(F.copy()).pin_memory()
        out = torch.empty(host.shape, dtype=host.dtype, pin_memory=True)
        dev = torch.empty(host.shape, dtype=host.dtype, device="cuda")
        reqs.append(serve.Request(tag=i, image=dev, lam=lam, adj=adj, arrival=float(a),
                                  host_in=host, host_out=out))
    copy_stream = torch.cuda.Stream()
    say("case serving replay from host memory")
    with thin.Context() as ctx:
        rep = serve.replay(ctx, reqs, rounds_per_step=2, copy_stream=copy_stream)
    torch.cuda.synchronize()
    assert rep.images == len(items) and (rep.latencies_s > 0).all()
    outs = [r.host_out.numpy() for r in reqs]
    _check_oracle(items, outs, rep.stats)


def test_device_blob_generator():
    a = synth.gen_blobs_device(300, 200, 11, synth.U16)
    b = synth.gen_blobs_device(300, 200, 11, synth.U16)
    assert a.dtype == torch.uint16 and tuple(a.shape) == (300, 200)
    assert torch.equal(a.to(torch.int32), b.to(torch.int32))
    ref = synth.gen_blobs(300, 200, 11, synth.U16).astype(np.int64)
    got = a.to(torch.int32).cpu().numpy().astype(np.int64)
    # Same blobs, different noise draw: within twice the noise amplitude.
    assert np.abs(got - ref).max() <= 2 * 10 * 257 + 257
