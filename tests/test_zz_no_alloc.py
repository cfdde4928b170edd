"""thin_run_noalloc (the entry point for callers that cannot allocate: its
scratch is the library's static per-device array) against thin_run through
the C ABI: identical bytes and statistics on two calls in a row, the second
on a smaller image (the array keeps the first call's contents), and a clear
THIN_ENOMEM, image untouched, for an image whose scratch does not fit."""
import sys

import numpy as np
import pytest

from paper_1603_09180_amd import synth, thin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call(fn, ctx, F, lam, adj):
    t = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    st = thin.thin_stats()
    torch.cuda.synchronize()
    dt = thin.THIN_U8 if F.dtype == np.uint8 else thin.THIN_U16
    rc = fn(ctx.handle, t.data_ptr(), F.shape[0], F.shape[1], dt, lam, adj, st)
    torch.cuda.synchronize()
    return rc, t.cpu().numpy(), thin.Stats.of(st)


CASES = [
    # (h, w, dtype, lambda, adjacency, seed): large first, then smaller
    [(1500, 1300, np.uint8, 20, 0, 11), (200, 333, np.uint8, 5, 0, 12)],
    [(1100, 1030, np.uint16, 300, 1, 13), (97, 131, np.uint16, 40, 1, 14)],
]


@pytest.mark.parametrize("pair", CASES, ids=["u8", "u16"])
def test_noalloc_matches_thin_run(pair):
    with thin.Context() as ctx:
        for h, w, dt, lam, adj, seed in pair:
            F = synth.gen_blobs(h, w, seed, dt, nblobs=12, sigma=(3.0, 14.0))
            say("case noalloc", h, w, np.dtype(dt).name, lam, adj)
            rc0, want, st0 = _call(thin.thin_run, ctx, F, lam, adj)
            rc1, got, st1 = _call(thin.thin_run_noalloc, ctx, F, lam, adj)
            assert rc0 == thin.THIN_OK and rc1 == thin.THIN_OK
            assert np.array_equal(got, want)
            assert (st1.passes, st1.lowerings, st1.converged) == (st0.passes, st0.lowerings,
                                                                  st0.converged)
            assert st1.passes > 1 and st1.lowerings > 0


def test_noalloc_refuses_what_does_not_fit():
    F = np.full((6000, 6000), 7, np.uint16)
    F[1:-1, 1:-1] = 200
    say("case noalloc too large")
    with thin.Context() as ctx:
        rc, got, st = _call(thin.thin_run_noalloc, ctx, F, 0, 0)
        assert rc == thin.THIN_ENOMEM
        assert "thin_run_noalloc" in thin.thin_last_error(ctx.handle)
        assert np.array_equal(got, F)
        # the context still works afterwards, with and without allocation
        small = synth.gen_blobs(90, 70, 15)
        rc0, want, _ = _call(thin.thin_run, ctx, small, 5, 0)
        rc1, got1, _ = _call(thin.thin_run_noalloc, ctx, small, 5, 0)
        assert rc0 == rc1 == thin.THIN_OK and np.array_equal(got1, want)
