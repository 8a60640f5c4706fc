"""The no-allocation row-start entry point against selfjoin_fetch_offsets,
through the C ABI: device and host outputs, a device-resident and a
host-resident (multi-batch) result, two calls in a row with the second on a
smaller input, and the size limit of its fixed array."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _offsets_both_ways(sj, P, eps, **opts):
    """(reference offsets, no-alloc offsets on the device, on the host)."""
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps, **opts)
    try:
        sj.selfjoin_run(h)
        n = len(P)
        ref = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        sj.selfjoin_fetch_offsets(h, ref)
        # garbage in the outputs first: the call must overwrite every entry
        got_d = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda")
        sj.selfjoin_fetch_offsets_noalloc(h, got_d)
        got_h = torch.full((n + 1,), -7, dtype=torch.int64)
        sj.selfjoin_fetch_offsets_noalloc(h, got_h)
        info = sj.selfjoin_get_info(h)
        torch.cuda.synchronize()
        return ref.cpu().numpy(), got_d.cpu().numpy(), got_h.numpy(), info
    finally:
        sj.selfjoin_free(h)


@pytest.mark.parametrize("opts", [dict(), dict(batch_pairs=4000, min_batches=3)])
def test_noalloc_offsets_match_fetch_offsets_twice(opts):
    from paper_1809_09930_amd import selfjoin as sj
    big = datagen.uniform_grid(6000, 12, 301)
    small = datagen.offgrid("normal_binades", 1500, 7, 302)
    for P, target in ((big, 25), (small, 12)):  # the second call on a smaller input
        eps, _ = oracle.calibrate_eps(P, target, np.arange(0, len(P), 5))
        print("case noalloc", len(P), opts, flush=True)
        ref, got_d, got_h, info = _offsets_both_ways(sj, P, eps, **opts)
        assert np.array_equal(got_d, ref)
        assert np.array_equal(got_h, ref)
        oi, _ = oracle.bruteforce(P, eps)
        assert np.array_equal(ref, np.searchsorted(oi, np.arange(len(P) + 1), side="left"))
        if opts:
            assert info["result_on_host"] == 1


def test_noalloc_offsets_query_handle_and_limit():
    """A query handle (rows may be empty), and a handle whose n is beyond the
    fixed array for host output: a clear error, and device output still works."""
    from paper_1809_09930_amd import selfjoin as sj
    E = datagen.uniform_grid(3000, 5, 303)
    Q = datagen.uniform_grid(800, 5, 304) * np.float32(1.5)
    eps = 0.08
    he = sj.selfjoin_build_index(torch.from_numpy(E).cuda(), eps)
    try:
        hq = sj.selfjoin_build_query(he, torch.from_numpy(Q).cuda())
        try:
            sj.selfjoin_run(hq)
            ref = torch.empty(len(Q) + 1, dtype=torch.int64, device="cuda")
            sj.selfjoin_fetch_offsets(hq, ref)
            got = torch.full((len(Q) + 1,), -1, dtype=torch.int64, device="cuda")
            sj.selfjoin_fetch_offsets_noalloc(hq, got)
            assert torch.equal(got, ref)
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)
    oi, _ = oracle.join(Q, E, eps)
    assert np.array_equal(ref.cpu().numpy(),
                          np.searchsorted(oi, np.arange(len(Q) + 1), side="left"))

    n = 7_000_000  # (n + 1) * 8 bytes of counts exceed the array for host output
    P = (np.arange(n, dtype=np.float64) * 2.0 ** -10).astype(np.float32).reshape(n, 1)
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), 2.0 ** -11)
    try:
        assert sj.selfjoin_run(h) == n  # points 2^-10 apart: only the self pairs
        with pytest.raises(sj.SelfJoinError) as e:
            sj.selfjoin_fetch_offsets_noalloc(h, torch.empty(n + 1, dtype=torch.int64))
        assert e.value.code == sj.SJ_ERR_INVALID_ARG
        got = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        sj.selfjoin_fetch_offsets_noalloc(h, got)
        assert torch.equal(got.cpu(), torch.arange(n + 1, dtype=torch.int64))
    finally:
        sj.selfjoin_free(h)
