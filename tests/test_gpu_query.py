"""GPU parity of the general join Q join_eps E (Section 3.1; the self-join is
the case Q = E) through the C ABI, against the oracle's nested-loop join.

Pair lists must match the oracle bit-exactly (same pairs, same sorted
order); distances are checked at 1e-5 relative against the oracle's FP64
distances.  Cases: separately drawn query sets, queries partly or wholly
outside E's range, Q = E, duplicates, exact ties at epsilon, ragged and
empty sides, every distance filter, the multi-batch path, the CSR table
with empty rows, error paths, and the 2M x 16 workload split into the
entity-partitioned query sets Q_l of the paper's distributed scheme."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FILTERS = [dict(), dict(fp32_form="difference"), dict(fp32_form="norm"),
           dict(precision="fp16"), dict(precision="bf16")]


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sj():
    from paper_1809_09930_amd import selfjoin as sj
    return sj


def gpu_query_join(Q, E, eps, with_dist=True, offsets=False, **opts):
    """Build E's index and Q's query handle, run, fetch everything."""
    sj = _sj()
    te = torch.from_numpy(np.ascontiguousarray(E, dtype=np.float32)).cuda()
    tq = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
    he = sj.selfjoin_build_index(te, eps, **opts)
    hq = None
    try:
        hq = sj.selfjoin_build_query(he, tq)
        total = sj.selfjoin_run(hq)
        oi = torch.empty(total, dtype=torch.int32, device="cuda")
        oj = torch.empty(total, dtype=torch.int32, device="cuda")
        od = torch.empty(total, dtype=torch.float32, device="cuda") if with_dist else None
        if total:
            assert sj.selfjoin_fetch_pairs(hq, 0, oi, oj, od, max_pairs=total) == total
        off = None
        if offsets:
            off = torch.empty(len(Q) + 1, dtype=torch.int64, device="cuda")
            sj.selfjoin_fetch_offsets(hq, off)
            off = off.cpu().numpy()
        info = sj.selfjoin_get_info(hq)
        torch.cuda.synchronize()
        res = (oi.cpu().numpy().view(np.uint32), oj.cpu().numpy().view(np.uint32),
               od.cpu().numpy() if with_dist else None, info, off)
    finally:
        if hq is not None:
            sj.selfjoin_free(hq)
        sj.selfjoin_free(he)
    return res


def assert_query_join_matches(Q, E, eps, **opts):
    gi, gj, gd, info, off = gpu_query_join(Q, E, eps, offsets=True, **opts)
    oi, oj, os_ = oracle.join(Q, E, eps, with_dist=True)
    assert len(gi) == len(oi), (len(gi), len(oi))
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
    np.testing.assert_allclose(gd, np.sqrt(os_), rtol=1e-5, atol=1e-30)
    assert info["pairs"] == len(oi) and info["n"] == len(Q)
    want = np.searchsorted(oi, np.arange(len(Q) + 1), side="left")
    assert np.array_equal(off, want)
    return info, oi


def calibrated(P, target, stride=3):
    eps, _ = oracle.calibrate_eps(P, target, np.arange(0, len(P), stride))
    return eps


# --------------------------------------------------------------------------
@pytest.mark.parametrize("opts", FILTERS)
@pytest.mark.parametrize("m,n,d,seed,target", [
    (3001, 6000, 16, 1, 30), (1777, 5000, 8, 2, 20), (2500, 4000, 18, 3, 25),
    (1200, 3000, 64, 4, 12), (700, 2000, 90, 5, 10)])
def test_separate_query_set_matches_oracle(opts, m, n, d, seed, target):
    E = datagen.uniform_grid(n, d, seed)
    Q = datagen.uniform_grid(m, d, seed + 50)
    print("case", m, n, d, seed, opts, flush=True)
    info, oi = assert_query_join_matches(Q, E, calibrated(E, target), **opts)
    assert len(oi) > m  # not vacuous


@pytest.mark.parametrize("opts", FILTERS)
def test_queries_partly_and_wholly_outside_the_indexed_range(opts):
    """Shifted queries: some overlap E's box, some lie just beyond its edge
    (they search clamped boundary cells), some are far away (no cells)."""
    E = datagen.uniform_grid(5000, 12, 21)
    eps = calibrated(E, 25)
    rng = np.random.default_rng(22)
    Q = datagen.uniform_grid(3000, 12, 23).astype(np.float64)
    Q[:1000, 0] += 0.6                       # half outside along dim 0
    Q[1000:1500, 3] = 1.0 + rng.random(500) * eps * 0.9   # just beyond the edge
    Q[1500:1700] += 5.0                      # far away: no neighbours
    Q[1700:1800, 7] = -3.0 * eps             # far along one dimension only
    Q = Q.astype(np.float32)
    print("case outside", opts, flush=True)
    info, oi = assert_query_join_matches(Q, E, eps, **opts)
    counts = np.bincount(oi, minlength=len(Q))
    assert (counts[1500:1800] == 0).all() and counts[1000:1500].sum() > 0


@pytest.mark.parametrize("opts", [dict(), dict(precision="fp16")])
def test_queries_equal_to_entries_give_the_self_join(opts):
    E = datagen.uniform_grid(4000, 16, 31)
    eps = calibrated(E, 30)
    gi, gj, _, _, _ = gpu_query_join(E, E, eps, with_dist=False, **opts)
    si, sj_ = oracle.bruteforce(E, eps)
    assert np.array_equal(gi, si) and np.array_equal(gj, sj_)


@pytest.mark.parametrize("opts", FILTERS)
def test_duplicates_and_exact_ties(opts):
    """Integer lattice points (exact distances): ties at exactly eps are in,
    and queries that duplicate indexed points find them at distance 0."""
    g = np.arange(0, 14, dtype=np.float32)
    E = np.array([(x, y, z) for x in g for y in g for z in g], dtype=np.float32)
    rng = np.random.default_rng(41)
    Q = np.concatenate([E[rng.choice(len(E), 300, replace=False)],
                        rng.integers(-2, 16, size=(500, 3)).astype(np.float32)])
    for eps in (1.0, 2.0, 3.0):
        print("case lattice", eps, opts, flush=True)
        info, oi = assert_query_join_matches(Q, E, eps, **opts)


@pytest.mark.parametrize("m", [0, 1, 63, 65, 129])
def test_ragged_and_empty_query_sets(m):
    E = datagen.uniform_grid(3000, 10, 51)
    eps = calibrated(E, 20)
    Q = datagen.uniform_grid(m, 10, 52) if m else np.zeros((0, 10), np.float32)
    for opts in (dict(), dict(precision="bf16")):
        assert_query_join_matches(Q, E, eps, **opts)


def test_empty_indexed_set():
    sj = _sj()
    he = sj.selfjoin_build_index(torch.zeros((0, 6), dtype=torch.float32, device="cuda"), 0.5)
    try:
        hq = sj.selfjoin_build_query(he, torch.rand(100, 6, device="cuda"))
        try:
            assert sj.selfjoin_run(hq) == 0
            off = torch.empty(101, dtype=torch.int64)
            sj.selfjoin_fetch_offsets(hq, off)
            assert int(off.abs().sum()) == 0
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)


@pytest.mark.parametrize("opts", [dict(min_batches=3), dict(batch_pairs=4000),
                                  dict(min_batches=4, precision="fp16")])
def test_multi_batch_query_join(opts):
    """Results streamed to pinned host memory in batches of query rows."""
    E = datagen.uniform_grid(5000, 16, 61)
    Q = datagen.uniform_grid(3500, 16, 62)
    eps = calibrated(E, 30)
    info, _ = assert_query_join_matches(Q, E, eps, **opts)
    assert info["batches"] >= 2 and info["result_on_host"] == 1


@pytest.mark.parametrize("opts", [dict(), dict(precision="bf16")])
def test_result_and_band_overflow_paths(opts, monkeypatch):
    """Undersized first result buffer and band list (host-side fault
    injection): the resize-and-rerun paths give the same result."""
    monkeypatch.setenv("SJ_DEBUG_UNDERSIZE", "1")
    E = datagen.uniform_grid(4000, 16, 71)
    Q = datagen.uniform_grid(2000, 16, 72)
    assert_query_join_matches(Q, E, calibrated(E, 40), **opts)


def test_host_inputs_and_outputs():
    sj = _sj()
    E = datagen.uniform_grid(3000, 8, 81)
    Q = datagen.uniform_grid(1500, 8, 82)
    eps = calibrated(E, 20)
    oi, oj = oracle.join(Q, E, eps)
    he = sj.selfjoin_build_index(torch.from_numpy(E), eps)
    try:
        hq = sj.selfjoin_build_query(he, torch.from_numpy(Q))
        try:
            total = sj.selfjoin_run(hq)
            gi = torch.empty(total, dtype=torch.int32)
            gj = torch.empty(total, dtype=torch.int32)
            sj.selfjoin_fetch_pairs(hq, 0, gi, gj, None, max_pairs=total)
            assert np.array_equal(gi.numpy().view(np.uint32), oi)
            assert np.array_equal(gj.numpy().view(np.uint32), oj)
            # the index itself still runs and fetches its own self-join
            assert sj.selfjoin_run(he) == len(oracle.bruteforce(E, eps)[0])
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)


def test_query_join_errors():
    sj = _sj()
    E = torch.rand(500, 4, device="cuda")
    he = sj.selfjoin_build_index(E, 0.1)
    try:
        bad = torch.rand(50, 4, device="cuda")
        bad[7, 2] = float("nan")
        with pytest.raises(sj.SelfJoinError) as e:
            sj.selfjoin_build_query(he, bad)
        assert e.value.code == sj.SJ_ERR_INVALID_ARG
        hq = sj.selfjoin_build_query(he, torch.rand(50, 4, device="cuda"))
        try:
            with pytest.raises(sj.SelfJoinError) as e:
                sj.selfjoin_build_query(hq, torch.rand(5, 4, device="cuda"))
            assert e.value.code == sj.SJ_ERR_INVALID_ARG
            with pytest.raises(sj.SelfJoinError) as e:
                sj.selfjoin_fetch_pairs(hq, 0, torch.empty(4, dtype=torch.int32), None, None)
            assert e.value.code == sj.SJ_ERR_STATE
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)
    # FP16 index whose epsilon reaches beyond the FP16 range for queries
    wide = torch.rand(400, 3, device="cuda") * 8000.0
    hf = sj.selfjoin_build_index(wide, 9000.0, precision="fp16")
    try:
        with pytest.raises(sj.SelfJoinError) as e:
            sj.selfjoin_build_query(hf, wide[:10])
        assert e.value.code == sj.SJ_ERR_INVALID_ARG
    finally:
        sj.selfjoin_free(hf)


# --------------------------------------------------------------------------
# The 2M x 16 workload split into the entity-partitioned query sets Q_l of
# the paper's distributed scheme (Q_l = every N_b-th point from offset l):
# the union of the rows of all Q_l join D is the self-join of D.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_uniform_2m_d16_query_set_sampled_rows(prec):
    import json
    import os
    from conftest import GOLDEN
    sj = _sj()
    with open(os.path.join(GOLDEN, "eps.json")) as f:
        table = json.load(f)
    eps = float.fromhex(table["uniform_2m_d16"]["eps"]["64"]["hex"])
    P = datagen.make_workload("uniform_2m_d16")
    n, nb, l = len(P), 32, 5
    Q = np.ascontiguousarray(P[l::nb])
    print("case 2m query set", prec, flush=True)
    he = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps, precision=prec)
    try:
        hq = sj.selfjoin_build_query(he, torch.from_numpy(Q).cuda())
        try:
            total = sj.selfjoin_run(hq)
            oi = torch.empty(total, dtype=torch.int32, device="cuda")
            oj = torch.empty(total, dtype=torch.int32, device="cuda")
            sj.selfjoin_fetch_pairs(hq, 0, oi, oj, None, max_pairs=total)
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)
    key = (oi.to(torch.int64) << 32) | oj.to(torch.int64)
    assert bool((key[1:] > key[:-1]).all())
    # every query finds itself (it is a point of D)
    qi = torch.arange(len(Q), device="cuda", dtype=torch.int64)
    assert bool(torch.isin((qi << 32) | (qi * nb + l), key).all())
    rng = np.random.default_rng(9)
    rows = np.sort(rng.choice(len(Q), size=32, replace=False))
    cnt, js = oracle.rows(P, eps, rows * nb + l)
    starts = torch.searchsorted(oi, torch.from_numpy(rows.astype(np.int32)).cuda()).tolist()
    off = 0
    for r, c, st in zip(rows, cnt, starts):
        got = oj[st:st + int(c)].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, js[off:off + c]), r
        if st + int(c) < total:
            assert int(oi[st + int(c)]) != r
        off += int(c)
    sd = total / len(Q) - 1.0
    assert 40 < sd < 90


def test_entries_freed_before_the_query_handle():
    """Freeing the index first keeps it alive for its query handles: the
    query handle still runs and fetches, and the last free releases both."""
    sj = _sj()
    E = datagen.uniform_grid(3000, 8, 91)
    Q = datagen.uniform_grid(900, 8, 92)
    eps = calibrated(E, 20)
    oi, oj = oracle.join(Q, E, eps)
    he = sj.selfjoin_build_index(torch.from_numpy(E).cuda(), eps)
    hq1 = sj.selfjoin_build_query(he, torch.from_numpy(Q).cuda())
    hq2 = sj.selfjoin_build_query(he, torch.from_numpy(Q[:100]).cuda())
    sj.selfjoin_free(he)
    for hq, m in ((hq1, len(Q)), (hq2, 100)):
        total = sj.selfjoin_run(hq)
        gi = torch.empty(total, dtype=torch.int32, device="cuda")
        gj = torch.empty(total, dtype=torch.int32, device="cuda")
        sj.selfjoin_fetch_pairs(hq, 0, gi, gj, None, max_pairs=total)
        keep = oi < m
        assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi[keep])
        assert np.array_equal(gj.cpu().numpy().view(np.uint32), oj[keep])
        sj.selfjoin_free(hq)


@pytest.mark.parametrize("opts", [dict(), dict(precision="fp16")])
def test_every_query_far_and_one_dimension(opts):
    """All queries beyond E's range (no query cell at all), and d = 1."""
    E = datagen.uniform_grid(2000, 4, 93)
    eps = calibrated(E, 15)
    far = datagen.uniform_grid(500, 4, 94) + np.float32(10.0)
    info, oi = assert_query_join_matches(far, E, eps, **opts)
    assert len(oi) == 0 and info["n_cells"] == 0
    E1 = datagen.uniform_grid(4000, 1, 95)
    Q1 = np.concatenate([datagen.uniform_grid(700, 1, 96), np.float32([[1.0], [-0.001]])])
    assert_query_join_matches(Q1, E1, 0.002, **opts)
