"""GPU parity of the batched path: many independent self-joins in one
persistent matrix-core launch under a hipGraph, each job's pairs compared
with the oracle bit-exactly."""
import os

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


def make_jobs(count, seed, n_lo=200, n_hi=3000, dims=(1, 3, 8, 16, 18, 32, 64, 77)):
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(count):
        n = int(rng.integers(n_lo, n_hi))
        d = int(rng.choice(dims))
        if rng.random() < 0.5:
            P = datagen.uniform_grid(n, d, seed * 100 + j)
        else:
            P = datagen.gaussian_mixture(n, d, 5, datagen.uniform_std(d, 0.01, 0.3, j), seed * 100 + j)
        target = float(rng.integers(2, 40))
        eps, _ = oracle.calibrate_eps(P, target, np.arange(0, n, 3))
        jobs.append((P, eps))
    return jobs


def fetch_job(sj, h, j):
    first, count = sj.selfjoin_batch_range(h, j)
    oi = torch.empty(count, dtype=torch.int32, device="cuda")
    oj = torch.empty(count, dtype=torch.int32, device="cuda")
    od = torch.empty(count, dtype=torch.float32, device="cuda")
    if count:
        assert sj.selfjoin_batch_fetch(h, j, 0, oi, oj, od, max_pairs=count) == count
    return (oi.cpu().numpy().view(np.uint32), oj.cpu().numpy().view(np.uint32),
            od.cpu().numpy())


def check_batch(jobs, precision="fp16", autotune=False):
    from paper_1809_09930_amd import selfjoin as sj
    pts = [torch.from_numpy(P).cuda() for P, _ in jobs]
    h = sj.selfjoin_run_batched(pts, [e for _, e in jobs], precision=precision, autotune=autotune)
    try:
        info = sj.selfjoin_batch_get_info(h)
        total = 0
        for j, (P, eps) in enumerate(jobs):
            gi, gj, gd = fetch_job(sj, h, j)
            ri, rj, rs = oracle.bruteforce(P, eps, with_dist=True)
            assert np.array_equal(gi, ri) and np.array_equal(gj, rj), j
            np.testing.assert_allclose(gd, np.sqrt(rs), rtol=1e-5, atol=1e-30)
            total += len(ri)
        assert info["pairs"] == total
        # a replay of the captured graph gives the same result
        sj.selfjoin_batch_replay(h)
        gi, gj, _ = fetch_job(sj, h, 0)
        ri, rj = oracle.bruteforce(*jobs[0])
        assert np.array_equal(gi, ri) and np.array_equal(gj, rj)
        return info
    finally:
        sj.selfjoin_batch_free(h)


def test_batched_mixed_jobs_match_oracle():
    info = check_batch(make_jobs(12, 1))
    assert info["njobs"] == 12 and info["n_wu"] > 0 and info["grid"] > 0


def test_batched_bf16_and_empty_job():
    jobs = make_jobs(5, 2)
    jobs.append((np.zeros((0, 4), np.float32), 0.5))
    jobs.append((np.full((50, 6), 0.25, np.float32), 1e-6))
    check_batch(jobs, precision="bf16")


def test_batched_autotune_then_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("SJ_TUNE_CACHE", str(tmp_path / "tune.txt"))
    jobs = make_jobs(6, 3)
    info = check_batch(jobs, autotune=True)
    assert info["tuned"] in (1, 2)
    info2 = check_batch(jobs, autotune=True)
    assert info2["tuned"] == 2
    assert info2["tile_candidates"] == info["tile_candidates"]


def test_overflow_detected_and_rerun(monkeypatch):
    """SJ_DEBUG_UNDERSIZE makes the first result buffer far too small: the
    device counter must detect it and the rerun must give the exact set."""
    monkeypatch.setenv("SJ_DEBUG_UNDERSIZE", "1")
    check_batch(make_jobs(4, 4))
    from test_gpu_parity import assert_same_as_oracle
    P = datagen.uniform_grid(3000, 16, 5)
    eps, _ = oracle.calibrate_eps(P, 30, np.arange(0, 3000, 3))
    for prec in ("fp32", "fp16", "bf16"):
        info = assert_same_as_oracle(P, eps, precision=prec)
        assert_same_as_oracle(P, eps, precision=prec, batch_pairs=20000)
        if prec == "bf16":
            assert info["rechecks"] > 16  # the 16-slot band list overflowed


def test_batched_argument_errors():
    from paper_1809_09930_amd import selfjoin as sj
    P = torch.zeros((10, 90), dtype=torch.float32, device="cuda")
    with pytest.raises(sj.SelfJoinError) as e:
        sj.selfjoin_run_batched([P], [0.1])
    assert e.value.code == sj.SJ_ERR_INVALID_ARG
    big = torch.zeros((1 << 20, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(sj.SelfJoinError) as e:
        sj.selfjoin_run_batched([big], [0.1])
    assert e.value.code == sj.SJ_ERR_INVALID_ARG


def test_batched_error_in_one_job_of_many():
    """A job that fails inside the (multi-threaded) index builds fails the
    whole call with that job's error; the library stays usable."""
    from paper_1809_09930_amd import selfjoin as sj
    good = [torch.from_numpy(datagen.uniform_grid(500 + 50 * i, 8, 40 + i)).cuda()
            for i in range(12)]
    bad = good[7].clone()
    bad[3, 2] = float("nan")
    with pytest.raises(sj.SelfJoinError) as e:
        sj.selfjoin_run_batched(good[:7] + [bad] + good[8:], [0.3] * 12)
    assert e.value.code == sj.SJ_ERR_INVALID_ARG
    assert "NaN" in str(e.value)
    wide = torch.zeros((40, 90), dtype=torch.float32, device="cuda")
    with pytest.raises(sj.SelfJoinError) as e:
        sj.selfjoin_run_batched(good[:5] + [wide] + good[5:], [0.3] * 13)
    assert e.value.code == sj.SJ_ERR_INVALID_ARG
    check_batch([(g.cpu().numpy(), 0.3) for g in good[:4]])


def test_batched_256_workload_sampled_jobs_and_replays():
    """The benchmark's 256-job batch (its job shapes and epsilons, autotuned
    as bench.py runs it): sampled jobs against the oracle (whole result for
    jobs up to 30,000 points, sampled full rows above), every job's pairs
    sorted and symmetric, and three replays of the captured graph, with
    eager device work and synchronisations between them, each giving the
    same pairs again."""
    import json
    from conftest import GOLDEN
    from paper_1809_09930_amd import selfjoin as sj
    with open(os.path.join(GOLDEN, "eps.json")) as f:
        entry = json.load(f)["batched_256"]
    specs = datagen.batched_job_specs(entry["n_jobs"], entry["seed"])
    pts_h = [datagen.make_job(sp) for sp in specs]
    eps = [float.fromhex(j["hex"]) for j in entry["jobs"]]
    pts = [torch.from_numpy(P).cuda() for P in pts_h]
    rng = np.random.default_rng(17)
    sizes = np.array([len(P) for P in pts_h])
    pick = sorted({int(sizes.argmax()), int(sizes.argmin())} |
                  set(rng.choice(len(pts), 4, replace=False).tolist()))
    h = sj.selfjoin_run_batched(pts, eps, precision="fp16", autotune=True)
    try:
        info = sj.selfjoin_batch_get_info(h)
        total = 0
        for j in range(len(pts)):
            first, count = sj.selfjoin_batch_range(h, j)
            total += count
        assert total == info["pairs"]
        first_fetch = {}
        for j in pick:
            P, e = pts_h[j], eps[j]
            gi, gj, _ = fetch_job(sj, h, j)
            first_fetch[j] = (gi, gj)
            key = gi.astype(np.uint64) << np.uint64(32) | gj.astype(np.uint64)
            assert (np.diff(key.astype(np.int64)) > 0).all(), j
            rkey = np.sort(gj.astype(np.uint64) << np.uint64(32) | gi.astype(np.uint64))
            assert np.array_equal(rkey, key), j
            if len(P) <= 30000:
                ri, rj = oracle.bruteforce(P, e)
                assert np.array_equal(gi, ri) and np.array_equal(gj, rj), j
            else:
                rows = np.sort(rng.choice(len(P), 16, replace=False))
                cnt, js = oracle.rows(P, e, rows)
                starts = np.searchsorted(gi, rows)
                off = 0
                for r, c, st in zip(rows, cnt, starts):
                    assert np.array_equal(gj[st:st + int(c)], js[off:off + c]), (j, r)
                    off += int(c)
        for rep in range(3):
            x = torch.randn(1 << 20, device="cuda")
            torch.cuda.synchronize()
            assert float((x * x).sum()) > 0
            sj.selfjoin_batch_replay(h)
            torch.cuda.synchronize()
            for j in pick:
                gi, gj, _ = fetch_job(sj, h, j)
                assert np.array_equal(gi, first_fetch[j][0]), (rep, j)
                assert np.array_equal(gj, first_fetch[j][1]), (rep, j)
    finally:
        sj.selfjoin_batch_free(h)
