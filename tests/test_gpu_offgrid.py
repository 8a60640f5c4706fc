"""GPU parity on float32 data off any coarse grid, through the C ABI.

The grid workloads of the other parity tests keep every float32 coordinate
difference exact, so the terms of the device error bands that cover a
rounded subtraction (FP32 difference form), rounded products against large
norms (FP32 norm form) and rounded centring and 16-bit quantisation (matrix
cores) are never reached there.  Here the coordinates are binary64 draws
rounded to the nearest float32: values of one dimension sit in different
binades and of both signs, so a - b rounds.  Every filter must still give
the canonical predicate's pair set (Section 3.1), bit-exactly and in (i, j)
order, and the partners placed within a few roundings of eps must reach the
FP64 recheck.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FILTERS = {
    "fp32_difference": dict(fp32_form="difference"),
    "fp32_norm": dict(fp32_form="norm"),
    "fp16": dict(precision="fp16"),
    "bf16": dict(precision="bf16"),
    "fp32_sortidu": dict(sortidu=True),
    "fp16_sortidu": dict(precision="fp16", sortidu=True),
}


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sj():
    from paper_1809_09930_amd import selfjoin as sj
    return sj


def gpu_join(P, eps, **opts):
    sj = _sj()
    t = torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32)).cuda()
    h = sj.selfjoin_build_index(t, eps, **opts)
    try:
        total = sj.selfjoin_run(h)
        oi = torch.empty(total, dtype=torch.int32, device="cuda")
        oj = torch.empty(total, dtype=torch.int32, device="cuda")
        od = torch.empty(total, dtype=torch.float32, device="cuda")
        if total:
            assert sj.selfjoin_fetch_pairs(h, 0, oi, oj, od, max_pairs=total) == total
        info = sj.selfjoin_get_info(h)
        torch.cuda.synchronize()
        return (oi.cpu().numpy().view(np.uint32), oj.cpu().numpy().view(np.uint32),
                od.cpu().numpy(), info)
    finally:
        sj.selfjoin_free(h)


def assert_same_as_oracle(P, eps, **opts):
    gi, gj, gd, info = gpu_join(P, eps, **opts)
    oi, oj, os_ = oracle.bruteforce(P, eps, with_dist=True)
    assert len(gi) == len(oi), (len(gi), len(oi))
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
    np.testing.assert_allclose(gd, np.sqrt(os_), rtol=1e-5, atol=1e-30)
    assert info["pairs"] == len(oi)
    return info


def calibrated(P, target, stride=3):
    eps, _ = oracle.calibrate_eps(P, target, np.arange(0, len(P), stride))
    return eps


CASES = [("uniform64", 3000, 16, 32), ("uniform64", 1500, 40, 20),
         ("normal_binades", 3000, 18, 30), ("normal_binades", 800, 90, 12),
         ("loguniform_signed", 2500, 8, 25), ("mixture_f32", 4000, 18, 40),
         ("normal_binades", 2049, 3, 10)]


@pytest.mark.parametrize("filt", list(FILTERS))
@pytest.mark.parametrize("kind,n,d,target", CASES)
def test_offgrid_matches_oracle(kind, n, d, target, filt):
    P = datagen.offgrid(kind, n, d, seed=1000 + n + d)
    print("case offgrid", kind, n, d, filt, flush=True)
    assert_same_as_oracle(P, calibrated(P, target), **FILTERS[filt])


@pytest.mark.parametrize("filt", list(FILTERS))
@pytest.mark.parametrize("kind,d", [("normal_binades", 6), ("uniform64", 16),
                                    ("loguniform_signed", 4), ("mixture_f32", 24)])
def test_offgrid_partners_at_radius(kind, d, filt):
    """Partners within a few float32 roundings of eps (un-snapped): the
    device band must hold them for the FP64 recheck and the result must be
    the oracle's."""
    base = datagen.offgrid(kind, 1200, d, seed=2000 + d)
    eps = calibrated(base, 8)
    near = datagen.partners_near_radius(base, eps, 600, seed=3000 + d)
    finer = datagen.partners_near_radius(base, eps, 300, seed=4000 + d, unit=2.0 ** -23)
    P = np.concatenate([base, near, finer])
    print("case partners", kind, d, filt, flush=True)
    info = assert_same_as_oracle(P, eps, **FILTERS[filt])
    assert info["rechecks"] > 0


@pytest.mark.parametrize("filt", ["fp32_difference", "fp32_norm", "fp16", "bf16"])
def test_offgrid_no_shortc_and_explicit_k(filt):
    P = datagen.offgrid("normal_binades", 2500, 12, seed=51)
    eps = calibrated(P, 20)
    assert_same_as_oracle(P, eps, shortc=False, **FILTERS[filt])
    assert_same_as_oracle(P, eps, k=2, reorder=False, **FILTERS[filt])


@pytest.mark.parametrize("filt", ["fp32_difference", "fp16", "bf16"])
def test_offgrid_multi_batch(filt):
    P = datagen.offgrid("uniform64", 2500, 16, seed=52)
    eps = calibrated(P, 30)
    info = assert_same_as_oracle(P, eps, batch_pairs=5000, **FILTERS[filt])
    assert info["batches"] >= 3


@pytest.mark.parametrize("filt", ["fp32_difference", "fp32_norm", "fp16", "bf16",
                                  "fp32_sortidu"])
def test_offgrid_query_join(filt):
    """Q join_eps E on off-grid sets, with Q shifted partly outside E's range
    and partners of E's points at eps placed in Q."""
    sj = _sj()
    E = datagen.offgrid("normal_binades", 3000, 10, seed=61)
    Q = datagen.offgrid("normal_binades", 1500, 10, seed=61)[:1000]
    Q[:200] += np.float32(0.75)
    eps = calibrated(E, 15)
    Q = np.concatenate([Q, datagen.partners_near_radius(E, eps, 500, seed=62)])
    te = torch.from_numpy(E).cuda()
    tq = torch.from_numpy(Q).cuda()
    he = sj.selfjoin_build_index(te, eps, **FILTERS[filt])
    try:
        hq = sj.selfjoin_build_query(he, tq)
        try:
            total = sj.selfjoin_run(hq)
            gi = torch.empty(total, dtype=torch.int32, device="cuda")
            gj = torch.empty(total, dtype=torch.int32, device="cuda")
            gd = torch.empty(total, dtype=torch.float32, device="cuda")
            if total:
                sj.selfjoin_fetch_pairs(hq, 0, gi, gj, gd, max_pairs=total)
            info = sj.selfjoin_get_info(hq)
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)
    oi, oj, os_ = oracle.join(Q, E, eps, with_dist=True)
    assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi)
    assert np.array_equal(gj.cpu().numpy().view(np.uint32), oj)
    np.testing.assert_allclose(gd.cpu().numpy(), np.sqrt(os_), rtol=1e-5, atol=1e-30)
    assert info["rechecks"] > 0


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_offgrid_batched_jobs(precision):
    """The persistent batched path on off-grid jobs of every kind, with
    partners at eps in half of them."""
    sj = _sj()
    rng = np.random.default_rng(71)
    jobs = []
    for j, kind in enumerate(datagen.OFFGRID_KINDS * 2):
        n = int(rng.integers(300, 2500))
        d = int(rng.choice([3, 8, 16, 18, 33, 64]))
        P = datagen.offgrid(kind, n, d, seed=7100 + j)
        eps = calibrated(P, float(rng.integers(3, 30)))
        if j % 2:
            P = np.concatenate([P, datagen.partners_near_radius(P, eps, n // 3, seed=7200 + j)])
        jobs.append((P, eps))
    pts = [torch.from_numpy(P).cuda() for P, _ in jobs]
    h = sj.selfjoin_run_batched(pts, [e for _, e in jobs], precision=precision)
    try:
        info = sj.selfjoin_batch_get_info(h)
        for j, (P, eps) in enumerate(jobs):
            first, count = sj.selfjoin_batch_range(h, j)
            oi = torch.empty(count, dtype=torch.int32, device="cuda")
            oj = torch.empty(count, dtype=torch.int32, device="cuda")
            if count:
                sj.selfjoin_batch_fetch(h, j, 0, oi, oj, None, max_pairs=count)
            ri, rj = oracle.bruteforce(P, eps)
            assert np.array_equal(oi.cpu().numpy().view(np.uint32), ri), j
            assert np.array_equal(oj.cpu().numpy().view(np.uint32), rj), j
        assert info["rechecks"] > 0
    finally:
        sj.selfjoin_batch_free(h)
