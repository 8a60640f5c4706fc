"""GPU parity: the HIP self-join against the CPU oracle, through the C ABI.

Pair lists must match the oracle bit-exactly (same pairs, same sorted
order); distances are checked at 1e-5 relative against the oracle's FP64
distances.  Sizes span several work units, ragged tails and the edge cases
(empty input, one point, duplicates, d = 1 .. 128)."""
import numpy as np
import pytest

import datagen
import oracle
from conftest import load_matrix, load_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_join(P, eps, with_dist=True, host_input=False, **opts):
    from paper_1809_09930_amd import selfjoin as sj
    t = torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32))
    if not host_input:
        t = t.cuda()
    h = sj.selfjoin_build_index(t, eps, **opts)
    try:
        total = sj.selfjoin_run(h)
        oi = torch.empty(total, dtype=torch.int32, device="cuda")
        oj = torch.empty(total, dtype=torch.int32, device="cuda")
        od = torch.empty(total, dtype=torch.float32, device="cuda") if with_dist else None
        if total:
            assert sj.selfjoin_fetch_pairs(h, 0, oi, oj, od, max_pairs=total) == total
        info = sj.selfjoin_get_info(h)
        torch.cuda.synchronize()
        res = (oi.cpu().numpy().view(np.uint32), oj.cpu().numpy().view(np.uint32),
               od.cpu().numpy() if with_dist else None, info)
    finally:
        sj.selfjoin_free(h)
    return res


def assert_same_as_oracle(P, eps, **opts):
    gi, gj, gd, info = gpu_join(P, eps, **opts)
    oi, oj, os_ = oracle.bruteforce(P, eps, with_dist=True)
    assert len(gi) == len(oi), (len(gi), len(oi))
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
    ref = np.sqrt(os_)
    np.testing.assert_allclose(gd, ref, rtol=1e-5, atol=1e-30)
    assert info["pairs"] == len(oi)
    return info


def calibrated(P, target, stride=3):
    eps, _ = oracle.calibrate_eps(P, target, np.arange(0, len(P), stride))
    return eps


# --------------------------------------------------------------------------
def test_fig1_worked_example():
    P = load_matrix("fig1_points.txt", np.float32)
    want = {(p, p) for p in range(len(P))}
    for a, b, _ in load_rows("fig1_pairs.txt"):
        want |= {(int(a), int(b)), (int(b), int(a))}
    gi, gj, gd, info = gpu_join(P, 1.0)
    assert set(zip(gi.tolist(), gj.tolist())) == want
    assert_same_as_oracle(P, 1.0)


@pytest.mark.parametrize("n,d,seed,target", [
    (3000, 16, 1, 32), (2500, 8, 2, 20), (1999, 18, 3, 40), (1500, 64, 4, 16),
    (777, 90, 5, 12), (640, 128, 6, 10), (1000, 1, 7, 5), (1234, 3, 8, 25),
    (4097, 16, 9, 3)])
def test_uniform_matches_oracle(n, d, seed, target):
    P = datagen.uniform_grid(n, d, seed)
    assert_same_as_oracle(P, calibrated(P, target))


@pytest.mark.parametrize("n,d,seed", [(5000, 18, 11), (3000, 12, 12), (2000, 32, 13)])
def test_clustered_many_cells_matches_oracle(n, d, seed):
    std = datagen.decaying_std(d, 0.2, 0.002, seed)
    P = datagen.gaussian_mixture(n, d, 20, std, seed)
    eps = calibrated(P, 30)
    info = assert_same_as_oracle(P, eps)
    assert info["n_cells"] > 1
    assert info["candidates"] < n * n


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("n,d,seed,target", [
    (3000, 16, 1, 32), (2500, 8, 2, 20), (1999, 18, 3, 40), (1500, 64, 4, 16),
    (777, 90, 5, 12), (640, 128, 6, 10), (1000, 1, 7, 5), (4097, 16, 9, 3)])
def test_matrix_core_uniform_matches_oracle(prec, n, d, seed, target):
    P = datagen.uniform_grid(n, d, seed)
    info = assert_same_as_oracle(P, calibrated(P, target), precision=prec)
    assert info["precision"] == {"fp16": 1, "bf16": 2}[prec]


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("n,d,seed", [(5000, 18, 11), (3000, 12, 12), (2000, 90, 13)])
def test_matrix_core_clustered_matches_oracle(prec, n, d, seed):
    std = datagen.decaying_std(d, 0.2, 0.002, seed)
    P = datagen.gaussian_mixture(n, d, 20, std, seed)
    assert_same_as_oracle(P, calibrated(P, 30), precision=prec)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_matrix_core_band_is_rechecked(prec):
    """Many pairs sit right at eps: the 16-bit form cannot decide them, the
    FP64 recheck must, and the result must still equal the oracle's."""
    u = 2.0 ** -24
    rng = np.random.default_rng(77)
    base = datagen.uniform_grid(400, 4, 78)
    eps = 0.1
    # partners at distance eps * (1 + k * 2^-20), k in -3..3, along random axes
    extra = []
    for p in base[:150]:
        axis = rng.integers(0, 4)
        k = rng.integers(-3, 4)
        q = p.astype(np.float64).copy()
        q[axis] += eps * (1 + k * 2.0 ** -20)
        extra.append(np.round(q / u) * u)
    P = np.concatenate([base, np.array(extra, dtype=np.float32)])
    info = assert_same_as_oracle(P, eps, precision=prec)
    assert info["rechecks"] > 0


def test_matrix_core_batched_and_filters():
    P = datagen.uniform_grid(2500, 16, 51)
    eps = calibrated(P, 30)
    info = assert_same_as_oracle(P, eps, precision="fp16", batch_pairs=5000)
    assert info["batches"] >= 3
    assert_same_as_oracle(P, eps, precision="bf16", k=2, reorder=False)


def test_empty_single_and_duplicates():
    gi, gj, gd, info = gpu_join(np.zeros((0, 5), np.float32), 0.5)
    assert len(gi) == 0 and info["pairs"] == 0
    for prec in ("fp16", "bf16"):
        assert_same_as_oracle(np.full((300, 4), 0.375, np.float32), 1e-6, precision=prec)
        gi, gj, gd, _ = gpu_join(np.array([[0.5, 0.25, 0.125]], np.float32), 1e-3,
                                 precision=prec)
        assert gi.tolist() == [0] and gj.tolist() == [0]
    gi, gj, gd, _ = gpu_join(np.array([[0.5, 0.25, 0.125]], np.float32), 1e-3)
    assert gi.tolist() == [0] and gj.tolist() == [0] and gd.tolist() == [0.0]
    P = np.repeat(datagen.uniform_grid(40, 6, 21), 3, axis=0)
    assert_same_as_oracle(P, 0.05)
    # all points identical: one cell, every pair at distance 0
    assert_same_as_oracle(np.full((300, 4), 0.375, np.float32), 1e-6)


def test_ties_exactly_at_epsilon():
    u = 2.0 ** -24
    base = datagen.uniform_grid(500, 4, 31)
    extra = np.array([[0, 0, 0, 0], [3000 * u, 4000 * u, 0, 0],
                      [3000 * u, 3999 * u, 89 * u, 0], [3000 * u, 4000 * u, u, 0]],
                     dtype=np.float32)
    P = np.concatenate([extra, base])
    eps = 5000 * u  # eps^2 equals the squared distance of points 0 and 1
    gi, gj, _, _ = gpu_join(P, eps)
    s = set(zip(gi.tolist(), gj.tolist()))
    assert (0, 1) in s and (1, 0) in s and (0, 2) in s and (0, 3) not in s
    assert_same_as_oracle(P, eps)


@pytest.mark.parametrize("opts", [
    dict(k=1), dict(k=2), dict(k=6), dict(k=8), dict(reorder=False), dict(shortc=False),
    dict(k=3, reorder=False, shortc=False)])
def test_filters_do_not_change_the_result(opts):
    std = datagen.uniform_std(10, 0.01, 0.3, 41)
    P = datagen.gaussian_mixture(3000, 10, 8, std, 41)
    assert_same_as_oracle(P, calibrated(P, 25), **opts)


@pytest.mark.parametrize("opts", [dict(batch_pairs=5000), dict(min_batches=3),
                                  dict(batch_pairs=777, min_batches=5)])
def test_batched_results_equal_single_batch(opts):
    P = datagen.uniform_grid(2500, 16, 51)
    eps = calibrated(P, 30)
    info = assert_same_as_oracle(P, eps, **opts)
    assert info["batches"] >= 3 and info["result_on_host"] == 1


def test_host_input_and_host_outputs():
    from paper_1809_09930_amd import selfjoin as sj
    P = datagen.uniform_grid(1500, 8, 61)
    eps = calibrated(P, 20)
    oi, oj, os_ = oracle.bruteforce(P, eps, with_dist=True)
    h = sj.selfjoin_build_index(torch.from_numpy(P), eps)
    try:
        total = sj.selfjoin_run(h)
        assert total == len(oi)
        ci = torch.empty(total, dtype=torch.int32)
        cj = torch.empty(total, dtype=torch.int32)
        cd = torch.empty(total, dtype=torch.float32)
        assert sj.selfjoin_fetch_pairs(h, 0, ci, cj, cd, max_pairs=total) == total
        assert np.array_equal(ci.numpy().view(np.uint32), oi)
        assert np.array_equal(cj.numpy().view(np.uint32), oj)
        np.testing.assert_allclose(cd.numpy(), np.sqrt(os_), rtol=1e-5)
        # partial fetch from an offset, and the end of the result
        part = torch.empty(100, dtype=torch.int32)
        assert sj.selfjoin_fetch_pairs(h, total - 40, None, part, None, max_pairs=100) == 40
        assert np.array_equal(part.numpy()[:40].view(np.uint32), oj[-40:])
        assert sj.selfjoin_fetch_pairs(h, total, None, part, None, max_pairs=100) == 0
        with pytest.raises(sj.SelfJoinError) as e:
            sj.selfjoin_fetch_pairs(h, total + 1, None, part, None, max_pairs=1)
        assert e.value.code == sj.SJ_ERR_RANGE
    finally:
        sj.selfjoin_free(h)


def test_state_and_input_errors():
    from paper_1809_09930_amd import selfjoin as sj
    P = datagen.uniform_grid(100, 4, 71)
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), 0.1)
    try:
        out = torch.empty(4, dtype=torch.int32, device="cuda")
        with pytest.raises(sj.SelfJoinError) as e:
            sj.selfjoin_fetch_pairs(h, 0, out, None, None, max_pairs=4)
        assert e.value.code == sj.SJ_ERR_STATE
    finally:
        sj.selfjoin_free(h)
    bad = torch.from_numpy(P).cuda()
    bad[17, 2] = float("nan")
    with pytest.raises(sj.SelfJoinError) as e:
        sj.selfjoin_build_index(bad, 0.1)
    assert e.value.code == sj.SJ_ERR_INVALID_ARG
    bad[17, 2] = float("inf")
    with pytest.raises(sj.SelfJoinError) as e:
        sj.selfjoin_build_index(bad, 0.1)
    assert e.value.code == sj.SJ_ERR_INVALID_ARG


def test_reorder_permutation_matches_oracle():
    from paper_1809_09930_amd import selfjoin as sj
    std = np.array([0.01, 0.3, 0.05, 0.2, 0.002, 0.1])
    P = datagen.gaussian_mixture(20000, 6, 5, std, 81)
    perm_ref, var = oracle.reorder_perm(P)
    # the sample variances here are far apart, so the order is unambiguous
    assert np.min(np.diff(np.sort(var))) > 1e-4
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), 0.05)
    try:
        assert sj.selfjoin_get_perm(h, 6) == perm_ref.tolist()
    finally:
        sj.selfjoin_free(h)


def test_uniform_20k_d16_full_result():
    """The 20,000 x 16 uniform workload at its calibrated epsilon (mean
    neighbours ~ 32): the whole pair list against the oracle."""
    P = datagen.make_workload("uniform_20k_d16")
    rows = datagen.calibration_rows(len(P), datagen.WORKLOADS["uniform_20k_d16"]["seed"])
    eps, _ = oracle.calibrate_eps(P, 32, rows)
    info = assert_same_as_oracle(P, eps)
    assert info["candidates"] == len(P) ** 2  # uniform data: every cell is adjacent


def test_uniform_2m_d16_sampled_rows_and_symmetry():
    """The 2,000,000 x 16 workload in the benchmark's configuration (auto k,
    one symmetric batch): sampled full rows against the oracle, plus the
    symmetry and self-pair invariants over the whole result."""
    import json
    import os
    from conftest import GOLDEN
    with open(os.path.join(GOLDEN, "eps.json")) as f:
        table = json.load(f)
    eps = float.fromhex(table["uniform_2m_d16"]["eps"]["64"]["hex"])
    P = datagen.make_workload("uniform_2m_d16")
    from paper_1809_09930_amd import selfjoin as sj
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps)
    try:
        total = sj.selfjoin_run(h)
        oi = torch.empty(total, dtype=torch.int32, device="cuda")
        oj = torch.empty(total, dtype=torch.int32, device="cuda")
        sj.selfjoin_fetch_pairs(h, 0, oi, oj, None, max_pairs=total)
        info = sj.selfjoin_get_info(h)
    finally:
        sj.selfjoin_free(h)
    n = len(P)
    key = (oi.to(torch.int64) << 32) | oj.to(torch.int64)
    assert bool((key[1:] > key[:-1]).all())  # strictly sorted, unique
    rkey = (oj.to(torch.int64) << 32) | oi.to(torch.int64)
    assert bool(torch.equal(torch.sort(rkey).values, key))  # symmetric
    self_pairs = (oi == oj)
    assert int(self_pairs.sum()) == n
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(n, size=48, replace=False))
    cnt, js = oracle.rows(P, eps, rows)
    starts = torch.searchsorted(oi, torch.from_numpy(rows.astype(np.int32)).cuda())
    off = 0
    for r, c, st in zip(rows, cnt, starts.tolist()):
        got = oj[st:st + int(c)].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, js[off:off + c]), r
        if st + int(c) < total:
            assert int(oi[st + int(c)]) != r
        off += int(c)
    assert info["candidates"] == n * n
    sd = (total - n) / n
    assert 40 < sd < 90


@pytest.mark.parametrize("workload,target,prec", [
    ("uniform_2m_d64", "16", "bf16"),
    ("uniform_2m_d64", "128", "fp16"),
    ("mixture50_5m_d18", "50", "fp16"),
    ("mixture50_5m_d18", "50", "fp32"),
    ("mixture20_515k_d90", "50", "fp16"),
])
def test_full_size_workloads_sampled_rows(workload, target, prec):
    """The other full-size workloads at their calibrated epsilons: sampled
    full rows against the oracle, and the symmetry / self-pair invariants of
    the whole result."""
    import json
    import os
    from conftest import GOLDEN
    with open(os.path.join(GOLDEN, "eps.json")) as f:
        table = json.load(f)
    eps = float.fromhex(table[workload]["eps"][target]["hex"])
    P = datagen.make_workload(workload)
    from paper_1809_09930_amd import selfjoin as sj
    print("case", workload, target, prec, flush=True)
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps, precision=prec)
    try:
        total = sj.selfjoin_run(h)
        oi = torch.empty(total, dtype=torch.int32, device="cuda")
        oj = torch.empty(total, dtype=torch.int32, device="cuda")
        sj.selfjoin_fetch_pairs(h, 0, oi, oj, None, max_pairs=total)
        info = sj.selfjoin_get_info(h)
    finally:
        sj.selfjoin_free(h)
    n = len(P)
    key = (oi.to(torch.int64) << 32) | oj.to(torch.int64)
    assert bool((key[1:] > key[:-1]).all())
    rkey = (oj.to(torch.int64) << 32) | oi.to(torch.int64)
    assert bool(torch.equal(torch.sort(rkey).values, key))
    assert int((oi == oj).sum()) == n
    del rkey
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(n, size=24, replace=False))
    cnt, js = oracle.rows(P, eps, rows)
    starts = torch.searchsorted(oi, torch.from_numpy(rows.astype(np.int32)).cuda()).tolist()
    off = 0
    for r, c, st in zip(rows, cnt, starts):
        got = oj[st:st + int(c)].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, js[off:off + c]), r
        if st + int(c) < total:
            assert int(oi[st + int(c)]) != r
        off += int(c)
    assert info["candidates"] >= total


@pytest.mark.parametrize("form", ["difference", "norm"])
@pytest.mark.parametrize("n,d,seed,target", [
    (3000, 16, 1, 32), (2500, 8, 2, 20), (1999, 18, 3, 40), (1500, 64, 4, 16),
    (777, 90, 5, 12), (640, 128, 6, 10), (1000, 1, 7, 5), (4097, 24, 9, 3)])
def test_fp32_forms_match_oracle(form, n, d, seed, target):
    """Both evaluations of the FP32 filter, forced, on the same inputs."""
    P = datagen.uniform_grid(n, d, seed)
    info = assert_same_as_oracle(P, calibrated(P, target), fp32_form=form)
    assert info["fp32_form"] == {"difference": 1, "norm": 2}[form]


@pytest.mark.parametrize("form", ["difference", "norm"])
def test_fp32_forms_band_and_ties(form):
    """Pairs at eps * (1 + k 2^-20) and exact ties: the norm form's wider
    band must send them to the FP64 recheck and still agree with the oracle;
    clustered data with offsets far from the origin as well."""
    u = 2.0 ** -24
    rng = np.random.default_rng(91)
    base = datagen.uniform_grid(400, 6, 92)
    eps = 0.1
    extra = []
    for p in base[:200]:
        axis = rng.integers(0, 6)
        k = rng.integers(-3, 4)
        q = p.astype(np.float64).copy()
        q[axis] += eps * (1 + k * 2.0 ** -20)
        extra.append(np.round(q / u) * u)
    P = np.concatenate([base, np.array(extra, dtype=np.float32)])
    info = assert_same_as_oracle(P, eps, fp32_form=form)
    assert info["rechecks"] > 0
    ties = np.array([[0, 0, 0, 0], [3000 * u, 4000 * u, 0, 0],
                     [3000 * u, 3999 * u, 89 * u, 0], [3000 * u, 4000 * u, u, 0]],
                    dtype=np.float32)
    P = np.concatenate([ties, datagen.uniform_grid(500, 4, 31)])
    assert_same_as_oracle(P, 5000 * u, fp32_form=form)
    std = datagen.decaying_std(12, 0.2, 0.002, 93)
    P = (datagen.gaussian_mixture(3000, 12, 10, std, 93) + np.float32(1.5)).astype(np.float32)
    assert_same_as_oracle(P, calibrated(P, 30), fp32_form=form)
    assert_same_as_oracle(P, calibrated(P, 30), fp32_form=form, shortc=False)


def test_fp32_form_automatic_choice():
    """Automatic choice: the norm form on unit-range data up to 16
    dimensions, the difference form above 16 dimensions or when eps is tiny
    against the squared norms."""
    P = datagen.uniform_grid(2000, 16, 95)
    assert gpu_join(P, calibrated(P, 20))[3]["fp32_form"] == 2
    R = datagen.uniform_grid(2000, 24, 96)
    assert gpu_join(R, calibrated(R, 20))[3]["fp32_form"] == 1
    Q = (P * np.float32(1e-3) + np.float32(100.0)).astype(np.float32)  # tiny eps, large norms
    info = assert_same_as_oracle(Q, calibrated(Q, 20))
    assert info["fp32_form"] == 1


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_both_unit_kinds_match_oracle(prec):
    """The build takes units of one cell's queries for large cells and the
    small-cell units (FP32: one query per lane; matrix cores: one wave) when
    most lane work of cell units would fall on idle query slots; both kinds
    give the oracle's result."""
    kinds = {}
    # 8 cells of about 500 points, 16 cells of about 250: cell units
    kinds["d1_large"] = assert_same_as_oracle(datagen.uniform_grid(4000, 1, 41), 0.125,
                                              precision=prec)["units"]
    kinds["d2_large"] = assert_same_as_oracle(datagen.uniform_grid(4000, 2, 42), 0.25,
                                              precision=prec)["units"]
    # two tight clusters in 16 dimensions, each within eps of itself
    std = np.full(16, 0.002)
    C = datagen.gaussian_mixture(3000, 16, 2, std, 43)
    kinds["d16_clusters"] = assert_same_as_oracle(C, 0.05, precision=prec)["units"]
    # cells of one or two points: small-cell units
    for d, seed in ((2, 44), (16, 45)):
        P = datagen.uniform_grid(3000, d, seed)
        kinds[f"d{d}_small"] = assert_same_as_oracle(P, calibrated(P, 4), precision=prec)["units"]
    assert kinds["d1_large"] == kinds["d2_large"] == 1, kinds
    assert kinds["d2_small"] == kinds["d16_small"] == 2, kinds


@pytest.mark.parametrize("opts", [dict(), dict(precision="fp16"), dict(batch_pairs=3000),
                                  dict(min_batches=4, precision="bf16")])
def test_csr_neighbour_table(opts):
    """Row starts plus the j column form the neighbour table: row i holds
    exactly the oracle's neighbours of i, in ascending order."""
    from paper_1809_09930_amd import selfjoin as sj
    P = datagen.uniform_grid(2200, 12, 71)
    eps = calibrated(P, 25)
    oi, oj = oracle.bruteforce(P, eps)
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps, **opts)
    try:
        total = sj.selfjoin_run(h)
        nb = torch.empty(total, dtype=torch.int32, device="cuda")
        sj.selfjoin_fetch_pairs(h, 0, None, nb, None, max_pairs=total)
        off_d = torch.empty(len(P) + 1, dtype=torch.int64, device="cuda")
        sj.selfjoin_fetch_offsets(h, off_d)
        off_h = torch.empty(len(P) + 1, dtype=torch.int64)
        sj.selfjoin_fetch_offsets(h, off_h)
    finally:
        sj.selfjoin_free(h)
    want = np.searchsorted(oi, np.arange(len(P) + 1), side="left")
    assert np.array_equal(off_d.cpu().numpy(), want)
    assert np.array_equal(off_h.numpy(), want)
    assert np.array_equal(nb.cpu().numpy().view(np.uint32), oj)


# --------------------------------------------------------------------------
# The paper's synthetic family (exponential, rate 40, in [0, 1); Section 5.1)
# at the paper's own epsilons.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("n,d,eps", [(20000, 16, 0.05), (12000, 32, 0.10), (6000, 64, 0.18)])
def test_exponential_family_full_result(prec, n, d, eps):
    P = datagen.exponential_syn(n, d, 40.0, 100 + d)
    print("case syn", n, d, eps, prec, flush=True)
    assert_same_as_oracle(P, eps, precision=prec)


@pytest.mark.parametrize("workload,eps,prec", [
    ("syn_2m_d16", 0.05, "fp32"), ("syn_2m_d16", 0.05, "fp16"),
    ("syn_2m_d32", 0.08, "bf16"), ("syn_2m_d64", 0.16, "fp16"),
    ("syn_2m_d64", 0.18, "fp16")])  # 4.7e9 pairs: more than 2^32 keys in one sorted batch
def test_exponential_family_full_size_sampled_rows(workload, eps, prec):
    """Syn16/32/64D2M-shaped inputs at the paper's epsilons: sampled full
    rows against the oracle, sorted order and the self pairs."""
    from paper_1809_09930_amd import selfjoin as sj
    P = datagen.make_workload(workload)
    n = len(P)
    print("case", workload, eps, prec, flush=True)
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps, precision=prec)
    try:
        total = sj.selfjoin_run(h)
        oi = torch.empty(total, dtype=torch.int32, device="cuda")
        oj = torch.empty(total, dtype=torch.int32, device="cuda")
        sj.selfjoin_fetch_pairs(h, 0, oi, oj, None, max_pairs=total)
    finally:
        sj.selfjoin_free(h)
    assert bool((oi[1:] >= oi[:-1]).all())
    assert int((oi == oj).sum()) == n
    rng = np.random.default_rng(13)
    rows = np.sort(rng.choice(n, size=24, replace=False))
    cnt, js = oracle.rows(P, eps, rows)
    starts = torch.searchsorted(oi, torch.from_numpy(rows.astype(np.int32)).cuda()).tolist()
    off = 0
    for r, c, st in zip(rows, cnt, starts):
        got = oj[st:st + int(c)].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, js[off:off + c]), r
        if st + int(c) < total:
            assert int(oi[st + int(c)]) != r
        off += int(c)


# --------------------------------------------------------------------------
# SORTIDU (Section 4.3): cells sorted by an un-indexed dimension u, each
# block of queries searching only the points within eps of its u-range.
# The result is unchanged; the evaluated pairs can only shrink.
# --------------------------------------------------------------------------
def _spread_along_u(n, seed):
    """Three dimensions of ranges 8, 4 and 0.1: indexed on the first alone
    (k = 1, about 70 cells of side 0.12, so every cell holds several blocks
    of queries), the second (u) spans about 33 eps, so a block of queries,
    a slab of its cell along u, finds only part of each adjacent cell."""
    rng = np.random.default_rng(seed)
    P = rng.random((n, 3)) * np.array([8.0, 4.0, 0.1])
    return (np.round(P * 2 ** 20) / 2 ** 20).astype(np.float32)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("case", ["uniform", "clustered", "spread"])
def test_sortidu_matches_oracle_and_prunes(prec, case):
    if case == "uniform":
        P = datagen.uniform_grid(3000, 16, 81)
        eps, k = calibrated(P, 30), 0
    elif case == "clustered":
        std = datagen.decaying_std(18, 0.2, 0.002, 82)
        P = datagen.gaussian_mixture(5000, 18, 12, std, 82)
        eps, k = calibrated(P, 25), 4
    else:
        P = _spread_along_u(60000, 83)
        eps, k = 0.12, 1
    print("case sortidu", case, prec, flush=True)
    info_u = assert_same_as_oracle(P, eps, precision=prec, k=k, sortidu=True)
    info_p = assert_same_as_oracle(P, eps, precision=prec, k=k)
    assert info_u["evaluated"] <= info_p["evaluated"]
    if case == "spread":  # blocks are slabs of about a quarter of u's range
        assert info_u["evaluated"] * 2 < info_p["evaluated"]


def test_sortidu_with_every_dimension_indexed_and_in_batches():
    """k = d (u is then an indexed dimension), and the multi-batch path."""
    P = datagen.uniform_grid(2500, 5, 84)
    eps = calibrated(P, 20)
    assert_same_as_oracle(P, eps, k=5, sortidu=True)
    assert_same_as_oracle(P, eps, sortidu=True, min_batches=3)
    assert_same_as_oracle(P, eps, sortidu=True, batch_pairs=4000, precision="fp16")


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_sortidu_general_join(prec):
    from paper_1809_09930_amd import selfjoin as sj
    E = _spread_along_u(30000, 85)
    Q = _spread_along_u(8000, 86)
    Q[:1000, 1] += 3.9  # partly beyond E's range along u
    eps = 0.12
    oi, oj = oracle.join(Q, E, eps)
    he = sj.selfjoin_build_index(torch.from_numpy(E).cuda(), eps, k=1, precision=prec,
                                 sortidu=True)
    try:
        hq = sj.selfjoin_build_query(he, torch.from_numpy(Q).cuda())
        try:
            total = sj.selfjoin_run(hq)
            gi = torch.empty(total, dtype=torch.int32, device="cuda")
            gj = torch.empty(total, dtype=torch.int32, device="cuda")
            sj.selfjoin_fetch_pairs(hq, 0, gi, gj, None, max_pairs=total)
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)
    assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi)
    assert np.array_equal(gj.cpu().numpy().view(np.uint32), oj)


@pytest.mark.parametrize("workload,target,k", [("uniform_2m_d16", "64", 0),
                                               ("mixture50_5m_d18", "50", 0)])
def test_full_size_results_identical_across_filters(workload, target, k):
    """At full size, every exact filter must give the same whole result: the
    FP32 difference and norm forms, FP16 and BF16 matrix cores, SORTIDU,
    and another k.  The CSR row starts and the neighbour column of each run
    are compared element by element with the first run's."""
    import json
    import os
    from conftest import GOLDEN
    from paper_1809_09930_amd import selfjoin as sj
    with open(os.path.join(GOLDEN, "eps.json")) as f:
        eps = float.fromhex(json.load(f)[workload]["eps"][target]["hex"])
    P = datagen.make_workload(workload)
    Pd = torch.from_numpy(P).cuda()
    runs = [dict(fp32_form="norm"), dict(fp32_form="difference"), dict(precision="fp16"),
            dict(precision="bf16"), dict(sortidu=True), dict(k=5, precision="fp16")]
    ref = None
    for opts in runs:
        print("case", workload, opts, flush=True)
        h = sj.selfjoin_build_index(Pd, eps, **opts)
        try:
            total = sj.selfjoin_run(h)
            nb = torch.empty(total, dtype=torch.int32, device="cuda")
            sj.selfjoin_fetch_pairs(h, 0, None, nb, None, max_pairs=total)
            off = torch.empty(len(P) + 1, dtype=torch.int64, device="cuda")
            sj.selfjoin_fetch_offsets(h, off)
        finally:
            sj.selfjoin_free(h)
        if ref is None:
            ref = (off, nb)
            assert int(off[-1]) == total and bool((off[1:] > off[:-1]).all())
        else:
            assert torch.equal(off, ref[0]), opts
            assert torch.equal(nb, ref[1]), opts


# --------------------------------------------------------------------------
# The metric's numerator: the ordered candidate count C of Section 3.2.1
# (every point's adjacent non-empty cells, summed) reported by the device
# equals the oracle's grid join at the same k, dimension order, origin and
# cell width, on workloads where the grid is not degenerate.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("opts", [dict(), dict(precision="fp16"), dict(sortidu=True),
                                  dict(k=3), dict(reorder=False)])
@pytest.mark.parametrize("case", ["mixture50_d18", "mixture20_d90", "syn_d16", "syn_d64",
                                  "offgrid_mixture"])
def test_candidates_equal_oracle_grid(case, opts):
    from paper_1809_09930_amd import selfjoin as sj
    if case == "mixture50_d18":
        P = datagen.make_workload("mixture50_5m_d18", n=30000)
        eps = calibrated(P, 50, stride=29)
    elif case == "mixture20_d90":
        P = datagen.make_workload("mixture20_515k_d90", n=8000)
        eps = calibrated(P, 50, stride=7)
    elif case == "syn_d16":
        P, eps = datagen.make_workload("syn_2m_d16", n=20000), 0.05
    elif case == "syn_d64":
        P, eps = datagen.make_workload("syn_2m_d64", n=6000), 0.16
    else:
        P = datagen.offgrid("mixture_f32", 30000, 18, 97)
        eps = calibrated(P, 50, stride=29)
    n, d = P.shape
    print("case candidates", case, opts, flush=True)
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps, **opts)
    try:
        total = sj.selfjoin_run(h)
        gi = torch.empty(total, dtype=torch.int32, device="cuda")
        gj = torch.empty(total, dtype=torch.int32, device="cuda")
        sj.selfjoin_fetch_pairs(h, 0, gi, gj, None, max_pairs=total)
        info = sj.selfjoin_get_info(h)
        perm = sj.selfjoin_get_perm(h, d)
    finally:
        sj.selfjoin_free(h)
    k = info["k"]
    oi, oj, cand = oracle.grid_join(P, eps, np.asarray(perm[:k], dtype=np.uint32))
    assert info["candidates"] == cand, (info["candidates"], cand, k)
    assert cand <= n * n
    if case in ("mixture50_d18", "offgrid_mixture"):
        assert cand * 4 < n * n  # clustered: far from the all-pairs count
    assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi)
    assert np.array_equal(gj.cpu().numpy().view(np.uint32), oj)
    # symmetric tiles: each unordered candidate pair once, plus the part of
    # the diagonal tiles (a query block against its own cell's run) above
    # the diagonal, bounded by a 256-query block per work unit
    lo = (cand + n) // 2
    if opts.get("sortidu"):
        assert info["evaluated"] <= lo + 256 * n
    else:
        assert lo <= info["evaluated"] <= lo + 256 * n, (info["evaluated"], lo)


# --------------------------------------------------------------------------
# Boundary cases of the index build and of the result budget.
# --------------------------------------------------------------------------
def test_explicit_k_overflows():
    """An explicit k whose cell id cannot be linearised in 63 bits, and one
    whose adjacency lists exceed 2^32 - 1 entries: both SJ_ERR_KEY_OVERFLOW;
    automatic k on the same sets stays within both limits and is exact."""
    from paper_1809_09930_amd import selfjoin as sj
    P = datagen.uniform_grid(3000, 16, 401)  # 20 cells per dimension at eps 0.05
    with pytest.raises(sj.SelfJoinError) as e:
        sj.selfjoin_build_index(torch.from_numpy(P).cuda(), 0.05, k=16)
    assert e.value.code == sj.SJ_ERR_KEY_OVERFLOW
    assert_same_as_oracle(P, 0.05)
    # 4^10 lattice points of spacing 1 at eps 0.9: one point per cell, each
    # cell adjacent to 2.5^10 non-empty cells on average, 10^10 entries
    g = np.indices((4,) * 10, dtype=np.float32).reshape(10, -1).T.copy()
    with pytest.raises(sj.SelfJoinError) as e:
        sj.selfjoin_build_index(torch.from_numpy(g).cuda(), 0.9, k=10)
    assert e.value.code == sj.SJ_ERR_KEY_OVERFLOW
    assert "2^32" in str(e.value)
    h = sj.selfjoin_build_index(torch.from_numpy(g).cuda(), 0.9)
    try:
        assert sj.selfjoin_run(h) == len(g)  # spacing 1 > eps: self pairs only
    finally:
        sj.selfjoin_free(h)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_mem_budget_forces_batches(prec):
    """A device budget too small for the result in one batch: the result is
    produced in several batches and streamed to host memory, unchanged."""
    P = datagen.offgrid("uniform64", 2500, 16, 402)
    eps = calibrated(P, 30)
    info = assert_same_as_oracle(P, eps, precision=prec, mem_budget=20 * 4000)
    assert info["batches"] >= 3 and info["result_on_host"] == 1


@pytest.mark.parametrize("mode", ["0", "1"])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_matrix_core_hit_modes(mode, prec, monkeypatch):
    """Both hit paths of the matrix-core kernels (per-tile minimum first, or
    the direct element scan the build picks when most tiles hold a hit),
    forced on the same inputs: clustered small cells (per-wave units),
    uniform data (workgroup units), off-grid partners at eps, a query join."""
    monkeypatch.setenv("SJ_DEBUG_HITS", mode)
    std = datagen.decaying_std(18, 0.2, 0.002, 11)
    P = datagen.gaussian_mixture(5000, 18, 20, std, 11)
    assert_same_as_oracle(P, calibrated(P, 30), precision=prec)
    P = datagen.uniform_grid(3000, 16, 1)
    assert_same_as_oracle(P, calibrated(P, 32), precision=prec)
    P = datagen.uniform_grid(1500, 64, 4)
    assert_same_as_oracle(P, calibrated(P, 16), precision=prec)
    base = datagen.offgrid("mixture_f32", 1500, 24, 5)
    eps = calibrated(base, 8)
    P = np.concatenate([base, datagen.partners_near_radius(base, eps, 700, 6)])
    assert assert_same_as_oracle(P, eps, precision=prec)["rechecks"] > 0
    from paper_1809_09930_amd import selfjoin as sj
    E = datagen.offgrid("normal_binades", 3000, 10, 7)
    Q = np.concatenate([E[:500], datagen.partners_near_radius(E, 0.3, 600, 8)])
    he = sj.selfjoin_build_index(torch.from_numpy(E).cuda(), 0.3, precision=prec)
    try:
        hq = sj.selfjoin_build_query(he, torch.from_numpy(Q).cuda())
        try:
            total = sj.selfjoin_run(hq)
            gi = torch.empty(total, dtype=torch.int32, device="cuda")
            gj = torch.empty(total, dtype=torch.int32, device="cuda")
            sj.selfjoin_fetch_pairs(hq, 0, gi, gj, None, max_pairs=total)
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)
    oi, oj = oracle.join(Q, E, 0.3)
    assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi)
    assert np.array_equal(gj.cpu().numpy().view(np.uint32), oj)


@pytest.mark.parametrize("box", ["0", "1"])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_matrix_core_query_box(box, prec, monkeypatch):
    """The workgroup matrix-core kernel with its query-box prefilter off and
    on, in both hit modes: uniform data (every cell adjacent), grid data and
    off-grid data with partners at eps, d from 2 to 32, the symmetric self-join,
    several batches and a query join."""
    from paper_1809_09930_amd import selfjoin as sj
    monkeypatch.setenv("SJ_DEBUG_BOX", box)
    for mode in ("0", "1"):
        monkeypatch.setenv("SJ_DEBUG_HITS", mode)
        for n, d, seed, target in ((4000, 16, 31, 8), (3000, 2, 32, 20), (2500, 32, 33, 12),
                                   (1999, 8, 34, 40)):
            P = datagen.uniform_grid(n, d, seed)
            assert_same_as_oracle(P, calibrated(P, target), precision=prec)
        base = datagen.offgrid("uniform64", 2500, 12, 35)
        eps = calibrated(base, 6)
        P = np.concatenate([base, datagen.partners_near_radius(base, eps, 800, 36)])
        assert assert_same_as_oracle(P, eps, precision=prec)["rechecks"] > 0
    assert_same_as_oracle(datagen.uniform_grid(3000, 16, 37), 0.55, precision=prec,
                          batch_pairs=6000)
    E = datagen.offgrid("uniform64", 5000, 16, 38)
    Q = np.concatenate([datagen.offgrid("uniform64", 1200, 16, 39),
                        datagen.partners_near_radius(E, 0.5, 500, 40)])
    he = sj.selfjoin_build_index(torch.from_numpy(E).cuda(), 0.5, precision=prec)
    try:
        hq = sj.selfjoin_build_query(he, torch.from_numpy(Q).cuda())
        try:
            total = sj.selfjoin_run(hq)
            gi = torch.empty(total, dtype=torch.int32, device="cuda")
            gj = torch.empty(total, dtype=torch.int32, device="cuda")
            sj.selfjoin_fetch_pairs(hq, 0, gi, gj, None, max_pairs=total)
        finally:
            sj.selfjoin_free(hq)
    finally:
        sj.selfjoin_free(he)
    oi, oj = oracle.join(Q, E, 0.5)
    assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi)
    assert np.array_equal(gj.cpu().numpy().view(np.uint32), oj)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_cached_blocks_reused(prec):
    """Freed device blocks are cached and handed to later runs: a run with
    many pairs leaves its buffers full of keys, and the smaller and larger
    runs after it (on the same and on differently sized blocks) must still
    give the oracle's result; releasing the cache frees what it held, and
    runs after the release are still exact."""
    from paper_1809_09930_amd import selfjoin as sj
    P = datagen.uniform_grid(6000, 12, 91)
    Q = datagen.offgrid("normal_binades", 3000, 7, 92)
    big, small = calibrated(P, 120), calibrated(P, 5)
    sj.selfjoin_release_cache()
    assert_same_as_oracle(P, big, precision=prec)
    assert_same_as_oracle(P, small, precision=prec)
    assert_same_as_oracle(Q, calibrated(Q, 30), precision=prec)
    assert_same_as_oracle(P, big, precision=prec, batch_pairs=40000)
    torch.cuda.synchronize()
    assert sj.selfjoin_release_cache() > 0
    assert sj.selfjoin_release_cache() == 0
    assert_same_as_oracle(P, small, precision=prec)


def _fetch_all(h, total, device):
    from paper_1809_09930_amd import selfjoin as sj
    dev = "cuda" if device else "cpu"
    oi = torch.empty(total, dtype=torch.int32, device=dev)
    oj = torch.empty(total, dtype=torch.int32, device=dev)
    if total:
        assert sj.selfjoin_fetch_pairs(h, 0, oi, oj, None, max_pairs=total) == total
    torch.cuda.synchronize()
    return oi.cpu().numpy().view(np.uint32), oj.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("order", ["random", "sorted", "reversed"])
@pytest.mark.parametrize("nbatch", [2, 5, 13])
def test_symmetric_result_batches(order, nbatch):
    """FP32 self-joins in several result batches take each unordered pair
    once: a batch skips candidates of earlier batches and mirrors its pairs,
    later batches' mirrors through a device spill.  The caller's row order
    decides how much is spilled: rows in random order, sorted along the
    first coordinate (partners mostly in the same or the next batch) and
    reversed.  The result must be the oracle's; the evaluated pairs must be
    about half of the one-directional count."""
    from paper_1809_09930_amd import selfjoin as sj
    P = datagen.offgrid("mixture_f32", 5000, 10, 93)
    if order != "random":
        P = P[np.argsort(P[:, 0], kind="stable")]
        if order == "reversed":
            P = P[::-1].copy()
    eps = calibrated(P, 40)
    oi, oj = oracle.bruteforce(P, eps)
    h = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps, min_batches=nbatch)
    try:
        total = sj.selfjoin_run(h)
        info = sj.selfjoin_get_info(h)
        assert info["batches"] == nbatch and info["result_on_host"] == 1
        for device in (True, False):
            gi, gj = _fetch_all(h, total, device)
            assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
        # pieces across batch boundaries, into host and device columns
        for first, cnt in ((0, 1), (total // 3, total // 2), (total - 7, 7), (1, total - 1)):
            for device in ("cpu", "cuda"):
                part = torch.empty(cnt, dtype=torch.int32, device=device)
                assert sj.selfjoin_fetch_pairs(h, first, part, None, None, max_pairs=cnt) == cnt
                assert np.array_equal(part.cpu().numpy().view(np.uint32), oi[first:first + cnt])
    finally:
        sj.selfjoin_free(h)
    one_way = sj.selfjoin_build_index(torch.from_numpy(P).cuda(), eps, min_batches=nbatch,
                                      precision="fp16")
    try:
        sj.selfjoin_run(one_way)
        ow = sj.selfjoin_get_info(one_way)["evaluated"]
    finally:
        sj.selfjoin_free(one_way)
    assert info["evaluated"] <= ow
    if order == "random":  # a candidate is in an earlier batch about half the time
        assert info["evaluated"] < (0.5 * (nbatch + 1) / nbatch + 0.05) * ow


@pytest.mark.parametrize("form", ["difference", "norm"])
def test_symmetric_batches_spill_overflow_falls_back(form, monkeypatch):
    """A spill too small for the mirrored pairs (forced by
    SJ_DEBUG_UNDERSIZE, which also undersizes every batch buffer) makes the
    run start over one-directionally; the result is still the oracle's."""
    monkeypatch.setenv("SJ_DEBUG_UNDERSIZE", "1")
    P = datagen.uniform_grid(3000, 12, 94)
    info = assert_same_as_oracle(P, calibrated(P, 25), min_batches=4, fp32_form=form)
    assert info["batches"] == 4


def test_symmetric_batches_edge_cases():
    """Batches that hold one row each, duplicates that straddle batches, a
    batch with no pairs beyond the diagonal and more batches than rows allow."""
    P = np.repeat(datagen.uniform_grid(40, 3, 95), 3, axis=0)
    assert_same_as_oracle(P, 0.05, min_batches=len(P))
    assert_same_as_oracle(P, 0.05, min_batches=7, shortc=False)
    far = np.arange(12, dtype=np.float32)[:, None] * np.ones((1, 4), np.float32)
    info = assert_same_as_oracle(far, 0.5, min_batches=5)
    assert info["pairs"] == 12


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_small_cell_groups(prec):
    """FP32 small-cell units take groups of up to three neighbouring cells
    along the last indexed dimension (one unit of up to 64 queries, the union
    of the cells' candidate runs); pairs inside a group, across groups and
    with cells that join no group must all be found once: 2-D cells of about
    18 points (groups of three), 3-D cells of a few points, clusters whose
    cells straddle the limit of 64 queries, and a multi-batch run.  The
    matrix-core precisions run the same cases with per-wave units."""
    P = datagen.uniform_grid(20000, 2, 96)
    info = assert_same_as_oracle(P, 0.03, precision=prec)
    assert info["units"] == 2
    Q = datagen.offgrid("uniform64", 8000, 3, 97)
    assert assert_same_as_oracle(Q, calibrated(Q, 6), precision=prec)["units"] == 2
    std = np.full(6, 0.01)
    C = datagen.gaussian_mixture(6000, 6, 40, std, 98)
    assert_same_as_oracle(C, 0.02, precision=prec)
    assert_same_as_oracle(P, 0.03, precision=prec, min_batches=3)
