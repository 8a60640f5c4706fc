"""Pins for the CPU oracle against facts fixed outside the oracle itself:
the paper's worked examples (Figures 1 and 2), closed forms, an exact-integer
join, scipy's KD-tree pair search, a sort-based 1-D join, and invariants the
paper states (Sections 3.1, 3.2.1, 4.1, 4.2)."""
import itertools

import numpy as np
import pytest

import datagen
import oracle
from conftest import load_keyed, load_matrix, load_rows


def pairset(i, j):
    return set(zip(np.asarray(i).tolist(), np.asarray(j).tolist()))


def all_oracles(P, eps):
    """O1, O1' and O2 (all k=min(d,3) first dims) on the same input."""
    i1, j1 = oracle.bruteforce(P, eps)
    i2, j2 = oracle.bruteforce_np(P, eps)
    k = min(P.shape[1], 3)
    i3, j3, _ = oracle.grid_join(P, eps, list(range(k)))
    return (i1, j1), (i2, j2), (i3, j3)


# --------------------------------------------------------------------------
# Hand cases: the predicate is dist <= eps (Section 3.1), ordered tuples,
# self pairs included.
# --------------------------------------------------------------------------
def test_pythagorean_tie_is_included_and_one_step_out_is_not():
    h = 2.0 ** -10
    P = np.array([[0.0, 0.0], [3 * h, 4 * h]], dtype=np.float32)
    eps = 5 * h  # squared distance 25 h^2 == eps^2 exactly
    for i, j in all_oracles(P, eps):
        assert pairset(i, j) == {(0, 0), (0, 1), (1, 0), (1, 1)}
    P2 = P.copy()
    P2[1, 0] += np.float32(2.0 ** -24)  # squared distance now > eps^2
    assert float(P2[1, 0]) > 3 * h
    for i, j in all_oracles(P2, eps):
        assert pairset(i, j) == {(0, 0), (1, 1)}


def test_duplicates_single_point_and_one_dimension():
    P = np.array([[0.25, 0.5], [0.25, 0.5], [0.75, 0.5]], dtype=np.float32)
    for i, j in all_oracles(P, 0.1):
        assert pairset(i, j) == {(0, 0), (0, 1), (1, 0), (1, 1), (2, 2)}
    one = np.array([[0.3, 0.7, 0.1]], dtype=np.float32)
    for i, j in all_oracles(one, 1e-6):
        assert pairset(i, j) == {(0, 0)}
    line = np.array([[0.0], [0.5], [1.0], [1.75]], dtype=np.float32)
    for i, j in all_oracles(line, 0.5):
        assert pairset(i, j) == {(0, 0), (1, 1), (2, 2), (3, 3),
                                 (0, 1), (1, 0), (1, 2), (2, 1)}


def test_empty_input():
    P = np.zeros((0, 4), dtype=np.float32)
    i, j = oracle.bruteforce(P, 0.5)
    assert len(i) == 0 and len(j) == 0


# --------------------------------------------------------------------------
# Figure 1 (Section 3.2.1)
# --------------------------------------------------------------------------
def fig1():
    return load_matrix("fig1_points.txt", np.float32)


def paper_cell_id(cx, cy):
    """Figure 1 numbering: rows counted from the top of a 7 x 7 grid."""
    return 7 * (6 - cy) + cx


def test_fig1_nonempty_cells_match_the_figure():
    P = fig1()
    c = oracle.cell_coords(P, 1.0, [0, 1], origin_zero=True, width_factor=1.0)
    ids = {paper_cell_id(int(x), int(y)) for x, y in c}
    assert ids == set(load_keyed("fig1_cells.txt")["nonempty"])


def test_fig1_cell24_searches_exactly_the_dashed_box():
    P = fig1()
    c = oracle.cell_coords(P, 1.0, [0, 1], origin_zero=True, width_factor=1.0)
    ids = [paper_cell_id(int(x), int(y)) for x, y in c]
    q = ids.index(24)
    cand = oracle.grid_candidates(P, 1.0, [0, 1], q, origin_zero=True,
                                  width_factor=1.0)
    assert {ids[j] for j in cand} == set(load_keyed("fig1_cells.txt")["adjacent_of_24"])
    # every point of those four cells is a candidate, nothing else
    assert sorted(cand.tolist()) == sorted(
        j for j, cid in enumerate(ids) if cid in (18, 23, 24, 32))


def test_fig1_join_matches_hand_worked_pairs():
    P = fig1()
    rows = load_rows("fig1_pairs.txt")
    want = {(p, p) for p in range(len(P))}
    for a, b, s in rows:
        a, b, s = int(a), int(b), float(s)
        want |= {(a, b), (b, a)}
    assert len(want) == 42
    for i, j in all_oracles(P, 1.0):
        assert pairset(i, j) == want
    i, j, s = oracle.bruteforce(P, 1.0, with_dist=True)
    got = {(a, b): v for a, b, v in zip(i.tolist(), j.tolist(), s.tolist())}
    for a, b, sd in rows:
        assert abs(got[(int(a), int(b))] - float(sd)) < 1e-5


def test_adjacent_cell_counts_2d_and_6d():
    """3^k cells around an interior cell: 9 in 2-D, 729 in 6-D (Section 4.1).
    One point at the centre of every cell of a 3^k (or 5^k) lattice."""
    for k, side in ((2, 3), (6, 3), (2, 5)):
        pts = np.array(list(itertools.product(range(side), repeat=k)),
                       dtype=np.float32) + np.float32(0.5)
        centre = [side // 2] * k
        q = [tuple(p) for p in (pts - 0.5).astype(int).tolist()].index(tuple(centre))
        cand = oracle.grid_candidates(pts, 1.0, list(range(k)), q,
                                      origin_zero=True, width_factor=1.0)
        assert len(cand) == 3 ** k


def test_indexing_fewer_dims_searches_fewer_cells():
    """Section 4.1 example: 5-D points indexed on 3 dims search 27 of the
    243 cells, a loss of (3^5 - 3^3)/3^5 = 88.9%; the join is unchanged."""
    pts = np.array(list(itertools.product(range(3), repeat=5)),
                   dtype=np.float32) + np.float32(0.5)
    q = 121  # the centre of the 3^5 lattice
    assert (pts[q] == 1.5).all()
    c5 = oracle.cell_coords(pts, 1.0, list(range(5)), origin_zero=True,
                            width_factor=1.0)
    c3 = oracle.cell_coords(pts, 1.0, list(range(3)), origin_zero=True,
                            width_factor=1.0)
    cells5 = {tuple(r) for r in c5[oracle.grid_candidates(
        pts, 1.0, list(range(5)), q, origin_zero=True, width_factor=1.0)]}
    cells3 = {tuple(r) for r in c3[oracle.grid_candidates(
        pts, 1.0, list(range(3)), q, origin_zero=True, width_factor=1.0)]}
    assert len(cells5) == 243 and len(cells3) == 27
    assert round(100 * (len(cells5) - len(cells3)) / len(cells5), 1) == 88.9
    a = pairset(*oracle.grid_join(pts, 1.0, [0, 1, 2], origin_zero=True)[:2])
    b = pairset(*oracle.bruteforce(pts, 1.0))
    assert a == b


# --------------------------------------------------------------------------
# Figure 2 (Section 4.2)
# --------------------------------------------------------------------------
def test_fig2_cells_per_dimension_and_dim4_occupancy():
    P = load_matrix("fig2_points.txt", np.float32)
    facts = load_keyed("fig2_facts.txt")
    c = oracle.cell_coords(P, 0.2, list(range(6)), origin_zero=True,
                           width_factor=1.0)
    assert [len(set(c[:, t])) for t in range(6)] == facts["cells_per_dim"]
    occ = np.bincount(c[:, 3] - c[:, 3].min())
    assert occ.tolist() == facts["dim4_cell_occupancy"]


def test_fig2_reorder_ranks_the_paper_dimensions():
    P = load_matrix("fig2_points.txt", np.float32)
    facts = load_keyed("fig2_facts.txt")
    perm, var = oracle.reorder_perm(P)
    one_based = [int(t) + 1 for t in perm]
    assert set(one_based[:3]) == set(facts["top3_set"])
    assert one_based[3:] == facts["rank4to6"]
    # textbook unbiased variance, written out
    X = P.astype(np.float64)
    m = X.mean(axis=0)
    v = ((X - m) ** 2).sum(axis=0) / (len(X) - 1)
    np.testing.assert_allclose(var, v, rtol=1e-12)
    # after reordering, each of the first three dims spans 5 cells
    c = oracle.cell_coords(P, 0.2, perm[:3], origin_zero=True, width_factor=1.0)
    assert [len(set(c[:, r])) for r in range(3)] == [5, 5, 5]


def test_reorder_does_not_change_the_join():
    P = datagen.gaussian_mixture(600, 6, 4, np.array([.3, .01, .2, .05, .1, .002]), 11)
    eps, _ = oracle.calibrate_eps(P, 10, np.arange(0, 600, 3))
    base = pairset(*oracle.bruteforce(P, eps))
    perm, _ = oracle.reorder_perm(P)
    for k in (1, 2, 3, 6):
        gi, gj, _ = oracle.grid_join(P, eps, perm[:k])
        assert pairset(gi, gj) == base
        gi, gj, _ = oracle.grid_join(P, eps, list(range(k)))
        assert pairset(gi, gj) == base


# --------------------------------------------------------------------------
# Independent implementations
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,d,seed,target", [
    (300, 1, 1, 5), (500, 2, 2, 8), (800, 5, 3, 12), (1200, 16, 4, 20),
    (700, 64, 5, 10), (400, 3, 6, 0.5)])
def test_o1_equals_exact_integer_join_and_numpy_twin(n, d, seed, target):
    g = datagen.GRID_UNIFORM
    P = datagen.uniform_grid(n, d, seed, g)
    eps, _ = oracle.calibrate_eps(P, target, np.arange(0, n, 2))
    eps2 = eps * eps
    T = int(np.floor(eps2 * float(2 ** (2 * g))))
    A = (P.astype(np.float64) * float(2 ** g)).astype(np.int64)
    exact = pairset(*oracle.exact_int_join(A, T))
    i1, j1 = oracle.bruteforce(P, eps)
    assert pairset(i1, j1) == exact
    assert pairset(*oracle.bruteforce_np(P, eps)) == exact
    # ordering: ascending (i, j), unique
    key = i1.astype(np.uint64) << np.uint64(32) | j1.astype(np.uint64)
    assert (np.diff(key.astype(np.int64)) > 0).all()


@pytest.mark.parametrize("n,d,seed", [(1500, 3, 7), (1000, 16, 8), (600, 40, 9)])
def test_o1_matches_scipy_kdtree(n, d, seed):
    sp = pytest.importorskip("scipy.spatial")
    P = datagen.uniform_grid(n, d, seed)
    eps, _ = oracle.calibrate_eps(P, 15, np.arange(0, n, 5))
    i, j = oracle.bruteforce(P, eps)
    ours = {(a, b) for a, b in zip(i.tolist(), j.tolist()) if a < b}
    tree = sp.cKDTree(P.astype(np.float64))
    theirs = tree.query_pairs(eps, p=2.0, output_type="set")
    assert ours == theirs
    assert all((a, a) in pairset(i, j) for a in range(n))


def test_one_dimension_matches_sort_and_search():
    """d = 1: the join is the set of |x_i - x_j| <= eps, found here by a
    sorted sweep (searchsorted) instead of distances."""
    g = datagen.GRID_UNIFORM
    P = datagen.uniform_grid(3000, 1, 21, g)
    eps = 777 * 2.0 ** -g * 16  # on the grid, so eps^2 is exact
    x = P[:, 0].astype(np.float64)
    order = np.argsort(x, kind="stable")
    xs = x[order]
    lo = np.searchsorted(xs, xs - eps, side="left")
    hi = np.searchsorted(xs, xs + eps, side="right")
    want = set()
    for r in range(len(xs)):
        for s in range(lo[r], hi[r]):
            want.add((int(order[r]), int(order[s])))
    assert pairset(*oracle.bruteforce(P, eps)) == want


@pytest.mark.parametrize("seed,k", [(31, 1), (32, 2), (33, 4), (34, 6)])
def test_grid_variant_equals_bruteforce(seed, k):
    P = datagen.uniform_grid(1500, 8, seed)
    eps, _ = oracle.calibrate_eps(P, 25, np.arange(0, 1500, 4))
    bi, bj = oracle.bruteforce(P, eps)
    gi, gj, cand = oracle.grid_join(P, eps, list(range(k)))
    assert (gi == bi).all() and (gj == bj).all()
    assert len(bi) <= cand <= 1500 * 1500


def test_grid_variant_on_clustered_data_with_many_cells():
    std = datagen.decaying_std(12, 0.2, 0.002, 5)
    P = datagen.gaussian_mixture(3000, 12, 20, std, 6)
    eps, _ = oracle.calibrate_eps(P, 30, np.arange(0, 3000, 10))
    perm, _ = oracle.reorder_perm(P)
    bi, bj = oracle.bruteforce(P, eps)
    for k in (2, 4, 6):
        gi, gj, cand = oracle.grid_join(P, eps, perm[:k])
        assert (gi == bi).all() and (gj == bj).all()
        assert cand < 3000 * 3000  # the grid really filters here


def test_boundary_pairs_at_eps2_plus_minus_one_grid_step():
    """Pairs whose exact squared distance is eps2 - 2^-48, eps2, eps2 + 2^-48
    (one step of the 2^-24 grid squared): O1 must agree with O0."""
    g = 24
    u = 2.0 ** -g
    base = np.zeros((1, 4))
    # (a*u)^2 + (b*u)^2 with a=3000,b=4000 -> 25e6 u^2; eps2 = that exactly
    pts = [base[0], [3000 * u, 4000 * u, 0, 0]]
    # 25e6 - 1 is not a sum of two squares near here, so use three coords:
    # 3000^2 + 3999^2 + 89^2 = 25e6 - 7999 + 7921 = 24999922 (< eps2)
    pts.append([3000 * u, 3999 * u, 89 * u, 0])
    # 3000^2 + 4000^2 + 1 = eps2 + u^2 (> eps2)
    pts.append([3000 * u, 4000 * u, 1 * u, 0])
    P = np.array(pts, dtype=np.float32)
    eps2_units = 25_000_000
    eps = float(np.sqrt(eps2_units)) * u  # 5000 u, exact
    assert eps * eps == eps2_units * u * u
    A = (P.astype(np.float64) / u).astype(np.int64)
    exact = pairset(*oracle.exact_int_join(A, eps2_units))
    assert (0, 1) in exact and (0, 2) in exact and (0, 3) not in exact
    assert pairset(*oracle.bruteforce(P, eps)) == exact


def test_symmetry_and_self_pairs_invariant():
    P = datagen.uniform_grid(2000, 10, 41)
    eps, _ = oracle.calibrate_eps(P, 40, np.arange(0, 2000, 7))
    i, j = oracle.bruteforce(P, eps)
    s = pairset(i, j)
    assert all((b, a) in s for a, b in s)
    assert all((a, a) in s for a in range(len(P)))


def test_rows_and_smallest_agree_with_full_join():
    P = datagen.uniform_grid(1500, 6, 51)
    eps, sd = oracle.calibrate_eps(P, 20, np.arange(0, 1500, 3))
    i, j, s = oracle.bruteforce(P, eps, with_dist=True)
    q = np.array([0, 17, 1499, 700])
    cnt, jj, ss = oracle.rows(P, eps, q, with_dist=True)
    off = 0
    for r, c in zip(q, cnt):
        sel = i == r
        assert (jj[off:off + c] == j[sel]).all()
        assert (ss[off:off + c] == s[sel]).all()
        off += c
    sm = oracle.rows_smallest(P, q, 10)
    for r, row in zip(q, sm):
        X = P.astype(np.float64)
        acc = np.zeros(len(P))
        for t in range(P.shape[1]):
            diff = X[r, t] - X[:, t]
            acc = acc + diff * diff
        acc[r] = np.inf
        assert (np.sort(acc)[:10] == row).all()


def test_calibration_hits_the_target_on_its_sample():
    P = datagen.uniform_grid(4000, 16, 61)
    q = datagen.calibration_rows(4000, 61)
    eps, sd = oracle.calibrate_eps(P, 32, q)
    cnt, _ = oracle.rows(P, eps, q)
    achieved = (cnt.sum() - len(q)) / len(q)
    assert achieved == pytest.approx(sd)
    assert abs(achieved - 32) <= 1.0 / len(q) + 1e-9
    # one ulp less epsilon loses at least one pair of the sample
    cnt2, _ = oracle.rows(P, float(np.nextafter(eps, 0)), q)
    assert cnt2.sum() < cnt.sum()


# --------------------------------------------------------------------------
# O1q: the general join Q join_eps E (Section 3.1; the self-join is E join E)
# --------------------------------------------------------------------------
def _r2(k):
    """Number of integer points (x, y) with x^2 + y^2 = k, from Jacobi's
    two-square formula r2(k) = 4 (d1(k) - d3(k)), d1 / d3 counting the
    divisors of k that are 1 / 3 mod 4 (r2(0) = 1)."""
    if k == 0:
        return 1
    d1 = sum(1 for t in range(1, k + 1) if k % t == 0 and t % 4 == 1)
    d3 = sum(1 for t in range(1, k + 1) if k % t == 0 and t % 4 == 3)
    return 4 * (d1 - d3)


@pytest.mark.parametrize("eps", [1.0, 2.0, 3.0, 5 ** 0.5, 8 ** 0.5, 10 ** 0.5, 2.5, 0.5])
def test_join_lattice_counts_follow_the_two_square_formula(eps):
    """Queries at integer points of the plane against the integer lattice
    [-6, 6]^2: each query's neighbour count is the number of lattice points
    in the closed disc of squared radius fl(eps*eps), i.e. the sum of r2(k)
    over integers k <= fl(eps*eps) (ties at exactly eps are included)."""
    g = np.arange(-6, 7, dtype=np.float32)
    E = np.array([(x, y) for x in g for y in g], dtype=np.float32)
    Q = np.array([(0, 0), (1, 0), (-2, 1), (3, 3)], dtype=np.float32)
    eps2 = eps * eps
    K = int(np.floor(eps2))
    expect = sum(_r2(k) for k in range(0, K + 1))
    qi, ej = oracle.join(Q, E, eps)
    counts = np.bincount(qi, minlength=len(Q))
    assert counts.tolist() == [expect] * len(Q)
    # and every reported pair is really within eps in exact arithmetic
    d2 = ((Q[qi].astype(np.int64) - E[ej].astype(np.int64)) ** 2).sum(1)
    assert (d2 <= K).all()


@pytest.mark.parametrize("m,n,d,seed,shift", [
    (300, 500, 2, 11, 0.0), (400, 700, 5, 12, 0.25), (250, 900, 16, 13, 0.5),
    (200, 300, 40, 14, 0.0)])
def test_join_equals_exact_integer_join_of_two_sets(m, n, d, seed, shift):
    """On 2^-g grid data the join equals the exact integer join; the query
    set is drawn separately and shifted so part of it lies outside E's box."""
    g = datagen.GRID_UNIFORM
    E = datagen.uniform_grid(n, d, seed, g)
    Q = datagen.uniform_grid(m, d, seed + 100, g) + np.float32(shift)
    eps, _ = oracle.calibrate_eps(E, 12, np.arange(0, n, 3))
    T = int(np.floor(eps * eps * float(2 ** (2 * g))))
    A = (Q.astype(np.float64) * float(2 ** g)).astype(np.int64)
    B = (E.astype(np.float64) * float(2 ** g)).astype(np.int64)
    exact = pairset(*oracle.exact_int_join(A, T, B))
    qi, ej = oracle.join(Q, E, eps)
    assert pairset(qi, ej) == exact
    key = qi.astype(np.uint64) << np.uint64(32) | ej.astype(np.uint64)
    assert (np.diff(key.astype(np.int64)) > 0).all()
    if shift == 0.0:
        assert len(exact) > m  # the case is not vacuous


def test_join_special_cases_self_join_and_transpose():
    """Q = E gives the self-join; swapping the sets transposes the pairs
    (the squared difference of two floats is the same in either order)."""
    E = datagen.uniform_grid(600, 8, 21)
    Q = datagen.uniform_grid(350, 8, 22)
    eps, _ = oracle.calibrate_eps(E, 20, np.arange(0, 600, 4))
    si, sj = oracle.bruteforce(E, eps)
    ji, jj = oracle.join(E, E, eps)
    assert np.array_equal(si, ji) and np.array_equal(sj, jj)
    a = pairset(*oracle.join(Q, E, eps))
    b = pairset(*oracle.join(E, Q, eps))
    assert a == {(y, x) for x, y in b}
    assert len(a) > 0


@pytest.mark.parametrize("m,n,d,seed", [(500, 2000, 3, 31), (400, 1500, 24, 32)])
def test_join_matches_scipy_kdtree_ball_query(m, n, d, seed):
    sp = pytest.importorskip("scipy.spatial")
    E = datagen.uniform_grid(n, d, seed)
    Q = datagen.uniform_grid(m, d, seed + 7)
    eps, _ = oracle.calibrate_eps(E, 15, np.arange(0, n, 5))
    tree = sp.cKDTree(E.astype(np.float64))
    theirs = set()
    for q, js in enumerate(tree.query_ball_point(Q.astype(np.float64), eps, p=2.0)):
        theirs.update((q, j) for j in js)
    assert pairset(*oracle.join(Q, E, eps)) == theirs


def test_join_empty_sides():
    E = datagen.uniform_grid(50, 4, 41)
    z = np.zeros((0, 4), np.float32)
    for Q, EE in ((z, E), (E, z), (z, z)):
        qi, ej = oracle.join(Q, EE, 0.3)
        assert len(qi) == 0 and len(ej) == 0


# --------------------------------------------------------------------------
# SORTIDU (Section 4.3): search along one un-indexed dimension u
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,d,k,u,seed", [(600, 6, 2, 3, 61), (800, 4, 1, 2, 62),
                                          (500, 8, 3, 0, 63)])
def test_sortidu_candidates_are_the_cells_points_within_eps_along_u(n, d, k, u, seed):
    """The binary search plus scan visits exactly the points of the adjacent
    cells whose u-coordinate is within eps of the query's (the definition,
    written here as a plain filter), each cell's in increasing u; and that
    set holds every neighbour of the query."""
    P = datagen.uniform_grid(n, d, seed)
    eps = oracle.calibrate_eps(P, 12, np.arange(0, n, 4))[0]
    dims = [r for r in range(d) if r != u][:k] if u < k else list(range(k))
    coords = oracle.cell_coords(P, eps, dims)
    for q in range(0, n, 37):
        grid = oracle.grid_candidates(P, eps, dims, q)
        want = {int(j) for j in grid
                if abs(float(P[j, u]) - float(P[q, u])) <= eps}
        got = oracle.sortidu_candidates(P, eps, dims, u, q)
        assert len(got) == len(set(got.tolist())) and set(got.tolist()) == want
        # grouped by cell, increasing u inside each cell
        keys = [tuple(coords[j]) for j in got]
        for a in range(1, len(got)):
            if keys[a] == keys[a - 1]:
                assert P[got[a], u] >= P[got[a - 1], u]
        _, js = oracle.rows(P, eps, [q])
        assert set(js.tolist()) <= want


def test_sortidu_prunes_when_u_spans_many_eps():
    """Points spread far along the un-indexed dimension: the search along u
    visits a small fraction of the cells' points (the case Section 4.3 is
    for), and nothing when the query is isolated along u."""
    rng = np.random.default_rng(64)
    P = np.empty((2000, 3), np.float32)
    P[:, 0] = rng.random(2000) * 0.2        # indexed: one or two cells
    P[:, 1] = rng.random(2000) * 0.2
    P[:, 2] = rng.random(2000) * 50.0       # u: 500 eps long
    eps = 0.1
    tot_grid = tot_u = 0
    for q in range(0, 2000, 50):
        tot_grid += len(oracle.grid_candidates(P, eps, [0, 1], q))
        tot_u += len(oracle.sortidu_candidates(P, eps, [0, 1], 2, q))
    assert tot_u * 50 < tot_grid
    P[0, 2] = 1000.0
    assert len(oracle.sortidu_candidates(P, eps, [0, 1], 2, 0)) == 1  # itself
