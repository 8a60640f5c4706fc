"""The synthetic inputs: distribution facts of the paper's exponential family
(Section 5.1) and the selectivity ranges it prints for it (Section 5.4), on
CPU with the oracle."""
import numpy as np
import pytest

import datagen
import oracle


def test_exponential_family_distribution():
    """Rate 40 restricted to [0, 1): mean 1/40 (the truncation at 1 removes
    a mass of e^-40), median ln 2 / 40, values on the 2^-24 grid."""
    X = datagen.exponential_syn(200_000, 4, 40.0, 3).astype(np.float64)
    assert X.min() >= 0.0 and X.max() < 1.0
    assert abs(X.mean() - 1 / 40) < 0.01 / 40
    assert abs(np.median(X) - np.log(2) / 40) < 0.02 / 40
    assert np.array_equal(X * 2.0 ** 24, np.round(X * 2.0 ** 24))


@pytest.mark.parametrize("name,lo,hi", [
    ("syn_2m_d16", 4, 1200), ("syn_2m_d32", 31, 1400), ("syn_2m_d64", 132, 2300)])
def test_paper_synthetic_workloads_land_in_the_printed_selectivity_ranges(name, lo, hi):
    """At the smallest and largest epsilon of the paper's sweep (Table 3) the
    mean neighbour count S_D of a 100-row sample is within a factor 1.5 of
    the range the paper prints for the dataset (Section 5.4)."""
    w = datagen.WORKLOADS[name]
    P = datagen.make_workload(name)
    assert P.shape == (w["n"], w["d"])
    rows = np.sort(np.random.default_rng(1).choice(len(P), 100, replace=False))
    sd = []
    for eps in w["eps_fixed"]:
        cnt, _ = oracle.rows(P, eps, rows)
        sd.append(cnt.mean() - 1.0)
    assert lo / 1.5 <= sd[0] <= lo * 1.5, sd
    assert hi / 1.5 <= sd[1] <= hi * 1.5, sd
