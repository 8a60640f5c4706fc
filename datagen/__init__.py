"""Seeded synthetic inputs for the epsilon self-join.

This module only draws random numbers: it holds none of the join's
arithmetic, and it is the one piece shared by the oracle tests, the GPU tests
and the benchmark.  Every generator is deterministic in its seed (numpy
PCG64 via ``default_rng``).

Value grids.  Uniform data are multiples of 2^-24 in [0, 1); mixtures are
clipped to [-2, 2) and rounded to multiples of 2^-22.  On such grids every
float32 coordinate difference is exact, its square is exact in binary64 and
partial sums stay exact below 2^(53-2g), so any summation order gives the same
include/exclude decision as the canonical FP64 order for every epsilon used
here.  That lets an exact-integer join check the floating-point oracle.

Workload shapes follow the paper's datasets (Table 1): 2*10^6 points in 16
and 64 dimensions like the Syn16D2M / Syn64D2M sets, 5*10^6 x 18 like SuSy,
515,000 x 90 like Songs.  The real datasets are not used; these draws stand
in for them.
"""
from __future__ import annotations

import math

import numpy as np

GRID_UNIFORM = 24
GRID_MIXTURE = 22


def uniform_grid(n: int, d: int, seed: int, g: int = GRID_UNIFORM) -> np.ndarray:
    """n x d float32, i.i.d. uniform over the multiples of 2^-g in [0, 1)."""
    rng = np.random.default_rng(seed)
    out = np.empty((n, d), dtype=np.float32)
    step = 1 << 20  # draw in row chunks to bound the int64 temporary
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        ints = rng.integers(0, 1 << g, size=(r1 - r0, d), dtype=np.int64)
        out[r0:r1] = (ints.astype(np.float64) * (2.0 ** -g)).astype(np.float32)
    return out


def _round_to_grid(x: np.ndarray, g: int, lo: float, hi: float) -> np.ndarray:
    x = np.clip(x, lo, hi - 2.0 ** -g)
    return (np.round(x * (1 << g)) * (2.0 ** -g)).astype(np.float32)


def gaussian_mixture(n: int, d: int, n_centers: int, std: np.ndarray,
                     seed: int, g: int = GRID_MIXTURE) -> np.ndarray:
    """n x d float32 mixture of isotropic-per-dimension Gaussians.

    Centres ~ U[0,1)^d, labels ~ U{0..n_centers-1}, x = centre + std * N(0,1)
    (std is a length-d vector shared by all components), clipped to [-2, 2)
    and rounded to multiples of 2^-g."""
    rng = np.random.default_rng(seed)
    std = np.asarray(std, dtype=np.float64)
    assert std.shape == (d,)
    centers = rng.random((n_centers, d))
    out = np.empty((n, d), dtype=np.float32)
    step = 1 << 19
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        lab = rng.integers(0, n_centers, size=r1 - r0)
        x = centers[lab] + rng.standard_normal((r1 - r0, d)) * std
        out[r0:r1] = _round_to_grid(x, g, -2.0, 2.0)
    return out


def decaying_std(d: int, hi: float, lo: float, seed: int) -> np.ndarray:
    """Per-dimension std decaying geometrically from hi to lo, then placed in
    a seeded shuffled dimension order."""
    j = np.arange(d, dtype=np.float64)
    std = hi * (lo / hi) ** (j / max(d - 1, 1))
    rng = np.random.default_rng(seed)
    return std[rng.permutation(d)]


def uniform_std(d: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=d)


def exponential_syn(n: int, d: int, lam: float, seed: int,
                    g: int = GRID_UNIFORM) -> np.ndarray:
    """The paper's synthetic family (Section 5.1): exponential coordinates
    with rate lam restricted to [0, 1) (values >= 1 are redrawn), on the 2^-g
    grid."""
    rng = np.random.default_rng(seed)
    out = np.empty((n, d), dtype=np.float64)
    fill = np.zeros((n, d), dtype=bool)
    while not fill.all():
        x = rng.exponential(1.0 / lam, size=(n, d))
        take = (~fill) & (x < 1.0)
        out[take] = x[take]
        fill |= take
    return _round_to_grid(out, g, 0.0, 1.0)


# ---------------------------------------------------------------------------
# Named workloads.  `targets` are mean neighbours per point (S_D) that the
# calibrated epsilons aim at; the epsilons themselves are stored values.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "uniform_20k_d16": dict(kind="uniform", n=20_000, d=16, seed=0,
                            targets=[32]),
    "uniform_2m_d16": dict(kind="uniform", n=2_000_000, d=16, seed=1,
                           targets=[8, 64, 512]),
    "uniform_2m_d64": dict(kind="uniform", n=2_000_000, d=64, seed=2,
                           targets=[16, 128]),
    "mixture50_5m_d18": dict(kind="mixture_decay", n=5_000_000, d=18, seed=3,
                             n_centers=50, std_hi=0.2, std_lo=0.002,
                             targets=[50]),
    "mixture20_515k_d90": dict(kind="mixture_uniform_std", n=515_000, d=90,
                               seed=4, n_centers=20, std_lo=0.01, std_hi=0.3,
                               targets=[50]),
    # The paper's synthetic family (Section 5.1, Table 1: Syn16D2M, Syn32D2M,
    # Syn64D2M) at the smallest and largest epsilon of its sweep (Table 3);
    # these use the paper's epsilons as given instead of calibrated ones.
    "syn_2m_d16": dict(kind="exponential", n=2_000_000, d=16, seed=21, lam=40.0,
                       eps_fixed=[0.03, 0.05]),
    "syn_2m_d32": dict(kind="exponential", n=2_000_000, d=32, seed=37, lam=40.0,
                       eps_fixed=[0.08, 0.10]),
    "syn_2m_d64": dict(kind="exponential", n=2_000_000, d=64, seed=69, lam=40.0,
                       eps_fixed=[0.16, 0.18]),
}


def make_workload(name: str, n: int | None = None) -> np.ndarray:
    """Draw the named workload, optionally with a different point count n
    (same seed and distribution)."""
    w = WORKLOADS[name]
    nn = w["n"] if n is None else n
    if w["kind"] == "uniform":
        return uniform_grid(nn, w["d"], w["seed"])
    if w["kind"] == "mixture_decay":
        std = decaying_std(w["d"], w["std_hi"], w["std_lo"], w["seed"] + 500)
        return gaussian_mixture(nn, w["d"], w["n_centers"], std, w["seed"])
    if w["kind"] == "mixture_uniform_std":
        std = uniform_std(w["d"], w["std_lo"], w["std_hi"], w["seed"] + 500)
        return gaussian_mixture(nn, w["d"], w["n_centers"], std, w["seed"])
    if w["kind"] == "exponential":
        return exponential_syn(nn, w["d"], w["lam"], w["seed"])
    raise KeyError(name)


def calibration_rows(n: int, seed: int, frac: float = 0.01,
                     min_rows: int = 256, max_rows: int = 4096) -> np.ndarray:
    """Seeded query rows (without replacement) for epsilon calibration:
    1% of n, at least min_rows and at most max_rows."""
    m = int(min(n, max(min_rows, min(max_rows, math.ceil(frac * n)))))
    rng = np.random.default_rng(seed + 1000)
    return np.sort(rng.choice(n, size=m, replace=False)).astype(np.int64)


def batched_job_specs(n_jobs: int = 256, seed: int = 7):
    """Specs for many independent self-joins of uneven size: n log-uniform in
    [1e3, 2e5], d from {8, 16, 32, 64}, uniform or a 10-Gaussian mixture,
    target mean neighbours log-uniform in [10, 200]."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_jobs):
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        d = int(rng.choice([8, 16, 32, 64]))
        kind = "uniform" if rng.random() < 0.5 else "mixture"
        target = int(round(math.exp(rng.uniform(math.log(10), math.log(200)))))
        specs.append(dict(n=n, d=d, kind=kind, target=target, seed=seed * 1000 + i))
    return specs


def make_job(spec) -> np.ndarray:
    if spec["kind"] == "uniform":
        return uniform_grid(spec["n"], spec["d"], spec["seed"])
    std = uniform_std(spec["d"], 0.01, 0.3, spec["seed"] + 500)
    return gaussian_mixture(spec["n"], spec["d"], 10, std, spec["seed"])


# ---------------------------------------------------------------------------
# Off-grid float32 inputs.  These are drawn in binary64 and rounded to the
# nearest float32 with no snapping to a coarse grid, so coordinates of one
# dimension sit in different binades and their float32 differences round.
# They exercise the error bounds of the device filters, which the grid data
# above (exact differences) never reach.
# ---------------------------------------------------------------------------
OFFGRID_KINDS = ("uniform64", "normal_binades", "loguniform_signed", "mixture_f32")


def offgrid(kind: str, n: int, d: int, seed: int) -> np.ndarray:
    """n x d float32 of one of OFFGRID_KINDS:
      uniform64          U[0,1) in binary64, rounded to float32;
      normal_binades     per dimension scale 10^U(-2,1) and an offset of 0 (values
                         of both signs around zero) or U(-2,2) scales, plus
                         scale * N(0,1);
      loguniform_signed  random sign times 2^U(-20,3): magnitudes over 23 binades;
      mixture_f32        10 Gaussians, centres U[0,1)^d, per-dimension std decaying
                         from 0.2 to 0.002 (shuffled), not clipped or rounded."""
    rng = np.random.default_rng(seed)
    if kind == "uniform64":
        x = rng.random((n, d))
    elif kind == "normal_binades":
        scale = 10.0 ** rng.uniform(-2.0, 1.0, size=d)
        offset = np.where(rng.random(d) < 0.5, 0.0, rng.uniform(-2.0, 2.0, size=d)) * scale
        x = offset + scale * rng.standard_normal((n, d))
    elif kind == "loguniform_signed":
        mag = np.exp2(rng.uniform(-20.0, 3.0, size=(n, d)))
        x = np.where(rng.random((n, d)) < 0.5, -mag, mag)
    elif kind == "mixture_f32":
        std = decaying_std(d, 0.2, 0.002, seed + 500)
        centers = rng.random((10, d))
        lab = rng.integers(0, 10, size=n)
        x = centers[lab] + rng.standard_normal((n, d)) * std
    else:
        raise KeyError(kind)
    return x.astype(np.float32)


def partners_near_radius(base: np.ndarray, eps: float, count: int, seed: int,
                         steps=(-3, -2, -1, 0, 1, 2, 3), unit: float = 2.0 ** -20):
    """For `count` rows p of `base`, a partner p + eps * (1 + s * unit) * v with
    v a random unit direction (binary64) and s drawn from `steps`, rounded to
    the nearest float32.  The partners' distances to their rows fall within a
    few float32 roundings of eps, inside the device filters' error bands."""
    rng = np.random.default_rng(seed)
    rows = rng.choice(len(base), size=count, replace=count > len(base))
    v = rng.standard_normal((count, base.shape[1]))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    s = rng.choice(np.asarray(steps, dtype=np.float64), size=count)
    q = base[rows].astype(np.float64) + (eps * (1.0 + s * unit))[:, None] * v
    return q.astype(np.float32)
