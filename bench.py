"""Benchmark of the epsilon self-join hot path on one MI355X.

One step = the whole path (index build with automatic k, estimate, join,
sort of the result in device memory) for every epsilon of the workload's
sweep, on synthetic data already resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

The default line (uniform 2*10^6 x 16, plain FP32, three epsilons) also
carries the comparison the benchmark is about: the same workload on the
matrix cores ("compare"), the paper's host-complete clock with every pair
stored in pinned host memory ("host_complete"), 256 joins in one persistent
launch against the same joins run one by one ("batched_256"), and the
2*10^6 x 64, 5*10^6 x 18 and 515,000 x 90 configurations with both filters
("other_configs"); --no-extras drops the last three.

Other lines (not the headline): --workload batched_256 (many joins in one
launch), --query-sets N (the general join of N entity-partitioned query
sets), --k-sweep (index-search against distance work per k), --host-io
(PCIe-inclusive), --sortidu (SORTIDU on), --precision / --compare (filters).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402

EPS_TABLE = os.path.join(ROOT, "tests", "golden", "eps.json")
TRAFFIC = os.path.join(ROOT, "profiles", "pmc_k_join_fp32_uniform_2m_d16.md")
JOIN_SRC = os.path.join(ROOT, "paper_1809_09930_amd", "csrc", "sj_join.hip")

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 FP32 lane
# instructions/s.  The published FP32 vector peak, 157.3 TFLOP/s, counts
# packed FMAs (2 lanes x 2 flops); packed FP32 math is disabled in this
# build, so one FMA per lane and cycle, 78.6 TFLOP/s, is its own ceiling.
# Both fractions are reported.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 78.6
VALU_LANE_OPS_PER_S = 3.93e13
# Dense FP16/BF16 matrix-core peak of MI355X.
PEAK_MFMA_16BIT_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uniform_2m_d16")
    ap.add_argument("--targets", default="", help="comma list of S_D targets (default: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="query rows for the CPU oracle sample (0: sized to ~15 s)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "bf16"],
                    help="distance filter of the headline line")
    ap.add_argument("--compare", default="fp16",
                    help="comma list of other precisions timed on the same workload ('' = none)")
    ap.add_argument("--query-sets", type=int, default=0,
                    help="instead of the self-join: the general join of N_b entity-partitioned "
                         "query sets Q_l (every N_b-th point from offset l) against the whole "
                         "workload, one query handle per set")
    ap.add_argument("--batch-pairs", type=float, default=0,
                    help="result batches of at most this many pairs (streamed to pinned host "
                         "memory); 0 = as the memory budget allows")
    ap.add_argument("--sortidu", action="store_true",
                    help="build every index with SORTIDU (search along one un-indexed dimension)")
    ap.add_argument("--host-io", action="store_true",
                    help="instead of the device-resident step: points handed over from host "
                         "memory and the whole result (i, j) fetched into pinned host memory, "
                         "timed per epsilon (PCIe-inclusive rate)")
    ap.add_argument("--k-sweep", default="",
                    help="comma list of explicit k: index and join the largest epsilon of the "
                         "workload at each k and report the index-search and distance work")
    ap.add_argument("--no-extras", action="store_true",
                    help="default line only: skip the host-complete clock, the batched "
                         "comparison and the other configurations")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only copy a buffer of this many MiB device-to-device 3 times (scales "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def candidate_prefix_mean(P, perm, k, eps, n_queries=96, per_query=16384, seed=99):
    """Mean number of dimensions a per-pair short-circuit evaluates, over
    the grid's CANDIDATE pairs: for seeded query points q, the points in the
    3^k cells around q's cell (cell side eps (1 + 2^-20) from the per-dimension
    minimum over the first k reordered dimensions), and per pair the first
    reordered dimension at which the binary64 partial sum of squares exceeds
    eps^2 (all d when it never does).  Each query's candidates are
    subsampled to per_query and weighted by their count, so the result
    estimates the mean over all candidate pairs (a ratio estimator)."""
    rng = np.random.default_rng(seed)
    n, d = P.shape
    X = P[:, perm]
    eps2 = eps * eps
    w = eps * (1.0 + 2.0 ** -20)
    lo = X[:, :k].astype(np.float64).min(axis=0)
    cells = np.floor((X[:, :k].astype(np.float64) - lo) / w).astype(np.int32)
    every_adjacent = bool((cells.max(axis=0) <= 1).all())  # all pairs are candidates
    # points ordered by their cell along the first two indexed dimensions,
    # so a query's neighbours along those come from three contiguous ranges
    k2 = min(k, 2)
    m1 = int(cells[:, 1].max()) + 3 if k2 == 2 else 1
    key = cells[:, 0].astype(np.int64) * m1 + (cells[:, 1] + 1 if k2 == 2 else 0)
    order = np.argsort(key, kind="stable")
    skey = key[order]
    num = den = 0.0
    for q in rng.choice(n, size=min(n_queries, n), replace=False):
        if every_adjacent:
            m = n
            take = rng.integers(0, n, size=per_query)
        else:
            parts = []
            for o in (-1, 0, 1):
                kq = (int(cells[q, 0]) + o) * m1 + (int(cells[q, 1]) + 1 if k2 == 2 else 0)
                lo_k, hi_k = (kq - 1, kq + 1) if k2 == 2 else (kq, kq)
                parts.append(order[np.searchsorted(skey, lo_k, "left"):
                                   np.searchsorted(skey, hi_k, "right")])
            cand = np.concatenate(parts)
            for r in range(k2, k):  # narrowed one indexed dimension at a time
                cand = cand[np.abs(cells[cand, r] - cells[q, r]) <= 1]
            m = len(cand)
            take = cand if m <= per_query else rng.choice(cand, size=per_query, replace=False)
        xq = X[q].astype(np.float64)
        acc = np.zeros(len(take))
        dims = np.full(len(take), float(d))
        done = np.zeros(len(take), dtype=bool)
        for r in range(d):
            diff = X[take, r].astype(np.float64) - xq[r]
            acc = acc + diff * diff
            newly = (~done) & (acc > eps2)
            dims[newly] = r + 1
            done |= newly
        num += m * float(dims.mean())
        den += m
    return num / den


def traffic_for_join():
    """HBM bytes per join launch from the committed rocprofv3 counter
    summary (its 'key: value' lines), valid only while the kernel source is
    unchanged."""
    if not os.path.exists(TRAFFIC):
        return None
    fields = {}
    with open(TRAFFIC) as f:
        for line in f:
            key, sep, val = line.partition(":")
            if sep and key.strip() in ("kernel", "source_sha256", "bytes_per_launch"):
                fields[key.strip()] = val.strip()
    sha = hashlib.sha256(open(JOIN_SRC, "rb").read()).hexdigest()
    if fields.get("source_sha256") != sha or "bytes_per_launch" not in fields:
        return None
    return int(fields["bytes_per_launch"])


def cpu_baseline(P, eps, rows_req):
    """The oracle (FP64 nested loop over candidate rows) on a bounded sample
    of query rows, on the host cores."""
    import oracle
    n = len(P)
    rng = np.random.default_rng(2024)
    if rows_req <= 0:
        # size the sample to about 15 s from a probe that fills every thread
        m = max(64, 4 * oracle.num_threads())
        probe = np.sort(rng.choice(n, size=m, replace=False))
        t0 = time.perf_counter()
        oracle.rows(P, eps, probe)
        dt = max(time.perf_counter() - t0, 1e-3)
        rows_req = int(min(8192, max(16, m * 15.0 / dt)))
    rows = np.sort(rng.choice(n, size=min(rows_req, n), replace=False))
    t0 = time.perf_counter()
    oracle.rows(P, eps, rows)
    dt = time.perf_counter() - t0
    cand = float(len(rows)) * n
    return {"value": cand / dt, "unit": "candidate distance evals/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d seeded query rows x all %d points (FP64 canonical predicate), %.1f s"
                      % (len(rows), n, dt)}


def bench_batched(a, table):
    """The batched comparison on its own line (--workload batched_256)."""
    from paper_1809_09930_amd import selfjoin as sj
    prec = a.precision if a.precision != "fp32" else "fp16"
    b = batched_comparison(sj, table, a.workload, a.steps, a.warmup, prec)
    out = {
        "metric": "candidate distance evals/s (exact pair set)",
        "value": b.pop("value"),
        "unit": "candidate distance evals/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": b.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": a.workload, "jobs": b["jobs"], "points": b["points"],
                   "path": b["path"]},
    }
    out.update(b)
    print(json.dumps(out), flush=True)


def bench_query_sets(a, table, P, Pd, targets, eps_list):
    """The general join Q_l join_eps D for the N_b entity-partitioned query
    sets of the paper's distributed scheme: one index of D, then one query
    handle per set (build, join, sort).  Reports the aggregate rate and the
    spread of the per-set join times (the load balance across sets)."""
    import torch
    from paper_1809_09930_amd import selfjoin as sj
    nb = a.query_sets
    n, d = P.shape
    sets = [Pd[l::nb].contiguous() for l in range(nb)]
    torch.cuda.synchronize()

    def step(record, precision):
        for t, eps in zip(targets, eps_list):
            he = sj.selfjoin_build_index(Pd, eps, precision=precision, sortidu=a.sortidu)
            e_info = sj.selfjoin_get_info(he)
            e_info["perm"] = sj.selfjoin_get_perm(he, d)
            rows = []
            for q in sets:
                hq = sj.selfjoin_build_query(he, q)
                total = sj.selfjoin_run(hq)
                rows.append((total, sj.selfjoin_get_info(hq)))
                sj.selfjoin_free(hq)
            sj.selfjoin_free(he)
            if record is not None:
                record.append((t, eps, e_info, rows))

    prec = a.precision
    for _ in range(a.warmup):
        step(None, prec)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step(recs, prec)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cand = sum(i["candidates"] for r in recs for _, i in r[3])
    pairs = sum(tot for r in recs for tot, _ in r[3])
    per_eps = {}
    flops_total = time_total = 0.0
    join_all = []
    for t, eps, e_info, rows in recs[:len(targets)]:
        join = np.array([i["ms_join"] / max(i["join_launches"], 1) for _, i in rows])
        c_sets = float(sum(i["candidates"] for _, i in rows))
        if prec == "fp32":  # operations the short-circuit leaves, per candidate (one direction)
            flops_total += 3.0 * candidate_prefix_mean(P, e_info["perm"], e_info["k"], eps) * c_sets
        else:               # one d-long dot product per candidate
            flops_total += 2.0 * d * c_sets
        time_total += float(join.sum()) / 1e3
        join_all.extend(join.tolist())
        run = np.array([i["ms_run"] for _, i in rows])
        build = np.array([i["ms_build"] for _, i in rows])
        tot = sum(x for x, _ in rows)
        per_eps[t] = {"eps": eps, "pairs": tot, "sd": (tot - n) / n, "k": e_info["k"],
                      "candidates": sum(i["candidates"] for _, i in rows),
                      "ms_index_build": round(e_info["ms_build"], 3),
                      "ms_query_build_sum": round(float(build.sum()), 3),
                      "ms_join_per_set": {"min": round(float(join.min()), 3),
                                          "max": round(float(join.max()), 3),
                                          "mean": round(float(join.mean()), 3)},
                      "ms_run_per_set": {"min": round(float(run.min()), 3),
                                         "max": round(float(run.max()), 3),
                                         "mean": round(float(run.mean()), 3)},
                      "max_over_min_join": round(float(join.max() / max(join.min(), 1e-9)), 4)}
    out = {
        "metric": "candidate distance evals/s (exact pair set)",
        "value": cand / elapsed,
        "unit": "candidate distance evals/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": elapsed * 1e3 / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else prec, "data": "synthetic",
        "config": {"workload": a.workload, "n": n, "d": d, "query_sets": nb,
                   "epsilons": eps_list,
                   "path": "general join Q_l join_eps D per query set (one direction, "
                           "%s filter), index of D built once per epsilon" % prec},
        "result_pairs_per_s": pairs / elapsed,
        "per_epsilon": per_eps,
    }
    achieved = flops_total / time_total / 1e12 if time_total > 0 else 0.0
    peak = PEAK_FP32_TFLOPS if prec == "fp32" else PEAK_MFMA_16BIT_TFLOPS
    out["roofline"] = {"bound": "alu" if prec == "fp32" else "mfma", "achieved": achieved,
                       "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                       "kernel": "k_join_fp32" if prec == "fp32" else "k_join_mfma",
                       "mean_launch_ms": float(np.mean(join_all)) if join_all else 0.0}
    print(json.dumps(out), flush=True)


def bench_host_io(a, P, targets, eps_list):
    """The whole call sequence with host buffers at both ends: build from a
    host array (the library copies it to the device), run, and fetch the i
    and j columns of the result into pinned host memory."""
    import torch
    from paper_1809_09930_amd import selfjoin as sj
    n, d = P.shape
    Ph = torch.from_numpy(P)
    rows = {}
    for t, eps in zip(targets, eps_list):
        for rep_ in range(a.warmup + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = sj.selfjoin_build_index(Ph, eps, precision=a.precision)
            t1 = time.perf_counter()
            total = sj.selfjoin_run(h)
            t2 = time.perf_counter()
            oi = torch.empty(total, dtype=torch.int32, pin_memory=True)
            oj = torch.empty(total, dtype=torch.int32, pin_memory=True)
            t3 = time.perf_counter()
            sj.selfjoin_fetch_pairs(h, 0, oi, oj, None, max_pairs=total)
            t4 = time.perf_counter()
            info = sj.selfjoin_get_info(h)
            sj.selfjoin_free(h)
        rows[t] = {"eps": eps, "pairs": total, "s_build_from_host": round(t1 - t0, 4),
                   "s_run": round(t2 - t1, 4), "s_fetch_to_pinned_host": round(t4 - t3, 4),
                   "s_total_excl_host_alloc": round((t4 - t0) - (t3 - t2), 4),
                   "candidates_per_s": info["candidates"] / ((t4 - t0) - (t3 - t2)),
                   "fetch_GB_per_s": total * 8 / max(t4 - t3, 1e-9) / 1e9}
    print(json.dumps({"metric": "PCIe-inclusive self-join (host input, host output)",
                      "workload": a.workload, "precision": a.precision, "n": n, "d": d,
                      "per_epsilon": rows}), flush=True)


def bench_k_sweep(a, P, Pd, eps):
    """Section 5.5 (Figure 8): index-search work against distance work as k
    grows, at one epsilon.  Per k: non-empty cells #G, adjacent-cell lookups
    (#G * 3^k here, one search per cell; |D| * 3^k in the paper's
    one-thread-per-point kernel), ordered candidates C and the coordinates a
    join without short-circuit would load (C * d), with the build and join
    times of the library."""
    import torch
    from paper_1809_09930_amd import selfjoin as sj
    n, d = P.shape
    rows = {}
    for k in [int(x) for x in a.k_sweep.split(",") if x.strip()]:
        for rep_ in range(a.warmup + 1):
            h = sj.selfjoin_build_index(Pd, eps, k=k, precision=a.precision, sortidu=a.sortidu)
            total = sj.selfjoin_run(h)
            info = sj.selfjoin_get_info(h)
            sj.selfjoin_free(h)
        torch.cuda.synchronize()
        rows[str(k)] = {"k": info["k"], "cells": info["n_cells"],
                        "lookups_per_cell_search": info["n_cells"] * 3 ** info["k"],
                        "lookups_per_point_search": n * 3 ** info["k"],
                        "candidates": info["candidates"],
                        "distance_coordinate_loads": info["candidates"] * d,
                        "pairs": total, "rechecks": info["rechecks"],
                        "batches": info["batches"], "join_launches": info["join_launches"],
                        "ms_build": round(info["ms_build"], 3),
                        "ms_join": round(info["ms_join"] / max(info["join_launches"], 1), 3),
                        "ms_sort": round(info["ms_sort"], 3), "ms_run": round(info["ms_run"], 3)}
    out = {"metric": "index-search vs distance work per k", "workload": a.workload,
           "eps": eps, "precision": a.precision, "n": n, "d": d, "per_k": rows}
    print(json.dumps(out), flush=True)


def selfjoin_step(sj, Pd, d, eps_list, targets, precision, sortidu, record, batch_pairs=0):
    """One step: build (automatic k), run (estimate, join, recheck, sort in
    device memory, or in batches to pinned host memory) and free, for every
    epsilon of the sweep."""
    for t, eps in zip(targets, eps_list):
        h = sj.selfjoin_build_index(Pd, eps, precision=precision, sortidu=sortidu,
                                    batch_pairs=batch_pairs)
        total = sj.selfjoin_run(h)
        info = sj.selfjoin_get_info(h)
        perm = sj.selfjoin_get_perm(h, d)
        sj.selfjoin_free(h)
        if record is not None:
            record.append((t, eps, total, info, perm))


def timed_steps(sj, Pd, d, eps_list, targets, precision, steps, warmup, sortidu=False,
                batch_pairs=0):
    import torch
    for _ in range(warmup):
        selfjoin_step(sj, Pd, d, eps_list, targets, precision, sortidu, None, batch_pairs)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        selfjoin_step(sj, Pd, d, eps_list, targets, precision, sortidu, recs, batch_pairs)
    torch.cuda.synchronize()
    return recs, time.perf_counter() - t0


def per_eps_table(P, recs, ntargets, precision):
    """Per-epsilon rows of the first recorded step, and the algorithmic work
    and join time summed over them.  FP32: 3 flops per dimension the ideal
    per-pair short-circuit evaluates (mean over candidate pairs), per
    unordered pair.  Matrix cores: one d-long dot product (2d flops) per
    unordered pair, and the floor max(MFMA time, one vector compare per
    pair)."""
    n, d = P.shape
    per_eps, flops_total, time_total = {}, 0.0, 0.0
    for t, eps, total, info, perm in recs[:ntargets]:
        # one join per epsilon: per launch (a rerun after an undersized
        # buffer repeats it), or the sum over result batches
        ms = (info["ms_join"] if info["batches"] > 1
              else info["ms_join"] / max(info["join_launches"], 1))
        npair = (info["candidates"] + n) / 2.0
        row = {"eps": eps, "pairs": total, "sd": (total - n) / n, "k": info["k"],
               "cells": info["n_cells"], "candidates": info["candidates"],
               "evaluated": info["evaluated"], "rechecks": info["rechecks"],
               "ms_build": round(info["ms_build"], 3), "ms_join": round(ms, 3),
               "ms_sort": round(info["ms_sort"], 3), "ms_run": round(info["ms_run"], 3),
               "batches": info["batches"], "join_launches": info["join_launches"]}
        if precision == "fp32":
            pbar = candidate_prefix_mean(P, perm, info["k"], eps)
            row["shortc_prefix_mean"] = round(pbar, 3)
            flops_total += 3.0 * pbar * npair
        else:
            flops_total += 2.0 * d * npair
            floor_s = max(2.0 * d * npair / (PEAK_MFMA_16BIT_TFLOPS * 1e12),
                          npair / VALU_LANE_OPS_PER_S)
            row["ms_floor_mfma_or_compare"] = round(floor_s * 1e3, 3)
        time_total += ms / 1e3
        per_eps[t] = row
    return per_eps, flops_total, time_total


def summarise(P, recs, elapsed, steps, ntargets, precision):
    """Rate, per-epsilon rows and the join kernel's roofline of one path."""
    cand = sum(r[3]["candidates"] for r in recs)
    pairs = sum(r[2] for r in recs)
    per_eps, flops, tjoin = per_eps_table(P, recs, ntargets, precision)
    achieved = flops / tjoin / 1e12 if tjoin > 0 else 0.0
    out = {"value": cand / elapsed, "ms_per_step": elapsed * 1e3 / steps,
           "result_pairs_per_s": pairs / elapsed, "per_epsilon": per_eps,
           "mean_join_launch_ms": float(np.mean([r[3]["ms_join"] / max(r[3]["join_launches"], 1)
                                                 for r in recs]))}
    if precision == "fp32":
        out["kernel_achieved_tflops"] = achieved
        out["kernel_frac_of_published_fp32_peak"] = achieved / PEAK_FP32_TFLOPS
        out["kernel_frac_of_nonpacked_fp32"] = achieved / PEAK_FP32_NONPACKED_TFLOPS
    else:
        floor_ms = sum(r["ms_floor_mfma_or_compare"] for r in per_eps.values())
        out["kernel_achieved_tflops"] = achieved
        out["kernel_frac_of_mfma_peak"] = achieved / PEAK_MFMA_16BIT_TFLOPS
        out["kernel_frac_of_floor"] = floor_ms / 1e3 / tjoin if tjoin > 0 else 0.0
    return out, flops, tjoin


def bench_host_complete(sj, P, Pd, eps_list, targets, precision):
    """The paper's response-time clock (Section 5.2): build, join and the
    whole (i, j) result stored in pinned host memory, per epsilon.  Inputs
    start in HBM; the pinned buffers are allocated once, before timing."""
    import torch
    n, d = P.shape
    totals = []
    for eps in eps_list:  # result sizes, and a warm run of each epsilon
        h = sj.selfjoin_build_index(Pd, eps, precision=precision)
        totals.append(sj.selfjoin_run(h))
        sj.selfjoin_free(h)
    cap = max(totals)
    oi = torch.empty(cap, dtype=torch.int32, pin_memory=True)
    oj = torch.empty(cap, dtype=torch.int32, pin_memory=True)
    torch.cuda.synchronize()
    rows, cand = {}, 0
    t_all = time.perf_counter()
    for t, eps in zip(targets, eps_list):
        t0 = time.perf_counter()
        h = sj.selfjoin_build_index(Pd, eps, precision=precision)
        total = sj.selfjoin_run(h)
        t1 = time.perf_counter()
        sj.selfjoin_fetch_pairs(h, 0, oi, oj, None, max_pairs=total)
        t2 = time.perf_counter()
        info = sj.selfjoin_get_info(h)
        sj.selfjoin_free(h)
        cand += info["candidates"]
        rows[t] = {"pairs": total, "s_build_and_run": round(t1 - t0, 4),
                   "s_fetch_to_pinned_host": round(t2 - t1, 4),
                   "fetch_GB_per_s": round(total * 8 / max(t2 - t1, 1e-9) / 1e9, 2)}
    elapsed = time.perf_counter() - t_all
    # the largest result again in batches of at most 1e8 pairs (Section
    # 3.2.2): each batch sorted and streamed to pinned host memory while the
    # next one computes; the best of two warm runs against the one-batch run
    t_big, eps_big = targets[-1], eps_list[-1]

    def once(batch_pairs):
        t0 = time.perf_counter()
        h = sj.selfjoin_build_index(Pd, eps_big, precision=precision, batch_pairs=batch_pairs)
        total = sj.selfjoin_run(h)
        sj.selfjoin_fetch_pairs(h, 0, oi, oj, None, max_pairs=total)
        dt = time.perf_counter() - t0
        info = sj.selfjoin_get_info(h)
        sj.selfjoin_free(h)
        return dt, info
    once(int(1e8))  # warm: the batches' pinned buffers
    single = min(once(0)[0] for _ in range(2))
    runs = [once(int(1e8)) for _ in range(2)]
    multi, minfo = min(runs, key=lambda r: r[0])
    batched = {"target": t_big, "batch_pairs": int(1e8), "batches": minfo["batches"],
               "s_one_batch": round(single, 4), "s_batched": round(multi, 4),
               "ratio": round(multi / single, 3), "evaluated": minfo["evaluated"],
               "ms_join": round(minfo["ms_join"], 1), "ms_sort": round(minfo["ms_sort"], 1)}
    return {"value": cand / elapsed, "ms_per_step": elapsed * 1e3,
            "result_pairs_per_s": sum(totals) / elapsed, "per_epsilon": rows,
            "clock": "build + join + sort + every (i, j) pair in pinned host memory",
            "batched": batched}


def workload_eps(table, name, targets_arg=""):
    w = datagen.WORKLOADS[name]
    if "eps_fixed" in w:  # the paper's own epsilons (its synthetic family)
        targets = [t.strip() for t in targets_arg.split(",") if t.strip()] or \
            [repr(e) for e in w["eps_fixed"]]
        return targets, [float(t) for t in targets]
    targets = [t.strip() for t in targets_arg.split(",") if t.strip()] or \
        [str(t) for t in w["targets"]]
    return targets, [float.fromhex(table[name]["eps"][t]["hex"]) for t in targets]


def bench_other_configs(sj, table):
    """The other configurations of the comparison, each with its matrix-core
    path against the plain FP32 path on the same data (few steps each)."""
    import torch
    out = {}
    # the 2M x 64 configuration names BF16 tiles; FP16 runs beside them
    plan = [("uniform_2m_d64", [("fp16", 2, 1), ("bf16", 2, 1), ("fp32", 1, 0)]),
            ("mixture50_5m_d18", [("fp16", 3, 1), ("fp32", 3, 1)]),
            ("mixture20_515k_d90", [("fp16", 3, 1), ("fp32", 2, 1)])]
    for name, runs in plan:
        targets, eps_list = workload_eps(table, name)
        P = datagen.make_workload(name)
        Pd = torch.from_numpy(P).cuda()
        row = {"n": P.shape[0], "d": P.shape[1], "epsilons": eps_list,
               "target_mean_neighbours": [int(t) for t in targets]}
        for prec, steps, warmup in runs:
            print("bench: %s %s" % (name, prec), file=sys.stderr, flush=True)
            recs, el = timed_steps(sj, Pd, P.shape[1], eps_list, targets, prec, steps, warmup)
            row[prec] = summarise(P, recs, el, steps, len(targets), prec)[0]
        for prec in ("fp16", "bf16"):
            if prec in row:
                row["speedup_%s_vs_fp32" % prec] = row[prec]["value"] / row["fp32"]["value"]
        out[name] = row
        del Pd
        torch.cuda.empty_cache()
    return out


def batched_comparison(sj, table, name="batched_256", steps=2, warmup=1, prec="fp16"):
    """Many independent self-joins in one persistent matrix-core launch under
    a captured hipGraph (autotuned), against the same jobs as sequential
    plain FP32 (and 16-bit) single joins on the same GPU."""
    import torch
    entry = table[name]
    specs = datagen.batched_job_specs(entry["n_jobs"], entry["seed"])
    pts = [torch.from_numpy(datagen.make_job(sp)).cuda() for sp in specs]
    eps = [float.fromhex(j["hex"]) for j in entry["jobs"]]
    torch.cuda.synchronize()

    def batched_once():
        h = sj.selfjoin_run_batched(pts, eps, precision=prec, autotune=True)
        return h, sj.selfjoin_batch_get_info(h)

    for _ in range(warmup):
        sj.selfjoin_batch_free(batched_once()[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        h, info = batched_once()
        infos.append(info)
        if len(infos) < steps:
            sj.selfjoin_batch_free(h)
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / steps
    replays = [sj.selfjoin_batch_replay(h) for _ in range(3)]  # outside the timed steps
    sj.selfjoin_batch_free(h)
    info = infos[-1]
    cand = info["candidates"]

    def sequential(precision):
        torch.cuda.synchronize()
        t = time.perf_counter()
        c = pairs = 0
        join_ms = 0.0
        for p, e in zip(pts, eps):
            hh = sj.selfjoin_build_index(p, e, precision=precision)
            pairs += sj.selfjoin_run(hh)
            inf = sj.selfjoin_get_info(hh)
            c += inf["candidates"]
            join_ms += inf["ms_join"]
            sj.selfjoin_free(hh)
        torch.cuda.synchronize()
        return time.perf_counter() - t, c, pairs, join_ms

    seq32 = sequential("fp32")
    seq16 = sequential(prec)
    graph_ms = float(np.median(replays))
    assert seq32[2] == info["pairs"] == seq16[2], "pair totals differ between paths"
    return {
        "value": cand / elapsed, "ms_per_step": elapsed * 1e3, "steps": steps, "warmup": warmup,
        "dtype": prec, "jobs": len(pts), "points": int(sum(p.shape[0] for p in pts)),
        "path": "one persistent %s matrix-core launch under hipGraph, autotuned" % prec,
        "result_pairs_per_s": info["pairs"] / elapsed,
        "batched": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in info.items()},
        "graph_replay_ms": graph_ms,
        "graph_candidates_per_s": cand / (graph_ms / 1e3),
        "sequential_fp32": {"s": seq32[0], "candidates_per_s": seq32[1] / seq32[0],
                            "pairs": seq32[2], "join_ms_sum": seq32[3]},
        "sequential_%s" % prec: {"s": seq16[0], "candidates_per_s": seq16[1] / seq16[0],
                                 "pairs": seq16[2], "join_ms_sum": seq16[3]},
        "speedup_vs_sequential_fp32": seq32[0] / elapsed,
        "speedup_graph_vs_sequential_fp32_joins": seq32[3] / graph_ms,
    }


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the self-join path here is single-GPU "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    if a.copy_probe_mib:
        src = torch.empty(a.copy_probe_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "copies": 3}))
        return
    from paper_1809_09930_amd import selfjoin as sj
    sj.load_library()
    with open(EPS_TABLE) as f:
        table = json.load(f)
    if a.workload.startswith("batched"):
        bench_batched(a, table)
        return
    w = datagen.WORKLOADS[a.workload]
    targets, eps_list = workload_eps(table, a.workload, a.targets)
    P = datagen.make_workload(a.workload)
    n, d = P.shape
    Pd = torch.from_numpy(P).cuda()
    torch.cuda.synchronize()
    if a.query_sets:
        bench_query_sets(a, table, P, Pd, targets, eps_list)
        return
    if a.k_sweep:
        bench_k_sweep(a, P, Pd, eps_list[-1])
        return
    if a.host_io:
        bench_host_io(a, P, targets, eps_list)
        return

    recs, elapsed = timed_steps(sj, Pd, d, eps_list, targets, a.precision, a.steps, a.warmup,
                                a.sortidu, int(a.batch_pairs))
    fp32 = a.precision == "fp32"
    head, flops, tjoin = summarise(P, recs, elapsed, a.steps, len(targets), a.precision)
    achieved = flops / tjoin / 1e12 if tjoin > 0 else 0.0
    cand = sum(r[3]["candidates"] for r in recs)
    # algorithmic HBM bytes of one join launch: the points once and 8 bytes
    # per emitted pair, at the epsilon the traffic counters were taken at
    # (the middle target of the sweep)
    mid_t = targets[len(targets) // 2]
    mid_pairs = next(r[2] for r in recs if r[0] == mid_t)
    alg_bytes = n * d * 4 + mid_pairs * 8
    traffic = traffic_for_join() if fp32 and a.workload == "uniform_2m_d16" else None
    out = {
        "metric": "candidate distance evals/s (exact pair set)",
        "value": head["value"],
        "unit": "candidate distance evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else a.precision,
        "data": "synthetic",
        "config": {"workload": a.workload, "n": n, "d": d, "distribution": w["kind"],
                   "target_mean_neighbours": ([int(t) for t in targets]
                                              if "eps_fixed" not in w else None),
                   "epsilons": eps_list,
                   "path": ("plain FP32 grid join" if fp32 else
                            "%s matrix-core join with FP64 band recheck" % a.precision)
                   + ", k auto in 4..8, symmetric tiles" + (", SORTIDU" if a.sortidu else "")
                   + (", result batches of at most %d pairs in pinned host memory"
                      % int(a.batch_pairs) if a.batch_pairs else "")},
        "result_pairs_per_s": head["result_pairs_per_s"],
        "per_epsilon": head["per_epsilon"],
        "roofline": {"bound": "alu" if fp32 else "mfma", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS if fp32 else PEAK_MFMA_16BIT_TFLOPS,
                     "unit": "TFLOP/s",
                     "frac": achieved / (PEAK_FP32_TFLOPS if fp32 else PEAK_MFMA_16BIT_TFLOPS),
                     "traffic": traffic,
                     "kernel": "k_join_fp32" if fp32 else "k_join_mfma",
                     "mean_launch_ms": head["mean_join_launch_ms"],
                     "algorithmic_bytes": alg_bytes,
                     "traffic_over_algorithmic": (traffic / alg_bytes) if traffic else None,
                     "traffic_epsilon": eps_list[len(targets) // 2]},
    }
    if fp32:
        out["roofline"]["peak_nonpacked"] = PEAK_FP32_NONPACKED_TFLOPS
        out["roofline"]["frac_nonpacked"] = achieved / PEAK_FP32_NONPACKED_TFLOPS
    compare = {}
    for prec in [x.strip() for x in a.compare.split(",") if x.strip() and x.strip() != a.precision]:
        print("bench: %s %s" % (a.workload, prec), file=sys.stderr, flush=True)
        crecs, celapsed = timed_steps(sj, Pd, d, eps_list, targets, prec, a.steps, a.warmup,
                                      a.sortidu)
        c = summarise(P, crecs, celapsed, a.steps, len(targets), prec)[0]
        c["speedup_vs_headline"] = c["value"] / head["value"]
        compare[prec] = c
    if compare:
        out["compare"] = compare
    default_line = (a.workload == "uniform_2m_d16" and not a.targets and not a.sortidu
                    and fp32 and not a.no_extras and not a.batch_pairs)
    if default_line:
        print("bench: host-complete", file=sys.stderr, flush=True)
        out["host_complete"] = bench_host_complete(sj, P, Pd, eps_list, targets, "fp32")
        del Pd
        torch.cuda.empty_cache()
        print("bench: batched_256", file=sys.stderr, flush=True)
        out["batched_256"] = batched_comparison(sj, table)
        out["other_configs"] = bench_other_configs(sj, table)
    if not a.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        mid = eps_list[len(eps_list) // 2]
        out["cpu_baseline"] = cpu_baseline(P, mid, a.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
