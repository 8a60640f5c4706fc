"""Write eps.json: the calibrated epsilon of every named workload and target
mean-neighbour count (S_D, Section 5.2).  Calls only the oracle and the input
generators.  Run from the repository root:  python tests/golden/make_eps.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "eps.json")


def batched(name="batched_256", n_jobs=256, seed=7):
    """Per-job epsilons of the many-joins workload (datagen.batched_job_specs):
    each job's own target mean-neighbour count on its own seeded sample."""
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    t0 = time.time()
    jobs = []
    for spec in datagen.batched_job_specs(n_jobs, seed):
        P = datagen.make_job(spec)
        rows = datagen.calibration_rows(len(P), spec["seed"])
        eps, sd = oracle.calibrate_eps(P, spec["target"], rows)
        jobs.append({"hex": float(eps).hex(), "value": float(eps), "sample_sd": sd,
                     "n": spec["n"], "d": spec["d"], "kind": spec["kind"],
                     "target": spec["target"]})
        if len(jobs) % 32 == 0:
            print(name, len(jobs), "%.1fs" % (time.time() - t0), flush=True)
    table[name] = {"n_jobs": n_jobs, "seed": seed, "jobs": jobs}
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def main(names):
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    for name in names:
        w = datagen.WORKLOADS[name]
        t0 = time.time()
        P = datagen.make_workload(name)
        rows = datagen.calibration_rows(len(P), w["seed"])
        entry = {"n": w["n"], "d": w["d"], "seed": w["seed"],
                 "sample_rows": int(len(rows)), "eps": {}}
        for target in w["targets"]:
            eps, sd = oracle.calibrate_eps(P, target, rows)
            entry["eps"][str(target)] = {"hex": float(eps).hex(),
                                         "value": float(eps),
                                         "sample_sd": sd}
            print(name, target, eps, sd, "%.1fs" % (time.time() - t0), flush=True)
        table[name] = entry
        with open(OUT, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args == ["batched_256"]:
        batched()
    else:
        main(args or list(datagen.WORKLOADS))
