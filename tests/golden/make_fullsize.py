"""Write the oracle digests of the full-size parity cases
(tests/golden/fullsize_<case>.json) by running the exact-integer oracle on
the seeded inputs of tests/fullsize_cases.py.  Nothing here touches the
GPU library.

Usage (from the repository root):
    python tests/golden/make_fullsize.py [--jobs J] [case ...]

At N = 32768 the oracle takes about 10 s per squaring with
relinearization on one core, so the whole set is several CPU-hours; units
run in parallel processes.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from tests import fullsize_cases as fc  # noqa: E402

_ENVS = {}


def _env(log2_n: int, alpha: int = 1) -> fc.Env:
    if (log2_n, alpha) not in _ENVS:
        _ENVS[(log2_n, alpha)] = fc.Env(log2_n, alpha=alpha)
    return _ENVS[(log2_n, alpha)]


def _run_unit(task):
    case, unit = task
    log2_n, units = fc.CASES[case]
    fn = dict(units)[unit]
    t0 = time.time()
    out = fn(_env(log2_n, fc.CASE_ALPHA.get(case, 1)))
    rec = {label: fc.record(arr) for label, arr in out.items()}
    print(f"{case}/{unit}: {time.time() - t0:.0f} s", flush=True)
    return case, unit, rec


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=list(fc.CASES))
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    args = ap.parse_args()
    tasks = [(c, u) for c in args.cases for u, _ in fc.CASES[c][1]]
    results = {c: {} for c in args.cases}
    with mp.get_context("fork").Pool(args.jobs, maxtasksperchild=4) as pool:
        for case, unit, rec in pool.imap_unordered(_run_unit, tasks):
            results[case][unit] = rec
            if len(results[case]) == len(fc.CASES[case][1]):
                outputs = {}
                for u, _ in fc.CASES[case][1]:
                    outputs.update(results[case][u])
                log2_n = fc.CASES[case][0]
                path = os.path.join(fc.GOLDEN_DIR, f"fullsize_{case}.json")
                with open(path, "w") as f:
                    json.dump({"case": case, "n": 1 << log2_n,
                               "written_by": "python tests/golden/make_fullsize.py " + case,
                               "outputs": outputs}, f, separators=(",", ":"))
                print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
