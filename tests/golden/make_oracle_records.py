"""Writes FP64 oracle records of the full-size workloads for the GPU parity tests.

Test infrastructure: it calls only the oracle (``oracle/``) and the seeded input
generators (``workloads/``); nothing here comes from the HIP path.  Output:

* ``oracle_lambda3.npz`` -- the three-level Lambda medium (32768 cells, 16 seeded
  materials, Gaussian pulse train, Alg. 1 over the full grid), all 200000 steps.
  Its 192 population traces are recorded every 10 steps; every 10th sample (one
  per 100 steps, 2000 per trace) is stored.  Within the run the first pulse of the
  train crosses the first 40 % of the grid (about 26 of the 64 probes).
* ``oracle_sweep_picks.npz`` -- the 8 seeded spot-check members of the 256-member
  batched sweep, each over its full 50000 steps, every recorded sample (E and the
  populations at two probes every 50 steps).

Each array is stored under its record name, prefixed by the problem, with the
problem's fingerprint (a hash of the generated description) so that a test can
tell when the generators have changed since the file was written.

Usage: python tests/golden/make_oracle_records.py [lambda3] [sweep] [--procs N]
(CPU only; the Lambda run takes roughly 45 minutes of one core, the sweep picks
about as much spread over the worker processes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LAMBDA_STRIDE = 10  # stored sample = every 10th recorded sample (one per 100 steps)
SWEEP_PICK_SEED_OFFSET = 3  # picks drawn like the batch test: default_rng(SEED_BASE + 3)


def fingerprint(prob) -> str:
    """Hash of a problem description (numbers and arrays), stable across runs."""
    import numpy as np

    def norm(v):
        if isinstance(v, dict):
            return {k: norm(v[k]) for k in sorted(v)}
        if isinstance(v, (list, tuple)):
            return [norm(x) for x in v]
        if isinstance(v, np.ndarray):
            return [norm(x) for x in v.tolist()]
        if isinstance(v, complex):
            return [repr(v.real), repr(v.imag)]
        if isinstance(v, float):
            return repr(v)
        if isinstance(v, (np.floating,)):
            return repr(float(v))
        if isinstance(v, (np.integer,)):
            return int(v)
        return v

    return hashlib.sha256(json.dumps(norm(prob), sort_keys=True).encode()).hexdigest()[:16]


def sweep_picks():
    import numpy as np
    import workloads as W

    return [int(k) for k in np.random.default_rng(W.SEED_BASE + SWEEP_PICK_SEED_OFFSET).choice(256, 8, replace=False)]


def _run_lambda3(_):
    import numpy as np
    import workloads as W
    from oracle import mb_oracle as O

    prob = W.lambda3()
    t0 = time.time()
    ref = O.run(prob)
    out = {"lambda3/fingerprint": np.array(fingerprint(prob)),
           "lambda3/n_steps": np.array(prob["n_steps"]),
           "lambda3/stride": np.array(LAMBDA_STRIDE)}
    for r in prob["records"]:
        out["lambda3/" + r["name"]] = np.asarray(ref[r["name"]])[LAMBDA_STRIDE - 1::LAMBDA_STRIDE]
    return "lambda3", out, time.time() - t0


def _run_sweep_pick(k):
    import numpy as np
    import workloads as W
    from oracle import mb_oracle as O

    prob = W.sweep(n_sims=256, precision=32)[k]
    t0 = time.time()
    ref = O.run(prob)
    tag = f"sweep{k}"
    out = {f"{tag}/fingerprint": np.array(fingerprint(prob)), f"{tag}/n_steps": np.array(prob["n_steps"])}
    for r in prob["records"]:
        out[f"{tag}/" + r["name"]] = np.asarray(ref[r["name"]])
    return tag, out, time.time() - t0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["lambda3", "sweep"])
    ap.add_argument("--procs", type=int, default=max(1, len(os.sched_getaffinity(0))))
    a = ap.parse_args(argv)
    # one BLAS thread per worker process
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor

    jobs = []
    if "lambda3" in a.which:
        jobs.append((_run_lambda3, 0))
    if "sweep" in a.which:
        jobs += [(_run_sweep_pick, k) for k in sweep_picks()]
    results = {}
    with ProcessPoolExecutor(max_workers=min(a.procs, len(jobs))) as ex:
        futs = [ex.submit(fn, arg) for fn, arg in jobs]
        for f in futs:
            tag, out, secs = f.result()
            print(f"{tag}: {secs:.0f} s", flush=True)
            results.update(out)
    if "lambda3" in a.which:
        np.savez_compressed(os.path.join(HERE, "oracle_lambda3.npz"),
                            **{k: v for k, v in results.items() if k.startswith("lambda3/")})
    if "sweep" in a.which:
        np.savez_compressed(os.path.join(HERE, "oracle_sweep_picks.npz"),
                            **{k: v for k, v in results.items() if k.startswith("sweep")})


if __name__ == "__main__":
    main()
