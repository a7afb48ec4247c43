"""Write the oracle's growth for the large workloads to ``oracle_growth.json``.

Run from the repository root: ``python tests/golden/make_oracle_fixtures.py
[name ...]``. It calls only the CPU oracle (``oracle/``) on inputs from
``paper_2509_19162_amd.inputs``; the GPU tests compare against the file.

* pancake_12:   S_12, prefix reversals (k = 11), full growth.
* lrx_16_prefix: S_16, LRX, every layer up to and including the first one
  larger than 2^26 (the GPU run goes on to 2^31; the oracle's hash set
  cannot hold that many states in host memory).
* batch_4096:   the 4096 batched jobs (n ~ U{7..10}, 2-4 random
  permutations plus inverses), full growth each.
"""

import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import native  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_growth.json")


def _load():
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def _save(d):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, OUT)


def _batch_job(j):
    n, gens = _JOBS[j]
    sizes, rc, _ = native.growth(n, gens)
    return j, sizes, rc


_JOBS = None


def _init_jobs():
    global _JOBS
    _JOBS = I.batch_jobs(4096)


def main(names):
    native.build(force=False)
    data = _load()
    if "pancake_12" in names:
        t = time.time()
        sizes, rc, _ = native.growth(12, I.pancake(12))
        data["pancake_12"] = {"n": 12, "family": "pancake", "sizes": sizes, "status": rc,
                              "oracle_seconds": round(time.time() - t, 1)}
        _save(data)
        print("pancake_12", sizes, flush=True)
    if "lrx_16_prefix" in names:
        t = time.time()
        sizes, rc, _ = native.growth(16, I.lrx(16), max_frontier=1 << 26)
        data["lrx_16_prefix"] = {"n": 16, "family": "lrx", "max_frontier": 1 << 26, "sizes": sizes,
                                 "status": rc, "oracle_seconds": round(time.time() - t, 1)}
        _save(data)
        print("lrx_16_prefix", sizes, flush=True)
    if "batch_4096" in names:
        t = time.time()
        with Pool(processes=max(1, (os.cpu_count() or 2) - 1), initializer=_init_jobs) as pool:
            res = sorted(pool.map(_batch_job, range(4096), chunksize=8))
        data["batch_4096"] = {"seed": I.SEED, "jobs": 4096,
                              "sizes": [r[1] for r in res], "status": [r[2] for r in res],
                              "oracle_seconds_wall": round(time.time() - t, 1)}
        _save(data)
        print("batch_4096 done", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["pancake_12", "lrx_16_prefix", "batch_4096"])
