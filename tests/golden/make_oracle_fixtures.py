"""Write the oracle's growth for the large workloads to ``oracle_growth.json``.

Run from the repository root: ``python tests/golden/make_oracle_fixtures.py
[name ...]``. It calls only the CPU oracle (``oracle/``) on inputs from
``paper_2509_19162_amd.inputs``; the GPU tests compare against the file.

* pancake_12:   S_12, prefix reversals (k = 11), full growth.
* lrx_16_prefix: S_16, LRX, every layer up to and including the first one
  larger than 2^28 (about 1.06e9 states; the GPU run goes on to 2^31, and
  the oracle's hash set of about 1e10 states would not fit in host memory).
* batch_4096:   the 4096 batched jobs (n ~ U{7..10}, 2-4 random
  permutations plus inverses), full growth each.
* family_11:    S_11 with prefix reversals, LRX and reversals, full growth
  each (one worker per family).
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


def _family_11(fam):
    t = time.time()
    sizes, rc, _ = native.growth(11, I.family(fam, 11))
    return fam, sizes, rc, round(time.time() - t, 1)


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
        sizes, rc, _ = native.growth(16, I.lrx(16), max_frontier=1 << 28)
        data["lrx_16_prefix"] = {"n": 16, "family": "lrx", "max_frontier": 1 << 28, "sizes": sizes,
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


    if "family_11" in names:
        fams = ["pancake", "lrx", "reversals"]
        with Pool(processes=len(fams)) as pool:
            res = pool.map(_family_11, fams)
        data["family_11"] = {f: {"sizes": sz, "status": rc, "oracle_seconds": sec} for f, sz, rc, sec in res}
        _save(data)
        print("family_11 done", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["pancake_12", "lrx_16_prefix", "batch_4096"])
