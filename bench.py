"""Benchmark: growth of permutation-group Cayley graphs on one MI355X.

A "step" is one pass of the whole hot path (expand, sort, unique + set
difference against layers d and d-1, compaction) over one growth job.
Inputs are synthetic by nature (the generators of the paper's families);
each job's start state is resident on the device before the timed region.

Default run (one JSON line): the headline is S_16 with the L, R, X
generators, every layer up to the first one larger than 2^31 (about 1e10
states, 44 layers): states expanded per second over K timed growths, with
the roofline of the dominant kernel (HIP events over the timed region) and
the CPU oracle's rate on the same workload's first layers. Beside it, as
extra keys: S_12 with the 11 prefix reversals (full growth, all layers
kept), the 4096-job batch (jobs/s against the same jobs run one at a time on
the same GPU, and the oracle on all host cores), one serving point
(p50/p99 latency at 0.9 x the measured capacity) and a plain copy kernel's
bandwidth as the measured HBM ceiling.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

--workload picks one leg alone (lrx16, pancake12, coxeter8, pancake13,
coxeter14, coset38, batch4096, serving).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    "lrx16": dict(n=16, family="lrx", keep_all=False, max_frontier=1 << 31,
                  desc="S_16, LRX (cyclic left shift, right shift, swap of positions 0 and 1), "
                       "layers up to the first one larger than 2^31"),
    "pancake12": dict(n=12, family="pancake", keep_all=True, max_frontier=None,
                      desc="S_12, 11 prefix reversals (pancake), full BFS, all layers kept"),
    "coxeter8": dict(n=8, family="coxeter", keep_all=False, max_frontier=None, on_chip=True,
                     desc="S_8, 7 adjacent transpositions (bubble-sort graph), full BFS"),
    # the bitmask engine (3 bits per state over the n! ranks) on groups the
    # sort path cannot hold
    "pancake13": dict(n=13, family="pancake", keep_all=False, max_frontier=None, bitmask=True,
                      desc="S_13, 12 prefix reversals (pancake), full BFS, bitmask engine"),
    "coxeter14": dict(n=14, family="coxeter", keep_all=False, max_frontier=None, bitmask=True,
                      desc="S_14, 13 adjacent transpositions, full BFS, bitmask engine"),
    # a Schreier coset graph with one bit per entry
    "coset38": dict(n=38, family="lrx", keep_all=False, max_frontier=None, binary_start=True,
                    desc="Schreier coset graph of the binary central state (19 zeros then 19 ones) under LRX, "
                         "n = 38: full BFS over all C(38,19) = 3.5e10 states, one bit per entry"),
}

# requests of the serving point in the default run (the full sweep takes 500)
DEFAULT_RUN_REQUESTS = 200

# Paper, table "Growth computations ... CPU on Kaggle cloud" (timing table
# with GAP): S_12 pancake took 4923 s with CayleyPy on a Kaggle CPU.
PAPER_PANCAKE12_SECONDS = 4923.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info() -> dict:
    """Host cores this process may use and the CPU model name."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if not model:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return {"nproc": cores, "cpu_model": model}


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs, or None when its device sources changed since the counters were
    taken."""
    from paper_2509_19162_amd.profiling import source_digest

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(workload, {}).get(kernel)
    if not e or e.get("source_digest") != source_digest(kernel):
        return None
    return e.get("bytes_per_launch")


def calibrate_copy(nbytes: int, repeats: int) -> None:
    """Runs the plain copy kernel `repeats` times over `nbytes` bytes: the
    known traffic that scales the hardware counters."""
    import torch

    from paper_2509_19162_amd import testing

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    testing.copy(src, dst, repeats=repeats)
    dt = time.perf_counter() - t
    print(json.dumps({"copy_bytes": nbytes, "repeats": repeats,
                      "gbs": round(2.0 * nbytes * repeats / dt / 1e9, 1)}), flush=True)


def copy_ceiling(nbytes: int = 4 << 30, repeats: int = 5) -> dict:
    """Measured HBM ceiling: the plain copy kernel over `nbytes` (read +
    write), timed with HIP events on the stream it runs on."""
    import torch

    from paper_2509_19162_amd import testing

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    testing.copy(src, dst, repeats=1)  # warm
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    testing.copy(src, dst, repeats=repeats)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    gbs = 2.0 * nbytes * repeats / (ms / 1000.0) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"gbs": round(gbs, 1), "bytes_copied": nbytes, "repeats": repeats,
            "frac_of_spec": round(gbs / HBM_PEAK_GBS, 4), "spec_gbs": HBM_PEAK_GBS,
            "timing": "HIP events around the launches"}


def cpu_baseline(workload: dict, budget_s: float, host: dict):
    """The CPU oracle (single thread) on the first layers of the same
    workload: the largest layer prefix whose expansion fits the budget."""
    from oracle import bfs_set, native
    from paper_2509_19162_amd import inputs as I

    native.build(force=False)
    n = workload["n"]
    gens = I.family(workload["family"], n)
    start = I.binary_central_state(n) if workload.get("binary_start") else None
    # the C oracle packs 4 bits per entry (n <= 16); longer binary states
    # take the Python set BFS
    use_c = n <= 16
    best = None
    layers = 2
    while True:
        t = time.perf_counter()
        if use_c:
            sizes, rc, _ = native.growth(n, gens, max_layers=layers, start=start)
        else:
            layers_found, complete = bfs_set.bfs_layers(n, gens, max_layers=layers, start=start)
            sizes, rc = [len(x) for x in layers_found], 0 if complete else 1
        dt = time.perf_counter() - t
        expanded = sum(sizes[:-1]) if rc == 1 else sum(sizes)
        best = (layers, expanded, dt, sizes)
        if rc == 0 or dt * max(3.0, sizes[-1] / max(1, sizes[-2])) > budget_s:
            break
        layers += 1
    layers, expanded, dt, sizes = best
    return {
        "value": round(expanded / dt, 1),
        "unit": "states/s",
        "cores": 1,
        "host_cores": host["nproc"],
        "cpu_model": host["cpu_model"],
        "kind": "oracle",
        "sample": f"first {layers} layers of the same workload ({expanded} states expanded, {sum(sizes)} "
                  f"states in its hash set, {dt:.1f} s); 1 of {host['nproc']} cores, single-threaded "
                  + ("C hash-set BFS" if use_c else "Python set BFS (the C oracle packs 4 bits per entry)"),
    }


def agg_kstats(results):
    agg = {}
    for r in results:
        for name, k in r.kstats.items():
            a = agg.setdefault(name, {"launches": 0, "total_ms": 0.0, "alg_bytes": 0.0, "items": 0.0})
            for f in a:
                a[f] += k[f]
    return agg


def growth_leg(name: str, steps: int, warmup: int) -> dict:
    """K timed growths of one workload on a reusable engine (its stream and
    device buffers warm): states/s, per-kernel HIP-event times, and the
    roofline of the dominant kernel."""
    import torch

    from paper_2509_19162_amd import api
    from paper_2509_19162_amd import inputs as I

    wl = WORKLOADS[name]
    n = wl["n"]
    gens = I.family(wl["family"], n)
    stream = torch.cuda.Stream()
    eng = api.Engine(stream=stream)
    bitmask = wl.get("bitmask", False)
    run_kw = dict(max_layers=512, keep_all_layers=wl["keep_all"], max_frontier=wl["max_frontier"],
                  bitmask=bitmask)
    if wl.get("binary_start"):
        run_kw.update(start=I.binary_central_state(n), max_layers=4096)
    for _ in range(warmup):
        eng.run(n, gens, **run_kw)
    torch.cuda.synchronize()
    api.memory_stats(reset_peak=True)
    t0 = time.perf_counter()
    results = [eng.run(n, gens, profile=not bitmask, **run_kw) for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mem = api.memory_stats()
    sizes = results[0].sizes
    for r in results[1:]:
        assert r.sizes == sizes, "growth differs between steps"
    if wl.get("binary_start"):
        assert sum(sizes) == math.comb(n, n // 2), "layer sizes do not sum to the orbit C(n, n/2)"
    elif wl["family"] in ("pancake", "coxeter") and wl["max_frontier"] is None:
        assert sum(sizes) == math.factorial(n), "layer sizes do not sum to n!"
    expanded = results[0].states_expanded
    elapsed = t1 - t0
    out = {
        "value": round(expanded * steps / elapsed, 1),
        "ms_per_step": round(1000.0 * elapsed / steps, 3),
        "steps": steps,
        "n": n, "generators": len(gens), "layers": len(sizes), "states": sum(sizes),
        "states_expanded_per_step": expanded, "candidates_per_step": results[0].candidates,
        "sizes": sizes, "desc": wl["desc"], "bitmask": bitmask,
        # the most device memory the library's buffers held during the
        # timed growths (layers, candidates, pipeline scratch)
        "device_memory": {"peak_held_bytes": mem["peak_held_bytes"], "arena_bytes": mem["arena_bytes"]},
    }
    out["layers_per_s"] = round(len(sizes) * steps / elapsed, 1)
    agg = agg_kstats(results)
    if agg and wl.get("on_chip"):
        # 40,320 states: every array fits in L2 and LDS, the run is bound by
        # launches and latency, and no HBM fraction means anything
        out["roofline"] = {"bound": "n/a (on-chip)", "achieved": None, "peak": None, "unit": None, "frac": None,
                           "traffic": None}
        out["kernel_ms_per_step"] = {k: round(v["total_ms"] / steps, 3) for k, v in sorted(agg.items())}
    elif agg:
        dom = max(agg, key=lambda k: agg[k]["total_ms"])
        d = agg[dom]
        achieved = d["alg_bytes"] / (d["total_ms"] / 1000.0) / 1e9
        out["roofline"] = {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(dom, name),
            "alg_bytes_per_launch": round(d["alg_bytes"] / d["launches"]),
            "avg_launch_ms": round(d["total_ms"] / d["launches"], 4),
            "launches": int(d["launches"]),
        }
        out["kernel_ms_per_step"] = {k: round(v["total_ms"] / steps, 3) for k, v in sorted(agg.items())}
        # bytes the kernels move by their own count (every sort pass
        # included), and the method's floor: per expanded layer d,
        # 8 [F + 2C + |L_d| + |L_{d-1}| + N] (frontier read, candidates
        # written and read once, both reference layers read, new layer
        # written)
        kern = sum(v["alg_bytes"] for v in agg.values()) / steps
        floor = 0
        k = len(gens)
        for d in range(len(sizes) - 1 if results[0].status == 1 else len(sizes)):
            F = sizes[d]
            prev = sizes[d - 1] if d > 0 else 0
            nxt = sizes[d + 1] if d + 1 < len(sizes) else 0
            floor += 8 * (F + 2 * k * F + F + prev + nxt)
        step_s = elapsed / steps
        out["pipeline"] = {"kernel_bytes_per_step": round(kern),
                           "kernel_gbs_over_wall": round(kern / step_s / 1e9, 1),
                           "floor_bytes_per_step": floor,
                           "floor_gbs_over_wall": round(floor / step_s / 1e9, 1),
                           "floor_frac_of_peak": round(floor / step_s / 1e9 / HBM_PEAK_GBS, 4)}
    if n <= 10 and not bitmask:
        # the same job as one workgroup-resident launch (a replayed hipGraph)
        geng = api.Engine(stream=stream)
        for _ in range(3):
            geng.run(n, gens, max_layers=512, small_job=True)
        torch.cuda.synchronize()
        reps = max(20, steps)
        tg = time.perf_counter()
        for _ in range(reps):
            rg = geng.run(n, gens, max_layers=512, small_job=True)
        torch.cuda.synchronize()
        g_ms = 1000.0 * (time.perf_counter() - tg) / reps
        assert rg.sizes == sizes, "small-job engine differs from the sort path"
        out["graph_variant"] = {"ms_per_run": round(g_ms, 3), "device_ms": round(rg.device_ms, 3),
                                "speedup_vs_plain": round(out["ms_per_step"] / g_ms, 1)}
        geng.close()
    eng.close()
    return out


def _oracle_job(job):
    from oracle import native

    n, gens = job
    t = time.perf_counter()
    native.growth(n, gens)
    return time.perf_counter() - t


def batch_leg(steps: int, warmup: int, tune: bool, n_jobs: int, cpu_budget: float, host: dict,
              seq_jobs: int = 4096) -> dict:
    """4096 independent jobs (n ~ U{7..10}, 2-4 uniform random permutations
    plus their inverses, full growth each) in one cg_growth_batch call,
    against the same jobs run one at a time through a reusable engine on the
    same GPU; the oracle on all host cores."""
    import torch

    from paper_2509_19162_amd import api
    from paper_2509_19162_amd import inputs as I

    jobs = I.batch_jobs(4096)[:n_jobs]
    # warm-up on the same batch: the library's device cache then holds every
    # buffer the timed runs need
    for _ in range(max(1, warmup)):
        api.growth_batch(jobs, max_layers=512, tune=tune)
    torch.cuda.synchronize()
    log("batch warm-up done")
    times, res = [], None
    for _ in range(steps):
        t = time.perf_counter()
        res = api.growth_batch(jobs, max_layers=512, tune=tune)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    elapsed = sum(times)
    states = sum(r.states_expanded for r in res)
    value = len(jobs) * steps / elapsed
    info = api.batch_info()
    # the one small-job launch's HIP-event time (every such job reports it)
    launch_ms = max((r.device_ms for r in res), default=0.0)
    log(f"batch: {value:.0f} jobs/s")
    # the plain one-job-at-a-time GPU path on the same jobs
    seq_line = None
    seq = jobs[:seq_jobs]
    if seq:
        eng = api.Engine()
        for n, gens in seq[:32]:
            eng.run(n, gens, max_layers=512)
        t = time.perf_counter()
        seq_states = 0
        for n, gens in seq:
            seq_states += eng.run(n, gens, max_layers=512).states_expanded
        seq_dt = time.perf_counter() - t
        eng.close()
        seq_jobs_s = len(seq) / seq_dt
        log(f"batch: sequential plain runs {seq_jobs_s:.0f} jobs/s")
        seq_line = {"jobs_per_s": round(seq_jobs_s, 2), "jobs": len(seq), "states_per_s": round(seq_states / seq_dt, 1),
                    "speedup_of_batch": round(value / seq_jobs_s, 1)}
    out = {
        "value": round(value, 2), "unit": "jobs/s", "ms_per_step": round(1000 * elapsed / steps, 2),
        "steps": steps, "jobs": len(jobs), "states_per_s": round(states * steps / elapsed, 1),
        "workload": f"{len(jobs)} jobs, n ~ U{{7..10}}, 2-4 uniform random permutations plus inverses, "
                    "full growth each (seed 19162)",
        "autotuned": bool(tune),
        "tuning": {"classes": info["tuned_classes"], "heavy_split": info["heavy_split"],
                   "file_entries": info["tune_file_entries"]} if tune else None,
        "graph": {"builds": int(info["graph_builds"]), "launches": int(info["graph_launches"]),
                  "replays": int(info["graph_launches"] - info["graph_builds"])},
        "small_job_launch_ms": round(launch_ms, 2),
        "host_ms_per_step": round(1000 * elapsed / steps - launch_ms, 2),
        "sequential_plain": seq_line,
        "cpu_baseline": None,
    }
    if cpu_budget > 0:
        # the oracle over the jobs on every host core (one job per worker),
        # stopped at the budget: all-core wall rate and the 1-core rate from
        # the summed per-job times
        from concurrent.futures import ProcessPoolExecutor, FIRST_COMPLETED, wait

        from oracle import native

        native.build(force=False)
        workers = max(1, host["nproc"])
        done, busy = [], set()
        t0 = time.perf_counter()
        it = iter(jobs)
        with ProcessPoolExecutor(max_workers=workers) as ex:
            for _ in range(2 * workers):
                j = next(it, None)
                if j is not None:
                    busy.add(ex.submit(_oracle_job, j))
            while busy:
                fin, busy = wait(busy, return_when=FIRST_COMPLETED)
                for f in fin:
                    done.append(f.result())
                if time.perf_counter() - t0 < cpu_budget:
                    for _ in range(len(fin)):
                        j = next(it, None)
                        if j is not None:
                            busy.add(ex.submit(_oracle_job, j))
        wall = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(len(done) / wall, 2), "unit": "jobs/s", "cores": workers,
            "host_cores": host["nproc"], "cpu_model": host["cpu_model"], "kind": "oracle",
            "one_core_jobs_per_s": round(len(done) / sum(done), 2),
            "sample": f"first {len(done)} of the {len(jobs)} jobs on {workers} worker processes "
                      f"(C hash-set BFS, one job per worker), {wall:.1f} s wall, {sum(done):.1f} s summed "
                      f"over jobs",
        }
    return out


def _replay_worker(reqs, conn):
    from oracle import native

    for n, fam, g in reqs:
        sizes, _, _ = native.growth(n, g, max_layers=512)
        conn.send(sum(sizes))
    conn.send(None)


def _oracle_replay(reqs, budget_s: float):
    """The oracle replays the requests in trace order in a child process,
    which is stopped at the budget (one large request alone can outlast
    it): returns (requests finished, states, seconds)."""
    import multiprocessing as mp

    from oracle import native

    native.build(force=False)
    ctx = mp.get_context("fork")
    a, b = ctx.Pipe(duplex=False)
    t0 = time.perf_counter()
    p = ctx.Process(target=_replay_worker, args=(reqs, b), daemon=True)
    p.start()
    b.close()
    m = st = 0
    while True:
        left = budget_s - (time.perf_counter() - t0)
        if left <= 0 or not a.poll(left):
            break
        try:
            v = a.recv()
        except EOFError:
            break
        if v is None:
            break
        m += 1
        st += v
    dt = time.perf_counter() - t0
    if p.is_alive():
        p.terminate()
    p.join(10)
    return m, st, dt


def serving_leg(n_requests: int, nmax: int, ratios, cpu_budget: float, host: dict, plain: bool = True) -> dict:
    """Poisson arrivals of growth requests (n ~ U{6..nmax}; family uniform
    over all transpositions, star, prefix reversals, LRX, 2-4 random
    involutions) at rates relative to the measured capacity; p50/p99
    latency from submit to completion, served states/s, and the same trace
    on the plain one-at-a-time GPU path and on the oracle (time-capped)."""
    import threading

    import numpy as np

    from paper_2509_19162_amd import api
    from paper_2509_19162_amd import inputs as I

    R = n_requests
    reqs = [I.serving_request(i, n_lo=6, n_hi=nmax) for i in range(R)]
    q = api.GrowthQueue(max_active=256)
    # warm-up: one request of every (n, family) shape of the trace
    seen, warm = set(), []
    for n, fam, g in reqs:
        if (n, fam) not in seen:
            seen.add((n, fam))
            warm.append((n, g))
    for t in [q.submit(n, g, max_layers=512) for n, g in warm]:
        q.wait(t)
    log(f"serving: warm-up on {len(warm)} request shapes done")
    plain_line = None
    if plain:
        eng = api.Engine()
        t0 = time.perf_counter()
        plain_states = 0
        for i, (n, fam, g) in enumerate(reqs):
            # the engine the queue picks for the request (from n = 12 the
            # bitmask engine)
            plain_states += eng.run(n, g, max_layers=512, bitmask=n >= 12).states_expanded
            if (i + 1) % 50 == 0:
                log(f"serving: plain one-at-a-time {i + 1}/{R} requests, {time.perf_counter() - t0:.1f} s")
        plain_dt = time.perf_counter() - t0
        eng.close()
        plain_line = {"req_per_s": round(R / plain_dt, 2), "states_per_s": round(plain_states / plain_dt, 1)}
        log(f"serving: plain one-at-a-time {R / plain_dt:.1f} req/s")
    # capacity: every request submitted at once
    t0 = time.perf_counter()
    ts = [q.submit(n, g, max_layers=512) for n, fam, g in reqs]
    outs = []
    for i, t in enumerate(ts):
        outs.append(q.wait(t))
        if (i + 1) % 100 == 0:
            log(f"serving: capacity run {i + 1}/{R} requests done, {time.perf_counter() - t0:.1f} s")
    cap_dt = time.perf_counter() - t0
    mu = R / cap_dt
    log(f"serving: capacity {mu:.1f} req/s")
    points = {}
    rng = np.random.default_rng(I.SEED)
    for ratio in ratios:
        lam = ratio * mu
        gaps = rng.exponential(1.0 / lam, size=R)
        tickets = [None] * R

        def producer():
            nxt = time.perf_counter()
            for i, (n, fam, g) in enumerate(reqs):
                nxt += gaps[i]
                d = nxt - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = q.submit(n, g, max_layers=512)

        t0 = time.perf_counter()
        th = threading.Thread(target=producer)
        th.start()
        while th.is_alive():
            th.join(timeout=30.0)
            if th.is_alive():
                log(f"serving: {ratio} x capacity: {sum(t is not None for t in tickets)}/{R} submitted, "
                    f"{time.perf_counter() - t0:.0f} s")
        out = [q.wait(t) for t in tickets]
        dt = time.perf_counter() - t0
        for a, b in zip(out, outs):
            assert a.sizes == b.sizes, "a request's growth differs between runs"
        lat = np.array([r.t_done - r.t_submit for r in out]) * 1000.0
        wait_ = np.array([r.t_admit - r.t_submit for r in out]) * 1000.0
        states = sum(r.states_expanded for r in out)
        points[str(ratio)] = {"lambda_req_s": round(lam, 2), "p50_ms": round(float(np.percentile(lat, 50)), 2),
                              "p99_ms": round(float(np.percentile(lat, 99)), 2),
                              "admit_wait_p50_ms": round(float(np.percentile(wait_, 50)), 2),
                              "states_per_s": round(states / dt, 1), "wall_s": round(dt, 2)}
        log(f"serving: {ratio} x capacity: p50 {points[str(ratio)]['p50_ms']} ms, "
            f"p99 {points[str(ratio)]['p99_ms']} ms")
    q.close()
    cpu = None
    if cpu_budget > 0:
        # the oracle holds every visited state in host memory: requests from
        # n = 11 on take it minutes to hours each, so it replays the n <= 10
        # requests of the trace, in order
        small = [r for r in reqs if r[0] <= 10]
        m, st, dt = _oracle_replay(small, cpu_budget)
        cpu = {"value": round(m / dt, 3), "unit": "req/s", "cores": 1, "host_cores": host["nproc"],
               "cpu_model": host["cpu_model"], "kind": "oracle", "states_per_s": round(st / dt, 1),
               "sample": f"sequential replay of the trace's {len(small)} requests with n <= 10, in order: {m} "
                         f"finished within {dt:.1f} s (the replay is stopped there), 1 of {host['nproc']} "
                         f"cores"}
    return {
        "requests": R, "n_range": [6, nmax],
        "workload": f"Poisson stream of {R} growth requests per rate, n ~ U{{6..{nmax}}}, families: all "
                    "transpositions, star, prefix reversals, LRX, 2-4 random involutions (seed 19162)",
        "capacity_req_per_s": round(mu, 2), "capacity_wall_s": round(cap_dt, 2),
        "plain_one_at_a_time": plain_line, "rates": points, "cpu_baseline": cpu,
    }


def _growth_line(name: str, leg: dict, steps: int, warmup: int, cpu) -> dict:
    n = leg["n"]
    return {
        "metric": "states expanded/sec",
        "value": leg["value"],
        "unit": "states/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # candidates of n <= 12 are sorted and deduplicated as 32-bit ranks
        "dtype": "u32" if n <= 12 else "u64",
        "data": "synthetic",
        "config": {"workload": leg["desc"], "n": n, "generators": leg["generators"], "layers": leg["layers"],
                   "states": leg["states"], "candidates_per_step": leg["candidates_per_step"]},
        "roofline": leg.get("roofline"),
        "cpu_baseline": cpu,
        "kernel_ms_per_step": leg.get("kernel_ms_per_step"),
        "pipeline": leg.get("pipeline"),
        "device_memory": leg.get("device_memory"),
        "layers_per_s": leg.get("layers_per_s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="default",
                    choices=["default"] + sorted(WORKLOADS) + ["batch4096", "serving"])
    ap.add_argument("--batch-jobs", type=int, default=4096)
    ap.add_argument("--seq-jobs", type=int, default=4096,
                    help="batch: jobs of the one-at-a-time comparison (0 = none)")
    ap.add_argument("--tune", action="store_true", help="batch: let the autotuner pick engines and launch shapes")
    ap.add_argument("--requests", type=int, default=500)
    ap.add_argument("--serving-nmax", type=int, default=13)
    ap.add_argument("--ratios", type=float, nargs="+", default=[0.25, 0.5, 0.75, 0.9, 1.0, 1.2])
    ap.add_argument("--no-plain", action="store_true", help="serving: skip the one-at-a-time comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-extras", action="store_true", help="default run: the headline only")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run the plain copy kernel over BYTES bytes (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this build has no multi-GPU path "
              "(its sharding is a design, not code)", file=sys.stderr)
        sys.exit(2)

    host = host_info()  # before the GPU is touched (it runs lscpu)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cpu_budget = 0.0 if args.no_cpu_baseline else args.cpu_budget
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy, max(1, args.steps))
    if args.workload == "batch4096":
        leg = batch_leg(args.steps, args.warmup, args.tune, args.batch_jobs, cpu_budget, host, args.seq_jobs)
        line = {"metric": "batched jobs/sec", "value": leg["value"], "unit": "jobs/s", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": leg["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                "data": "synthetic", "config": {"workload": leg["workload"], "jobs": leg["jobs"]}}
        line.update({k: v for k, v in leg.items() if k not in ("value", "ms_per_step", "workload", "jobs")})
        print(json.dumps(line), flush=True)
        return
    if args.workload == "serving":
        leg = serving_leg(args.requests, args.serving_nmax, args.ratios, cpu_budget, host, plain=not args.no_plain)
        ref = leg["rates"].get("0.9") or list(leg["rates"].values())[-1]
        line = {"metric": "p99 job latency", "value": ref["p99_ms"], "unit": "ms", "n_gpus": 1,
                "steps": len(args.ratios), "warmup": 1, "ms_per_step": round(1000 * leg["capacity_wall_s"], 2),
                "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                "data": "synthetic", "config": {"workload": leg["workload"] + "; value = p99 at 0.9 x capacity",
                                                "requests": leg["requests"]}}
        line.update({k: v for k, v in leg.items() if k not in ("workload", "requests")})
        print(json.dumps(line), flush=True)
        return
    if args.workload != "default":
        leg = growth_leg(args.workload, args.steps, args.warmup)
        cpu = cpu_baseline(WORKLOADS[args.workload], cpu_budget, host) if cpu_budget > 0 else None
        line = _growth_line(args.workload, leg, args.steps, args.warmup, cpu)
        if args.workload == "pancake12":
            line["paper_context"] = {"s12_pancake_full_growth_s": PAPER_PANCAKE12_SECONDS,
                                     "hardware": "Kaggle CPU (another machine; context only)"}
        if leg.get("graph_variant"):
            line["graph_variant"] = leg["graph_variant"]
        if leg["bitmask"]:
            line["engine"] = "bitmask (3 bits per state; VALU and atomic bound, no HBM roofline)"
        print(json.dumps(line), flush=True)
        return

    # ---- default: the headline (S_16 LRX to 2^31) and the other legs ----
    log(f"S_16 LRX: {args.warmup} warm-up + {args.steps} timed growths")
    head = growth_leg("lrx16", args.steps, args.warmup)
    log(f"S_16 LRX: {head['value']:.3e} states/s, {head['ms_per_step']:.1f} ms per growth")
    cpu = cpu_baseline(WORKLOADS["lrx16"], cpu_budget, host) if cpu_budget > 0 else None
    line = _growth_line("lrx16", head, args.steps, args.warmup, cpu)
    line["config"]["layer_sizes"] = head["sizes"]
    line["host"] = host
    if not args.no_extras:
        torch.cuda.synchronize()
        from paper_2509_19162_amd import api

        api.release_cached_memory()
        torch.cuda.empty_cache()
        line["copy_ceiling"] = copy_ceiling()
        log(f"copy ceiling {line['copy_ceiling']['gbs']} GB/s")
        p12 = growth_leg("pancake12", 5, 1)
        log(f"S_12 pancake: {p12['value']:.3e} states/s")
        line["pancake12"] = {k: p12[k] for k in ("value", "ms_per_step", "steps", "states", "layers")}
        line["pancake12"].update({"unit": "states/s", "workload": p12["desc"], "roofline": p12.get("roofline"),
                                  "kernel_ms_per_step": p12.get("kernel_ms_per_step"),
                                  "pipeline": p12.get("pipeline"), "device_memory": p12.get("device_memory"),
                                  "paper_context": {"s12_pancake_full_growth_s": PAPER_PANCAKE12_SECONDS,
                                                    "hardware": "Kaggle CPU (another machine; context only)"}})
        api.release_cached_memory()
        line["batch4096"] = batch_leg(3, 1, True, 4096, min(cpu_budget, 10.0), host)
        api.release_cached_memory()
        sv = serving_leg(DEFAULT_RUN_REQUESTS, 13, [0.9], min(cpu_budget, 10.0), host, plain=False)
        sv["note"] = (f"one rate point (0.9 x capacity) with {DEFAULT_RUN_REQUESTS} requests, to fit the "
                      "default run's time; the full sweep (500 requests per rate) is --workload serving")
        line["serving"] = sv
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
