"""Benchmark of the multispin Kob-Andersen sweep on one MI355X.

Workload (default "cubic128"): 3D cubic lattice L=128 with periodic boundaries, z=6, m=3,
256 replicas (4 uint64 words per site), 10^4 sweeps per job, overlap and persistence
observed on a 38-point log-spaced grid (0 and the distinct floor(10^(k/10)) <= 10^4).  One
step is one whole job: initial state (uniform K-subset per replica) + all sweeps + all
observations, with rho cycling through 0.80, 0.85, 0.88.  Inputs are synthetic (the
dynamics needs no data); the lattice and all state are resident on the GPU during the
timed region.

Metric: site-replica move attempts per second = N * R * sweeps * steps / wall time (one
sweep attempts every edge once per replica, N attempts per replica in the paper's time
unit).  Also reported: the rate without the observations, and the roofline of the dominant
kernel (the global-memory class pass).  Its average launch time is the HIP-event stream time
of the timed jobs' sweep loops, less the same number of observations timed on their own,
divided by the number of class-pass launches; so it includes the short gaps between
back-to-back launches.  With --plane-streams a sim with two or more word planes runs them as
separate launches on two streams that overlap, and this figure is each launch's share of the
wall time (the launches' own durations overlap and are longer).  Last, the oracle's rate on
a bounded sample on this host's cores.

After the headline (default workload only): the same pass on 3D L=256 x 256 replicas, whose
state exceeds the 256 MiB Infinity Cache, so that its words run one at a time ("hbm_regime");
then the batched form (256 uneven instances) and the continuous-batching server (a Poisson
trace, --jobs jobs at --rate per second and at half the measured capacity), measured against
one job at a time ("batch256", "serve").  --no-extras skips them.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload cubic128]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "cubic128": dict(kind="lattice", d=3, L=128, m=3, rhos=[0.80, 0.85, 0.88], R=256, sweeps=10_000,
                     desc="3D cubic lattice L=128 periodic, z=6, m=3, rho in {0.80,0.85,0.88}, 256 replicas "
                          "(4 uint64 words/site), 10^4 sweeps, overlap+persistence on a 38-point log grid"),
    "square64": dict(kind="lattice", d=2, L=64, m=2, rhos=[0.70], R=64, sweeps=1000, obs_every=10,
                     desc="2D square lattice L=64 periodic, z=4, m=2, rho=0.70, 64 replicas, 1000 sweeps, "
                          "observables every 10 sweeps"),
    "rrg20": dict(kind="rrg", N=1 << 20, z=4, m=2, rhos=[0.50, 0.55, 0.60, 0.65, 0.70, 0.75], R=64,
                  sweeps=10_000, graph_seed=1,
                  desc="random regular graph N=2^20, z=4, m=2, rho 0.50-0.75, 64 replicas, 10^4 sweeps"),
    "cubic256": dict(kind="lattice", d=3, L=256, m=3, rhos=[0.85], R=256, sweeps=200,
                     desc="3D cubic lattice L=256 periodic, z=6, m=3, rho=0.85, 256 replicas, 200 sweeps "
                          "(state beyond the 256 MiB Infinity Cache)"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def class_pass_bytes(w, N, W, with_moved_ever=False):
    """Algorithmic HBM bytes of one global class pass over all words, per-pass model: every
    site's words are read once as endpoint or neighbour (8 B) and the endpoints (half of the
    sites) are written (8 B): 12 B per site-word.  with_moved_ever adds a read of every
    endpoint's moved-ever word (8 B per endpoint, 16 B per site-word in all); the kernel reads
    it only where an exchange happens, and writes it only where it gains a bit."""
    if w["kind"] == "lattice":
        b = N * W * 8 + (N // 2) * W * 8
        if with_moved_ever:
            b += (N // 2) * W * 8
        return b
    return None


def measured_traffic(kernel_sources, counters_file, key="traffic_bytes_per_launch"):
    """A figure from a committed rocprofv3 counter summary (by default the HBM bytes per
    launch), or None when the kernel sources no longer hash to the ones the counters were
    taken with."""
    import hashlib
    try:
        kv = {}
        with open(counters_file) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        h = hashlib.sha256()
        for path in kernel_sources:
            with open(path, "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != kv.get("source_sha256"):
            return None
        return float(kv[key])
    except (OSError, KeyError, ValueError):
        return None


def obs_grid(w):
    """Observation times of one job; the last one is the job's final sweep, so that a job
    always runs exactly w["sweeps"] sweeps."""
    from paper_1710_05155_amd import workloads
    if "obs_every" in w:
        grid = list(range(0, w["sweeps"] + 1, w["obs_every"]))
    else:
        grid = workloads.log_time_grid(w["sweeps"])
    if grid[-1] != w["sweeps"]:
        grid.append(w["sweeps"])
    return grid


def cpu_baseline(w, seconds_target=15.0):
    """The oracle (plain scalar C, one replica per thread) on a bounded sample."""
    from oracle import oracle as o
    if w["kind"] == "lattice":
        g = o.lattice(w["d"], w["L"])
    else:
        g = o.rrg(w["N"], w["z"], w["graph_seed"])
    threads = o.threads()
    rho = w["rhos"][0]
    K = o.k_from_rho(g.N, rho)
    reps = list(range(threads))
    s = o.Sim(g, w["m"], K, 1, reps)
    t0 = time.perf_counter()
    s.sweep(1)
    one = time.perf_counter() - t0
    n = max(1, int(seconds_target / max(one, 1e-6)) - 1)
    t0 = time.perf_counter()
    s.sweep(n)
    dt = time.perf_counter() - t0
    total_sweeps = n + 1
    rate = g.N * len(reps) * total_sweeps / (dt + one)
    return {"value": rate, "unit": "site-replica move attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(reps)} replicas x {total_sweeps} sweeps of the same "
                      f"{'lattice' if w['kind'] == 'lattice' else 'graph'} at rho={rho} "
                      f"(one replica per thread), sweeps only"}


def graph_bytes_model(adj, eu, ev, ec, C, z, W):
    """Algorithmic bytes of one sweep over a general graph, summed over its class passes:
    per class, the distinct sites read (endpoints and their neighbours, at most N) x 8 B per
    word, the class records (16 B per edge), the neighbour lists (2(z-1) x 4 B per edge),
    the endpoint words written (2 x 8 B per edge and word) and their moved-ever words read
    (2 x 8 B per edge and word; as for lattices, the rare moved-ever stores are left out)."""
    import numpy as np
    N = adj.shape[0]
    total = 0
    for c in range(C):
        sel = ec == c
        Ec = int(sel.sum())
        touched = np.zeros(N, dtype=bool)
        touched[eu[sel]] = True
        touched[ev[sel]] = True
        touched[adj[eu[sel]].ravel()] = True
        touched[adj[ev[sel]].ravel()] = True
        total += int(touched.sum()) * 8 * W + Ec * (16 + 2 * 4 * (z - 1) + 2 * 8 * W + 2 * 8 * W)
    return total


def hbm_regime_measure(stream, jobs=2):
    """3D L=256 x 256 replicas, rho = 0.85, 200 sweeps per job with the 38-point log grid cut at
    200 (state 3 x 512 MiB, beyond the 256 MiB Infinity Cache; the library runs its four words
    one at a time, one launch per word and class step): rate and the class pass's roofline
    under the 12 B model, per launch, timed like the headline (HIP events around each job's
    sweep loop, less the observations timed on their own)."""
    import torch
    from paper_1710_05155_amd import ka
    w = WORKLOADS["cubic256"]
    g = ka.ka_graph_lattice(w["d"], w["L"])
    grid = obs_grid(w)
    run_ms = []
    launches = 0
    for k in range(jobs + 1):
        sim = ka.ka_init(g, w["m"], w["rhos"][0], 1, w["R"], stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dens, _, _ = ka.ka_run(sim, grid)
        e1.record(stream)
        torch.cuda.synchronize()
        assert (dens == sim.K).all()
        if k > 0:    # the first job is a warm-up
            run_ms.append(e0.elapsed_time(e1))
            launches += ka.ka_timing(sim)[0]
        sim.free()
    sim = ka.ka_init(g, w["m"], w["rhos"][0], 1, w["R"], stream=stream)
    torch.cuda.synchronize()
    oa, ob = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    oa.record(stream)
    ka.ka_run(sim, [0] * len(grid))
    ob.record(stream)
    torch.cuda.synchronize()
    obs_ms = oa.elapsed_time(ob)
    sim.free()
    N, W = g.N, w["R"] // 64
    sweep_ms = sum(run_ms) - jobs * obs_ms
    avg_s = sweep_ms / launches / 1000.0
    # the model is per class step over all words; a step is one launch per group of word
    # planes (the words of this lattice run one group at a time), so scale to one launch
    per_launch = w["sweeps"] * g.C * jobs / launches
    B = class_pass_bytes(w, N, W) * per_launch
    B16 = class_pass_bytes(w, N, W, with_moved_ever=True) * per_launch
    srcs = [os.path.join(ROOT, "paper_1710_05155_amd", "csrc", f) for f in ("ka_device.h", "ka_pass.hip", "ka_host.cpp")]
    cfile = os.path.join(ROOT, "profiles", "k_pass_lattice_cubic256.counters.txt")
    traffic = measured_traffic(srcs, cfile)
    return {"workload": w["desc"], "value": N * w["R"] * w["sweeps"] * jobs / (sum(run_ms) / 1000.0),
            "unit": "site-replica move attempts/s", "jobs": jobs,
            "roofline": {"bound": "hbm", "achieved": B / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": B / avg_s / 1e9 / HBM_PEAK_GBS, "kernel": "k_pass_lattice",
                         "avg_launch_us": avg_s * 1e6, "bytes_per_launch": B,
                         "frac_with_moved_ever_reads": B16 / avg_s / 1e9 / HBM_PEAK_GBS,
                         "traffic": traffic,
                         "traffic_source": "profiles/k_pass_lattice_cubic256.counters.txt" if traffic else None}}


def batch_measure(steps, warmup, sweeps=1000, serial=True, solo_bytes=32 << 20):
    """256 uneven instances advanced together by one batch (timed `steps` times after
    `warmup` untimed runs), against the same jobs run one at a time with the single-instance
    path (once).  Members whose n and f take at least solo_bytes (the 3D L=128 ones) run one
    at a time inside the batch through their own pass kernels (KA_BOPT_SOLO_BYTES; 0: every
    member in the step kernel).  Returns a dict."""
    import torch
    from paper_1710_05155_amd import ka, workloads

    man = workloads.batch_manifest(256, sweeps=sweeps)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    graphs, bytes_per_sweep = {}, {}
    for inst in man:
        key = (inst["kind"], inst.get("d"), inst.get("L"), inst.get("N"), inst.get("z"), inst.get("graph_seed"))
        inst["key"] = key
        if key in graphs:
            continue
        if inst["kind"] == "lattice":
            graphs[key] = ka.ka_graph_lattice(inst["d"], inst["L"])
            bytes_per_sweep[key] = 12 * inst["N"] * (inst["R"] // 64) * 4 * inst["d"]
        else:
            g = ka.ka_graph_rrg(inst["N"], inst["z"], inst["graph_seed"])
            graphs[key] = g
            adj, eu, ev, ec = ka.ka_graph_export(g)
            bytes_per_sweep[key] = graph_bytes_model(adj, eu, ev, ec, g.C, g.z, inst["R"] // 64)
    log(f"batch: built {len(graphs)} graphs in {time.perf_counter() - t0:.1f} s")
    n_solo = sum(1 for i in man if solo_bytes > 0 and 2 * graphs[i["key"]].N * (i["R"] // 64) * 8 >= solo_bytes)
    attempts = sum(graphs[i["key"]].N * i["R"] * i["sweeps"] for i in man)
    model_bytes = sum(bytes_per_sweep[i["key"]] * i["sweeps"] for i in man)

    shape = {}
    # The members' initial states are built on a few streams of their own, so that the
    # one-workgroup-per-replica-pair init kernels of different members run side by side;
    # ka_batch_add orders each member's init before the batch's steps.
    init_streams = [torch.cuda.Stream() for _ in range(4)]

    def batched(timed_kernel):
        sims = [ka.ka_init(graphs[i["key"]], i["m"], i["rho"], i["seed"], i["R"],
                           stream=init_streams[k % len(init_streams)]) for k, i in enumerate(man)]
        b = ka.ka_batch_create(len(sims), stream=stream)
        ka.ka_batch_set_option(b, ka.KA_BOPT_SOLO_BYTES, solo_bytes)
        if shape:
            ka.ka_batch_set_option(b, ka.KA_BOPT_BLOCK, shape["block"])
        for s, i in zip(sims, man):
            ka.ka_batch_add(b, s, i["sweeps"])
        steps = ka.ka_batch_steps_left(b)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ka.ka_batch_run(b, steps)
        e1.record(stream)
        _, _, block, _ = ka.ka_batch_info(b)
        ka.ka_batch_wait_all(b)
        for s in sims:
            _, dens, _, _ = ka.ka_observe(s)
            assert (dens == s.K).all(), "particle number not conserved"
        b.free()
        for s in sims:
            s.free()
        shape.update(block=block)
        if timed_kernel is not None:
            timed_kernel.append((e0.elapsed_time(e1), steps))
        return steps

    def one_at_a_time():
        for i in man:
            s = ka.ka_init(graphs[i["key"]], i["m"], i["rho"], i["seed"], i["R"], stream=stream)
            ka.ka_sweep(s, i["sweeps"])
            _, dens, _, _ = ka.ka_observe(s)
            assert (dens == s.K).all()
            s.free()

    for k in range(warmup):
        t = time.perf_counter()
        batched(None)
        log(f"batch warmup {k}: {time.perf_counter() - t:.2f} s, tuned shape {shape}")
    kern = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(steps):
        n_steps = batched(kern)
        log(f"batch step {k}: step kernels {n_steps}, {kern[-1][0]:.1f} ms of them")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    ms = sum(k[0] for k in kern)
    launches = sum(k[1] for k in kern)
    achieved = model_bytes * steps / (ms / 1000.0) / 1e9
    out = {"value": attempts * steps / wall, "unit": "site-replica move attempts/s",
           "ms_per_batch": wall * 1000.0 / steps, "instances": len(man), "sweeps_each": sweeps,
           "sites_total": int(sum(graphs[i["key"]].N for i in man)), "launch_shape": dict(shape),
           "solo_bytes": solo_bytes, "solo_members": n_solo,
           # one batch step: the step kernel over the batched members and one launch of the
           # running solo member's pass kernel, whichever are present
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "k_batch_step and the solo members' k_pass_lattice",
                        "steps_per_batch": launches // steps, "avg_step_us": ms * 1000.0 / launches,
                        "bytes_per_step": model_bytes / (launches / steps), "kernel_ms_per_batch": ms / steps,
                        "byte_model": "12 B per site-word per lattice class pass; graph members as bench.graph_bytes_model"}}
    if serial:
        log("batch: one-at-a-time baseline ...")
        torch.cuda.synchronize()
        t = time.perf_counter()
        one_at_a_time()
        torch.cuda.synchronize()
        ws = time.perf_counter() - t
        out["one_at_a_time"] = {"value": attempts / ws, "ms": ws * 1000.0}
        out["speedup_vs_one_at_a_time"] = ws / (wall / steps)
    return out


def run_batch_workload(args):
    """The batched workload as the bench line."""
    r = batch_measure(args.steps, args.warmup, sweeps=args.sweeps or 1000, serial=not args.no_serial,
                      solo_bytes=args.solo_bytes)
    result = {
        "metric": "site-replica move attempts/s (1 GPU)",
        "value": r["value"],
        "unit": "site-replica move attempts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_batch"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "256 uneven instances (2D L 32-512, 3D L 16-128, RRG N 2^12-2^18 z 3-5, "
                               f"m 1..z-1, rho U[0.5,0.9], 64 replicas), {r['sweeps_each']} sweeps each, batched "
                               "step kernel in captured graphs, autotuned launch shape; members whose n and f take "
                               f"at least {r['solo_bytes']} bytes run one at a time through their own pass kernels",
                   "instances": r["instances"], "sites_total": r["sites_total"], "launch_shape": r["launch_shape"],
                   "solo_members": r["solo_members"]},
        "roofline": r["roofline"],
    }
    for k in ("one_at_a_time", "speedup_vs_one_at_a_time"):
        if k in r:
            result[k] = r[k]
    print(json.dumps(result), flush=True)


def serve_measure(n_jobs, rate_per_s, serial=True):
    """Continuous-batching job server on a Poisson trace of n_jobs jobs at the stated rate and
    at half of the measured capacity, each against serial per-job launches.  Returns a dict."""
    import numpy as np
    import torch
    from paper_1710_05155_amd import ka, workloads

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    graphs = {}

    def graph_for(inst):
        # random regular graphs of one (N, z) share one graph (seed 1000 + N + z)
        key = (inst["kind"], inst.get("d"), inst.get("L"), inst.get("N"), inst.get("z"))
        if key not in graphs:
            if inst["kind"] == "lattice":
                graphs[key] = ka.ka_graph_lattice(inst["d"], inst["L"])
            else:
                graphs[key] = ka.ka_graph_rrg(inst["N"], inst["z"], 1000 + inst["N"] + inst["z"])
        return graphs[key]

    def trace(rate):
        jobs = workloads.serving_trace(n_jobs, rate, seed=5)
        for j in jobs:
            j["graph"] = graph_for(j)
            j["obs"] = workloads.log_time_grid(j["sweeps"])
            if j["obs"][-1] != j["sweeps"]:
                j["obs"].append(j["sweeps"])
        return jobs

    base = trace(rate_per_s)
    log(f"serve: built {len(graphs)} graphs in {time.perf_counter() - t0:.1f} s")
    work = [j["graph"].N * j["R"] * j["sweeps"] for j in base]
    mean_work = float(np.mean(work))

    def served(jobs):
        props = torch.cuda.get_device_properties(0)
        budget = int(props.total_memory * 0.8)
        sv = ka.ka_server_create(budget, 256)
        start = time.perf_counter()
        ids = []
        for j in jobs:
            dt = j["arrival_s"] - (time.perf_counter() - start)
            if dt > 0:
                time.sleep(dt)
            ids.append(ka.ka_server_submit(sv, j["graph"], j["m"], j["rho"], j["seed"], j["R"], j["sweeps"],
                                           obs_times=j["obs"]))
            if len(ids) % 500 == 0:
                log(f"serve: {len(ids)}/{len(jobs)} jobs submitted at {time.perf_counter() - start:.1f} s")
        while True:
            done = ka.ka_server_stats(sv)["jobs_done"]
            if done >= len(ids):
                break
            log(f"serve: {done}/{len(ids)} jobs done at {time.perf_counter() - start:.1f} s")
            time.sleep(min(30.0, max(0.05, 0.25 * (time.perf_counter() - start))))
        ka.ka_server_wait_idle(sv)
        end = time.perf_counter()
        lat = []
        for jid, j in zip(ids, jobs):
            r = ka.ka_server_result(sv, jid)
            assert (r["density"] == r["density"][0, 0]).all()
            lat.append(r["latency_s"])
        stats = ka.ka_server_stats(sv)
        sv.free()
        return end - start, np.array(lat), stats

    def serial_run(jobs):
        stream = torch.cuda.Stream()
        start = time.perf_counter()
        lat = []
        for j in jobs:
            dt = j["arrival_s"] - (time.perf_counter() - start)
            if dt > 0:
                time.sleep(dt)
            s = ka.ka_init(j["graph"], j["m"], j["rho"], j["seed"], j["R"], stream=stream)
            ka.ka_run(s, j["obs"])
            s.free()
            lat.append(time.perf_counter() - start - j["arrival_s"])
            if len(lat) % 250 == 0:
                log(f"serve: serial {len(lat)}/{len(jobs)} jobs done at {time.perf_counter() - start:.1f} s")
        return time.perf_counter() - start, np.array(lat)

    def pct(a, q):
        return float(np.percentile(a, q))

    out = {}
    rates = [("stated", rate_per_s)]
    # a warm-up pass at the stated rate measures capacity for the half-load rate
    wall, lat, stats = served(base)
    capacity = stats["attempts"] / wall
    rates.append(("half_capacity", 0.5 * capacity / mean_work))
    log(f"serve: capacity estimate {capacity:.3e} attempts/s -> half-load rate {rates[1][1]:.2f} jobs/s")
    for name, rate in rates:
        jobs = trace(rate)
        total = float(sum(j["graph"].N * j["R"] * j["sweeps"] for j in jobs))
        wall, lat, stats = served(jobs)
        entry = {"rate_jobs_per_s": rate, "offered_attempts_per_s": rate * mean_work,
                 "throughput": total / wall, "makespan_s": wall, "p50_latency_s": pct(lat, 50),
                 "p99_latency_s": pct(lat, 99), "peak_active": stats["peak_active"]}
        log(f"served {name}: {entry}")
        if serial:
            sw, slat = serial_run(jobs)
            entry["serial"] = {"throughput": total / sw, "makespan_s": sw, "p50_latency_s": pct(slat, 50),
                               "p99_latency_s": pct(slat, 99)}
            log(f"serial {name}: {entry['serial']}")
        out[name] = entry
    return {"jobs": n_jobs, "capacity_attempts_per_s": capacity, "rates": out}


def run_serve_workload(args):
    r = serve_measure(args.jobs, args.rate, serial=not args.no_serial)
    main_entry = r["rates"]["stated"]
    result = {
        "metric": "site-replica move attempts/s (1 GPU); p50/p99 job latency served",
        "value": main_entry["throughput"],
        "unit": "site-replica move attempts/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": main_entry["makespan_s"] * 1000.0,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{args.jobs} Poisson-arriving jobs (rate {args.rate}/s, seed 5) from the 256-instance "
                               "size mix, sweeps log-uniform in [10^2, 10^4], observations on a log grid, "
                               "continuous batching with admission by device footprint",
                   "jobs": args.jobs},
        "serving": r["rates"],
        "capacity_attempts_per_s": r["capacity_attempts_per_s"],
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cubic128", choices=sorted(WORKLOADS) + ["batch256", "serve"])
    ap.add_argument("--timing-every", type=int, default=0,
                    help="also bracket every k-th class-pass launch with HIP events (each bracket adds "
                         "the events' own stream time to that launch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweeps", type=int, default=None,
                    help="override the sweeps per job (profiling runs only; the default is the workload's)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB, so that a "
                         "hardware-counter run can scale HBM byte counters by a kernel of known traffic")
    ap.add_argument("--calibrate-alu", action="store_true",
                    help="also time register-only VALU chains (v_xor_b32, v_mad_u64_u32) on the whole "
                         "device and report their issue rates under \"calibration\"")
    ap.add_argument("--plane-streams", action="store_true",
                    help="lattice workloads: run the word planes on two streams of each sim's own "
                         "(KA_OPT_PLANE_STREAMS=1) instead of one launch per class pass")
    ap.add_argument("--no-serial", action="store_true", help="batch workload: skip the one-at-a-time baseline")
    ap.add_argument("--solo-bytes", type=int, default=32 << 20,
                    help="batch workload: KA_BOPT_SOLO_BYTES (members whose n and f take at least this many "
                         "bytes run one at a time inside the batch; 0: all in the step kernel)")
    ap.add_argument("--no-extras", action="store_true",
                    help="cubic128: skip the batch256 and serve figures after the headline")
    ap.add_argument("--replicas", type=int, default=None, help="override the replica count (exploration only)")
    ap.add_argument("--jobs", type=int, default=200, help="serve workload: jobs in the trace")
    ap.add_argument("--rate", type=float, default=200.0, help="serve workload: mean arrivals per second")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (use --gpus 1). The replica planes of a job would shard "
              "across GPUs with no communication, but no multi-GPU path is implemented.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch256":
        run_batch_workload(args)
        return
    if args.workload == "serve":
        run_serve_workload(args)
        return

    import torch
    from paper_1710_05155_amd import ka

    w = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if w["kind"] == "lattice":
        g = ka.ka_graph_lattice(w["d"], w["L"])
    else:
        g = ka.ka_graph_rrg(w["N"], w["z"], w["graph_seed"])
    if args.sweeps is not None:
        w = dict(w, sweeps=args.sweeps)
    if args.replicas is not None:
        w = dict(w, R=args.replicas, desc=w["desc"] + f" [replicas overridden: {args.replicas}]")
    N, R, sweeps = g.N, w["R"], w["sweeps"]
    if args.calibrate_copy_mib > 0:
        # A plain device-to-device copy (rocclr copyBuffer) and fill of known size: the scale
        # for hardware byte counters, and the box's practical streaming rates.
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nbytes} bytes read + {nbytes} bytes written")
        # rates: the mean over 20 back-to-back operations, best of 3 rounds (below 256 MiB per
        # buffer pair the data stays in the Infinity Cache between operations)
        best = {"copy": float("inf"), "fill": float("inf")}
        reps = 20
        for _ in range(3):
            for kind in ("copy", "fill"):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    if kind == "copy":
                        dst.copy_(src)
                    else:
                        dst.fill_(7)
                b.record()
                torch.cuda.synchronize()
                best[kind] = min(best[kind], a.elapsed_time(b) / 1000.0 / reps)
        log(f"calibration rates: copy {2 * nbytes / best['copy'] / 1e12:.2f} TB/s (read + write), "
            f"fill {nbytes / best['fill'] / 1e12:.2f} TB/s")
        del src, dst
    W = R // 64
    grid = obs_grid(w)

    pass_ms_total = 0.0
    pass_timed = 0
    pass_launches = 0
    run_events = []

    def job(step_idx, timed):
        rho = w["rhos"][step_idx % len(w["rhos"])]
        sim = ka.ka_init(g, w["m"], rho, 1, R, stream=stream)
        if args.timing_every > 0:
            ka.ka_set_option(sim, ka.KA_OPT_TIMING, args.timing_every)
        if args.plane_streams:
            ka.ka_set_option(sim, ka.KA_OPT_PLANE_STREAMS, 1)
        if timed:
            evs = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            evs[0].record(stream)
        dens, ov, pers = ka.ka_run(sim, grid)
        if timed:
            evs[1].record(stream)
            run_events.append(evs)
        K = sim.K
        assert (dens == K).all(), "particle number not conserved"
        C, chi4, P = ka.ka_derived(N, K, ov, pers)
        stats = ka.ka_timing(sim)
        path = ka.ka_sim_path(sim)
        sim.free()
        return rho, C, chi4, P, stats, path

    for k in range(args.warmup):
        rho, C, chi4, P, _, _ = job(k, False)
        log(f"warmup {k}: rho={rho} C(t_max)={C[-1]:.4f} P(t_max)={P[-1]:.4f}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    path = None
    for k in range(args.steps):
        rho, C, chi4, P, (launches, timed, ms), path = job(args.warmup + k, True)
        pass_launches += launches
        pass_timed += timed
        pass_ms_total += ms
        log(f"step {k}: rho={rho} C(t_max)={C[-1]:.4f} chi4_max={max(chi4[1:]):.3f} P(t_max)={P[-1]:.4f} "
            f"passes={launches}")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    run_ms = sum(a.elapsed_time(b) for a, b in run_events)

    # Observation cost on its own: the same number of observations of a fresh state with no
    # sweeps in between, timed the same way.  Subtracted from the sweep loops' stream time
    # it leaves the time of the class passes (kernels and the gaps between them).
    sim = ka.ka_init(g, w["m"], w["rhos"][0], 1, R, stream=stream)
    torch.cuda.synchronize()
    oa, ob = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    oa.record(stream)
    ka.ka_run(sim, [0] * len(grid))
    ob.record(stream)
    torch.cuda.synchronize()
    obs_ms = oa.elapsed_time(ob)
    sim.free()
    sweep_ms = run_ms - args.steps * obs_ms

    attempts = N * R * sweeps * args.steps
    value = attempts / wall
    edges = (N * g.z // 2)
    result = {
        "metric": "site-replica move attempts/s (1 GPU)",
        "value": value,
        "unit": "site-replica move attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1000.0 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "sites": N, "replicas": R, "sweeps_per_step": sweeps,
                   "observations_per_step": len(grid), "path": {1: "global class passes", 2: "LDS-resident"}[path],
                   "plane_streams": bool(args.plane_streams)},
        "edge_replica_updates_per_s": edges * R * sweeps * args.steps / wall,
        "stream_event_ms": gpu_ms,
        "rate_excluding_observe": attempts / (sweep_ms / 1000.0) if path == 1 else None,
        "observe_ms_per_step": obs_ms,
    }
    B = class_pass_bytes(w, N, W)
    B16 = class_pass_bytes(w, N, W, with_moved_ever=True)
    kernel = "k_pass_lattice"
    if w["kind"] != "lattice":
        adj, eu, ev, ec = ka.ka_graph_export(g)
        B = graph_bytes_model(adj, eu, ev, ec, g.C, g.z, W) / g.C
        B16 = None
        kernel = "k_pass_graph"
    if path == 1 and pass_launches > 0 and B:
        # B is one class step over all word planes; a lattice sim with two or more planes
        # launches one kernel per plane and class step (on two streams, overlapping), so the
        # bytes of one launch are the step's bytes over the launches per step
        class_steps = sweeps * g.C * args.steps
        per_launch = class_steps / pass_launches
        B = B * per_launch
        avg_s = sweep_ms / pass_launches / 1000.0
        achieved = B / avg_s / 1e9
        csrc = os.path.join(ROOT, "paper_1710_05155_amd", "csrc")
        traffic = valu = trace_us = None
        cfile = None
        counters = {"cubic128": "k_pass_lattice_cubic128.counters.txt",
                    "cubic256": "k_pass_lattice_cubic256.counters.txt",
                    "rrg20": "k_pass_graph_rrg20.counters.txt"}.get(args.workload)
        expected_R = {"cubic128": 256, "cubic256": 256, "rrg20": 64}.get(args.workload)
        if counters and R == expected_R and not args.plane_streams and sweeps == WORKLOADS[args.workload]["sweeps"]:
            # kernels, and the host code that chooses the launches (plane groups, chunk order)
            srcs = [os.path.join(csrc, f) for f in ("ka_device.h", "ka_pass.hip", "ka_host.cpp")]
            if w["kind"] != "lattice":
                srcs.append(os.path.join(csrc, "ka_plan.cpp"))   # the graph's device numbering
            cfile = os.path.join(ROOT, "profiles", counters)
            traffic = measured_traffic(srcs, cfile)
            valu = measured_traffic(srcs, cfile, key="valu_busy_pct")
            trace_us = measured_traffic(srcs, cfile, key="trace_avg_launch_us")
        result["roofline"] = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_source": (f"profiles/{os.path.basename(cfile)}: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE "
                               "runs, scaled by a plain copy's counts; null when the kernel sources no "
                               "longer hash to the ones counted") if traffic is not None else None,
            "valu_busy_pct": valu, "kernel": kernel, "avg_launch_us": avg_s * 1e6,
            "bytes_per_launch": B,
            "byte_model": ("12 B per site-word: every site's words read once, the endpoints' written"
                           if w["kind"] == "lattice" else
                           "per class: touched sites x 8 B per word + records + neighbour lists + endpoint "
                           "writes and moved-ever reads"),
            "launches": pass_launches,
            "sampled_launch_us": pass_ms_total / pass_timed * 1000.0 if pass_timed else None}
        if trace_us:
            # the same figure from the committed rocprofv3 kernel trace of this command
            result["roofline"]["trace_avg_launch_us"] = trace_us
            result["roofline"]["trace_frac"] = B / (trace_us / 1e6) / 1e9 / HBM_PEAK_GBS
        if B16:
            b16 = B16 * per_launch
            result["roofline"]["with_moved_ever_reads"] = {
                "bytes_per_launch": b16, "achieved": b16 / avg_s / 1e9,
                "frac": b16 / avg_s / 1e9 / HBM_PEAK_GBS,
                "model": "16 B per site-word: also a moved-ever read at every endpoint"}
        if w["kind"] == "lattice":
            # For comparison only: the floor of a schedule that would read and write each n word
            # once per sweep (all classes fused), 16 B per 64 site-replica attempts.
            floor_gbs = (attempts / (sweep_ms / 1000.0)) * 0.25 / 1e9
            result["roofline"]["fused_floor"] = {"bytes_per_attempt": 0.25, "achieved": floor_gbs,
                                                 "frac": floor_gbs / HBM_PEAK_GBS}
    if args.calibrate_alu:
        cal = {}
        for kind, name in ((0, "v_xor_b32"), (1, "v_mad_u64_u32")):
            ips, lops = ka.ka_probe_valu(kind, stream=stream)
            cal[name] = {"wave_instr_per_s": ips, "lane_ops_per_s": lops}
            log(f"calibration {name}: {ips:.4g} wave instructions/s, {lops:.4g} lane ops/s")
        result["calibration"] = cal
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(w)
    if args.workload == "cubic128" and not args.no_extras and args.sweeps is None and args.replicas is None:
        # After the headline's timed region: the same pass beyond the Infinity Cache (3D
        # L=256), then the batched and served forms against one job at a time on the same GPU
        # (their own workloads: --workload cubic256 / batch256 / serve).
        log("extra: 3D L=256 (state beyond the Infinity Cache) ...")
        result["hbm_regime"] = hbm_regime_measure(stream)
        log("extra: batch of 256 uneven instances ...")
        b = batch_measure(1, 1)
        result["batch256"] = {
            "value": b["value"], "unit": b["unit"], "ms_per_batch": b["ms_per_batch"],
            "one_at_a_time_value": b["one_at_a_time"]["value"], "one_at_a_time_ms": b["one_at_a_time"]["ms"],
            "speedup_vs_one_at_a_time": b["speedup_vs_one_at_a_time"], "launch_shape": b["launch_shape"],
            "solo_members": b["solo_members"],
            "config": "256 uneven instances (2D L 32-512, 3D L 16-128, RRG N 2^12-2^18 z 3-5), 64 replicas, "
                      f"1000 sweeps each; the {b['solo_members']} whose n and f take 32 MiB or more run one at a "
                      "time inside the batch; 1 warm-up batch, 1 timed"}
        log(f"extra: serving trace of {args.jobs} jobs ...")
        sv = serve_measure(args.jobs, args.rate)
        result["serve"] = {
            name: {"rate_jobs_per_s": e["rate_jobs_per_s"], "throughput": e["throughput"],
                   "p50_latency_s": e["p50_latency_s"], "p99_latency_s": e["p99_latency_s"],
                   "serial_throughput": e["serial"]["throughput"],
                   "serial_p50_latency_s": e["serial"]["p50_latency_s"],
                   "serial_p99_latency_s": e["serial"]["p99_latency_s"]}
            for name, e in sv["rates"].items()}
        result["serve"]["jobs"] = sv["jobs"]
        result["serve"]["capacity_attempts_per_s"] = sv["capacity_attempts_per_s"]
        result["serve"]["config"] = (f"{args.jobs} Poisson-arriving jobs (seed 5) from the 256-instance mix, "
                                     "sweeps log-uniform in [10^2, 10^4], at the stated rate and at half the "
                                     "measured capacity")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
