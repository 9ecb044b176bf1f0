#!/usr/bin/env python3
"""Throughput of the multi-objective Digital Annealer on the bi-objective QAP.

One bench step is one pass of the whole hot path over one batch: for every
instance of the workload, all replicas start from random bits, run every
annealing step (energy differences of both objectives for all m bits,
acceptance with the dynamic offset, choice of one flip, field update, archive
update; Algorithm 3 with Eqs. cale, pacceptms), the per-replica non-dominated
flags are computed and the merged non-dominated archive of each instance is
copied to the host.  The QUBO operands are built once, before the timed region.

Metric: bit-trials/s = sum over instances of replicas * m * annealing steps,
divided by the wall time of the step.  The plain GPU form (one launch per
annealing step, replica state in HBM) runs the same workload beside it, and
the oracle is timed on a bounded sample on the host's cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

# Workloads: (n, rho values, seed config, replicas, annealing steps, path, structured)
WORKLOADS = {
    # the headline: three n = 50 instances (2500 bits), correlations -0.75, 0, 0.75,
    # 4096 replicas x 1e5 steps each, Kronecker field updates, one batched launch
    "bqap-n50-x3-kron": dict(n=50, rhos=(-0.75, 0.0, 0.75), cfg=2, replicas=4096, steps=100_000,
                             path="kron", structured=True),
    "bqap-n25-kron": dict(n=25, rhos=(0.75,), cfg=1, replicas=1024, steps=100_000, path="kron",
                          structured=True),
    "bqap-n25-dense": dict(n=25, rhos=(0.75,), cfg=1, replicas=1024, steps=100_000, path="dense",
                           structured=True),
    "bqap-n8-dense": dict(n=8, rhos=(0.0,), cfg=0, replicas=16, steps=10_000, path="dense",
                          structured=False),
}

# K objectives on a generic QUBO (the extension beyond two objectives): K dense
# upper-triangular matrices from synth.make_gqubo, default schedule scaled to
# max|C|, one wave per replica, one persistent launch
GENERIC = {
    "gqubo-k3-m1024": dict(K=3, m=1024, density=0.05, rho=0.0, seed=3, replicas=1024, steps=200_000),
}

# Peak of plain 32-bit integer VALU work: 256 CUs x 4 SIMDs x 16 lanes per clock
# x 2.4 GHz (a wave64 VALU instruction occupies a 16-lane SIMD for 4 clocks).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# MI355X HBM3E bandwidth (vendor figure), GB/s
HBM_PEAK_GBS = 8000.0

OPMODEL_PATH = os.path.join(ROOT, "paper_2205_13399_amd", "opmodel.json")


def load_opmodel() -> dict:
    """The algorithmic op model (versioned file): lane-ops per bit-trial, per
    moved bit and per random block."""
    with open(OPMODEL_PATH) as f:
        return json.load(f)


def alu_roofline(opm, bit_trials, m, moves, rng_blocks, kernel_ms, kernel="k_persistent", traffic=None):
    ops = (opm["ops"]["per_bit_trial"] * bit_trials + opm["ops"]["per_move_bit"] * m * moves
           + opm["ops"]["per_random_block"] * 64 * rng_blocks)
    achieved = ops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "TOP/s",
            "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic, "kernel": kernel,
            "kernel_ms": round(kernel_ms, 3), "ops_per_launch": int(ops), "opmodel_version": opm["version"]}


def hbm_roofline_dense(m, moves, kernel_ms, traffic=None):
    """Dense update path: each move streams the flipped bit's row of P_1 and
    P_2 restricted to the m bits, 2 x 4 B per bit (8 B per bit-trial that
    moves)."""
    nbytes = 8.0 * m * moves
    achieved = nbytes / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": "k_persistent",
            "kernel_ms": round(kernel_ms, 3), "algorithmic_bytes_per_launch": int(nbytes)}


# sources of each measured kernel (the per-tile translation units only name a tile)
KERNEL_SOURCES = {
    "k_persistent": ("paper_2205_13399_amd/csrc/mda_wave.h", "paper_2205_13399_amd/csrc/mda_wave_tile.h",
                     "paper_2205_13399_amd/csrc/mda_device.h", "paper_2205_13399_amd/csrc/mda_desc.h"),
    "k_generic": ("paper_2205_13399_amd/csrc/mda_generic.h", "paper_2205_13399_amd/csrc/mda_generic_tile.h",
                  "paper_2205_13399_amd/csrc/mda_device.h"),
}


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash(kernel: str = "k_persistent") -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str = "k_persistent"):
    """HBM bytes per launch of a kernel from the committed counter summary, or
    None when there is none or the kernel source has changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != kernel_source_hash(kernel):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_instances(w):
    out = []
    for idx, rho in enumerate(w["rhos"]):
        seed = 0 if w["cfg"] == 0 else synth.instance_seed(w["cfg"], idx)
        out.append(synth.make_instance(w["n"], rho, seed, structured=w["structured"]))
    return out


# ---------------------------------------------------------------- oracle leg

def _pin_worker(cores, counter):
    """Pins this oracle worker process to one host core of its own."""
    with counter.get_lock():
        k = counter.value
        counter.value += 1
    try:
        os.sched_setaffinity(0, {cores[k % len(cores)]})
    except (AttributeError, OSError):
        pass


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_job(args):
    import oracle
    (n, F1, F2, D, r, steps, seed) = args
    F1 = np.frombuffer(F1, np.int32).reshape(n, n)
    F2 = np.frombuffer(F2, np.int32).reshape(n, n)
    D = np.frombuffer(D, np.int32).reshape(n, n)
    q = oracle.Qubo(F1, F2, D, 0)
    d0, df, xi, beta = oracle.default_schedule(q.maxabs_c, steps)
    t0 = time.perf_counter()
    res = oracle.run_replica(q, r, steps, d0, df, xi, beta, seed)
    dt = time.perf_counter() - t0
    return r, dt, (res["E1"], res["E2"], res["Eoff"], res["moves"], res["arch_size"],
                   res["arch_e1"].tobytes(), res["arch_e2"].tobytes())


def cpu_baseline(inst, steps, replicas, cores):
    """The oracle, unmodified, on a sample of replicas: one process per replica,
    each worker pinned to a host core of its own."""
    import multiprocessing as mp
    jobs = [(inst.n, inst.F1.tobytes(), inst.F2.tobytes(), inst.D.tobytes(), r, steps, inst.seed)
            for r in replicas]
    ctx = mp.get_context("spawn")
    avail = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else list(range(os.cpu_count() or 1))
    counter = ctx.Value("i", 0)
    t0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_pin_worker, initargs=(avail[:cores], counter)) as pool:
        res = pool.map(_oracle_job, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    return wall, {r: (dt, out) for r, dt, out in res}


# ---------------------------------------------------------------- serving

SERVE = dict(count=48, n_lo=10, n_hi=100, replicas=256, steps=50_000, config=4)


def serving_measure(mda, w, factors=(0.5, 0.9, 1.2)):
    """Poisson stream of bQAP solves through the serving engine: the saturated
    rate first (everything submitted at once), then arrivals at the given
    multiples of it; per-request latency (submission to results on the
    device) and throughput."""
    import threading
    insts = synth.mixed_batch(count=w["count"], n_lo=w["n_lo"], n_hi=w["n_hi"], config=w["config"])
    params = [mda.make_params(w["replicas"], w["steps"], i.seed) for i in insts]
    srv = mda.Server(max_inflight=4)

    def run_stream(gaps):
        infos = [None] * len(insts)
        tickets = [None] * len(insts)
        ready = threading.Semaphore(0)

        def collect():
            for k in range(len(insts)):
                ready.acquire()
                _, infos[k] = srv.wait(tickets[k], keep=False)
        th = threading.Thread(target=collect)
        th.start()
        start = time.perf_counter()
        due = 0.0
        for k, inst in enumerate(insts):
            due += gaps[k]
            delay = start + due - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets[k] = srv.submit(inst.F1, inst.F2, inst.D, params[k])
            ready.release()
        th.join()
        lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
        span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
        bt = sum(i["bit_trials"] for i in infos)
        return dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    mean_s=float(lat.mean()), span_s=span, bit_trials_per_s=bt / span,
                    requests_per_s=len(insts) / span,
                    mean_batch=float(np.mean([i["batch"] for i in infos])))

    # warm-up: compile paths and fill the memory pool
    _log("serving: warm-up")
    t = srv.submit(insts[0].F1, insts[0].F2, insts[0].D, mda.make_params(8, 1000, 1))
    srv.wait(t, keep=False)
    _log("serving: saturated (%d requests at once)" % len(insts))
    sat = run_stream(np.zeros(len(insts)))
    rates = {"saturated": sat}
    rng = np.random.default_rng(w["config"])
    for f in factors:
        lam = f * sat["requests_per_s"]
        _log("serving: Poisson arrivals at %.2f requests/s (%.1f x saturated)" % (lam, f))
        res = run_stream(rng.exponential(1.0 / lam, len(insts)))
        res["arrival_rate"] = lam
        rates["%.1fx" % f] = res
        _log("serving: p50 %.3f s, p99 %.3f s, %.3g bit-trials/s" % (res["p50_s"], res["p99_s"],
                                                                   res["bit_trials_per_s"]))
    srv.close()
    return rates, insts


def serve_config(w, insts):
    return {"workload": "bqap-serve-n10-100", "requests": len(insts), "n": [w["n_lo"], w["n_hi"]],
            "replicas": w["replicas"], "anneal_steps": w["steps"], "path": "automatic (Kronecker)",
            "arrivals": "all at once (saturated), then Poisson at the stated multiples of the saturated rate",
            "server": "admission by device footprint, up to 4 launches in flight"}


def serve_bench(args, mda):
    w = dict(SERVE)
    if args.anneal_steps:
        w["steps"] = args.anneal_steps
    if args.replicas:
        w["replicas"] = args.replicas
    if args.serve_requests:
        w["count"] = args.serve_requests
    rates, insts = serving_measure(mda, w)
    sat = rates["saturated"]
    out = {
        "metric": "bit-trials/s", "value": sat["bit_trials_per_s"], "unit": "bit-trials/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(sat["span_s"] * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": serve_config(w, insts),
        "latency": rates,
    }
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- runs and legs

def timed_launches(mda, qs, params, steps, warmup, label):
    """warmup untimed, then steps timed bench steps of one batched launch of
    qs (plus the merged front of each run copied to the host)."""
    import torch

    def one_step():
        runs = mda.da_run_batch(qs, params)
        fronts = [r.archive(-1, bits=False) for r in runs]
        return runs, fronts

    for k in range(warmup):
        runs, _ = one_step()
        _log("%s warmup %d: kernel %.1f ms" % (label, k, runs[0].kernel_ms()))
        for r in runs:
            r.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms, ems, runs_last, fronts_last, stats = [], [], None, None, None
    for k in range(steps):
        if runs_last:
            # done with the previous step: its device memory goes back to the pool
            for r in runs_last:
                r.close()
        runs, fronts = one_step()
        kms.append(runs[0].kernel_ms())
        ems.append(runs[0].elapsed_ms())
        stats = [r.stats() for r in runs]
        runs_last, fronts_last = runs, fronts
        _log("%s step %d: kernel %.1f ms, launch %.1f ms" % (label, k, kms[-1], ems[-1]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(wall=wall, kernel_ms=float(np.mean(kms)), launch_ms=float(np.mean(ems)), runs=runs_last,
                fronts=fronts_last, stats=stats)


def plain_compare(mda, q, inst, R, steps, ref_run, ref_front, label):
    """The plain GPU form (one launch per annealing step, state in HBM) of one
    instance: wall time and whether it equals the batched launch."""
    import torch
    pp = mda.make_params(R, steps, inst.seed, variant=mda.VARIANT_PLAIN)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pr = mda.da_run(q, pp)
    fr = pr.archive(-1, bits=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    same = True
    for r in sorted({0, R // 2, R - 1}):
        a, b = pr.state(r), ref_run.state(r)
        same &= (a["E1"], a["E2"], a["moves"]) == (b["E1"], b["E2"], b["moves"])
    same &= np.array_equal(fr.e1, ref_front.e1) and np.array_equal(fr.e2, ref_front.e2)
    _log("%s plain: %.2f s, identical to the persistent launch: %s" % (label, dt, same))
    pr.close()
    return dt, bool(same)


def leg_single(mda, opm, name, steps_timed, warmup):
    """One of the single-instance workloads (n = 25 dense or Kronecker):
    persistent launch, its roofline, the plain form beside it."""
    w = WORKLOADS[name]
    R, steps, n = w["replicas"], w["steps"], w["n"]
    m = n * n
    path = mda.PATH_KRON if w["path"] == "kron" else mda.PATH_DENSE
    insts = make_instances(w)
    qs = [mda.Qubo(i.F1, i.F2, i.D, path=path) for i in insts]
    params = [mda.make_params(R, steps, i.seed) for i in insts]
    res = timed_launches(mda, qs, params, steps_timed, warmup, name)
    bt = len(insts) * R * m * steps
    moves = sum(s["moves"] for s in res["stats"])
    rngb = sum(s["rng_blocks"] for s in res["stats"])
    traffic = measured_traffic(name)
    if path == mda.PATH_DENSE:
        roof = hbm_roofline_dense(m, moves, res["kernel_ms"], traffic)
        roof["note"] = ("P_1 and P_2 of n = 25 hold %.1f MB on the device, which stays in the L2 caches "
                        "(4 MB per XCD) and the 256 MB MALL: the rows stream from cache, not HBM"
                        % (qs[0].info().device_bytes / 1e6))
        roof["alu"] = alu_roofline(opm, bt, m, moves, rngb, res["kernel_ms"])
    else:
        roof = alu_roofline(opm, bt, m, moves, rngb, res["kernel_ms"], traffic=traffic)
    value = bt * steps_timed / res["wall"]
    dt, same = plain_compare(mda, qs[0], insts[0], R, steps, res["runs"][0], res["fronts"][0], name)
    out = {"value": value, "unit": "bit-trials/s", "steps": steps_timed, "warmup": warmup,
           "ms_per_step": round(res["wall"] * 1e3 / steps_timed, 3),
           "config": {"workload": name, "n": n, "m": m, "rho": list(w["rhos"]), "replicas": R,
                      "anneal_steps": steps, "path": w["path"]},
           "roofline": roof,
           "p_move": moves / (R * steps * len(insts)),
           "plain": {"value": R * m * steps / dt, "unit": "bit-trials/s", "identical_results": same},
           "vs_plain": round(value / (R * m * steps / dt), 3)}
    for r in res["runs"]:
        r.close()
    return out


def front_points(run):
    """Merged non-dominated front of a run: all points and the feasible ones
    (permutation matrices), as (E1, E2) = (f1, f2) pairs."""
    f = run.archive(-1, bits=True)
    pts = np.stack([f.e1, f.e2], axis=1).astype(np.float64)
    return pts, pts[f.feasible == 1]


def leg_quality(mda, name, qs_2max, runs_2max):
    """Quality of the headline runs (Sec. Performance Criteria): the same
    instances, replicas, steps and seeds run again with the Verma-Lewis
    penalty (Eqs. vermap, wvermaa); per instance and penalty, the merged
    front's size, how many of its points are permutations, and the 2-D
    hypervolume of the feasible points, normalised to [1, 2] over both
    penalties' feasible points together, reference point (2.1, 2.1)."""
    from paper_2205_13399_amd import quality
    w = WORKLOADS[name]
    R, steps = w["replicas"], w["steps"]
    insts = make_instances(w)
    qv = [mda.Qubo(i.F1, i.F2, i.D, path=mda.PATH_KRON, penalty=mda.PEN_VL) for i in insts]
    pv = [mda.make_params(R, steps, i.seed) for i in insts]
    t0 = time.perf_counter()
    runs_vl = mda.da_run_batch(qv, pv)
    for r in runs_vl:
        r.sync()
    dt = time.perf_counter() - t0
    out = []
    for k, inst in enumerate(insts):
        a_all, a_feas = front_points(runs_2max[k])
        b_all, b_feas = front_points(runs_vl[k])
        sets = [s for s in (a_feas, b_feas) if len(s)]
        norm = quality.normaliser(sets) if sets else None
        hv = lambda s: float(quality.hypervolume_2d(norm(s))) if len(s) and norm else 0.0
        out.append({"rho": inst.rho,
                    "penalty_2max": {"alpha": [int(qs_2max[k].info().alpha1), int(qs_2max[k].info().alpha2)],
                                     "front": int(len(a_all)), "feasible": int(len(a_feas)), "hv_feasible": hv(a_feas)},
                    "penalty_vl": {"alpha": [int(qv[k].info().alpha1), int(qv[k].info().alpha2)],
                                   "front": int(len(b_all)), "feasible": int(len(b_feas)), "hv_feasible": hv(b_feas)}})
        _log("quality rho %+.2f: 2max front %d (%d feasible), Verma-Lewis front %d (%d feasible, hv %.4f)"
             % (inst.rho, len(a_all), len(a_feas), len(b_all), len(b_feas), out[-1]["penalty_vl"]["hv_feasible"]))
    for r in runs_vl:
        r.close()
    return {"per_instance": out, "vl_run_s": round(dt, 3),
            "note": "hypervolume of the feasible front points, normalised over both penalties' feasible points "
                    "of the instance (the reference fronts of the paper's instances are not available)"}


BATCH = dict(count=256, n_lo=10, n_hi=60, replicas=64, steps=100_000, config=3, plain_sample=4)


def leg_batch(mda, opm, steps_timed, warmup, plain=True):
    """Configuration of many uneven instances: 256 bQAP instances, n uniform on
    {10..60}, 64 replicas x 1e5 steps each, Kronecker updates, one batched
    launch captured as a HIP graph; the plain form of a sample of instances
    (the smallest, the largest and two more) beside it."""
    import torch
    w = BATCH
    insts = synth.mixed_batch(count=w["count"], n_lo=w["n_lo"], n_hi=w["n_hi"], config=w["config"])
    qs = [mda.Qubo(i.F1, i.F2, i.D, path=mda.PATH_KRON) for i in insts]
    stream = torch.cuda.Stream()
    params = [mda.make_params(w["replicas"], w["steps"], i.seed, graph=True, stream=stream.cuda_stream)
              for i in insts]
    with torch.cuda.stream(stream):
        res = timed_launches(mda, qs, params, steps_timed, warmup, "batch")
    bt = sum(w["replicas"] * i.m * w["steps"] for i in insts)
    value = bt * steps_timed / res["wall"]
    moves = sum(s["moves"] for s in res["stats"])
    rngb = sum(s["rng_blocks"] for s in res["stats"])
    moved_bits = sum(s["moves"] * i.m for s, i in zip(res["stats"], insts))
    ops_roof = alu_roofline(opm, bt, 1, moved_bits, rngb, res["kernel_ms"], kernel="graph of k_persistent launches")
    ns = [i.n for i in insts]
    sample = sorted({int(np.argmin(ns)), int(np.argmax(ns)), 1, len(insts) // 2})[:w["plain_sample"]] if plain else []
    pl_bt, pl_s, same = 0, 0.0, True
    for k in sample:
        dt, ok = plain_compare(mda, qs[k], insts[k], w["replicas"], w["steps"], res["runs"][k], res["fronts"][k],
                               "batch instance %d (n=%d)" % (k, insts[k].n))
        pl_bt += w["replicas"] * insts[k].m * w["steps"]
        pl_s += dt
        same &= ok
    out = {"value": value, "unit": "bit-trials/s", "steps": steps_timed, "warmup": warmup,
           "ms_per_step": round(res["wall"] * 1e3 / steps_timed, 3),
           "config": {"workload": "bqap-batch-n10-60-x256", "instances": len(insts), "n": [min(ns), max(ns)],
                      "replicas": w["replicas"], "anneal_steps": w["steps"], "path": "kron",
                      "launch": "one HIP graph of persistent launches (one per register tile)",
                      "bit_trials_per_step": bt},
           "roofline": ops_roof,
           "moves": moves,
           "plain": ({"value": pl_bt / pl_s, "unit": "bit-trials/s",
                      "sample": "instances %s (n = %s), one plain run each" % (sample, [ns[k] for k in sample]),
                      "identical_results": bool(same)} if sample else None),
           "vs_plain": round(value / (pl_bt / pl_s), 3) if sample else None}
    for r in res["runs"]:
        r.close()
    return out


def _goracle_job(args):
    import oracle
    (K, m, Qb, qb, r, steps, seed) = args
    g = oracle.GQubo(np.frombuffer(Qb, np.int32).reshape(K, m, m), np.frombuffer(qb, np.int64))
    d0, df, xi, beta = oracle.gdefault_schedule(g.maxabs_c, steps)
    t0 = time.perf_counter()
    res = oracle.run_greplica(g, r, steps, d0, df, xi, beta, seed)
    dt = time.perf_counter() - t0
    return r, dt, (tuple(res["E"]), res["Eoff"], res["moves"], res["arch_size"], res["arch_e"].tobytes())


def generic_measure(mda, opm, name, steps_timed, warmup, cpu_replicas=2):
    """K objectives on a generic QUBO: timed persistent launches (each with the
    merged K-way front copied to the host), the ALU roofline of the kernel,
    and the oracle on a bounded sample (the first replicas of the workload,
    checked bit for bit against the last timed launch)."""
    import multiprocessing as mp
    import torch
    w = GENERIC[name]
    K, m, R, steps = w["K"], w["m"], w["replicas"], w["steps"]
    Q, q = synth.make_gqubo(K, m, seed=w["seed"], density=w["density"], rho=w["rho"])
    g = mda.GQubo(Q, q)
    params = mda.make_params(R, steps, w["seed"])

    def one_step():
        run = mda.gda_run(g, params)
        front = run.archive(-1, bits=False)
        return run, front

    for k in range(warmup):
        run, _ = one_step()
        _log("%s warmup %d: kernel %.1f ms" % (name, k, run.kernel_ms()))
        run.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms, run, front, last = [], None, None, None
    for k in range(steps_timed):
        if last is not None:
            last.close()
        run, front = one_step()
        kms.append(run.kernel_ms())
        last = run
        _log("%s step %d: kernel %.1f ms" % (name, k, kms[-1]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = run.stats()
    bt = R * m * steps
    kernel_ms = float(np.mean(kms))
    go = opm["generic"]
    ops = (go["per_bit_trial_per_objective"] * K * bt + go["per_move_bit_per_objective"] * K * m * st["moves"]
           + go["per_random_block"] * 64 * st["rng_blocks"])
    achieved = ops / (kernel_ms * 1e-3) / 1e12
    nbytes = go["breakdown"]["hbm_bytes_per_move_bit_per_objective"] * K * m * st["moves"]
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "TOP/s",
            "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": measured_traffic(name, "k_generic"),
            "kernel": "k_generic<%d,%d>" % (K, _slots(m, K)),
            "kernel_ms": round(kernel_ms, 3), "ops_per_launch": int(ops), "opmodel_version": opm["version"],
            "hbm": {"algorithmic_bytes_per_launch": int(nbytes),
                    "achieved_GBs": round(nbytes / (kernel_ms * 1e-3) / 1e9, 2), "peak_GBs": HBM_PEAK_GBS,
                    "note": "rows of P_k streamed per move; P_1..P_K hold %.1f MB and stay in the L2 caches and MALL"
                            % (K * m * 64 * _slots(m, K) * 4 / 1e6)}}
    out = {"value": bt * steps_timed / wall, "unit": "bit-trials/s", "steps": steps_timed, "warmup": warmup,
           "ms_per_step": round(wall * 1e3 / steps_timed, 3),
           "config": {"workload": name, "K": K, "m": m, "density": w["density"], "replicas": R, "anneal_steps": steps,
                      "launch": "persistent, one wave per replica", "bit_trials_per_step": bt},
           "roofline": roof, "p_move": st["moves"] / (R * steps), "front_size": int(len(front))}
    if cpu_replicas > 0:
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        cores = max(1, min(cpu_replicas, ncpu, 16))
        jobs = [(K, m, Q.tobytes(), q.tobytes(), r, steps, w["seed"]) for r in range(cpu_replicas)]
        ctx = mp.get_context("spawn")
        avail = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else list(range(ncpu))
        counter = ctx.Value("i", 0)
        t1 = time.perf_counter()
        with ctx.Pool(cores, initializer=_pin_worker, initargs=(avail[:cores], counter)) as pool:
            res = pool.map(_goracle_job, jobs, chunksize=1)
        cw = time.perf_counter() - t1
        exact = True
        for r, dt, o in res:
            s_ = run.state(r)
            a = run.archive(r, raw=True, bits=False)
            exact &= (tuple(s_["E"]), s_["Eoff"], s_["moves"], len(a), a.e.tobytes()) == o
        out["cpu_baseline"] = {"value": cpu_replicas * m * steps / cw, "unit": "bit-trials/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "replicas 0..%d of the workload (%d annealing steps each), one process per "
                                         "replica, each pinned to its own core, %.1f s wall"
                                         % (cpu_replicas - 1, steps, cw),
                               "bit_exact_vs_gpu": bool(exact)}
    run.close()
    return out


def _slots(m, K):
    for S in (8, 16, 32, 64):
        if 64 * S >= m and K * S <= 64:
            return S
    return 0


def copy_calibration():
    """A 1 GiB fill, then a 1 GiB device-to-device copy: known bytes for
    scaling the HBM counters."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    return {"read": a.numel() * 4, "write": b.numel() * 4}


def generic_bench(args, mda):
    name = args.workload
    opm = load_opmodel()
    leg = generic_measure(mda, opm, name, args.steps, args.warmup,
                          cpu_replicas=2 if args.cpu_replicas > 0 else 0)
    out = {"metric": "bit-trials/s", "value": leg["value"], "unit": "bit-trials/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": leg["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic"}
    out.update({k: v for k, v in leg.items() if k not in ("value", "unit", "steps", "warmup", "ms_per_step")})
    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration()
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- SB-DA vs MDA

def sbda_vs_mda(args, mda):
    """The paper's comparison on synthetic instances: MDA (strict, explore) and
    SB-DA (11 weights), 20 runs each at I_max = 0.25 m^2 steps, Verma-Lewis
    penalty for both, on the QUBOs as given and with both objectives normalised
    to one largest coefficient 2^L (Sec. Parameter Settings); per run the
    non-dominated feasible set in the true (f1, f2), normalised together, its
    hypervolume and size; and each method's throughput."""
    import torch
    from paper_2205_13399_amd import quality, sbda
    runs = args.replicas or 20
    n = 20   # the largest size at which the Verma-Lewis weight keeps every field in int32 here
    m = n * n
    steps = args.anneal_steps or int(round(0.25 * m * m))
    insts = [synth.make_instance(n, rho, seed=synth.instance_seed(5, k)) for k, rho in enumerate((-0.75, 0.0, 0.75))]
    per_inst = []
    tot = {"mda": [0, 0.0], "sbda": [0, 0.0]}
    for inst in insts:
        q = mda.Qubo(inst.F1, inst.F2, inst.D, penalty=mda.PEN_VL, path=mda.PATH_KRON)
        qn = mda.Qubo(inst.F1, inst.F2, inst.D, penalty=mda.PEN_VL, path=mda.PATH_KRON, normalise=mda.NORM_AUTO)

        def mda_runs(escape, qq=q):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run = mda.da_run(qq, mda.make_params(runs, steps, inst.seed, escape=escape))
            run.sync()
            dt = time.perf_counter() - t0
            scaled = qq.info().normalise_log2 != 0
            sets = []
            for r in range(runs):
                a = run.archive(r, raw=True, bits=scaled)
                ok = a.feasible == 1
                if not len(a) or not ok.any():
                    sets.append(np.zeros((0, 2)))
                    continue
                if scaled:   # energies in scaled units: cost the permutations in the true objectives
                    pts = np.array([(sbda.qap_cost(inst.F1, inst.D, p), sbda.qap_cost(inst.F2, inst.D, p))
                                    for p in a.perm[ok]], np.int64)
                else:
                    pts = np.stack([a.e1[ok], a.e2[ok]], axis=1)
                sets.append(pts[quality.nondominated(pts)])
            return sets, dt

        mda_sets, t_mda = mda_runs(mda.ESC_OFFSET)
        rst_sets, t_rst = mda_runs(mda.ESC_ARCHIVE)
        mdan_sets, _ = mda_runs(mda.ESC_OFFSET, qn)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = sbda.sbda(inst.F1, inst.F2, inst.D, runs, steps, inst.seed)
        t_sb = time.perf_counter() - t0
        resn = sbda.sbda(inst.F1, inst.F2, inst.D, runs, steps, inst.seed, normalise=mda.NORM_AUTO)
        sets = mda_sets + rst_sets + res.points + mdan_sets + resn.points
        qual = quality.compare([s for s in sets if len(s)] or [np.zeros((1, 2))])
        norm = quality.normaliser([s for s in sets if len(s)])
        hv = lambda ss: [quality.hypervolume_2d(norm(s)) if len(s) else 0.0 for s in ss]
        hv_m, hv_r, hv_s = hv(mda_sets), hv(rst_sets), hv(res.points)
        hv_mn, hv_sn = hv(mdan_sets), hv(resn.points)
        per_inst.append({"rho": inst.rho,
                         "mda": {"hv_mean": float(np.mean(hv_m)), "nondominated_mean": float(np.mean([len(s) for s in mda_sets])),
                                 "seconds": t_mda},
                         "mda_restart": {"hv_mean": float(np.mean(hv_r)),
                                         "nondominated_mean": float(np.mean([len(s) for s in rst_sets])), "seconds": t_rst},
                         "sbda": {"hv_mean": float(np.mean(hv_s)), "nondominated_mean": float(np.mean([len(s) for s in res.points])),
                                  "seconds": t_sb},
                         "mda_normalised": {"hv_mean": float(np.mean(hv_mn)), "log2": int(qn.info().normalise_log2),
                                            "nondominated_mean": float(np.mean([len(s) for s in mdan_sets]))},
                         "sbda_normalised": {"hv_mean": float(np.mean(hv_sn)), "log2": int(resn.normalise_log2),
                                             "nondominated_mean": float(np.mean([len(s) for s in resn.points]))}})
        tot["mda"][0] += runs * m * steps
        tot["mda"][1] += t_mda
        tot["sbda"][0] += len(res.weights) * runs * m * steps
        tot["sbda"][1] += t_sb
        _log("rho %+.2f: MDA hv %.4f (%.1f points/run, %.2f s), MDA restarting from the archive hv %.4f (%.1f), "
             "SB-DA hv %.4f (%.1f points/run, %.2f s)"
             % (inst.rho, per_inst[-1]["mda"]["hv_mean"], per_inst[-1]["mda"]["nondominated_mean"], t_mda,
                per_inst[-1]["mda_restart"]["hv_mean"], per_inst[-1]["mda_restart"]["nondominated_mean"],
                per_inst[-1]["sbda"]["hv_mean"], per_inst[-1]["sbda"]["nondominated_mean"], t_sb))
        _log("rho %+.2f normalised to 2^%d / 2^%d: MDA hv %.4f (%.1f points/run), SB-DA hv %.4f (%.1f points/run)"
             % (inst.rho, per_inst[-1]["mda_normalised"]["log2"], per_inst[-1]["sbda_normalised"]["log2"],
                per_inst[-1]["mda_normalised"]["hv_mean"], per_inst[-1]["mda_normalised"]["nondominated_mean"],
                per_inst[-1]["sbda_normalised"]["hv_mean"], per_inst[-1]["sbda_normalised"]["nondominated_mean"]))
        del qual
    out = {"metric": "bit-trials/s", "value": tot["sbda"][0] / tot["sbda"][1], "unit": "bit-trials/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": round(tot["sbda"][1] * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "sbda-vs-mda-n20", "n": n, "instances": 3, "runs": runs, "anneal_steps": steps,
                      "weights": 11, "penalty": "Verma-Lewis"},
           "mda_bit_trials_per_s": tot["mda"][0] / tot["mda"][1],
           "quality": per_inst}
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed bench steps")
    ap.add_argument("--warmup", type=int, default=1, help="untimed bench steps")
    ap.add_argument("--workload", default="bqap-n50-x3-kron",
                    choices=sorted(WORKLOADS) + sorted(GENERIC) + ["bqap-batch-n10-60-x256", "bqap-serve-n10-100",
                                                                   "sbda-vs-mda-n20"])
    ap.add_argument("--anneal-steps", type=int, default=0, help="override the workload's annealing steps")
    ap.add_argument("--replicas", type=int, default=0, help="override the workload's replicas")
    ap.add_argument("--plain", type=int, default=1, help="plain-form comparison runs (0 = none)")
    ap.add_argument("--cpu-replicas", type=int, default=16, help="oracle sample size (0 = skip)")
    ap.add_argument("--cpu-cores", type=int, default=8, help="oracle worker processes")
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 1 GiB (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=0, help="requests of the serving workload")
    ap.add_argument("--legs", type=int, default=1,
                    help="also measure the other configurations (n = 25 dense and Kronecker, the uneven batch, "
                         "serving) as legs of the JSON line (0 = headline only)")
    ap.add_argument("--leg-steps", type=int, default=2, help="timed bench steps of each leg")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the replicas of this workload are independent and would "
              "shard across GPUs with no per-step communication, but only the one-GPU path is "
              "built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2205_13399_amd import mda

    if args.workload == "bqap-serve-n10-100":
        torch.cuda.set_device(0)
        mda.use_torch_allocator()
        serve_bench(args, mda)
        return
    if args.workload in GENERIC:
        torch.cuda.set_device(0)
        mda.use_torch_allocator()
        generic_bench(args, mda)
        return
    if args.workload == "bqap-batch-n10-60-x256":
        # the uneven batch alone (its leg of the default line), e.g. for a
        # kernel trace of the graph's launches
        torch.cuda.set_device(0)
        mda.use_torch_allocator()
        leg = leg_batch(mda, load_opmodel(), args.steps, args.warmup, plain=args.plain > 0)
        line = {"metric": "bit-trials/s", "value": leg["value"], "unit": "bit-trials/s", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": leg["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
                "data": "synthetic"}
        line.update({k: v for k, v in leg.items() if k not in line})
        print(json.dumps(line))
        return
    if args.workload == "sbda-vs-mda-n20":
        torch.cuda.set_device(0)
        mda.use_torch_allocator()
        sbda_vs_mda(args, mda)
        return

    w = dict(WORKLOADS[args.workload])
    if args.anneal_steps:
        w["steps"] = args.anneal_steps
    if args.replicas:
        w["replicas"] = args.replicas
    R, steps, n = w["replicas"], w["steps"], w["n"]
    m = n * n
    path = mda.PATH_KRON if w["path"] == "kron" else mda.PATH_DENSE
    opm = load_opmodel()

    torch.cuda.set_device(0)
    mda.use_torch_allocator()
    insts = make_instances(w)
    _log("workload %s: %d instance(s) n=%d, %d replicas x %d steps, path %s"
         % (args.workload, len(insts), n, R, steps, w["path"]))
    qs = [mda.Qubo(i.F1, i.F2, i.D, path=path) for i in insts]
    params = [mda.make_params(R, steps, i.seed, waves_per_block=args.waves_per_block) for i in insts]
    tuning = None
    if not args.waves_per_block:
        # launch shape from the autotuner (probe runs, outside the timed region)
        tuning = mda.autotune(qs[0], params[0], probe_steps=2000)
        params = [mda.tuned(p, tuning) for p in params]
        _log("autotuner: %d waves per replica, %d waves per block, occupancy build %d (%s)"
             % (tuning["waves_per_replica"], tuning["waves_per_block"], tuning["occupancy"],
                ", ".join("%d/%d/%d: %.1f ms" % c for c in tuning["candidates"])))
    torch.cuda.synchronize()

    bit_trials_step = len(insts) * R * m * steps
    res = timed_launches(mda, qs, params, args.steps, args.warmup, "")
    runs_last, fronts_last = res["runs"], res["fronts"]
    wall = res["wall"]
    ms_per_step = wall * 1e3 / max(1, args.steps)
    value = bit_trials_step * args.steps / wall

    # roofline of the persistent kernel: algorithmic lane-ops per launch / kernel time
    st = res["stats"]
    moves = sum(s["moves"] for s in st)
    rng_blocks = sum(s["rng_blocks"] for s in st)
    traffic = measured_traffic(args.workload)
    if path == mda.PATH_DENSE:
        roofline = hbm_roofline_dense(m, moves, res["kernel_ms"], traffic)
    else:
        roofline = alu_roofline(opm, bit_trials_step, m, moves, rng_blocks, res["kernel_ms"], traffic=traffic)

    out = {
        "metric": "bit-trials/s", "value": value, "unit": "bit-trials/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "instances": len(insts),
                   "rho": list(w["rhos"]), "replicas": R, "anneal_steps": steps,
                   "path": w["path"], "launch": "persistent, all instances in one launch",
                   "bit_trials_per_step": bit_trials_step,
                   "launch_shape": ({"waves_per_replica": tuning["waves_per_replica"],
                                     "waves_per_block": tuning["waves_per_block"],
                                     "occupancy_build": tuning["occupancy"], "autotuned": True}
                                    if tuning else {"waves_per_block": args.waves_per_block})},
        "roofline": roofline,
        "run_stats": {"moves_per_replica": moves / (len(insts) * R),
                      "p_move": moves / (len(insts) * R * steps),
                      "rng_blocks_per_replica": rng_blocks / (len(insts) * R),
                      "archived_per_replica": sum(s["archived"] for s in st) / (len(insts) * R),
                      "front_sizes": [len(f) for f in fronts_last],
                      "front_feasible": [int(f.feasible.sum()) for f in fronts_last]},
    }

    # plain GPU form: one launch per annealing step, one instance per call
    if args.plain > 0:
        pl_bt, pl_s, same = 0, 0.0, True
        for idx in range(min(args.plain, len(insts))):
            dt, ok = plain_compare(mda, qs[idx], insts[idx], R, steps, runs_last[idx], fronts_last[idx],
                                   "instance %d" % idx)
            pl_bt += R * m * steps
            pl_s += dt
            same &= ok
        pv = pl_bt / pl_s
        out["plain"] = {"value": pv, "unit": "bit-trials/s", "instances": min(args.plain, len(insts)),
                        "launch": "one launch per annealing step, state in HBM",
                        "identical_results": bool(same)}
        out["vs_plain"] = round(value / pv, 3)

    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration()

    # the oracle on a bounded sample, on host cores (rank 0, one GPU)
    if args.cpu_replicas > 0:
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        cores = max(1, min(args.cpu_replicas, args.cpu_cores, ncpu, 16))
        sample = list(range(args.cpu_replicas))
        idx = len(insts) // 2
        inst = insts[idx]
        _log("oracle: %d replicas of instance %d on %d pinned cores" % (len(sample), idx, cores))
        cw, ores = cpu_baseline(inst, steps, sample, cores)
        exact = True
        for r, (dt, o) in ores.items():
            g = runs_last[idx].state(r)
            a = runs_last[idx].archive(r, raw=True, bits=False)
            exact &= (g["E1"], g["E2"], g["Eoff"], g["moves"], len(a)) == o[:5]
            exact &= a.e1.tobytes() == o[5] and a.e2.tobytes() == o[6]
        per_core = float(np.mean([m * steps / dt for dt, _ in ores.values()]))
        out["cpu_baseline"] = {"value": len(sample) * m * steps / cw, "unit": "bit-trials/s",
                               "cores": cores, "kind": "oracle",
                               "sample": "%d replicas x %d steps of the n=%d rho=%g instance, one process "
                                         "per replica, each pinned to its own core, %.1f s wall"
                                         % (len(sample), steps, n, inst.rho, cw),
                               "per_core": per_core, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                               "affinity_cores": ncpu, "bit_exact_vs_gpu": bool(exact)}
    # the other configurations, each a bench leg of its own
    if args.legs:
        legs = {}
        if args.workload == "bqap-n50-x3-kron":
            _log("leg quality (Verma-Lewis penalty beside 2 max|C|)")
            out["quality"] = leg_quality(mda, args.workload, qs, runs_last)
    for r in runs_last:
        r.close()
    if args.legs:
        for name in ("bqap-n25-dense", "bqap-n25-kron"):
            if name != args.workload:
                _log("leg %s" % name)
                legs[name] = leg_single(mda, opm, name, args.leg_steps, 1)
        _log("leg batch")
        legs["bqap-batch-n10-60-x256"] = leg_batch(mda, opm, args.leg_steps, 1)
        for name in GENERIC:
            _log("leg %s" % name)
            legs[name] = generic_measure(mda, opm, name, args.leg_steps, 1,
                                         cpu_replicas=2 if args.cpu_replicas > 0 else 0)
        _log("leg serving")
        sw = dict(SERVE)
        rates, sinsts = serving_measure(mda, sw, factors=(0.9,))
        legs["bqap-serve-n10-100"] = {"config": serve_config(sw, sinsts), "latency": rates,
                                      "value": rates["saturated"]["bit_trials_per_s"], "unit": "bit-trials/s",
                                      "p50_s_at_0.9x": rates["0.9x"]["p50_s"], "p99_s_at_0.9x": rates["0.9x"]["p99_s"]}
        out["legs"] = legs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
